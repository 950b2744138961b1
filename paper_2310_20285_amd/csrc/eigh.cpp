// Symmetric eigendecomposition in FP64 on the host for the B x B matrix M of
// the virtual solver run (Algorithm 3: M = U Lambda U^T, eigenvalues sorted
// in decreasing order).  B is at most a few hundred, so this O(B^3) step is
// small next to the products with K.
//
// Method (Golub & Van Loan, "Matrix Computations", Sec. 8.3):
//  1. Householder reduction to tridiagonal form T = Z^T A Z, with Z
//     accumulated backwards from the reflectors;
//  2. implicit symmetric QR steps with a Wilkinson shift on T, chasing the
//     bulge with Givens rotations that are accumulated into Z;
//  3. deflation when |e_i| <= eps (|d_i| + |d_{i+1}|).
// Z is kept column-major so that every rotation and reflector update runs
// over contiguous columns.  Host-only code (built with the host C++ compiler):
// the dot products run with four partial sums so that they vectorise.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "itergp.h"

namespace igp {

void set_error(const char* fmt, ...);
int eigh_desc(int n, const double* A, double* w_out, double* Z_out);

namespace {

// sum_i a[i] b[i] in four interleaved partial sums, added in a fixed order
inline double dot4(const double* a, const double* b, int m) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = 0;
  for (; i + 4 <= m; i += 4) {
    s0 += a[i] * b[i];
    s1 += a[i + 1] * b[i + 1];
    s2 += a[i + 2] * b[i + 2];
    s3 += a[i + 3] * b[i + 3];
  }
  for (; i < m; ++i) s0 += a[i] * b[i];
  return (s0 + s1) + (s2 + s3);
}

void tridiagonalize(int n, std::vector<double>& a, std::vector<double>& Z, std::vector<double>& d,
                    std::vector<double>& e) {
  // a: n x n row-major, full symmetric.  Reflector k (acting on indices
  // k+1..n-1) is stored in vs[k], with scale betas[k].
  std::vector<std::vector<double>> vs(n);
  std::vector<double> betas(n, 0.0), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    std::vector<double>& v = vs[k];
    v.assign(m, 0.0);
    for (int i = 0; i < m; ++i) v[i] = a[static_cast<size_t>(k + 1 + i) * n + k];
    const double sig = dot4(v.data(), v.data(), m);
    const double xnorm = std::sqrt(sig);
    if (xnorm == 0.0) continue;
    const double alpha = v[0] >= 0.0 ? -xnorm : xnorm;   // H x = alpha e_1
    v[0] -= alpha;
    const double vtv = dot4(v.data(), v.data(), m);
    if (vtv == 0.0) continue;
    const double beta = 2.0 / vtv;
    betas[k] = beta;
    // p = beta * A22 v
    for (int i = 0; i < m; ++i)
      p[i] = beta * dot4(&a[static_cast<size_t>(k + 1 + i) * n + (k + 1)], v.data(), m);
    const double ptv = dot4(p.data(), v.data(), m);
    const double c = 0.5 * beta * ptv;
    for (int i = 0; i < m; ++i) w[i] = p[i] - c * v[i];
    // A22 -= v w^T + w v^T
    for (int i = 0; i < m; ++i) {
      double* row = &a[static_cast<size_t>(k + 1 + i) * n + (k + 1)];
      const double vi = v[i], wi = w[i];
      for (int j = 0; j < m; ++j) row[j] -= vi * w[j] + wi * v[j];
    }
    a[static_cast<size_t>(k + 1) * n + k] = alpha;
    a[static_cast<size_t>(k) * n + k + 1] = alpha;
    for (int i = 1; i < m; ++i) {
      a[static_cast<size_t>(k + 1 + i) * n + k] = 0.0;
      a[static_cast<size_t>(k) * n + k + 1 + i] = 0.0;
    }
  }
  d.resize(n);
  e.assign(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = a[static_cast<size_t>(i) * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = a[static_cast<size_t>(i + 1) * n + i];
  // Z = H_0 H_1 ... H_{n-3}, accumulated from the last reflector.
  Z.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) Z[static_cast<size_t>(i) * n + i] = 1.0;
  for (int k = n - 3; k >= 0; --k) {
    if (betas[k] == 0.0) continue;
    const std::vector<double>& v = vs[k];
    const int m = n - k - 1;
    for (int j = k + 1; j < n; ++j) {
      double* col = &Z[static_cast<size_t>(j) * n + (k + 1)];
      const double s = betas[k] * dot4(v.data(), col, m);
      for (int i = 0; i < m; ++i) col[i] -= s * v[i];
    }
  }
}

inline void rotate_cols(double* zk, double* zk1, int n, double c, double s) {
  for (int i = 0; i < n; ++i) {
    const double a = zk[i], b = zk1[i];
    zk[i] = c * a + s * b;
    zk1[i] = -s * a + c * b;
  }
}

// One implicit QR step with Wilkinson shift on the unreduced block [l, m].
void qr_step(int n, int l, int m, std::vector<double>& d, std::vector<double>& e,
             std::vector<double>& Z) {
  const double dd = 0.5 * (d[m - 1] - d[m]);
  const double em = e[m - 1];
  const double den = dd + std::copysign(std::sqrt(dd * dd + em * em), dd == 0.0 ? 1.0 : dd);
  const double mu = den != 0.0 ? d[m] - em * em / den : d[m] - std::fabs(em);
  double x = d[l] - mu, z = e[l];
  double bulge = 0.0;
  for (int k = l; k < m; ++k) {
    if (k > l) {
      x = e[k - 1];
      z = bulge;
    }
    const double r = std::sqrt(x * x + z * z);   // entries far from overflow
    double c = 1.0, s = 0.0;
    if (r != 0.0) {
      c = x / r;
      s = z / r;
    }
    if (k > l) e[k - 1] = r;
    const double a = d[k], b = e[k], cc = d[k + 1];
    d[k] = c * c * a + 2.0 * c * s * b + s * s * cc;
    d[k + 1] = s * s * a - 2.0 * c * s * b + c * c * cc;
    e[k] = c * s * (cc - a) + (c * c - s * s) * b;
    if (k + 1 < m) {
      bulge = s * e[k + 1];
      e[k + 1] = c * e[k + 1];
    }
    rotate_cols(&Z[static_cast<size_t>(k) * n], &Z[static_cast<size_t>(k + 1) * n], n, c, s);
  }
}

}  // namespace

int eigh_desc(int n, const double* A, double* w_out, double* Z_out) {
  if (n <= 0) return IGP_OK;
  std::vector<double> a(static_cast<size_t>(n) * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      const double v = A[static_cast<size_t>(i) * n + j];
      a[static_cast<size_t>(i) * n + j] = v;
      a[static_cast<size_t>(j) * n + i] = v;
    }
  std::vector<double> Z, d, e;
  tridiagonalize(n, a, Z, d, e);
  const double eps = 2.220446049250313e-16;
  int iter = 0;
  const int max_iter = 60 * n + 100;
  int hi = n - 1;
  while (hi > 0) {
    for (int i = 0; i < hi; ++i)
      if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
    while (hi > 0 && e[hi - 1] == 0.0) --hi;
    if (hi == 0) break;
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    if (++iter > max_iter) {
      set_error("symmetric eigensolver did not converge (n = %d)", n);
      return IGP_EDEVICE;
    }
    qr_step(n, lo, hi, d, e, Z);
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return d[i] > d[j]; });
  for (int k = 0; k < n; ++k) {
    w_out[k] = d[order[k]];
    std::copy(&Z[static_cast<size_t>(order[k]) * n], &Z[static_cast<size_t>(order[k]) * n] + n,
              Z_out + static_cast<size_t>(k) * n);
  }
  return IGP_OK;
}

}  // namespace igp
