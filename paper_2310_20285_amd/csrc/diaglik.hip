// Likelihoods whose negative Hessian W(f) is diagonal, elementwise over the
// n = N C latent values (CN-ordering):
//
//   Poisson, log link (appendix on the Poisson log likelihood):
//     grad = y - exp(f),  W^{-1} = diag(exp(-f)),
//     log p = y f - exp(f) - log(y!)
//   Gaussian, observation variance s2 (the conjugate case):
//     grad = (y - f) / s2,  W^{-1} = s2 I,
//     log p = -(y - f)^2 / (2 s2) - log(2 pi s2) / 2
//
// The Newton step's pseudo-targets are yhat - m = f + W^{-1} grad (section 3.1
// with m = 0): f + y exp(-f) - 1 for Poisson, y for Gaussian.  The update
// statistics below also serve the block likelihood (no y; log p left NaN).
#include "iter_ops.hpp"

namespace igp {
namespace {

constexpr int NTD = 256;

template <typename T>
__device__ inline double target(int lik, const void* y, int64_t i) {
  return lik == IGP_LIK_GAUSSIAN ? static_cast<double>(static_cast<const T*>(y)[i])
                                 : static_cast<double>(static_cast<const int32_t*>(y)[i]);
}

template <typename T>
__global__ void __launch_bounds__(NTD)
k_diag_begin(int lik, const T* __restrict__ f, const void* __restrict__ y, int64_t n, double s2,
             T* __restrict__ winv, T* __restrict__ rhs) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(NTD) + threadIdx.x;
  if (i >= n) return;
  const double fi = static_cast<double>(f[i]);
  const double yi = target<T>(lik, y, i);
  if (lik == IGP_LIK_POISSON) {
    const double e = exp(-fi);
    winv[i] = static_cast<T>(e);
    rhs[i] = static_cast<T>(fi + yi * e - 1.0);
  } else {
    winv[i] = static_cast<T>(s2);
    rhs[i] = static_cast<T>(yi);
  }
}

// Out[:, b] = winv .* V[:, b] (+ Add[:, b])
template <typename T>
__global__ void __launch_bounds__(NTD)
k_diag_apply(const T* __restrict__ winv, int64_t n, const T* __restrict__ V, int64_t ldv,
             const T* __restrict__ Add, int64_t lda, T* __restrict__ Out, int64_t ldo,
             const int* gate) {
  if (gate_closed(gate)) return;
  const int64_t i = blockIdx.x * static_cast<int64_t>(NTD) + threadIdx.x;
  if (i >= n) return;
  iter::winv_diag<T>(winv, i, V, blockIdx.y, ldv, Add, lda, Out, ldo);
}

template <typename T>
__global__ void __launch_bounds__(NTD)
k_diag_stats(int lik, double s2, const T* __restrict__ fnew, const T* __restrict__ f,
             const T* __restrict__ v, const void* __restrict__ y, int64_t n,
             double* __restrict__ part) {
  __shared__ double red[NTD / 64];
  const int64_t i = blockIdx.x * static_cast<int64_t>(NTD) + threadIdx.x;
  double dd = 0.0, ff = 0.0, ll = 0.0, gv = 0.0;
  if (i < n) {
    const double a = static_cast<double>(fnew[i]);
    const double b = static_cast<double>(f[i]);
    dd = (a - b) * (a - b);
    ff = a * a;
    gv = a * static_cast<double>(v[i]);
    if (lik == IGP_LIK_POISSON) {
      const double yi = target<T>(lik, y, i);
      ll = yi * a - exp(a) - lgamma(yi + 1.0);
    } else if (lik == IGP_LIK_GAUSSIAN) {
      const double r = target<T>(lik, y, i) - a;
      ll = -0.5 * r * r / s2 - 0.5 * log(2.0 * 3.14159265358979323846 * s2);
    } else {
      ll = __builtin_nan("");   // block likelihood: log p is the caller's
    }
  }
  const int nb = gridDim.x;
  double s;
  s = block_sum(dd, red); if (threadIdx.x == 0) part[0 * nb + blockIdx.x] = s;
  s = block_sum(ff, red); if (threadIdx.x == 0) part[1 * nb + blockIdx.x] = s;
  s = block_sum(ll, red); if (threadIdx.x == 0) part[2 * nb + blockIdx.x] = s;
  s = block_sum(gv, red); if (threadIdx.x == 0) part[3 * nb + blockIdx.x] = s;
}

// sums rows r < 4 of part (nblk entries each, fixed order) into out[slot[r]]
__global__ void __launch_bounds__(NTD)
k_diag_finish(const double* __restrict__ part, int nblk, double* __restrict__ scal) {
  __shared__ double red[NTD / 64];
  const int slots[4] = {SC_DIFF2, SC_FNEW2, SC_LOGLIK, SC_GV};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += NTD) s += part[r * nblk + b];
    s = block_sum(s, red);
    if (threadIdx.x == 0) scal[slots[r]] = s;
    __syncthreads();
  }
}

__global__ void k_check_counts(const int32_t* __restrict__ y, int64_t n, int* bad) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    if (y[i] < 0) atomicAdd(bad, 1);
}

template <typename T>
__global__ void k_check_finite(const T* __restrict__ y, int64_t n, int* bad) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    if (!isfinite(static_cast<double>(y[i]))) atomicAdd(bad, 1);
}

}  // namespace

template <typename T>
int diag_begin(int lik, const T* f, const void* y, int64_t n, double s2, T* winv, T* rhs,
               hipStream_t s) {
  if (n == 0) return IGP_OK;
  k_diag_begin<T><<<static_cast<unsigned>(ceil_div(n, NTD)), NTD, 0, s>>>(lik, f, y, n, s2, winv,
                                                                          rhs);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int diag_apply(const T* winv, int64_t n, const T* V, int64_t nb, int64_t ldv, const T* Add,
               int64_t lda, T* Out, int64_t ldo, hipStream_t s, const int* gate) {
  if (n == 0 || nb == 0) return IGP_OK;
  dim3 grid(static_cast<unsigned>(ceil_div(n, NTD)), static_cast<unsigned>(nb));
  k_diag_apply<T><<<grid, NTD, 0, s>>>(winv, n, V, ldv, Add, lda, Out, ldo, gate);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int diag_stats(int lik, double s2, const T* fnew, const T* f, const T* v, const void* y,
               int64_t n, double* part, double* scal, hipStream_t s) {
  const int g = static_cast<int>(ceil_div(n, NTD));
  if (g == 0) return IGP_OK;
  k_diag_stats<T><<<g, NTD, 0, s>>>(lik, s2, fnew, f, v, y, n, part);
  k_diag_finish<<<1, NTD, 0, s>>>(part, g, scal);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int diag_check_targets(int lik, const void* y, int64_t n, int* flag, hipStream_t s) {
  if (n == 0) return IGP_OK;
  if (lik == IGP_LIK_POISSON)
    k_check_counts<<<256, 256, 0, s>>>(static_cast<const int32_t*>(y), n, flag);
  else
    k_check_finite<T><<<256, 256, 0, s>>>(static_cast<const T*>(y), n, flag);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

#define IGP_DIAG_INST(T)                                                                      \
  template int diag_begin<T>(int, const T*, const void*, int64_t, double, T*, T*, hipStream_t); \
  template int diag_apply<T>(const T*, int64_t, const T*, int64_t, int64_t, const T*, int64_t, \
                             T*, int64_t, hipStream_t, const int*);                           \
  template int diag_stats<T>(int, double, const T*, const T*, const T*, const void*, int64_t, \
                             double*, double*, hipStream_t);                                  \
  template int diag_check_targets<T>(int, const void*, int64_t, int*, hipStream_t);
IGP_DIAG_INST(float)
IGP_DIAG_INST(double)
#undef IGP_DIAG_INST

}  // namespace igp
