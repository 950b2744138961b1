// Softmax likelihood pieces, one thread per data point with its C logits in
// registers (CN-ordering keeps a point's C entries contiguous, so a wave's
// loads cover one contiguous 64*C-element span).
//
//   pi_n  = softmax(F_n)                          (log-sum-exp)
//   rhs_n = F_n + W_n^+ (onehot(y_n) - pi_n)       pseudo-targets minus m (m = 0)
//   W_n   v = pi_n * v - pi_n (pi_n^T v)
//   W_n^+ v = P ((P v) / pi_n),  P = I - 11^T / C  (explicit pseudo-inverse from
//             the paper's appendix lemma for multi-class classification)
#include "iter_ops.hpp"

namespace igp {
namespace {

using iter::apply_block;
using iter::load_softmax;

template <typename T, int CMAX>
__global__ void __launch_bounds__(256)
k_softmax_pi_rhs(const T* __restrict__ F, const int32_t* __restrict__ y, int64_t N, int C,
                 T* __restrict__ pi, T* __restrict__ rhs, double* __restrict__ ll_part) {
  __shared__ double red[4];
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  double ll = 0.0;
  if (n < N) {
    T p[CMAX], u[CMAX];
    load_softmax<T, CMAX>(F, n, C, p);
    const int yn = y[n];
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) {
        u[c] = (c == yn ? T(1) : T(0)) - p[c];
        pi[n * C + c] = p[c];
      }
    // log p(y_n | f_n) = f_y - lse(f_n), in FP64
    double mx = -INFINITY;
    for (int c = 0; c < C; ++c) mx = fmax(mx, static_cast<double>(F[n * C + c]));
    double se = 0.0;
    for (int c = 0; c < C; ++c) se += exp(static_cast<double>(F[n * C + c]) - mx);
    ll = static_cast<double>(F[n * C + yn]) - mx - log(se);
    apply_block<T, CMAX>(IGP_W_PINV, C, p, u);
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) rhs[n * C + c] = F[n * C + c] + u[c];
  }
  const double s = block_sum(ll, red);
  if (threadIdx.x == 0) ll_part[blockIdx.x] = s;
}

template <typename T, int CMAX>
__global__ void __launch_bounds__(256)
k_winv_apply(const T* __restrict__ pi, int logits, int mode, int64_t N, int C,
             const T* __restrict__ V, int64_t nb, int64_t ldv, const T* __restrict__ Add,
             int64_t lda, T* __restrict__ Out, int64_t ldo, const int* gate) {
  if (gate_closed(gate)) return;
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t b = blockIdx.y;
  if (n >= N || b >= nb) return;
  iter::winv_point<T, CMAX>(pi, logits, mode, n, C, V, b, ldv, Add, lda, Out, ldo);
}

// The residual of a solver iteration with the W^+ v it needs, one thread per
// point: wv = W^+ v (kept), r = rhs - kv - wv, and the block partials of r^T r
template <typename T, int CMAX>
__global__ void __launch_bounds__(256)
k_winv_residual(const T* __restrict__ pi, int64_t N, int C, const T* __restrict__ v,
                const T* __restrict__ rhs, const T* __restrict__ kv, T* __restrict__ wv,
                T* __restrict__ r, double* __restrict__ part, const int* gate) {
  if (gate_closed(gate)) return;
  __shared__ double red[4];
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  double acc = 0.0;
  if (n < N) {
    T p[CMAX], u[CMAX];
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) {
        p[c] = pi[n * C + c];
        u[c] = v[n * C + c];
      }
    iter::apply_block<T, CMAX>(IGP_W_PINV, C, p, u);
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) {
        const int64_t i = n * C + c;
        wv[i] = u[c];
        const T ri = rhs[i] - kv[i] - u[c];
        r[i] = ri;
        acc += static_cast<double>(ri) * static_cast<double>(ri);
      }
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// The append step and the residual of a solver iteration in one pass, one
// thread per point (softmax likelihood, recurrence residual): every block
// finishes alpha and eta from their partials (the fixed-order sum, so all
// blocks hold the same values; block 0 stores them), then each point takes
// its append and residual, and the block partials of r^T r are those of
// k_winv_residual.
template <typename T, int CMAX>
__global__ void __launch_bounds__(256)
k_append_winv_residual(const T* __restrict__ d, const double* __restrict__ apart, int anblk,
                       const double* __restrict__ epart, int enblk, double* __restrict__ scal,
                       T* __restrict__ qcol, T* __restrict__ v, const T* __restrict__ kd,
                       T* __restrict__ kqcol, T* __restrict__ kv, const T* __restrict__ pi,
                       int64_t N, int C, const T* __restrict__ rhs, T* __restrict__ wv,
                       T* __restrict__ r, double* __restrict__ part, const int* gate) {
  if (gate_closed(gate)) return;
  __shared__ double red[4];
  const int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  iter::AppendPoint<T, CMAX> pt;
  if (n < N) pt.load_point(d, v, kd, kv, pi, rhs, n, C);   // in flight over the sums below
  double a = 0.0, e = 0.0;
  for (int i = threadIdx.x; i < anblk; i += 256) a += apart[i];
  a = block_sum(a, red);
  for (int i = threadIdx.x; i < enblk; i += 256) e += epart[i];
  e = block_sum(e, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[SC_ALPHA] = a;
    scal[SC_ETA] = e;
  }
  double acc = 0.0;
  if (n < N) acc = pt.append_residual(a, e, qcol, v, kqcol, kv, wv, r, n, C);
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

}  // namespace

#define IGP_DISPATCH_C(C, BODY)                    \
  do {                                             \
    if ((C) <= 4) {                                \
      constexpr int CM = 4;                        \
      BODY;                                        \
    } else if ((C) <= 8) {                         \
      constexpr int CM = 8;                        \
      BODY;                                        \
    } else if ((C) <= 16) {                        \
      constexpr int CM = 16;                       \
      BODY;                                        \
    } else {                                       \
      constexpr int CM = 64;                       \
      BODY;                                        \
    }                                              \
  } while (0)

template <typename T>
int softmax_pi_rhs(const T* F, const int32_t* y, int64_t N, int64_t C, T* pi, T* rhs,
                   double* ll_part, int* nblocks_out, hipStream_t s) {
  if (C > 64) {
    set_error("C = %lld classes exceeds the supported maximum of 64", (long long)C);
    return IGP_EUNSUPPORTED;
  }
  const int blocks = static_cast<int>(ceil_div(N, 256));
  *nblocks_out = blocks;
  if (blocks == 0) return IGP_OK;
  IGP_DISPATCH_C(C, (k_softmax_pi_rhs<T, CM><<<blocks, 256, 0, s>>>(F, y, N, (int)C, pi, rhs, ll_part)));
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int winv_apply(const T* pi, bool pi_is_logits, int mode, int64_t N, int64_t C, const T* V,
               int64_t nb, int64_t ldv, const T* Add, int64_t lda, T* Out, int64_t ldo,
               hipStream_t s, const int* gate) {
  if (C > 64) {
    set_error("C = %lld classes exceeds the supported maximum of 64", (long long)C);
    return IGP_EUNSUPPORTED;
  }
  if (N == 0 || nb == 0) return IGP_OK;
  dim3 grid(static_cast<unsigned>(ceil_div(N, 256)), static_cast<unsigned>(nb));
  IGP_DISPATCH_C(C, (k_winv_apply<T, CM><<<grid, 256, 0, s>>>(pi, pi_is_logits ? 1 : 0, mode, N, (int)C, V, nb, ldv, Add, lda, Out, ldo, gate)));
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int winv_residual(const T* pi, int64_t N, int64_t C, const T* v, const T* rhs, const T* kv,
                  T* wv, T* r, double* part, int* nblk_out, hipStream_t s, const int* gate) {
  if (C > 64) {
    set_error("C = %lld classes exceeds the supported maximum of 64", (long long)C);
    return IGP_EUNSUPPORTED;
  }
  const int blocks = static_cast<int>(ceil_div(N, 256));
  *nblk_out = blocks;
  if (blocks == 0) return IGP_OK;
  IGP_DISPATCH_C(C, (k_winv_residual<T, CM><<<blocks, 256, 0, s>>>(pi, N, (int)C, v, rhs, kv, wv, r, part, gate)));
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int append_winv_residual(const T* d, const double* apart, const double* epart, double* scal,
                         T* qcol, T* v, const T* kd, T* kqcol, T* kv, const T* pi, int64_t N,
                         int64_t C, const T* rhs, T* wv, T* r, double* part, int* nblk_out,
                         hipStream_t s, const int* gate) {
  if (C > 64) {
    set_error("C = %lld classes exceeds the supported maximum of 64", (long long)C);
    return IGP_EUNSUPPORTED;
  }
  const int blocks = static_cast<int>(ceil_div(N, 256));
  *nblk_out = blocks;
  if (blocks == 0) return IGP_OK;
  const int anblk = iter::grid_for(N * C), enblk = static_cast<int>(ceil_div(N * C, iter::NT));
  IGP_DISPATCH_C(C, (k_append_winv_residual<T, CM><<<blocks, 256, 0, s>>>(d, apart, anblk, epart, enblk, scal, qcol, v, kd, kqcol, kv, pi, N, (int)C, rhs, wv, r, part, gate)));
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template int append_winv_residual<float>(const float*, const double*, const double*, double*,
                                         float*, float*, const float*, float*, float*,
                                         const float*, int64_t, int64_t, const float*, float*,
                                         float*, double*, int*, hipStream_t, const int*);
template int append_winv_residual<double>(const double*, const double*, const double*, double*,
                                          double*, double*, const double*, double*, double*,
                                          const double*, int64_t, int64_t, const double*,
                                          double*, double*, double*, int*, hipStream_t,
                                          const int*);
template int winv_residual<float>(const float*, int64_t, int64_t, const float*, const float*,
                                  const float*, float*, float*, double*, int*, hipStream_t,
                                  const int*);
template int winv_residual<double>(const double*, int64_t, int64_t, const double*,
                                   const double*, const double*, double*, double*, double*,
                                   int*, hipStream_t, const int*);
template int softmax_pi_rhs<float>(const float*, const int32_t*, int64_t, int64_t, float*,
                                   float*, double*, int*, hipStream_t);
template int softmax_pi_rhs<double>(const double*, const int32_t*, int64_t, int64_t, double*,
                                    double*, double*, int*, hipStream_t);
template int winv_apply<float>(const float*, bool, int, int64_t, int64_t, const float*, int64_t,
                               int64_t, const float*, int64_t, float*, int64_t, hipStream_t,
                               const int*);
template int winv_apply<double>(const double*, bool, int, int64_t, int64_t, const double*,
                                int64_t, int64_t, const double*, int64_t, double*, int64_t,
                                hipStream_t, const int*);

}  // namespace igp
