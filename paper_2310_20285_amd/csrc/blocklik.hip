// Likelihoods given by the caller as per-point blocks: the gradient of log p
// and the C x C negative-Hessian block W_n at each point (symmetric positive
// definite).  The Newton step (section 3.1 with m = 0) needs the pseudo-
// targets f + W^{-1} grad and products with W^{-1}, which is block diagonal
// over the points: each block is inverted once per step.
#include "iter_ops.hpp"

namespace igp {
namespace {

constexpr int NTB = 256;   // threads per block (four points per block in k_block_begin)

// One wave per point; lane j < C holds column j of the block in FP64.
// Gauss-Jordan elimination without pivoting leaves W^{-1} in place; for a
// positive definite block every pivot is the diagonal of a Schur complement,
// hence positive.  Lanes >= C carry zero columns and take no part.
template <typename T, int CMAX>
__global__ void __launch_bounds__(NTB)
k_block_begin(const T* __restrict__ W, const T* __restrict__ grad, const T* __restrict__ f,
              int64_t N, int C, T* __restrict__ winv, T* __restrict__ rhs, int* bad) {
  const int64_t pt = blockIdx.x * static_cast<int64_t>(NTB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (pt >= N) return;
  const int64_t base = pt * C * C;
  double a[CMAX];
#pragma unroll
  for (int i = 0; i < CMAX; ++i)
    a[i] = (i < C && lane < C) ? static_cast<double>(W[base + static_cast<int64_t>(i) * C + lane])
                               : 0.0;
  bool ok = true;
  for (int k = 0; k < C; ++k) {
    double akk = 0.0, aik[CMAX];
    // column k (the multipliers) from lane k, before this step changes it;
    // register arrays are indexed only by unrolled constants (selects on k)
#pragma unroll
    for (int i = 0; i < CMAX; ++i) {
      aik[i] = __shfl(a[i], k, 64);
      if (i == k) akk = aik[i];
    }
    if (!(akk > 0.0)) ok = false;   // the same value on every lane
    const double inv = 1.0 / akk;
    // row k scaled; in column k the pivot entry becomes 1 / akk
#pragma unroll
    for (int i = 0; i < CMAX; ++i)
      if (i == k) a[i] = (lane == k ? 1.0 : a[i]) * inv;
    // every other row: A[i][j] -= A[i][k] A[k][j]; column k: -A[i][k] / akk
    double rowk = 0.0;
#pragma unroll
    for (int i = 0; i < CMAX; ++i)
      if (i == k) rowk = a[i];
#pragma unroll
    for (int i = 0; i < CMAX; ++i)
      if (i < C && i != k) a[i] = (lane == k ? 0.0 : a[i]) - aik[i] * rowk;
  }
  if (!ok) {
    if (lane == 0) atomicAdd(bad, 1);
#pragma unroll
    for (int i = 0; i < CMAX; ++i) a[i] = __builtin_nan("");
  }
  // W^{-1} is symmetric: lane j's column is row j
  if (lane < C) {
#pragma unroll
    for (int i = 0; i < CMAX; ++i)
      if (i < C) winv[base + static_cast<int64_t>(i) * C + lane] = static_cast<T>(a[i]);
    double s = static_cast<double>(f[pt * C + lane]);
#pragma unroll
    for (int i = 0; i < CMAX; ++i)
      if (i < C) s += a[i] * static_cast<double>(grad[pt * C + i]);
    rhs[pt * C + lane] = static_cast<T>(s);
  }
}

// Out[n] = W_n^{-1} V[n] (+ Add[n]) for column b = blockIdx.y; one thread per point
template <typename T, int CMAX>
__global__ void __launch_bounds__(NTB)
k_block_apply(const T* __restrict__ winv, int64_t N, int C, const T* __restrict__ V,
              int64_t ldv, const T* __restrict__ Add, int64_t lda, T* __restrict__ Out,
              int64_t ldo, const int* gate) {
  if (gate_closed(gate)) return;
  const int64_t pt = blockIdx.x * static_cast<int64_t>(NTB) + threadIdx.x;
  if (pt >= N) return;
  const int64_t b = blockIdx.y;
  const T* vb = V + b * ldv + pt * C;
  double v[CMAX];
#pragma unroll
  for (int i = 0; i < CMAX; ++i) v[i] = i < C ? static_cast<double>(vb[i]) : 0.0;
  const T* w = winv + pt * C * C;
  for (int j = 0; j < C; ++j) {
    double s = Add ? static_cast<double>(Add[b * lda + pt * C + j]) : 0.0;
#pragma unroll
    for (int i = 0; i < CMAX; ++i)
      if (i < C) s += static_cast<double>(w[static_cast<int64_t>(j) * C + i]) * v[i];
    Out[b * ldo + pt * C + j] = static_cast<T>(s);
  }
}

}  // namespace

#define IGP_BLOCK_C(C, BODY)  \
  do {                        \
    if ((C) <= 4) {           \
      constexpr int CM = 4;   \
      BODY;                   \
    } else if ((C) <= 16) {   \
      constexpr int CM = 16;  \
      BODY;                   \
    } else {                  \
      constexpr int CM = 64;  \
      BODY;                   \
    }                         \
  } while (0)

template <typename T>
int block_begin(const T* W, const T* grad, const T* f, int64_t N, int64_t C, T* winv, T* rhs,
                int* bad, hipStream_t s) {
  if (C < 1 || C > 64) {
    set_error("block likelihood: C = %lld outside [1, 64]", (long long)C);
    return IGP_EUNSUPPORTED;
  }
  if (N == 0) return IGP_OK;
  const unsigned blocks = static_cast<unsigned>(ceil_div(N, NTB / 64));
  IGP_BLOCK_C(C, (k_block_begin<T, CM><<<blocks, NTB, 0, s>>>(W, grad, f, N, (int)C, winv, rhs,
                                                               bad)));
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int block_apply(const T* winv, int64_t N, int64_t C, const T* V, int64_t nb, int64_t ldv,
                const T* Add, int64_t lda, T* Out, int64_t ldo, hipStream_t s, const int* gate) {
  if (C < 1 || C > 64) {
    set_error("block likelihood: C = %lld outside [1, 64]", (long long)C);
    return IGP_EUNSUPPORTED;
  }
  if (N == 0 || nb == 0) return IGP_OK;
  dim3 grid(static_cast<unsigned>(ceil_div(N, NTB)), static_cast<unsigned>(nb));
  IGP_BLOCK_C(C, (k_block_apply<T, CM><<<grid, NTB, 0, s>>>(winv, N, (int)C, V, ldv, Add, lda,
                                                             Out, ldo, gate)));
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

#define IGP_BLOCK_INST(T)                                                                     \
  template int block_begin<T>(const T*, const T*, const T*, int64_t, int64_t, T*, T*, int*,   \
                              hipStream_t);                                                   \
  template int block_apply<T>(const T*, int64_t, int64_t, const T*, int64_t, int64_t,         \
                              const T*, int64_t, T*, int64_t, hipStream_t, const int*);
IGP_BLOCK_INST(float)
IGP_BLOCK_INST(double)
#undef IGP_BLOCK_INST

}  // namespace igp
