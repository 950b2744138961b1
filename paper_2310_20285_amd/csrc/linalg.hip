// Skinny linear algebra of the IterGP loop and of the virtual solver run.
// Every reduction accumulates in FP64 and is finished by a single block in a
// fixed order, so repeated runs are bitwise identical.
//
// Buffers S, T, Q are stored column by column: column b of an n-row buffer
// starts at element b*ld (each column is one CN-ordered vector).
#include <algorithm>

#include "iter_ops.hpp"

namespace igp {
namespace {

using iter::GV_ROWS;
using iter::MAXCOLS_LDS;
using iter::NT;
using iter::grid_for;

__global__ void k_finish_sum(const double* __restrict__ part, int nblk, double* __restrict__ out,
                             const int* gate) {
  if (gate_closed(gate)) return;
  __shared__ double red[NT / 64];
  iter::finish_sum(part, nblk, out, red);
}

template <typename T>
__global__ void __launch_bounds__(NT)
k_residual(const T* __restrict__ rhs, const T* __restrict__ kv, const T* __restrict__ wv,
           T* __restrict__ r, int64_t n, double* __restrict__ part, const int* gate) {
  if (gate_closed(gate)) return;
  __shared__ double red[NT / 64];
  iter::residual<T>(rhs, kv, wv, r, n, part, blockIdx.x, gridDim.x, red);
}

// rr = sum of the residual partials, then the end of the solver iteration
__global__ void k_finish_rr_consume(const double* __restrict__ part, int nblk,
                                    double* __restrict__ scal, double thresh, int* gate,
                                    double* rec) {
  if (gate_closed(gate)) return;
  __shared__ double red[NT / 64];
  iter::finish_sum(part, nblk, scal + SC_RR, red);
  if (threadIdx.x == 0) iter::consume_iteration(scal, thresh, 1, gate, rec);
}

template <typename T>
__global__ void __launch_bounds__(NT)
k_dot(const T* __restrict__ a, const T* __restrict__ b, int64_t n, double* __restrict__ part,
      const int* gate) {
  if (gate_closed(gate)) return;
  __shared__ double red[NT / 64];
  iter::dot<T>(a, b, n, part, blockIdx.x, gridDim.x, red);
}

// CG action s = r / sqrt(r^T r) and the partials of alpha = s^T r in one pass
// (the partials of a separate k_dot over s and r)
template <typename T>
__global__ void __launch_bounds__(NT)
k_action_cg_dot(const T* __restrict__ r, const double* __restrict__ rr, T* __restrict__ s,
                int64_t n, double* __restrict__ part, const int* gate) {
  if (gate_closed(gate)) return;
  __shared__ double red[NT / 64];
  const double inv = 1.0 / sqrt(coherent_load(rr));
  double acc = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(NT) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * NT) {
    const T ri = r[i];
    const T si = static_cast<T>(static_cast<double>(ri) * inv);
    s[i] = si;
    acc += static_cast<double>(si) * static_cast<double>(ri);
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// the previous iteration's end (k_finish_rr_consume) and this iteration's CG
// action (k_action_cg_dot) in one launch
template <typename T>
__global__ void __launch_bounds__(NT)
k_consume_action_cg_dot(const T* __restrict__ r, const double* __restrict__ rpart, int rnblk,
                        double* __restrict__ scal, double thresh, int* gate, double* rec,
                        T* __restrict__ s, int64_t n, double* __restrict__ part) {
  if (gate_closed(gate)) return;
  __shared__ double red[NT / 64];
  // rr in the order of iter::finish_sum: the same value in every block
  double rr = 0.0;
  for (int i = threadIdx.x; i < rnblk; i += NT) rr += rpart[i];
  rr = block_sum(rr, red);
  const double eta = coherent_load(scal + SC_ETA);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[SC_RR] = rr;
    iter::consume_iteration(scal, thresh, 1, gate, rec);
  }
  // the decision consume_iteration takes, in every block
  if (!(eta > 0.0) || !(sqrt(rr) >= thresh)) return;
  const double inv = 1.0 / sqrt(rr);
  double acc = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(NT) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * NT) {
    const T ri = r[i];
    const T si = static_cast<T>(static_cast<double>(ri) * inv);
    s[i] = si;
    acc += static_cast<double>(si) * static_cast<double>(ri);
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

template <typename T>
__global__ void __launch_bounds__(NT) k_fill_unit(T* __restrict__ s, int64_t n, int64_t idx,
                                                  const int* gate) {
  if (gate_closed(gate)) return;
  iter::fill_unit<T>(s, n, idx, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void k_fill_zero(T* __restrict__ a, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    a[i] = T(0);
}

template <typename T>
__global__ void __launch_bounds__(NT) k_copy(const T* __restrict__ a, T* __restrict__ b, int64_t n,
                                             const int* gate) {
  if (gate_closed(gate)) return;
  iter::copy<T>(a, b, n, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void k_add(const T* __restrict__ a, const T* __restrict__ b, T* __restrict__ o, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    o[i] = a[i] + b[i];
}

// y = Q^T z for a column-major Q: one wave per (column, chunk of GV_ROWS rows),
// each lane accumulating GV_ROWS/64 consecutive-in-wave elements in FP64, a
// single wave reduction per (column, chunk); chunk partials are summed in a
// fixed order by k_finish_cols.
template <typename T>
__global__ void __launch_bounds__(NT)
k_gemv_t(const T* __restrict__ Q, int64_t ldq, int64_t n, int ncols, const T* __restrict__ z,
         double* __restrict__ part, int nchunks, const int* gate) {
  if (gate_closed(gate)) return;
  iter::gemv_t<T>(Q, ldq, n, ncols, z, part, nchunks, blockIdx.x);
}

__global__ void __launch_bounds__(NT)
k_finish_cols(const double* __restrict__ part, int nrow_blocks, int ncols,
              double* __restrict__ y, const int* gate) {
  if (gate_closed(gate)) return;
  iter::finish_col(part, nrow_blocks, ncols, blockIdx.x * (NT / 64) + (threadIdx.x >> 6), y);
}

// d = s - Q y ; eta partial = z^T d.  One row per thread; y staged in LDS.
template <typename T, bool KQ>
__global__ void __launch_bounds__(NT)
k_dir_update(const T* __restrict__ sv, const T* __restrict__ Q, int64_t ldq, int64_t n,
             int ncols, const double* __restrict__ y, const T* __restrict__ z,
             T* __restrict__ d, double* __restrict__ epart, const T* __restrict__ tv,
             const T* __restrict__ KQm, T* __restrict__ kd, const int* gate) {
  if (gate_closed(gate)) return;
  __shared__ double sy[MAXCOLS_LDS];
  __shared__ double red[NT / 64];
  iter::dir_update<T, KQ>(sv, Q, ldq, n, ncols, y, z, d, epart, tv, KQm, kd, blockIdx.x, sy,
                          red);
}

template <typename T>
__global__ void k_gemv_n(const T* __restrict__ Q, int64_t ldq, int64_t n, int ncols,
                         const double* __restrict__ y, T* __restrict__ out) {
  __shared__ double sy[MAXCOLS_LDS];
  for (int b = threadIdx.x; b < ncols; b += blockDim.x) sy[b] = y[b];
  __syncthreads();
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int b = 0; b < ncols; ++b) acc += static_cast<double>(Q[static_cast<int64_t>(b) * ldq + i]) * sy[b];
  out[i] = static_cast<T>(acc);
}

// every block finishes alpha and eta from their partials (the fixed-order sum
// of k_finish_sum, so all blocks hold the same values); block 0 stores them
template <typename T, bool KQ>
__global__ void __launch_bounds__(NT)
k_append_step(const T* __restrict__ d, const double* __restrict__ apart, int anblk,
              const double* __restrict__ epart, int enblk, double* __restrict__ scal,
              T* __restrict__ qcol, T* __restrict__ v, int64_t n, const T* __restrict__ kd,
              T* __restrict__ kqcol, T* __restrict__ kv, const int* gate) {
  if (gate_closed(gate)) return;
  __shared__ double red[NT / 64];
  double a = 0.0, e = 0.0;
  for (int i = threadIdx.x; i < anblk; i += NT) a += apart[i];
  a = block_sum(a, red);
  for (int i = threadIdx.x; i < enblk; i += NT) e += epart[i];
  e = block_sum(e, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[SC_ALPHA] = a;
    scal[SC_ETA] = e;
  }
  iter::append_step_vals<T, KQ>(d, a, e, qcol, v, n, kd, kqcol, kv, blockIdx.x, gridDim.x);
}

// Gram matrix M = A^T B over a chunk of rows; 32 x 32 output tile per block,
// 4 outputs per thread, rows staged in LDS 32 at a time.
constexpr int GT = 32;
template <typename T>
__global__ void __launch_bounds__(NT)
k_gram(const T* __restrict__ A, const T* __restrict__ B, int64_t ld, int64_t n, int ncols,
       int64_t rows_per_chunk, double* __restrict__ part) {
  __shared__ double sA[GT][GT + 1];
  __shared__ double sB[GT][GT + 1];
  const int tid = threadIdx.x;
  const int a0 = blockIdx.x * GT, b0 = blockIdx.y * GT;
  const int64_t i_begin = static_cast<int64_t>(blockIdx.z) * rows_per_chunk;
  const int64_t i_end = i_begin + rows_per_chunk < n ? i_begin + rows_per_chunk : n;
  const int ta = tid % 16, tb = tid / 16;   // outputs (a0+ta+16*u, b0+tb+16*v)
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int64_t i0 = i_begin; i0 < i_end; i0 += GT) {
#pragma unroll 4
    for (int e = tid; e < GT * GT; e += NT) {
      const int col = e / GT, row = e % GT;     // column-major: rows contiguous
      const int64_t gi = i0 + row;
      const int ga = a0 + col, gb = b0 + col;
      sA[col][row] = (gi < i_end && ga < ncols) ? static_cast<double>(A[static_cast<int64_t>(ga) * ld + gi]) : 0.0;
      sB[col][row] = (gi < i_end && gb < ncols) ? static_cast<double>(B[static_cast<int64_t>(gb) * ld + gi]) : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < GT; ++k) {
      const double x0 = sA[ta][k], x1 = sA[ta + 16][k];
      const double y0 = sB[tb][k], y1 = sB[tb + 16][k];
      acc[0][0] += x0 * y0;
      acc[0][1] += x0 * y1;
      acc[1][0] += x1 * y0;
      acc[1][1] += x1 * y1;
    }
    __syncthreads();
  }
  double* P = part + static_cast<int64_t>(blockIdx.z) * ncols * ncols;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int a = a0 + ta + 16 * u, b = b0 + tb + 16 * v;
      if (a < ncols && b < ncols) P[static_cast<int64_t>(a) * ncols + b] = acc[u][v];
    }
}

__global__ void k_finish_gram(const double* __restrict__ part, int nchunks, int ncols,
                              double* __restrict__ M) {
  const int64_t total = static_cast<int64_t>(ncols) * ncols;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int c = 0;
    for (; c + 4 <= nchunks; c += 4) {
      s0 += part[c * total + e];
      s1 += part[(c + 1) * total + e];
      s2 += part[(c + 2) * total + e];
      s3 += part[(c + 3) * total + e];
    }
    for (; c < nchunks; ++c) s0 += part[c * total + e];
    M[e] = (s0 + s1) + (s2 + s3);
  }
}

// Out[:, r] = (A U[:, r]) * colscale[r]; 16 output columns per block, U tile in LDS.
constexpr int RM_COLS = 16;
template <typename T>
__global__ void __launch_bounds__(NT)
k_right_mul(const T* __restrict__ A, int64_t lda, int64_t n, int ncols,
            const double* __restrict__ U, int R, const double* __restrict__ colscale,
            T* __restrict__ Out, int64_t ldo) {
  extern __shared__ double sU[];   // ncols x RM_COLS
  const int r0 = blockIdx.y * RM_COLS;
  for (int e = threadIdx.x; e < ncols * RM_COLS; e += NT) {
    const int b = e / RM_COLS, rr = e % RM_COLS;
    sU[e] = (r0 + rr < R) ? U[static_cast<int64_t>(r0 + rr) * ncols + b] : 0.0;
  }
  __syncthreads();
  const int64_t i = blockIdx.x * static_cast<int64_t>(NT) + threadIdx.x;
  if (i >= n) return;
  double acc[RM_COLS];
#pragma unroll
  for (int rr = 0; rr < RM_COLS; ++rr) acc[rr] = 0.0;
#pragma unroll 4
  for (int b = 0; b < ncols; ++b) {
    const double a = static_cast<double>(A[static_cast<int64_t>(b) * lda + i]);
#pragma unroll
    for (int rr = 0; rr < RM_COLS; ++rr) acc[rr] += a * sU[b * RM_COLS + rr];
  }
#pragma unroll
  for (int rr = 0; rr < RM_COLS; ++rr)
    if (r0 + rr < R) {
      const double sc = colscale ? colscale[r0 + rr] : 1.0;
      Out[static_cast<int64_t>(r0 + rr) * ldo + i] = static_cast<T>(acc[rr] * sc);
    }
}

template <typename T>
__global__ void __launch_bounds__(NT)
k_newton_stats(const T* __restrict__ fnew, const T* __restrict__ f, const T* __restrict__ v,
               const int32_t* __restrict__ y, int64_t N, int C, double* __restrict__ part) {
  __shared__ double red[NT / 64];
  const int64_t n = blockIdx.x * static_cast<int64_t>(NT) + threadIdx.x;
  double dd = 0.0, ff = 0.0, ll = 0.0, gv = 0.0;
  if (n < N) {
    double mx = -INFINITY;
    for (int c = 0; c < C; ++c) {
      const double a = static_cast<double>(fnew[n * C + c]);
      const double b = static_cast<double>(f[n * C + c]);
      dd += (a - b) * (a - b);
      ff += a * a;
      gv += a * static_cast<double>(v[n * C + c]);
      mx = fmax(mx, a);
    }
    double se = 0.0;
    for (int c = 0; c < C; ++c) se += exp(static_cast<double>(fnew[n * C + c]) - mx);
    ll = static_cast<double>(fnew[n * C + y[n]]) - mx - log(se);
  }
  const int nb = gridDim.x;
  double s;
  s = block_sum(dd, red); if (threadIdx.x == 0) part[0 * nb + blockIdx.x] = s;
  s = block_sum(ff, red); if (threadIdx.x == 0) part[1 * nb + blockIdx.x] = s;
  s = block_sum(ll, red); if (threadIdx.x == 0) part[2 * nb + blockIdx.x] = s;
  s = block_sum(gv, red); if (threadIdx.x == 0) part[3 * nb + blockIdx.x] = s;
}

struct PriorVar {
  double v[64];   // k_c(x, x) per class
};

template <typename T>
__global__ void k_predict_epilogue(const T* __restrict__ A, int64_t lda, int64_t nrows,
                                   int ncols, PriorVar os, const T* __restrict__ mean, int64_t Ns,
                                   int C, T* __restrict__ var, T* __restrict__ probs) {
  const int64_t s = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (s >= Ns) return;
  double z[64];
  double mx = -INFINITY;
  for (int c = 0; c < C; ++c) {
    const int64_t row = s * C + c;
    double acc = 0.0;
    for (int b = 0; b < ncols; ++b) {
      const double a = static_cast<double>(A[static_cast<int64_t>(b) * lda + row]);
      acc += a * a;
    }
    const double vv = os.v[c] - acc;
    if (var) var[row] = static_cast<T>(vv);
    if (probs) {
      const double vz = vv > 0.0 ? vv : 0.0;
      z[c] = static_cast<double>(mean[row]) / sqrt(1.0 + 0.39269908169872414 * vz);
      mx = fmax(mx, z[c]);
    }
  }
  if (probs) {
    double se = 0.0;
    for (int c = 0; c < C; ++c) {
      z[c] = exp(z[c] - mx);
      se += z[c];
    }
    for (int c = 0; c < C; ++c) probs[s * C + c] = static_cast<T>(z[c] / se);
  }
}

__global__ void k_iter_gate_init(int* gate, double* rec) {
  if (threadIdx.x != 0) return;
  *gate = 0;
  for (int k = 0; k < REC_COUNT; ++k) rec[k] = 0.0;
  rec[REC_ETAMIN] = INFINITY;
}

__global__ void k_iter_consume(const double* __restrict__ scal, double thresh, int next_r,
                               int* gate, double* rec) {
  if (threadIdx.x == 0) iter::consume_iteration(scal, thresh, next_r, gate, rec);
}

}  // namespace

// ------------------------------ launchers ---------------------------------------

int iter_gate_init(int* gate, double* rec, hipStream_t s) {
  k_iter_gate_init<<<1, 64, 0, s>>>(gate, rec);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

int iter_consume(const double* scal, double thresh, int next_r, int* gate, double* rec,
                 hipStream_t s) {
  k_iter_consume<<<1, 64, 0, s>>>(scal, thresh, next_r, gate, rec);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int residual(const T* rhs, const T* kv, const T* wv, T* r, int64_t n, double* part,
             double* out, hipStream_t s, const int* gate) {
  const int g = grid_for(n);
  k_residual<T><<<g, NT, 0, s>>>(rhs, kv, wv, r, n, part, gate);
  k_finish_sum<<<1, NT, 0, s>>>(part, g, out, gate);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int dot_into(const T* a, const T* b, int64_t n, double* part, double* out, hipStream_t s,
             const int* gate) {
  const int g = grid_for(n);
  k_dot<T><<<g, NT, 0, s>>>(a, b, n, part, gate);
  if (out) k_finish_sum<<<1, NT, 0, s>>>(part, g, out, gate);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int action_cg_dot(const T* r, const double* rr, T* sv, int64_t n, double* part, double* alpha,
                  const int* gate, hipStream_t s) {
  const int g = grid_for(n);
  k_action_cg_dot<T><<<g, NT, 0, s>>>(r, rr, sv, n, part, gate);
  if (alpha) k_finish_sum<<<1, NT, 0, s>>>(part, g, alpha, gate);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int consume_action_cg_dot(const T* r, const double* rpart, int rnblk, double* scal,
                          double thresh, int* gate, double* rec, T* sv, int64_t n,
                          double* apart, hipStream_t s) {
  k_consume_action_cg_dot<T><<<grid_for(n), NT, 0, s>>>(r, rpart, rnblk, scal, thresh, gate, rec,
                                                        sv, n, apart);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

int rr_consume(const double* part, int nblk, double* scal, double thresh, int* gate, double* rec,
               hipStream_t s) {
  k_finish_rr_consume<<<1, NT, 0, s>>>(part, nblk, scal, thresh, gate, rec);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int residual_consume(const T* rhs, const T* kv, const T* wv, T* r, int64_t n, double* part,
                     double* scal, double thresh, int* gate, double* rec, hipStream_t s) {
  const int g = grid_for(n);
  k_residual<T><<<g, NT, 0, s>>>(rhs, kv, wv, r, n, part, gate);
  k_finish_rr_consume<<<1, NT, 0, s>>>(part, g, scal, thresh, gate, rec);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int fill_unit(T* sv, int64_t n, int64_t idx, hipStream_t s, const int* gate) {
  k_fill_unit<T><<<grid_for(n), NT, 0, s>>>(sv, n, idx, gate);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int fill_zero(T* a, int64_t n, hipStream_t s) {
  k_fill_zero<T><<<grid_for(n), NT, 0, s>>>(a, n);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int copy_vec(const T* a, T* b, int64_t n, hipStream_t s, const int* gate) {
  k_copy<T><<<grid_for(n), NT, 0, s>>>(a, b, n, gate);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int add_vec(const T* a, const T* b, T* o, int64_t n, hipStream_t s) {
  k_add<T><<<grid_for(n), NT, 0, s>>>(a, b, o, n);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int gemv_t(const T* Q, int64_t ldq, int64_t n, int ncols, const T* z, double* part, double* y,
           hipStream_t s, const int* gate) {
  if (ncols == 0) return IGP_OK;
  const int nchunks = static_cast<int>(ceil_div(n, GV_ROWS));
  const int64_t waves = static_cast<int64_t>(nchunks) * ncols;
  k_gemv_t<T><<<static_cast<unsigned>(ceil_div(waves, NT / 64)), NT, 0, s>>>(Q, ldq, n, ncols, z,
                                                                             part, nchunks, gate);
  k_finish_cols<<<static_cast<unsigned>(ceil_div(ncols, NT / 64)), NT, 0, s>>>(part, nchunks,
                                                                              ncols, y, gate);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int dir_update(const T* sv, const T* Q, int64_t ldq, int64_t n, int ncols, const double* y,
               const T* z, T* d, double* part, double* eta_out, hipStream_t s, const T* tv,
               const T* KQm, T* kd, const int* gate) {
  if (ncols > MAXCOLS_LDS) {
    set_error("buffer of %d columns exceeds %d", ncols, MAXCOLS_LDS);
    return IGP_EUNSUPPORTED;
  }
  const int g = static_cast<int>(ceil_div(n, NT));
  if (KQm)
    k_dir_update<T, true><<<g, NT, 0, s>>>(sv, Q, ldq, n, ncols, y, z, d, part, tv, KQm, kd,
                                           gate);
  else
    k_dir_update<T, false><<<g, NT, 0, s>>>(sv, Q, ldq, n, ncols, y, z, d, part, nullptr,
                                            nullptr, nullptr, gate);
  if (eta_out) k_finish_sum<<<1, NT, 0, s>>>(part, g, eta_out, gate);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int append_and_step(const T* d, const double* apart, const double* epart, double* scal, T* qcol,
                    T* v, int64_t n, hipStream_t s, const T* kd, T* kqcol, T* kv,
                    const int* gate) {
  const int anblk = grid_for(n), enblk = static_cast<int>(ceil_div(n, NT));
  if (kd)
    k_append_step<T, true><<<grid_for(n), NT, 0, s>>>(d, apart, anblk, epart, enblk, scal, qcol,
                                                      v, n, kd, kqcol, kv, gate);
  else
    k_append_step<T, false><<<grid_for(n), NT, 0, s>>>(d, apart, anblk, epart, enblk, scal, qcol,
                                                       v, n, nullptr, nullptr, nullptr, gate);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int gemv_n(const T* Q, int64_t ldq, int64_t n, int ncols, const double* y, T* out,
           hipStream_t s) {
  if (ncols > MAXCOLS_LDS) {
    set_error("buffer of %d columns exceeds %d", ncols, MAXCOLS_LDS);
    return IGP_EUNSUPPORTED;
  }
  k_gemv_n<T><<<static_cast<unsigned>(ceil_div(n, NT)), NT, 0, s>>>(Q, ldq, n, ncols, y, out);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int gram(const T* A, const T* B, int64_t ld, int64_t n, int ncols, double* part,
         size_t part_cap, double* M, hipStream_t s) {
  if (ncols == 0) return IGP_OK;
  const int tiles = static_cast<int>(ceil_div(ncols, GT));
  // enough row chunks (each a block per output tile) to keep every CU busy: the
  // kernel is bound by the latency of its 32-row passes, not by bandwidth
  int64_t nchunks = std::min<int64_t>(256, ceil_div(4096, static_cast<int64_t>(tiles) * tiles));
  const size_t per = static_cast<size_t>(ncols) * ncols;
  if (nchunks * per > part_cap) nchunks = static_cast<int64_t>(part_cap / per);
  if (nchunks < 1) {
    set_error("Gram workspace too small for %d columns", ncols);
    return IGP_ENOMEM;
  }
  int64_t rows_per = ceil_div(ceil_div(n, nchunks), GT) * GT;
  if (rows_per < GT) rows_per = GT;
  nchunks = ceil_div(n, rows_per);
  if (nchunks < 1) nchunks = 1;
  dim3 grid(tiles, tiles, static_cast<unsigned>(nchunks));
  k_gram<T><<<grid, NT, 0, s>>>(A, B, ld, n, ncols, rows_per, part);
  k_finish_gram<<<static_cast<unsigned>(ceil_div(static_cast<int64_t>(per), NT)), NT, 0, s>>>(
      part, static_cast<int>(nchunks), ncols, M);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int right_mul(const T* A, int64_t lda, int64_t n, int ncols, const double* U, int R,
              const double* colscale, T* Out, int64_t ldo, hipStream_t s) {
  if (R == 0 || n == 0) return IGP_OK;
  const size_t lds = static_cast<size_t>(ncols) * RM_COLS * sizeof(double);
  if (lds > 150 * 1024) {
    set_error("buffer of %d columns too wide for the re-weighting kernel", ncols);
    return IGP_EUNSUPPORTED;
  }
  dim3 grid(static_cast<unsigned>(ceil_div(n, NT)), static_cast<unsigned>(ceil_div(R, RM_COLS)));
  k_right_mul<T><<<grid, NT, lds, s>>>(A, lda, n, ncols, U, R, colscale, Out, ldo);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int newton_stats(const T* fnew, const T* f, const T* v, const int32_t* y, int64_t N, int64_t C,
                 double* part, double* scal, hipStream_t s) {
  const int g = static_cast<int>(ceil_div(N, NT));
  if (g == 0) return IGP_OK;
  k_newton_stats<T><<<g, NT, 0, s>>>(fnew, f, v, y, N, static_cast<int>(C), part);
  k_finish_sum<<<1, NT, 0, s>>>(part + 0 * g, g, scal + SC_DIFF2, nullptr);
  k_finish_sum<<<1, NT, 0, s>>>(part + 1 * g, g, scal + SC_FNEW2, nullptr);
  k_finish_sum<<<1, NT, 0, s>>>(part + 2 * g, g, scal + SC_LOGLIK, nullptr);
  k_finish_sum<<<1, NT, 0, s>>>(part + 3 * g, g, scal + SC_GV, nullptr);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <typename T>
int predict_epilogue(const T* A, int64_t lda, int64_t nrows, int ncols, const double* os_c,
                     const T* mean, int64_t Ns, int64_t C, T* var, T* probs, hipStream_t s) {
  (void)nrows;
  if (Ns == 0) return IGP_OK;
  IGP_REQUIRE(C <= 64, "C must be <= 64");
  PriorVar pv{};
  for (int c = 0; c < C; ++c) pv.v[c] = os_c[c];
  k_predict_epilogue<T><<<static_cast<unsigned>(ceil_div(Ns, 128)), 128, 0, s>>>(
      A, lda, nrows, ncols, pv, mean, Ns, static_cast<int>(C), var, probs);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

#define IGP_INST(T)                                                                             \
  template int residual<T>(const T*, const T*, const T*, T*, int64_t, double*, double*,        \
                           hipStream_t, const int*);                                           \
  template int residual_consume<T>(const T*, const T*, const T*, T*, int64_t, double*,         \
                                   double*, double, int*, double*, hipStream_t);               \
  template int dot_into<T>(const T*, const T*, int64_t, double*, double*, hipStream_t,         \
                           const int*);                                                        \
  template int action_cg_dot<T>(const T*, const double*, T*, int64_t, double*, double*,        \
                                const int*,                                                    \
                                hipStream_t);                                                  \
  template int consume_action_cg_dot<T>(const T*, const double*, int, double*, double, int*,   \
                                        double*, T*, int64_t, double*, hipStream_t);           \
  template int fill_unit<T>(T*, int64_t, int64_t, hipStream_t, const int*);                    \
  template int copy_vec<T>(const T*, T*, int64_t, hipStream_t, const int*);                    \
  template int fill_zero<T>(T*, int64_t, hipStream_t);                                         \
  template int add_vec<T>(const T*, const T*, T*, int64_t, hipStream_t);                       \
  template int gemv_t<T>(const T*, int64_t, int64_t, int, const T*, double*, double*,         \
                         hipStream_t, const int*);                                             \
  template int dir_update<T>(const T*, const T*, int64_t, int64_t, int, const double*,         \
                             const T*, T*, double*, double*, hipStream_t, const T*, const T*,  \
                             T*, const int*);                                                  \
  template int append_and_step<T>(const T*, const double*, const double*, double*, T*, T*,   \
                                  int64_t, hipStream_t, const T*, T*, T*, const int*);         \
  template int gemv_n<T>(const T*, int64_t, int64_t, int, const double*, T*, hipStream_t);     \
  template int gram<T>(const T*, const T*, int64_t, int64_t, int, double*, size_t, double*,   \
                       hipStream_t);                                                           \
  template int right_mul<T>(const T*, int64_t, int64_t, int, const double*, int,              \
                            const double*, T*, int64_t, hipStream_t);                          \
  template int newton_stats<T>(const T*, const T*, const T*, const int32_t*, int64_t, int64_t, \
                               double*, double*, hipStream_t);                                 \
  template int predict_epilogue<T>(const T*, int64_t, int64_t, int, const double*, const T*, int64_t, \
                                   int64_t, T*, T*, hipStream_t);
IGP_INST(float)
IGP_INST(double)

}  // namespace igp
