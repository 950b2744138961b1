// Device bodies of the per-iteration vector operations of the IterGP loop,
// shared by the single-model kernels (linalg.hip, hessian.hip) and by the
// batched kernels that run the same operation for many models in one launch
// (batched_ops.hip).  Each body takes its block index and block count within
// the operation, so a batched launch gives every model exactly the blocks and
// the summation order of its own single-model launch.
#pragma once

#include "ops.hpp"

namespace igp {
namespace iter {

constexpr int NT = 256;
constexpr int GV_ROWS = QTZ_ROWS;    // rows per wave of the Q^T z pass
constexpr int MAXCOLS_LDS = 4096;    // y staged in LDS by the direction update

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// blocks of a grid-stride reduction over n elements
__host__ __device__ inline int grid_for(int64_t n) {
  int64_t b = cdiv(n, NT * 4);
  if (b > RED_BLOCKS) b = RED_BLOCKS;
  if (b < 1) b = 1;
  return static_cast<int>(b);
}

// fixed-order sum of nblk partials (one block)
__device__ inline void finish_sum(const double* __restrict__ part, int nblk, double* out,
                                  double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += NT) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

// end of a solver iteration (one thread): unless the gate is closed, count it,
// close the gate on a breakdown (eta <= 0) or convergence, keep min eta and rr
__device__ inline void consume_iteration(const double* __restrict__ scal, double thresh,
                                         int next_r, int* gate, double* rec) {
  if (gate_closed(gate)) return;
  rec[REC_EXEC] = coherent_load(rec + REC_EXEC) + 1.0;
  const double eta = coherent_load(scal + SC_ETA);
  if (!(eta > 0.0)) {   // breakdown: the iteration's column was not appended
    rec[REC_BREAK] = 1.0;
    __hip_atomic_store(gate, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  rec[REC_APPEND] = coherent_load(rec + REC_APPEND) + 1.0;
  rec[REC_ETAMIN] = fmin(coherent_load(rec + REC_ETAMIN), eta);
  if (next_r) {
    const double rr = coherent_load(scal + SC_RR);
    rec[REC_RR] = rr;
    if (!(sqrt(rr) >= thresh)) {
      rec[REC_CONV] = 1.0;
      __hip_atomic_store(gate, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// r = rhs - kv - wv ; part[bid] = sum of r^2 over this block's rows
template <typename T>
__device__ inline void residual(const T* __restrict__ rhs, const T* __restrict__ kv,
                                const T* __restrict__ wv, T* __restrict__ r, int64_t n,
                                double* __restrict__ part, int64_t bid, int64_t nblk,
                                double* red) {
  double acc = 0.0;
  for (int64_t i = bid * NT + threadIdx.x; i < n; i += nblk * NT) {
    const T ri = rhs[i] - kv[i] - wv[i];
    r[i] = ri;
    acc += static_cast<double>(ri) * static_cast<double>(ri);
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[bid] = acc;
}

template <typename T>
__device__ inline void dot(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                           double* __restrict__ part, int64_t bid, int64_t nblk, double* red) {
  double acc = 0.0;
  for (int64_t i = bid * NT + threadIdx.x; i < n; i += nblk * NT)
    acc += static_cast<double>(a[i]) * static_cast<double>(b[i]);
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[bid] = acc;
}

// s = r / sqrt(r^T r)
template <typename T>
__device__ inline void action_cg(const T* __restrict__ r, const double* __restrict__ rr,
                                 T* __restrict__ s, int64_t n, int64_t bid, int64_t nblk) {
  const double inv = 1.0 / sqrt(coherent_load(rr));
  for (int64_t i = bid * NT + threadIdx.x; i < n; i += nblk * NT)
    s[i] = static_cast<T>(static_cast<double>(r[i]) * inv);
}

template <typename T>
__device__ inline void fill_unit(T* __restrict__ s, int64_t n, int64_t idx, int64_t bid,
                                 int64_t nblk) {
  for (int64_t i = bid * NT + threadIdx.x; i < n; i += nblk * NT) s[i] = (i == idx) ? T(1) : T(0);
}

template <typename T>
__device__ inline void copy(const T* __restrict__ a, T* __restrict__ b, int64_t n, int64_t bid,
                            int64_t nblk) {
  for (int64_t i = bid * NT + threadIdx.x; i < n; i += nblk * NT) b[i] = a[i];
}

// partial Q^T z: one wave per (column, chunk of GV_ROWS rows); wave index
// wid = bid * 4 + wave of the block
template <typename T>
__device__ inline void gemv_t(const T* __restrict__ Q, int64_t ldq, int64_t n, int ncols,
                              const T* __restrict__ z, double* __restrict__ part, int nchunks,
                              int64_t bid) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = bid * (NT / 64) + (threadIdx.x >> 6);
  if (wid >= static_cast<int64_t>(nchunks) * ncols) return;
  const int b = static_cast<int>(wid % ncols);
  const int64_t chunk = wid / ncols;
  const int64_t r0 = chunk * GV_ROWS;
  const T* q = Q + static_cast<int64_t>(b) * ldq;
  double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
  for (int k = 0; k < GV_ROWS / 64; k += 2) {
    const int64_t i0 = r0 + k * 64 + lane, i1 = i0 + 64;
    if (i0 < n) acc0 += static_cast<double>(q[i0]) * static_cast<double>(z[i0]);
    if (i1 < n) acc1 += static_cast<double>(q[i1]) * static_cast<double>(z[i1]);
  }
  const double s = wave_sum(acc0 + acc1);
  if (lane == 0) part[static_cast<int64_t>(b) * nchunks + chunk] = s;   // column-major
}

// y[b] = fixed-order sum of the chunk partials of column b (one thread per column)
__device__ inline void finish_col(const double* __restrict__ part, int nchunks, int ncols,
                                  int b, double* __restrict__ y) {
  // one wave per column b: lane l adds the chunk partials l, l + 64, ..., then
  // a fixed butterfly over the wave
  if (b >= ncols) return;
  const int lane = threadIdx.x & 63;
  const double* p = part + static_cast<int64_t>(b) * nchunks;
  double s = 0.0;
  for (int r = lane; r < nchunks; r += 64) s += p[r];
  s = wave_sum(s);
  if (lane == 0) y[b] = s;
}

// d = s - Q y (and kd = t - KQ y) ; epart[bid] = z^T d over this block's rows.
// sy: LDS staging of y (MAXCOLS_LDS doubles)
template <typename T, bool KQ>
__device__ inline void dir_update(const T* __restrict__ sv, const T* __restrict__ Q, int64_t ldq,
                                  int64_t n, int ncols, const double* __restrict__ y,
                                  const T* __restrict__ z, T* __restrict__ d,
                                  double* __restrict__ epart, const T* __restrict__ tv,
                                  const T* __restrict__ KQm, T* __restrict__ kd, int64_t bid,
                                  double* sy, double* red) {
  for (int b = threadIdx.x; b < ncols; b += NT) sy[b] = y[b];
  __syncthreads();
  const int64_t i = bid * NT + threadIdx.x;
  double e = 0.0;
  if (i < n) {
    double acc = 0.0, acck = 0.0;
    int b = 0;
    for (; b + 4 <= ncols; b += 4) {
      const double q0 = Q[static_cast<int64_t>(b) * ldq + i];
      const double q1 = Q[static_cast<int64_t>(b + 1) * ldq + i];
      const double q2 = Q[static_cast<int64_t>(b + 2) * ldq + i];
      const double q3 = Q[static_cast<int64_t>(b + 3) * ldq + i];
      acc += q0 * sy[b] + q1 * sy[b + 1] + q2 * sy[b + 2] + q3 * sy[b + 3];
      if constexpr (KQ) {
        const double k0 = KQm[static_cast<int64_t>(b) * ldq + i];
        const double k1 = KQm[static_cast<int64_t>(b + 1) * ldq + i];
        const double k2 = KQm[static_cast<int64_t>(b + 2) * ldq + i];
        const double k3 = KQm[static_cast<int64_t>(b + 3) * ldq + i];
        acck += k0 * sy[b] + k1 * sy[b + 1] + k2 * sy[b + 2] + k3 * sy[b + 3];
      }
    }
    for (; b < ncols; ++b) {
      acc += static_cast<double>(Q[static_cast<int64_t>(b) * ldq + i]) * sy[b];
      if constexpr (KQ) acck += static_cast<double>(KQm[static_cast<int64_t>(b) * ldq + i]) * sy[b];
    }
    const T di = static_cast<T>(static_cast<double>(sv[i]) - acc);
    d[i] = di;
    if constexpr (KQ) kd[i] = static_cast<T>(static_cast<double>(tv[i]) - acck);
    e = static_cast<double>(z[i]) * static_cast<double>(di);
  }
  e = block_sum(e, red);
  if (threadIdx.x == 0) epart[bid] = e;
}

// eta > 0: Q column = d / sqrt(eta), v += (alpha / eta) d (and the K Q / K v twins)
template <typename T, bool KQ>
__device__ inline void append_step_vals(const T* __restrict__ d, double alpha, double eta,
                                        T* __restrict__ qcol, T* __restrict__ v, int64_t n,
                                        const T* __restrict__ kd, T* __restrict__ kqcol,
                                        T* __restrict__ kv, int64_t bid, int64_t nblk) {
  if (!(eta > 0.0)) return;
  const double qs = 1.0 / sqrt(eta);
  const double step = alpha / eta;
  for (int64_t i = bid * NT + threadIdx.x; i < n; i += nblk * NT) {
    const double di = static_cast<double>(d[i]);
    qcol[i] = static_cast<T>(di * qs);
    v[i] = static_cast<T>(static_cast<double>(v[i]) + step * di);
    if constexpr (KQ) {
      const double ki = static_cast<double>(kd[i]);
      kqcol[i] = static_cast<T>(ki * qs);
      kv[i] = static_cast<T>(static_cast<double>(kv[i]) + step * ki);
    }
  }
}

// the same with alpha and eta read from scal
template <typename T, bool KQ>
__device__ inline void append_step(const T* __restrict__ d, const double* __restrict__ scal,
                                   T* __restrict__ qcol, T* __restrict__ v, int64_t n,
                                   const T* __restrict__ kd, T* __restrict__ kqcol,
                                   T* __restrict__ kv, int64_t bid, int64_t nblk) {
  append_step_vals<T, KQ>(d, coherent_load(scal + SC_ALPHA), coherent_load(scal + SC_ETA), qcol,
                          v, n, kd, kqcol, kv, bid, nblk);
}

// ---- softmax-Hessian blocks (one thread per data point) ----------------------

template <typename T, int CMAX>
__device__ inline void load_softmax(const T* F, int64_t n, int C, T (&p)[CMAX]) {
  T mx = -INFINITY;
#pragma unroll
  for (int c = 0; c < CMAX; ++c)
    if (c < C) {
      p[c] = F[n * C + c];
      mx = p[c] > mx ? p[c] : mx;
    }
  T sum = T(0);
#pragma unroll
  for (int c = 0; c < CMAX; ++c)
    if (c < C) {
      p[c] = exp(p[c] - mx);
      sum += p[c];
    }
  const T inv = T(1) / sum;
#pragma unroll
  for (int c = 0; c < CMAX; ++c)
    if (c < C) p[c] *= inv;
}

// u <- W^+ u (mode IGP_W_PINV) or u <- W u (mode IGP_W), in place
template <typename T, int CMAX>
__device__ inline void apply_block(int mode, int C, const T (&p)[CMAX], T (&u)[CMAX]) {
  if (mode == IGP_W_PINV) {
    T m = T(0);
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) m += u[c];
    m /= T(C);
    T m2 = T(0);
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) {
        u[c] = (u[c] - m) / p[c];
        m2 += u[c];
      }
    m2 /= T(C);
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) u[c] -= m2;
  } else {
    T pv = T(0);
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) pv += p[c] * u[c];
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) u[c] = p[c] * u[c] - p[c] * pv;
  }
}

// Out_b (point n) = W_n^+ V_b (+ Add_b) for data point n of column b
template <typename T, int CMAX>
__device__ inline void winv_point(const T* __restrict__ pi, int logits, int mode, int64_t n,
                                  int C, const T* __restrict__ V, int64_t b, int64_t ldv,
                                  const T* __restrict__ Add, int64_t lda, T* __restrict__ Out,
                                  int64_t ldo) {
  T p[CMAX], u[CMAX];
  if (logits) {
    load_softmax<T, CMAX>(pi, n, C, p);
  } else {
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) p[c] = pi[n * C + c];
  }
#pragma unroll
  for (int c = 0; c < CMAX; ++c)
    if (c < C) u[c] = V[b * ldv + n * C + c];
  apply_block<T, CMAX>(mode, C, p, u);
#pragma unroll
  for (int c = 0; c < CMAX; ++c)
    if (c < C) {
      T o = u[c];
      if (Add) o += Add[b * lda + n * C + c];
      Out[b * ldo + n * C + c] = o;
    }
}

// Out_b[i] = winv[i] V_b[i] (+ Add_b[i]) (diagonal W^{-1})
template <typename T>
__device__ inline void winv_diag(const T* __restrict__ winv, int64_t i, const T* __restrict__ V,
                                 int64_t b, int64_t ldv, const T* __restrict__ Add, int64_t lda,
                                 T* __restrict__ Out, int64_t ldo) {
  T o = winv[i] * V[b * ldv + i];
  if (Add) o += Add[b * lda + i];
  Out[b * ldo + i] = o;
}

// The append step of a solver iteration followed by its residual, for data
// point n (softmax likelihood, recurrence residual), in two parts so that a
// kernel can issue the point's loads before it finishes alpha and eta:
// load_point takes the point's d, v, K d, K v, pi and rhs; append_residual
// then, with eta > 0, sets the point's Q and K Q entries and advances v, K v
// (the values of append_step_vals), and forms wv = W^+ v and
// r = rhs - K v - wv.  Returns the point's part of r^T r.
template <typename T, int CMAX>
struct AppendPoint {
  T d[CMAX], v[CMAX], kd[CMAX], kv[CMAX], p[CMAX], rhs[CMAX];

  __device__ inline void load_point(const T* __restrict__ dg, const T* __restrict__ vg,
                                    const T* __restrict__ kdg, const T* __restrict__ kvg,
                                    const T* __restrict__ pi, const T* __restrict__ rhsg,
                                    int64_t n, int C) {
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) {
        const int64_t i = n * C + c;
        d[c] = dg[i];
        v[c] = vg[i];
        kd[c] = kdg[i];
        kv[c] = kvg[i];
        p[c] = pi[i];
        rhs[c] = rhsg[i];
      }
  }

  __device__ inline double append_residual(double alpha, double eta, T* __restrict__ qcol,
                                           T* __restrict__ vg, T* __restrict__ kqcol,
                                           T* __restrict__ kvg, T* __restrict__ wv,
                                           T* __restrict__ r, int64_t n, int C) {
    const bool app = eta > 0.0;
    const double qs = app ? 1.0 / sqrt(eta) : 0.0;
    const double step = app ? alpha / eta : 0.0;
    if (app) {
#pragma unroll
      for (int c = 0; c < CMAX; ++c)
        if (c < C) {
          const int64_t i = n * C + c;
          const double di = static_cast<double>(d[c]);
          qcol[i] = static_cast<T>(di * qs);
          v[c] = static_cast<T>(static_cast<double>(v[c]) + step * di);
          vg[i] = v[c];
          const double kdi = static_cast<double>(kd[c]);
          kqcol[i] = static_cast<T>(kdi * qs);
          kv[c] = static_cast<T>(static_cast<double>(kv[c]) + step * kdi);
          kvg[i] = kv[c];
        }
    }
    T u[CMAX];
#pragma unroll
    for (int c = 0; c < CMAX; ++c) u[c] = c < C ? v[c] : T(0);
    apply_block<T, CMAX>(IGP_W_PINV, C, p, u);
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < CMAX; ++c)
      if (c < C) {
        const int64_t i = n * C + c;
        wv[i] = u[c];
        const T ri = rhs[c] - kv[c] - u[c];
        r[i] = ri;
        acc += static_cast<double>(ri) * static_cast<double>(ri);
      }
    return acc;
  }
};

}  // namespace iter
}  // namespace igp
