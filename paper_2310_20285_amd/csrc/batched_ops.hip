// The per-iteration vector operations of IterGP (Algorithm 2) for many models
// in one launch each: a block finds its model by binary search over the
// prefix of per-model block counts and runs the same device body, with the
// same block index and block count, as that model's single-model launch, so
// the batched iteration computes bit for bit what the models would compute
// one at a time.
#include "iter_ops.hpp"

namespace igp {
namespace {

using iter::NT;

// a model whose append step and residual run as one pass over its points
// (softmax likelihood, residual after the iteration): the single-model
// k_append_winv_residual, with alpha and eta from the finished scalars
__device__ __host__ inline bool fused_resid(const BIter& t, bool residual) {
  return residual && t.lik == IGP_LIK_SOFTMAX;
}

__device__ inline int find_model(const int64_t* __restrict__ pre, int nm, int64_t bid) {
  int lo = 0, hi = nm;            // pre[lo] <= bid < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= bid) lo = mid; else hi = mid;
  }
  return lo;
}

template <int OP>
__global__ void __launch_bounds__(NT)
kb_iter(const BIter* __restrict__ tab, const int64_t* __restrict__ pre, int nm) {
  const int m = find_model(pre, nm, blockIdx.x);
  const BIter& t = tab[m];
  if (t.gate && gate_closed(t.gate)) return;
  const int64_t bid = blockIdx.x - pre[m];
  const int64_t nblk = pre[m + 1] - pre[m];
  if constexpr (OP == BOP_ACTION) {
    if (t.policy == IGP_POLICY_CG)
      iter::action_cg<float>(t.r, t.scal + SC_RR, t.s, t.n, bid, nblk);
    else if (t.policy == IGP_POLICY_UNIT)
      iter::fill_unit<float>(t.s, t.n, t.unit_idx, bid, nblk);
    else
      iter::copy<float>(t.user, t.s, t.n, bid, nblk);
  } else if constexpr (OP == BOP_DOT_ALPHA) {
    __shared__ double red[NT / 64];
    iter::dot<float>(t.s, t.r, t.n, t.part, bid, nblk, red);
  } else if constexpr (OP == BOP_FIN_ALPHA || OP == BOP_FIN_ETA || OP == BOP_FIN_RR) {
    __shared__ double red[NT / 64];
    const int slot = OP == BOP_FIN_ALPHA ? SC_ALPHA : OP == BOP_FIN_ETA ? SC_ETA : SC_RR;
    const int np = OP == BOP_FIN_ETA ? static_cast<int>(iter::cdiv(t.n, NT))
                   : OP == BOP_FIN_RR && fused_resid(t, t.next_r) ? static_cast<int>(iter::cdiv(t.N, NT))
                                                                   : iter::grid_for(t.n);
    const double* part = OP == BOP_FIN_ETA ? t.epart : t.part;
    if (OP != BOP_FIN_RR || t.next_r) iter::finish_sum(part, np, t.scal + slot, red);
    if constexpr (OP == BOP_FIN_RR) {
      // device control: the end of the iteration (finish_sum wrote rr from thread 0)
      if (t.gate && threadIdx.x == 0)
        iter::consume_iteration(t.scal, t.thresh, t.next_r, t.gate, t.rec);
    }
  } else if constexpr (OP == BOP_WINV_Z || OP == BOP_WINV_V) {
    // z = t + W^+ s, or wv = W^+ v
    const float* V = OP == BOP_WINV_Z ? t.s : t.v;
    const float* Add = OP == BOP_WINV_Z ? t.t : nullptr;
    float* Out = OP == BOP_WINV_Z ? t.z : t.wv;
    const int64_t i = bid * NT + threadIdx.x;
    if (t.lik == IGP_LIK_SOFTMAX) {
      if (i < t.N) iter::winv_point<float, 8>(t.pi, 0, IGP_W_PINV, i, t.C, V, 0, t.n, Add, t.n,
                                              Out, t.n);
    } else {
      if (i < t.n) iter::winv_diag<float>(t.pi, i, V, 0, t.n, Add, t.n, Out, t.n);
    }
  } else if constexpr (OP == BOP_GEMV) {
    iter::gemv_t<float>(t.Q, t.ld, t.n, t.ncols, t.z, t.part, t.nchunks, bid);
  } else if constexpr (OP == BOP_FIN_COLS) {
    iter::finish_col(t.part, t.nchunks, t.ncols,
                     static_cast<int>(bid * (NT / 64) + (threadIdx.x >> 6)), t.yb);
  } else if constexpr (OP == BOP_DIR) {
    __shared__ double sy[iter::MAXCOLS_LDS];
    __shared__ double red[NT / 64];
    iter::dir_update<float, true>(t.s, t.Q, t.ld, t.n, t.ncols, t.yb, t.z, t.d, t.epart, t.t,
                                  t.KQ, t.kd, bid, sy, red);
  } else if constexpr (OP == BOP_APPEND) {
    if (fused_resid(t, t.next_r)) {
      // append and residual per point; the r^T r partials go to part (the
      // Q^T z partials there were summed by BOP_FIN_COLS; eta's are in epart)
      __shared__ double red[NT / 64];
      const int64_t i = bid * NT + threadIdx.x;
      double acc = 0.0;
      if (i < t.N) {
        iter::AppendPoint<float, 8> pt;
        pt.load_point(t.d, t.v, t.kd, t.kv, t.pi, t.rhs, i, t.C);
        acc = pt.append_residual(coherent_load(t.scal + SC_ALPHA), coherent_load(t.scal + SC_ETA),
                                 t.qcol, t.v, t.kqcol, t.kv, t.wv, t.r, i, t.C);
      }
      acc = block_sum(acc, red);
      if (threadIdx.x == 0) t.part[bid] = acc;
    } else {
      iter::append_step<float, true>(t.d, t.scal, t.qcol, t.v, t.n, t.kd, t.kqcol, t.kv, bid,
                                     nblk);
    }
  } else if constexpr (OP == BOP_RESID) {
    __shared__ double red[NT / 64];
    iter::residual<float>(t.rhs, t.kv, t.wv, t.r, t.n, t.part, bid, nblk, red);
  }
}

}  // namespace

int64_t biter_blocks(int op, const BIter& t, bool residual) {
  switch (op) {
    case BOP_ACTION:
    case BOP_DOT_ALPHA: return iter::grid_for(t.n);
    case BOP_APPEND: return fused_resid(t, residual) ? ceil_div(t.N, NT) : iter::grid_for(t.n);
    case BOP_FIN_ALPHA:
    case BOP_FIN_ETA: return 1;
    case BOP_WINV_Z: return ceil_div(t.lik == IGP_LIK_SOFTMAX ? t.N : t.n, NT);
    case BOP_GEMV: return t.ncols == 0 ? 0 : ceil_div(static_cast<int64_t>(t.nchunks) * t.ncols, NT / 64);
    case BOP_FIN_COLS: return t.ncols == 0 ? 0 : ceil_div(t.ncols, NT / 64);
    case BOP_DIR: return ceil_div(t.n, NT);
    case BOP_WINV_V:
      return residual && !fused_resid(t, residual)
                 ? ceil_div(t.lik == IGP_LIK_SOFTMAX ? t.N : t.n, NT) : 0;
    case BOP_RESID: return residual && !fused_resid(t, residual) ? iter::grid_for(t.n) : 0;
    case BOP_FIN_RR: return residual || t.gate ? 1 : 0;   // device control: always the end
    default: return 0;
  }
}

int biter_launch(int op, const BIter* tab, const int64_t* pre, int nm, int64_t total,
                 hipStream_t s) {
  if (total == 0 || nm == 0) return IGP_OK;
  if (total > INT32_MAX) {
    set_error("batched iteration launch too large");
    return IGP_EINVAL;
  }
  const dim3 grid(static_cast<unsigned>(total));
  switch (op) {
    case BOP_ACTION: kb_iter<BOP_ACTION><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    case BOP_DOT_ALPHA: kb_iter<BOP_DOT_ALPHA><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    case BOP_FIN_ALPHA: kb_iter<BOP_FIN_ALPHA><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    case BOP_WINV_Z: kb_iter<BOP_WINV_Z><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    case BOP_GEMV: kb_iter<BOP_GEMV><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    case BOP_FIN_COLS: kb_iter<BOP_FIN_COLS><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    case BOP_DIR: kb_iter<BOP_DIR><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    case BOP_FIN_ETA: kb_iter<BOP_FIN_ETA><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    case BOP_APPEND: kb_iter<BOP_APPEND><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    case BOP_WINV_V: kb_iter<BOP_WINV_V><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    case BOP_RESID: kb_iter<BOP_RESID><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    case BOP_FIN_RR: kb_iter<BOP_FIN_RR><<<grid, NT, 0, s>>>(tab, pre, nm); break;
    default: set_error("unknown batched operation %d", op); return IGP_EINVAL;
  }
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

}  // namespace igp
