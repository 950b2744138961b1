// Internal launchers of the HIP kernels (not part of the public ABI).
#pragma once
#include "common.hpp"

// Host-side handle behind the opaque igp_model of the public header.
struct igp_model {
  virtual ~igp_model() = default;
  virtual int newton_step(igp_step_info* info) = 0;
  virtual int predict(const void* Xs, int64_t Ns, void* mean, void* var, void* probs, void* ws,
                      size_t ws_bytes, hipStream_t s) const = 0;
  virtual size_t predict_ws_bytes(int64_t Ns) const = 0;
  virtual int view(int which, const void** ptr, int64_t* rows, int64_t* cols,
                   int64_t* ld) const = 0;
  virtual int set_user_actions(const void* a, int64_t ncols, int64_t ld) = 0;
  virtual int set_profiling(int enable) = 0;
  virtual int set_block_likelihood(const void* grad, const void* W) = 0;
  virtual int get_profile(igp_profile* out) const = 0;
  virtual int compress(int32_t rank_limit, int32_t* kept) = 0;
  virtual int step_begin() = 0;
  virtual int step_iterate(int64_t max_iters, int32_t* done) = 0;
  virtual int step_end(igp_step_info* info) = 0;
};

namespace igp {

// ---- matrix-free kernel product ------------------------------------------
// Out_b = os * (K_X(X1, X2) (x) I_C) V_b + beta * Out_b for b < nb.
// `skip` (device, nullable): when *skip != 0 the launch does nothing.
struct KVProblem {
  igp_kernel_params kp;
  int precision;          // igp_precision
  const void* X1;         // n1 x d (T); for IGP_BF16 float rows (centred)
  const void* X2;
  int64_t n1, n2, d;
  const void* V;          // nb CN vectors, stride ldv
  int64_t C, nb, ldv;
  void* Out;
  int64_t ldo;
  double beta;
  // optional prepared rows for the matrix-core paths: X - centre (common
  // centre for X1 and X2), zero-padded to a multiple of 16 features, and the
  // squared norms of those rows.  When absent the launcher prepares them in ws.
  const void* X1p = nullptr;     // float rows (FP32 path) or __bf16 rows (BF16 path)
  const void* X2p = nullptr;
  const float* norm1 = nullptr;
  const float* norm2 = nullptr;
  const int* skip = nullptr;
  // set by the launcher when non-null: 1 if the product evaluated each pair of
  // rows once (same prepared rows on both sides), else 0
  int* symmetric_out = nullptr;
  // one kernel per latent function (same family, class-specific lengthscale and
  // outputscale): kpc[c] for c < C when n_kp == C > 1
  const igp_kernel_params* kpc = nullptr;
  int n_kp = 1;
  // split the X2 rows into fixed ranges regardless of n1 (4096 rows; on the
  // FP32 matrix cores 512 rows for outputs at most 16 wide and about n2 / 20
  // rows, at least 1024, for outputs at most 512 wide), so that each output
  // row is summed in the same order whatever rows share the launch
  bool fixed_split = false;
  // optional epilogue of the final reduction (one vector, nb == 1, beta == 0):
  // z = Out + W^+ s at every point, W^+ the pseudo-inverse of the softmax
  // Hessian block from the probabilities epi_pi (N x C), s = epi_s (N x C),
  // into epi_z (N x C); the launcher sets *epi_applied to 1 when it took it
  // (else the caller forms z itself)
  const void* epi_pi = nullptr;
  const void* epi_s = nullptr;
  void* epi_z = nullptr;
  int* epi_applied = nullptr;
};
constexpr int64_t FIXED_SPLIT_ROWS = 4096;
constexpr int64_t FIXED_SPLIT_ROWS_NARROW = 512;
// rows per wave of the Q^T z pass of a solver iteration (partials per column: n / QTZ_ROWS)
constexpr int QTZ_ROWS = 1024;

size_t kv_ws_bytes(int64_t n1, int64_t n2, int64_t d, int64_t C, int64_t nb, int precision,
                   bool fixed_split = false);
// bytes of ws needed when X1p/X2p/norms are supplied (partials only)
size_t kv_ws_bytes_prepared(int64_t n1, int64_t n2, int64_t d, int64_t C, int64_t nb,
                            int precision, bool fixed_split = false);
int kv_launch(const KVProblem& p, void* ws, size_t ws_bytes, hipStream_t s);
// whether (precision, kind, d) runs on the matrix cores from prepared rows
bool kv_uses_prepared(int precision, int kind, int64_t d);

// FP32 matrix-core kernel product (kv_mfma.hip)
bool mfma_f32_supported(int kind, int64_t d);
size_t mfma_f32_partial_bytes(int64_t n1, int64_t n2, int64_t d, int64_t W, bool fixed = false);
int64_t padded_dim(int64_t d);
int column_mean_f32(const float* X, int64_t n, int64_t d, float* mean, double* part,
                    int64_t part_cap, hipStream_t s);
int prep_rows_f32(const float* X, int64_t n, int64_t d, const float* centre, float* Xp,
                  float* norms, hipStream_t s);
// a per-class FP32 product that the symmetric matrix-core kernel can take
bool mfma_f32_perclass_ok(const KVProblem& p);
int kv_mfma_f32_launch(const KVProblem& p, const float* X1p, const float* n1p,
                       const float* X2p, const float* n2p, float* P, size_t P_bytes,
                       hipStream_t s, int* nsplit_out);

// Batched persistent product (kv_mfma.hip): one launch covers the narrow
// products (W <= 8) of many independent problems.
struct BatchProblem {
  const void* X1p;          // prepared rows: float (FP32 models) or __bf16 (BF16 models)
  const float* nrm1;
  const void* X2p;
  const float* nrm2;
  int64_t n1, n2;
  const float* V;
  int64_t ldv;
  int C, W;
  float* P;                 // split partials: nsplit * n1 * W floats
  int64_t cols_per_split;
  int nsplit, gx;
  float cnorm, cdot, os;
  float* Out;
  int64_t ldo;
  int64_t tile_begin;       // prefix over problems of gx * nsplit
  int64_t out_begin;        // prefix over problems of n1 * W
  const int* gate;          // device control: the problem's iteration gate (or null)
  // symmetric plan (FP32, K(X, X) V): sym_q super-blocks of sym_g row blocks,
  // sym_q (sym_q + 1) / 2 items, nsplit = sym_q partial slots, sym_kb feature
  // k-blocks of the distance; sym_q = 0: one-sided tiles
  int sym_g, sym_q, sym_kb;
};
// One model's part of a batched solver iteration (recurrence residual, FP32):
// the vectors and scalars the per-iteration operations touch.
struct BIter {
  float *r, *s, *t, *z, *d, *v, *kv, *kd, *rhs, *wv, *Q, *KQ, *qcol, *kqcol;
  const float* pi;          // softmax probabilities, or the diagonal of W^{-1}
  const float* user;        // this iteration's user action (policy USER)
  double *scal, *part, *epart, *yb;
  int64_t n, N, ld, unit_idx;
  int C, ncols, lik, policy, nchunks, pad;
  // device control (null gate: the host decides after every round): every
  // operation of a closed gate returns at once; BOP_FIN_RR ends the iteration
  // (iter::consume_iteration with thresh and next_r) even without a residual
  int* gate;
  double* rec;
  double thresh;
  int next_r, pad2;
};
// operations of a batched iteration, in launch order
enum BIterOp {
  BOP_ACTION = 0, BOP_DOT_ALPHA, BOP_FIN_ALPHA,               // s_j, alpha_j
  BOP_WINV_Z, BOP_GEMV, BOP_FIN_COLS, BOP_DIR, BOP_FIN_ETA,   // z_j, Q^T z_j, d_j, eta_j
  BOP_APPEND,                                                 // Q, K Q, v, K v
  BOP_WINV_V, BOP_RESID, BOP_FIN_RR,                          // r_j, ||r_j||^2
  BOP_COUNT
};
// blocks of operation `op` for one model (0: the model skips it)
int64_t biter_blocks(int op, const BIter& t, bool residual);
// runs operation `op` for nm models: tab[nm] (device), pre[nm + 1] (device,
// prefix of biter_blocks), total = pre[nm]
int biter_launch(int op, const BIter* tab, const int64_t* pre, int nm, int64_t total,
                 hipStream_t s);
bool batched_supported(int kind, int64_t d, int64_t W);
void batched_plan(int64_t n1, int64_t n2, int64_t W, int ns, int64_t split_rows, BatchProblem* bp);
// The symmetric plan of an FP32 product K(X, X) V (n rows, d features, W
// columns) in the batched launch: sets sym_g, sym_q and nsplit and returns
// true, or returns false (the problem takes one-sided tiles).  The plan is the
// single-problem launch's, so the product equals that launch's bit for bit.
bool batched_sym_plan(int64_t n, int64_t d, int64_t W, BatchProblem* bp);
// LDS bytes of a symmetric problem's items; workgroup tiles of a problem
size_t batched_sym_lds(const BatchProblem& bp, int dch);
int64_t batched_tiles(const BatchProblem& bp);
// The symmetric problems of one output width W and distance k-block count kb:
// dprobs[first, first + count), tile prefixes over them from 0, `tiles` items,
// `lds` the largest plan's LDS.
struct SymGroup {
  int first, count, W, kb;
  int64_t tiles;
  size_t lds;
};
// 64-bit queue counters a batched launch needs (one per symmetric group, one
// for the one-sided problems)
constexpr int BATCH_COUNTERS = 32;
// The products of a batch: the symmetric groups (problems sorted by (W, kb), first
// in the table), then dprobs[nsym, np) one-sided (tile prefixes from 0, ntiles
// tiles), then one reduction over all np (out_begin prefixes over all).
int kv_batched_run(int kind, int dch, int ns, bool bf16, const BatchProblem* dprobs, int np,
                   const SymGroup* groups, int ngroups, int64_t ntiles, int64_t total_out,
                   int* counter, hipStream_t s);
float kv_kappa(int kind);
// BF16 products with few features on the narrow BF16 tile (kv_mfma.hip)
bool bf16_narrow_supported(int kind, int64_t d, int64_t W);
size_t bf16_narrow_partial_bytes(int64_t n1, int64_t n2, int64_t W, bool fixed);
int kv_bf16_narrow_launch(const KVProblem& p, const void* X1b, const float* n1p,
                          const void* X2b, const float* n2p, float* P, size_t P_bytes,
                          hipStream_t s, int* nsplit_out);

// BF16 matrix-core kernel product (kv_bf16.hip): rows rounded to BF16, padded
// to a multiple of 32 features, norms of the rounded rows.
int64_t bf16_padded_dim(int64_t d);
// the BF16 matrix-core modes (plain, and hi/lo split of the inputs)
inline bool is_bf16(int precision) { return precision == IGP_BF16 || precision == IGP_BF16X3; }
// BF16 elements of n prepared rows: the high parts, then (IGP_BF16X3) the low parts
inline int64_t bf16_rows_elems(int precision, int64_t n, int64_t d) {
  return n * bf16_padded_dim(d) * (precision == IGP_BF16X3 ? 2 : 1);
}
size_t bf16_partial_bytes(int64_t n1, int64_t n2, int64_t W, bool fixed = false);
int prep_rows_bf16(int precision, const float* X, int64_t n, int64_t d, const float* centre, void* Xb,
                   float* norms, hipStream_t s);
int kv_bf16_launch(const KVProblem& p, const void* X1b, const float* n1p, const void* X2b,
                   const float* n2p, float* P, size_t P_bytes, hipStream_t s, int* nsplit_out);
// bytes of one prepared row set (rows + norms) for (precision, d)
size_t prepared_rows_bytes(int precision, int64_t n, int64_t d);
int prep_rows_any(int precision, const float* X, int64_t n, int64_t d, const float* centre,
                  void* rows, float* norms, hipStream_t s);

// ---- softmax Hessian blocks ---------------------------------------------------
// pi = softmax(F) per point; rhs = F + W^+ (onehot(y) - pi); loglik partials.
template <typename T>
int softmax_pi_rhs(const T* F, const int32_t* y, int64_t N, int64_t C, T* pi, T* rhs,
                   double* loglik_partials, int* nblocks_out, hipStream_t s);
// Out_b = W^+ V_b (+ Add_b) using stored pi, or from logits when pi_is_logits.
template <typename T>
int winv_apply(const T* pi, bool pi_is_logits, int mode, int64_t N, int64_t C,
               const T* V, int64_t nb, int64_t ldv, const T* Add, int64_t lda,
               T* Out, int64_t ldo, hipStream_t s, const int* gate = nullptr);

// ---- reductions and projections (FP64 accumulation) ---------------------------
constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 1024;   // max partial blocks of a grid-stride reduction

enum Scalar {
  SC_RR = 0,       // ||r||^2
  SC_ALPHA,        // s^T r
  SC_ETA,          // z^T d
  SC_RHS2,         // ||rhs||^2
  SC_DIFF2,        // ||f_new - f||^2
  SC_FNEW2,        // ||f_new||^2
  SC_LOGLIK,       // log p(y | f)
  SC_GV,           // g^T v
  SC_COUNT
};

// The launchers below that take `gate` skip their work (every kernel returns at
// once) while *gate != 0: the solver enqueues iterations ahead of their
// convergence test and the test closes the gate (iter_consume).
template <typename T>
int residual(const T* rhs, const T* kv, const T* wv, T* r, int64_t n, double* partials,
             double* out_scalar, hipStream_t s, const int* gate = nullptr);
// the residual of a solver iteration, its norm finished together with the
// iteration's end (iter_consume with next_r = 1)
// rr = the fixed-order sum of nblk residual partials into scal[SC_RR], then
// the end of the solver iteration as in residual_consume
int rr_consume(const double* partials, int nblk, double* scal, double thresh, int* gate,
               double* rec, hipStream_t s);
// The append step (Q and K Q columns, v, K v; alpha and eta finished from
// their partials and stored to scal) and the residual r = rhs - K v - W^+ v
// with wv = W^+ v in one pass over the N points (softmax likelihood,
// recurrence residual); part: the ceil(N / 256) block partials of r^T r
// (must not alias epart).
template <typename T>
int append_winv_residual(const T* d, const double* apart, const double* epart, double* scal,
                         T* qcol, T* v, const T* kd, T* kqcol, T* kv, const T* pi, int64_t N,
                         int64_t C, const T* rhs, T* wv, T* r, double* part, int* nblk_out,
                         hipStream_t s, const int* gate);
// softmax: wv = W^+ v, r = rhs - kv - wv and ceil(N / 256) partials of r^T r
// (one thread per point), *nblk_out = their count
template <typename T>
int winv_residual(const T* pi, int64_t N, int64_t C, const T* v, const T* rhs, const T* kv,
                  T* wv, T* r, double* partials, int* nblk_out, hipStream_t s,
                  const int* gate = nullptr);
template <typename T>
int residual_consume(const T* rhs, const T* kv, const T* wv, T* r, int64_t n, double* partials,
                     double* scal, double thresh, int* gate, double* rec, hipStream_t s);
// a^T b: grid_for(n) block partials, then (when out_scalar is non-null) their
// fixed-order sum into out_scalar
template <typename T>
int dot_into(const T* a, const T* b, int64_t n, double* partials, double* out_scalar,
             hipStream_t s, const int* gate = nullptr);
// s = r / sqrt(rr) and the grid_for(n) partials of alpha = s^T r in one pass
// over r, then (when alpha is non-null) their sum into alpha
template <typename T>
int action_cg_dot(const T* r, const double* rr, T* s_out, int64_t n, double* partials,
                  double* alpha, const int* gate, hipStream_t s);
// The end of the previous solver iteration and the CG action of this one in
// one launch: rr = the fixed-order sum of the previous residual's rnblk
// partials (rpart), stored to scal[SC_RR] with that iteration's end
// (iter_consume with next_r = 1) by one thread; every block takes the same
// stop decision (breakdown or rr below thresh^2) and, when it goes on, forms
// s = r / sqrt(rr) and the grid_for(n) partials of alpha = s^T r (apart)
template <typename T>
int consume_action_cg_dot(const T* r, const double* rpart, int rnblk, double* scal,
                          double thresh, int* gate, double* rec, T* s_out, int64_t n,
                          double* apart, hipStream_t s);
template <typename T>
int fill_unit(T* s_out, int64_t n, int64_t idx, hipStream_t s, const int* gate = nullptr);
template <typename T>
int copy_vec(const T* src, T* dst, int64_t n, hipStream_t s, const int* gate = nullptr);
template <typename T>
int fill_zero(T* a, int64_t n, hipStream_t s);
template <typename T>
int add_vec(const T* a, const T* b, T* out, int64_t n, hipStream_t s);
// y[b] = sum_i Q[b*ldq + i] z[i], b < ncols
template <typename T>
int gemv_t(const T* Q, int64_t ldq, int64_t n, int ncols, const T* z, double* partials,
           double* y, hipStream_t s, const int* gate = nullptr);
// d = s - Q y ; the ceil(n / 256) partials of eta = z^T d, summed into eta_out
// when it is non-null ; with KQ: also kd = t - KQ y (= K d)
template <typename T>
int dir_update(const T* sv, const T* Q, int64_t ldq, int64_t n, int ncols, const double* y,
               const T* z, T* d, double* partials, double* eta_out, hipStream_t s,
               const T* tv = nullptr, const T* KQ = nullptr, T* kd = nullptr,
               const int* gate = nullptr);
// alpha and eta from their partials (alpha_part: the grid_for(n) partials of
// dot_into / action_cg_dot; eta_part: the ceil(n / 256) partials of
// dir_update), summed in the same fixed order as the finishing kernel by every
// block and stored in scal[SC_ALPHA], scal[SC_ETA]; then
// Q[:, col] = d / sqrt(eta); v += (alpha/eta) d   (no-op when eta <= 0)
// with kd: also KQ[:, col] = kd / sqrt(eta); kv += (alpha/eta) kd
template <typename T>
int append_and_step(const T* d, const double* alpha_part, const double* eta_part, double* scal,
                    T* qcol, T* v, int64_t n, hipStream_t s, const T* kd = nullptr,
                    T* kqcol = nullptr, T* kv = nullptr, const int* gate = nullptr);
// Device-side end of a solver iteration (after its eta and, when next_r, its
// residual norm are in scal): unless the gate is already closed, count the
// iteration in rec, close the gate on a breakdown (eta <= 0) or when
// sqrt(rr) < thresh, and keep the smallest eta and the last rr.
enum IterRecord { REC_EXEC = 0, REC_APPEND, REC_BREAK, REC_CONV, REC_ETAMIN, REC_RR, REC_COUNT };
int iter_gate_init(int* gate, double* rec, hipStream_t s);
int iter_consume(const double* scal, double thresh, int next_r, int* gate, double* rec,
                 hipStream_t s);
// v = Q y
template <typename T>
int gemv_n(const T* Q, int64_t ldq, int64_t n, int ncols, const double* y, T* out,
           hipStream_t s);
// Gram partials: M = A^T B (ncols x ncols), FP64 out (row-major, ld = ncols)
template <typename T>
int gram(const T* A, const T* B, int64_t ld, int64_t n, int ncols, double* partials,
         size_t partial_cap, double* M, hipStream_t s);
// Out[:, r] = A U[:, r] * scale[r] for r < R (U: ncols x R col-major FP64)
template <typename T>
int right_mul(const T* A, int64_t lda, int64_t n, int ncols, const double* U, int R,
              const double* colscale, T* Out, int64_t ldo, hipStream_t s);
// likelihoods with diagonal W (igp_likelihood POISSON / GAUSSIAN), elementwise
// over n = N C values: W^{-1} diagonal and pseudo-targets f + W^{-1} grad;
// Out = W^{-1} V (+ Add); Newton bookkeeping as newton_stats; target checks
template <typename T>
int diag_begin(int lik, const T* f, const void* y, int64_t n, double s2, T* winv, T* rhs,
               hipStream_t s);
template <typename T>
int diag_apply(const T* winv, int64_t n, const T* V, int64_t nb, int64_t ldv, const T* Add,
               int64_t lda, T* Out, int64_t ldo, hipStream_t s, const int* gate = nullptr);
template <typename T>
int diag_stats(int lik, double s2, const T* fnew, const T* f, const T* v, const void* y,
               int64_t n, double* part, double* scal, hipStream_t s);
template <typename T>
int diag_check_targets(int lik, const void* y, int64_t n, int* flag, hipStream_t s);
// Block likelihood (per-point C x C negative-Hessian blocks, C <= 64):
// winv[n] = W_n^{-1} (Gauss-Jordan in FP64, one wave per point; a point with a
// pivot <= 0 counts in *bad and leaves NaN) and rhs[n] = f[n] + W_n^{-1} grad[n]
template <typename T>
int block_begin(const T* W, const T* grad, const T* f, int64_t N, int64_t C, T* winv, T* rhs,
                int* bad, hipStream_t s);
// Out[:, b] = W^{-1} V[:, b] (+ Add[:, b]) with the inverted blocks, b < nb
template <typename T>
int block_apply(const T* winv, int64_t N, int64_t C, const T* V, int64_t nb, int64_t ldv,
                const T* Add, int64_t lda, T* Out, int64_t ldo, hipStream_t s,
                const int* gate = nullptr);
// Newton update bookkeeping: ||fnew - f||^2, ||fnew||^2, loglik(fnew), fnew^T v
template <typename T>
int newton_stats(const T* fnew, const T* f, const T* v, const int32_t* y, int64_t N,
                 int64_t C, double* partials, double* scal, hipStream_t s);
// predict epilogue: var = os - sum_b A_b^2 ; probs = softmax(mean / sqrt(1 + pi/8 var))
// os_c: the prior variance k_c(x, x) of each class (C values, host)
template <typename T>
int predict_epilogue(const T* A, int64_t lda, int64_t nrows, int ncols, const double* os_c,
                     const T* mean, int64_t Ns, int64_t C, T* var, T* probs, hipStream_t s);

// ---- host FP64 symmetric eigensolver ---------------------------------------------
// A (n x n, row-major, symmetric; only the lower triangle is read) =
// Z diag(w) Z^T, eigenvalues descending, Z column-major (column k at Z + k*n).
int eigh_desc(int n, const double* A, double* w, double* Z);

}  // namespace igp
