/*
 * itergp.h -- C ABI of the MI355X (gfx950) IterNCGP hot path.
 *
 * Method: Tatzel, Wenger, Schneider, Hennig, "Accelerating Non-Conjugate
 * Gaussian Processes By Trading Off Computation For Uncertainty" (TMLR 2025).
 * Multi-class GP classification with a softmax likelihood, Laplace
 * approximation and Newton's method, each Newton step solved approximately by
 * IterGP (Algorithm 2) with recycling and compression (Algorithm 3) inside
 * the IterNCGP outer loop (Algorithm 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named X*, V, Out, F, mean, var, probs, y, arena and ws are DEVICE
 *   pointers owned by the caller.  The library never allocates device memory:
 *   calls that need scratch space take a caller-provided workspace whose size
 *   is given by the matching *_ws_bytes / *_state_bytes query.  (A model keeps
 *   two HIP events and a 224-byte pinned host buffer for reading the solver's
 *   scalars back, created on its first Newton step and freed by
 *   itergp_destroy.)
 * - Vectors in R^{NC} use CN-ordering (the paper's appendix on orderings):
 *   entry n*C + c belongs to point n and latent function c.  A set of nb such
 *   vectors is stored column by column: vector b starts at element b*ld.
 * - Inputs X are row-major N x D.  Floating-point arrays are double when the
 *   precision argument is IGP_FP64 and float otherwise (IGP_FP32, IGP_BF16).
 * - Calls are asynchronous on the caller's HIP stream unless stated.
 * - Return value: IGP_OK (0) or a negative igp_status.  No C++ exception
 *   crosses this boundary.  igp_last_error() returns a thread-local message
 *   describing the last failure of the calling thread.
 * - By default all latent functions share one kernel k with the same
 *   hyperparameters, as in every experiment of the paper, so K = K_X (x) I_C
 *   in CN-ordering; with n_kp == C kernel parameter sets each latent function
 *   has its own lengthscale and outputscale (one kernel family), K =
 *   sum_c K_c (x) e_c e_c^T.
 */
#ifndef ITERGP_H
#define ITERGP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status ------------------------------------------------------------ */
typedef enum igp_status {
  IGP_OK = 0,
  IGP_EINVAL = -1,       /* bad shape, NULL pointer, non-finite hyperparameter */
  IGP_ENOMEM = -2,       /* workspace or arena smaller than the query says */
  IGP_EDEVICE = -3,      /* a HIP runtime call failed */
  IGP_EUNSUPPORTED = -4  /* valid but not implemented combination */
} igp_status;

/* ---- kernels (paper: RBF and Matern kernels with a lengthscale and an
 * outputscale; the outputscale multiplies).  With r = ||x - x'|| / l:
 *   RBF os*exp(-r^2/2); Matern-1/2 os*exp(-r);
 *   Matern-3/2 os*(1+sqrt3 r)exp(-sqrt3 r); Matern-5/2 os*(1+sqrt5 r+5r^2/3)exp(-sqrt5 r) */
typedef enum igp_kernel_kind {
  IGP_RBF = 0, IGP_MATERN12 = 1, IGP_MATERN32 = 2, IGP_MATERN52 = 3
} igp_kernel_kind;

typedef struct igp_kernel_params {
  int32_t kind;          /* igp_kernel_kind */
  int32_t reserved;      /* must be 0 */
  double lengthscale;    /* > 0 */
  double outputscale;    /* > 0 */
} igp_kernel_params;

/* ---- arithmetic of the kernel-matrix product ----------------------------
 * IGP_FP64: FP64 throughout.  IGP_FP32: FP32 storage and arithmetic, FP64
 * reductions in the solver.  IGP_BF16: as FP32, but the distance product
 * X1 X2^T runs on BF16 MFMA with FP32 accumulation (inputs rounded to BF16,
 * squared norms taken of the rounded values).  IGP_BF16X3: as IGP_BF16 with
 * each (centred) input split into BF16 high and low parts, x = xh + xl, and
 * x1.x2 taken as xh1.xh2 + xl1.xh2 + xh1.xl2 (three BF16 products; inputs
 * kept to about 2^-17 relative instead of 2^-9, at three times the distance
 * work).  The element type of the BF16 modes is float. */
typedef enum igp_precision {
  IGP_FP64 = 0, IGP_FP32 = 1, IGP_BF16 = 2, IGP_BF16X3 = 3
} igp_precision;

/* ======================================================================
 * glm_kernel_matmul -- the matrix-free product with the prior covariance.
 *
 * Computes, for b = 0..nb-1,
 *     Out_b <- (K_X(X1, X2) (x) I_C) V_b + beta * Out_b
 * i.e. Out[n*C + c + b*ldo] = sum_m k(x1_n, x2_m) V[m*C + c + b*ldv] (+ beta*Out).
 * This is the product w -> K w that Algorithms 1 and 2 take as input (the
 * paper's appendix on matrix-vector products: K is evaluated lazily and
 * never formed; cost quadratic in N).  With n_kp == C each latent function
 * has its own kernel k_c (same family, its own lengthscale and outputscale):
 * Out[n*C + c] = sum_m k_c(x1_n, x2_m) V[m*C + c] (FP64 and FP32; the
 * direct-difference kernel evaluates the C kernels on shared distances).
 *   kp      kernel and hyperparameters: n_kp entries, n_kp == 1 (shared by
 *           all classes) or n_kp == C (one per class, one kernel family).
 *   X1      n1 x d row-major (device), X2 n2 x d row-major (device).
 *   V       nb vectors of length n2*C, vector b at V + b*ldv (ldv >= n2*C).
 *   Out     nb vectors of length n1*C, vector b at Out + b*ldo (ldo >= n1*C);
 *           must not alias V, X1 or X2.
 *   beta    0 overwrites Out (Out may hold NaN then); otherwise accumulates.
 *   precision  igp_precision; selects the element type (see conventions).
 *   ws      device workspace of at least glm_kernel_matmul_ws_bytes(...) bytes.
 * n1 == 0 or nb == 0 is a no-op; n2 == 0 gives Out = beta*Out.
 * Errors: IGP_EINVAL (NULL pointer with non-zero size, d < 1, C < 1,
 * ld too small, non-positive hyperparameter, n_kp not 1 or C, mixed kernel
 * families), IGP_EUNSUPPORTED (n_kp > 1 in a BF16 mode), IGP_ENOMEM (ws too
 * small), IGP_EDEVICE (launch failure).
 * ====================================================================== */
size_t glm_kernel_matmul_ws_bytes(int64_t n1, int64_t n2, int64_t d, int64_t C,
                                  int64_t nb, int32_t precision);
int glm_kernel_matmul(const igp_kernel_params* kp, int32_t n_kp,
                      const void* X1, int64_t n1, const void* X2, int64_t n2, int64_t d,
                      const void* V, int64_t C, int64_t nb, int64_t ldv,
                      void* Out, int64_t ldo, double beta, int32_t precision,
                      void* ws, size_t ws_bytes, hipStream_t stream);

/* ----------------------------------------------------------------------
 * glm_kernel_matmul_noalloc -- glm_kernel_matmul without a workspace, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, result and errors as glm_kernel_matmul, except that the
 * scratch space (split partials, centred rows and their norms) comes from a
 * static device array of glm_kernel_matmul_noalloc_max_bytes() bytes (64 MiB)
 * that the library holds on each GPU it runs on until the process ends; the
 * call itself allocates nothing.  The array of the CURRENT device is used, so
 * `stream` must belong to the current device.  Products whose
 * glm_kernel_matmul_ws_bytes(...) exceeds the maximum fail with IGP_ENOMEM
 * before any work is queued (FP32, D = 16, 5 output columns: n1 = n2 = 20000
 * needs about 33 MiB, n1 = n2 = 30000 about 72 MiB).
 * All calls on one GPU share its array: calls that overlap in time on one GPU
 * (different streams, different host threads without ordering) race and give
 * undefined results; calls ordered on one stream are safe.  The array keeps
 * the last call's contents; every byte a call reads it has written first.
 * ---------------------------------------------------------------------- */
size_t glm_kernel_matmul_noalloc_max_bytes(void);
int glm_kernel_matmul_noalloc(const igp_kernel_params* kp, int32_t n_kp,
                              const void* X1, int64_t n1, const void* X2, int64_t n2, int64_t d,
                              const void* V, int64_t C, int64_t nb, int64_t ldv,
                              void* Out, int64_t ldo, double beta, int32_t precision,
                              hipStream_t stream);

/* ======================================================================
 * glm_softmax_hessian_apply -- products with the per-point C x C blocks of
 * the negative Hessian of the softmax log likelihood at logits F.
 *   mode IGP_W:       Out_n = W_n V_n,  W_n = diag(pi_n) - pi_n pi_n^T
 *   mode IGP_W_PINV:  Out_n = W_n^+ V_n, W_n^+ = P diag(1/pi_n) P,
 *                     P = I - 11^T/C  (the paper's explicit pseudo-inverse,
 *                     appendix lemma for multi-class classification)
 * with pi_n = softmax(F_n) formed in-kernel by log-sum-exp.
 *   F      N x C logits (CN-ordered vector of length N*C).
 *   V/Out  nb CN-ordered vectors (strides ldv, ldo >= N*C); Out may equal V.
 *   precision IGP_FP64 (double) or IGP_FP32 (float).
 * Cost O(N C) per vector.  Errors: IGP_EINVAL, IGP_EDEVICE.
 * ====================================================================== */
typedef enum igp_hessian_mode { IGP_W = 0, IGP_W_PINV = 1 } igp_hessian_mode;
int glm_softmax_hessian_apply(const void* F, int64_t N, int64_t C,
                              const void* V, int64_t nb, int64_t ldv,
                              void* Out, int64_t ldo, int32_t mode, int32_t precision,
                              hipStream_t stream);

/* ======================================================================
 * IterNCGP model: Algorithm 1 with Algorithm 2 (IterGP) as inner solver and
 * Algorithm 3 (virtual solver run + compression) at the start of each step.
 * ====================================================================== */
typedef enum igp_policy {
  IGP_POLICY_CG = 0,    /* s_j = r_{j-1} / ||r_{j-1}||  (residual actions = CG) */
  IGP_POLICY_UNIT = 1,  /* s_j = e_j (partial Cholesky / subset of data); no recycling */
  IGP_POLICY_USER = 2   /* s_j = column j-1 of caller-supplied actions; the step
                           ends when they are used up */
} igp_policy;

typedef enum igp_residual_mode {
  IGP_RESIDUAL_EXPLICIT = 0,    /* r = (yhat - m) - K v - W^+ v with a fresh K product */
  IGP_RESIDUAL_RECURRENCE = 1   /* K v kept up to date from K d_j (one K product per iteration) */
} igp_residual_mode;

/* Likelihood of the observations.  Softmax: multi-class classification, y
 * int32 labels in [0, C), W_n the C x C softmax Hessian block (applied through
 * its pseudo-inverse).  Poisson (log link) and Gaussian: one observation per
 * latent value, y with N*C entries in CN-ordering (int32 counts >= 0 for
 * Poisson; finite targets of the model's element type for Gaussian), W^{-1}
 * diagonal: exp(-f) (appendix on the Poisson log likelihood) or noise_var.
 * Block: any likelihood that factorises over the N points, supplied by the
 * caller before each Newton step (and before itergp_compress) through
 * itergp_set_block_likelihood as the gradient of log p at the current f and
 * the per-point C x C blocks W_n of its negative Hessian (symmetric positive
 * definite); the step uses yhat - m = f + W^{-1} grad (section 3.1 with m = 0)
 * and per-point C x C solves; y is unused (may be NULL) and psi is NaN (log p
 * at the new iterate is the caller's). */
typedef enum igp_likelihood {
  IGP_LIK_SOFTMAX = 0,
  IGP_LIK_POISSON = 1,
  IGP_LIK_GAUSSIAN = 2,
  IGP_LIK_BLOCK = 3
} igp_likelihood;

typedef struct igp_solver_config {
  int32_t policy;        /* igp_policy */
  int32_t j_max;         /* maximum new actions per Newton step (>= 0) */
  int32_t rank_limit;    /* R: eigenpairs kept by the virtual solver run; < 0 = no limit */
  int32_t recycle;       /* 1: run Algorithm 3 at the start of every Newton step */
  double tol_abs;        /* inner stop: ||r|| < max(tol_abs, tol_rel ||yhat - m||) */
  double tol_rel;
  int32_t precision;     /* igp_precision of K products and NC-vector storage */
  int32_t residual_mode; /* igp_residual_mode */
  int32_t max_buffer;    /* columns reserved for S, T, Q (>= j_max; >= R + j_max
                            with recycling and a rank limit) */
  int32_t likelihood;    /* igp_likelihood (0: softmax) */
  double noise_var;      /* Gaussian observation variance (> 0); unused otherwise */
} igp_solver_config;

typedef struct igp_step_info {
  int32_t iters;          /* new actions taken in this step (j at exit) */
  int32_t buffer_cols;    /* columns of S, T, Q at exit */
  int32_t recycled_cols;  /* columns kept by the virtual solver run */
  int32_t eig_dropped;    /* eigenpairs dropped by the tiny-eigenvalue floor */
  int32_t converged;      /* inner tolerance reached */
  int32_t breakdown;      /* eta_j <= 0 met (the offending action was removed) */
  int32_t k_products;     /* products with K issued (incl. the Newton update) */
  int32_t reserved;
  double res_norm;        /* last residual norm formed */
  double rhs_norm;        /* ||yhat - m|| */
  double eta_min;         /* smallest accepted eta_j */
  double rel_change;      /* ||g_{i+1} - g_i|| / ||g_{i+1}|| */
  double psi;             /* log posterior at f_{i+1}: log p(y|f) - g^T v / 2 (FP64) */
} igp_step_info;

typedef struct igp_model igp_model;

/* Device bytes needed for a model of N points, D features, C classes. */
size_t itergp_state_bytes(int64_t N, int64_t D, int64_t C, const igp_solver_config* cfg);

/* Create a model with f_0 = m = 0 and empty buffers (Algorithm 1, start).
 *   kp     n_kp kernel parameter sets: 1 (shared by all latent functions) or
 *          C (one per latent function, one kernel family; the products then
 *          run on the direct-difference kernel and the batched form is not
 *          available; not with IGP_BF16).
 *   X      N x D row-major (double for IGP_FP64, float otherwise); copied
 *          into the arena, the caller may free it after the call returns.
 *   y      observations (see igp_likelihood): N int32 labels in [0, C) for
 *          softmax; N*C int32 counts >= 0 for Poisson; N*C targets of the
 *          model's element type for Gaussian.  Read by every Newton step, so
 *          the caller keeps it alive for the model's lifetime.
 *   arena  device memory of >= itergp_state_bytes(...) bytes, 256-byte
 *          aligned, owned by the caller, alive for the model's lifetime.
 * Synchronises `stream`.  The model runs all its work on `stream`. */
int itergp_init(igp_model** out, const igp_kernel_params* kp, int32_t n_kp,
                const igp_solver_config* cfg,
                const void* X, const void* y, int64_t N, int64_t D, int64_t C,
                void* arena, size_t arena_bytes, hipStream_t stream);

/* Actions for IGP_POLICY_USER in the next Newton step: ncols CN-ordered
 * vectors of length N*C (device, element type of the model), column j at
 * actions + j*ld.  The pointer must stay valid until that step returns. */
int itergp_set_user_actions(igp_model* m, const void* actions, int64_t ncols, int64_t ld);

/* One Newton step (the body of Algorithm 1's loop):
 *   pseudo-targets yhat - m = g + W(f)^+ (onehot(y) - pi);
 *   C_0, S, T <- virtual solver run (Algorithm 3), if recycling;
 *   v <- IterGP (Algorithm 2);  f <- K v + m.
 * Host control flow; synchronises the model's stream.  info may be NULL. */
int itergp_newton_step(igp_model* m, igp_step_info* info);

/* The same Newton step in three calls, so that a caller (a scheduler sharing
 * the GPU, a progress monitor) can do other work between solver iterations:
 *   itergp_newton_step_begin    pseudo-targets, Algorithm 3, v_0 and r_0;
 *   itergp_newton_step_iterate  up to max_iters iterations of Algorithm 2;
 *                               done (nullable) = 1 once the solver has stopped
 *                               (tolerance, j_max, breakdown, actions used up);
 *   itergp_newton_step_end      f = K v + m and the step record (info nullable);
 *                               IGP_EINVAL unless the solver has stopped.
 * Between the calls itergp_predict gives the IterGP posterior at the current
 * iteration; itergp_compress and the batched step refuse a model in a step.
 * Each call synchronises the model's stream. */
int itergp_newton_step_begin(igp_model* m);
int itergp_newton_step_iterate(igp_model* m, int64_t max_iters, int32_t* done);
int itergp_newton_step_end(igp_model* m, igp_step_info* info);

/* Compression of the fitted state for serving (Algorithm 3 alone): the
 * virtual solver run over the stored buffer S, T with W(f)^+ at the current
 * iterate f, keeping at most rank_limit eigendirections (-1: all above the
 * tiny-eigenvalue floor).  Replaces S, T and the root Q by S U, T U and
 * S U Lambda^{-1/2}; v and f are unchanged, so the predictive mean is too and
 * the marginal variance uses the compressed root.  kept (nullable) receives
 * the number of columns left.  Synchronises the model's stream. */
int itergp_compress(igp_model* m, int32_t rank_limit, int32_t* kept);

/* Predictive mean, marginal variance and probit class probabilities at Xs
 * (paper eqs. for m_{i,j} and k_{i,j}; probit as in its large-scale
 * experiment), using the v and root Q of the last Newton step:
 *   mean[s*C+c] = sum_n k(xs_s, x_n) v[n*C+c]
 *   var[s*C+c]  = k(xs,xs) - sum_b (sum_n k(xs_s, x_n) Q[n*C+c, b])^2
 *   probs[s*C+c]= softmax_c(mean / sqrt(1 + pi/8 var))
 *   Xs   Ns x D row-major (model element type); mean (required), var and
 *        probs (nullable) Ns*C each.  probs requires var and the softmax
 *        likelihood.
 *   ws   >= itergp_predict_ws_bytes(m, Ns) bytes. Asynchronous on `stream`. */
size_t itergp_predict_ws_bytes(const igp_model* m, int64_t Ns);
int itergp_predict(const igp_model* m, const void* Xs, int64_t Ns, void* mean,
                   void* var, void* probs, void* ws, size_t ws_bytes, hipStream_t stream);

/* Read-only device views into the model state (for tests and checkpoints).
 *   which: IGP_VIEW_F (N*C logits f_i), IGP_VIEW_V (representer weights),
 *   IGP_VIEW_Q / IGP_VIEW_S / IGP_VIEW_T (rows=N*C, cols=buffer columns,
 *   column j at ptr + j*ld), IGP_VIEW_RHS (yhat - m of the last step),
 *   IGP_VIEW_X (the model's copy of X; centred for FP32/BF16). */
typedef enum igp_view {
  IGP_VIEW_F = 0, IGP_VIEW_V = 1, IGP_VIEW_Q = 2, IGP_VIEW_S = 3, IGP_VIEW_T = 4,
  IGP_VIEW_RHS = 5, IGP_VIEW_X = 6
} igp_view;
int itergp_get_view(const igp_model* m, int32_t which, const void** ptr,
                    int64_t* rows, int64_t* cols, int64_t* ld);

/* Tracing: device time of the kernel-matrix products inside Newton steps,
 * measured with HIP events recorded on the model's stream around a product
 * (kernel evaluation, reduction of split partials).  Each event adds a few
 * microseconds of stream time, so the products may be sampled: with
 * enable = k > 0 every k-th product of the model is timed (k = 1: all of them);
 * products of solver iterations that did not run are never counted.
 * Counters cover every itergp_newton_step since the last itergp_set_profiling
 * call; enable = 0 turns tracing off. */
typedef struct igp_profile {
  int64_t kv_launches;   /* products timed */
  double kv_ms;          /* sum of their device durations, milliseconds */
  double kv_evals;       /* kernel evaluations performed: n1*n2, or n(n+1)/2 for a
                            symmetric product (same rows on both sides, each pair once) */
  double kv_flops;       /* algorithmic flops of the method that ran: 2*n1*n2*(d + C*nb),
                            or n(n+1)*d + 2*n*n*C*nb for a symmetric product */
  double step_ms;        /* device time of whole Newton steps (first to last kernel) */
  int64_t steps;         /* Newton steps timed */
  int64_t kv_symmetric;  /* products among kv_launches that ran symmetric */
} igp_profile;
/* Block likelihood (IGP_LIK_BLOCK): gradient and negative-Hessian blocks at the
 * model's current f (Algorithm 1, the per-step W and pseudo-targets), for the
 * next itergp_newton_step or itergp_compress, which consume them.
 *   grad  N*C values, CN-ordering (grad[n*C + c] = d log p / d f_{n,c}).
 *   W     N*C*C values: W[(n*C + a)*C + b] = -d^2 log p / d f_{n,a} d f_{n,b};
 *         each block symmetric positive definite.
 * Device pointers of the model's element type; read on the model's stream
 * before the call returns (the call synchronises it), then free.  Each block
 * is inverted on the device (Gauss-Jordan in FP64, one wave per point) and
 * f + W^{-1} grad formed.  Errors: IGP_EINVAL for a model of another
 * likelihood, NULL pointers, or a block whose pivots are not all positive
 * (not positive definite), with the count in the message. */
int itergp_set_block_likelihood(igp_model* m, const void* grad, const void* W);

int itergp_set_profiling(igp_model* m, int32_t enable);   /* 0: off; k > 0: time every k-th product; resets */
int itergp_get_profile(const igp_model* m, igp_profile* out);

/* Batched form: one Newton step of n independent models together.  Every
 * solver iteration issues ONE persistent launch covering the products K s of
 * all models still iterating (a work queue of (model, row block, split)
 * tiles), then the per-model projections; the host reads all models' scalars
 * with one transfer per iteration, and the eigendecompositions of the virtual
 * solver runs run in parallel host threads.  Results match itergp_newton_step
 * on each model up to the summation order of the products (the batched launch
 * may split the X2 rows differently).
 * Requirements: FP32 models, or BF16 models (all of one precision; their
 * products run a BF16 tile of the same launch), on one stream, recurrence
 * residual, RBF or Matern-3/2 or -5/2, D <= 32, C <= 8, each model at most
 * once.  The launch
 * shape (rows per wave, X2 rows per split) is chosen by timing candidates on
 * the first batch of each (precision, kernel, feature class, size class) and
 * cached for the process; itergp_batched_tuning returns the table as JSON.
 *   ws  device workspace of >= itergp_batched_ws_bytes(models, n) bytes.
 *   infos  n entries (nullable).  Synchronises the models' stream. */
size_t itergp_batched_ws_bytes(igp_model* const* models, int32_t n);
int itergp_newton_step_batched(igp_model* const* models, int32_t n, igp_step_info* infos,
                               void* ws, size_t ws_bytes);
/* The batched step with flags (itergp_newton_step_batched is flags = 0).
 * IGP_BATCH_DEVICE_CONTROL moves the solver's control flow onto the device:
 * the host enqueues windows of up to 8 solver iterations (Algorithm 2) for
 * every model still iterating, as if each took all of them (bounded by its
 * j_max, its buffer and its user actions), and reads the models' iteration
 * records once per window instead of their scalars once per iteration.  On
 * the device each model's end of iteration (breakdown eta <= 0, or
 * ||r|| < tolerance, as in the single-model step) closes that model's gate,
 * and every later operation and product tile of the model returns at once.
 * The arithmetic is that of flags = 0, so results, iteration counts and
 * flags are the same.  A window whose launch shape (see above) has not been
 * timed yet runs one iteration under host control first.  Same requirements,
 * workspace and errors as itergp_newton_step_batched, and IGP_EINVAL for an
 * unknown flag. */
enum { IGP_BATCH_DEVICE_CONTROL = 1 };
int itergp_newton_step_batched_ex(igp_model* const* models, int32_t n, igp_step_info* infos,
                                  void* ws, size_t ws_bytes, int32_t flags);
int itergp_batched_tuning(char* buf, size_t len);
/* Seeds the launch-shape table from JSON in the format itergp_batched_tuning
 * writes (an array of objects with kind, feature_chunks, log2_rows, strips,
 * split_rows; us and precision optional, precision "fp32"), e.g. a table
 * saved by an earlier process on the same kind of GPU, so that batches of
 * those shapes skip the timing.  Entries already in the table are kept.
 * loaded (nullable) receives the number of entries added.  Host only.
 * Errors: IGP_EINVAL (NULL text, a malformed entry, values outside the
 * candidate set: strips 1 or 2, split_rows 1024 or 4096). */
int itergp_batched_tuning_load(const char* json, int32_t* loaded);

/* Release the host-side handle (the arena stays the caller's). */
int itergp_destroy(igp_model* m);

/* Thread-local description of the last error of this thread ("" if none). */
const char* igp_last_error(void);

/* Library version string. */
const char* igp_version(void);

/* The host FP64 symmetric eigensolver used by Algorithm 3 for M = U Lambda U^T
 * (host pointers, no device work):  A is n x n row-major symmetric (only its
 * lower triangle is read); on return w holds the eigenvalues in decreasing
 * order and Z (n x n, column k at Z + k*n) the matching orthonormal
 * eigenvectors.  Errors: IGP_EINVAL (n < 0 or NULL pointer with n > 0),
 * IGP_EDEVICE (no convergence). */
int igp_host_eigh(int32_t n, const double* A, double* w, double* Z);

#ifdef __cplusplus
}
#endif
#endif /* ITERGP_H */
