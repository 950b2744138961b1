// IterNCGP driver: Algorithm 1 (outer Newton loop), Algorithm 2 (IterGP) and
// Algorithm 3 (virtual solver run with compression), with every NC-sized
// operation running in the library's HIP kernels and only B x B algebra and
// scalar control on the host.
#include <algorithm>
#include <cstdint>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "ops.hpp"

namespace igp {
size_t state_bytes(int64_t N, int64_t D, int64_t C, const igp_solver_config* cfg);

namespace {

constexpr int PARTIAL_DOUBLES = 1 << 16;

template <typename T>
struct Layout {
  T *X, *f, *fnew, *pi, *rhs, *v, *r, *z, *d, *kv, *wv;
  T *S, *Tb, *Q, *S2, *T2;
  T *KQ, *kd;   // recurrence mode: K Q and K d
  T* wblk;      // block likelihood: the inverted C x C blocks W_n^{-1}
  double *part, *scal, *yb, *M, *U, *lamscale, *gram_part;
  double* apart;  // partials of a solver iteration's alpha (finished by the append step)
  double* epart;  // partials of a solver iteration's eta (the direction update's blocks)
  size_t gram_cap;
  void* kvws;
  size_t kvws_bytes;
  int* flags;
  int* gate;      // closed (1) once the solver has stopped: later iteration kernels return
  double* rec;    // device record of the iterations (IterRecord)
  // matrix-core paths: common centre, centred zero-padded rows (float or
  // BF16), squared norms of those rows
  float* centre;
  void* Xp;
  float* nrm;
  double* meanpart;
};

int64_t col_stride(int64_t n) { return ceil_div(n, 64) * 64; }

constexpr int64_t MEAN_BLOCKS = 1024;

template <typename T>
Layout<T> carve(Carver& cv, int64_t N, int64_t D, int64_t C, const igp_solver_config& cfg,
                bool prepared) {
  Layout<T> L{};
  const int64_t n = N * C, ld = col_stride(n);
  const int64_t B = cfg.max_buffer;
  L.X = cv.take<T>(N * D);
  L.f = cv.take<T>(n);
  L.fnew = cv.take<T>(n);
  L.pi = cv.take<T>(n);
  L.rhs = cv.take<T>(n);
  L.v = cv.take<T>(n);
  L.r = cv.take<T>(n);
  L.z = cv.take<T>(n);
  L.d = cv.take<T>(n);
  L.kv = cv.take<T>(n);
  L.wv = cv.take<T>(n);
  L.S = cv.take<T>(ld * B);
  L.Tb = cv.take<T>(ld * B);
  L.Q = cv.take<T>(ld * B);
  L.S2 = cv.take<T>(ld * B);
  L.T2 = cv.take<T>(ld * B);
  if (cfg.residual_mode == IGP_RESIDUAL_RECURRENCE) {
    L.KQ = cv.take<T>(ld * B);
    L.kd = cv.take<T>(n);
  }
  if (cfg.likelihood == IGP_LIK_BLOCK) L.wblk = cv.take<T>(n * C);
  int64_t npart = PARTIAL_DOUBLES;
  const int64_t gemv_need = (ceil_div(n, QTZ_ROWS) + 1) * std::max<int64_t>(B, 1);
  npart = std::max(npart, gemv_need);
  npart = std::max(npart, 4 * ceil_div(N, 256) + 64);
  L.part = cv.take<double>(npart);
  // the scalars and, right after them, the iteration record: one copy to the
  // host per window of iterations
  L.scal = cv.take<double>(SC_COUNT + REC_COUNT);
  L.yb = cv.take<double>(std::max<int64_t>(B, 1));
  L.M = cv.take<double>(std::max<int64_t>(B * B, 1));
  L.U = cv.take<double>(std::max<int64_t>(B * B, 1));
  L.lamscale = cv.take<double>(std::max<int64_t>(B, 1));
  L.gram_cap = static_cast<size_t>(std::max<int64_t>(B * B, 1)) * 16;
  L.gram_part = cv.take<double>(L.gram_cap);
  L.kvws_bytes = prepared ? kv_ws_bytes_prepared(N, N, D, C, 1, cfg.precision)
                          : kv_ws_bytes(N, N, D, C, 1, cfg.precision);
  L.kvws = cv.take<char>(L.kvws_bytes);
  L.flags = cv.take<int>(64);
  L.gate = cv.take<int>(1);
  L.rec = L.scal + SC_COUNT;
  L.apart = cv.take<double>(RED_BLOCKS);
  L.epart = cv.take<double>(ceil_div(n, 256) + 1);
  if (prepared) {
    L.centre = cv.take<float>(D);
    L.Xp = is_bf16(cfg.precision)
               ? static_cast<void*>(cv.take<uint16_t>(bf16_rows_elems(cfg.precision, N, D)))
               : static_cast<void*>(cv.take<float>(N * padded_dim(D)));
    L.nrm = cv.take<float>(N);
    L.meanpart = cv.take<double>(MEAN_BLOCKS * D);
  }
  return L;
}

template <typename T>
struct Model final : igp_model {
  igp_kernel_params kp{};
  std::vector<igp_kernel_params> kps;   // one per class when n_kp == C > 1
  int n_kp = 1;
  std::vector<double> prior_var;        // k_c(x, x) per class
  igp_solver_config cfg{};
  int64_t N = 0, D = 0, C = 0, n = 0, ld = 0;
  const void* y = nullptr;       // observations (igp_likelihood decides the type)
  hipStream_t stream = nullptr;
  Layout<T> L{};
  int ncols = 0;                 // columns of S, T and Q
  const T* user = nullptr;
  int64_t user_cols = 0, user_ld = 0;
  int steps_done = 0;
  std::vector<double> hM, hMs, hU, hlam, hscale, hL;
  // tracing: every prof_every-th product is timed (prof_seq counts them)
  bool prof = false;
  int prof_every = 1;
  int64_t prof_seq = 0;
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  igp_profile pstat{};
  double pending_evals = 0.0, pending_flops = 0.0;
  int64_t pending_sym = 0;
  std::vector<char> pair_skipped;   // per event pair
  // products of iterations enqueued ahead of their convergence test: counted
  // once the iteration is known to have run
  struct SpecProduct {
    size_t pair;
    double evals, flops;
    bool sym;
    int iter;
  };
  std::vector<SpecProduct> spec_products;

  ~Model() override {
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
    for (hipEvent_t e : win_ev)
      if (e) (void)hipEventDestroy(e);
    if (win_host) (void)hipHostFree(win_host);
  }

  int event_pair(hipEvent_t* a, hipEvent_t* b) {
    while (evpool.size() < evused + 2) {
      hipEvent_t e;
      IGP_CHECK_HIP(hipEventCreate(&e));
      evpool.push_back(e);
    }
    *a = evpool[evused];
    *b = evpool[evused + 1];
    evused += 2;
    pair_skipped.resize(evused / 2, 0);
    pair_skipped[evused / 2 - 1] = 0;
    return IGP_OK;
  }

  // after a stream synchronisation: fold the recorded pairs into the counters
  int collect_profile() {
    if (!prof) return IGP_OK;
    // pair 0 brackets the whole step; the rest bracket products with K
    for (size_t i = 0; i + 1 < evused; i += 2) {
      if (pair_skipped[i / 2]) continue;   // a product of an iteration that did not run
      float ms = 0.f;
      IGP_CHECK_HIP(hipEventElapsedTime(&ms, evpool[i], evpool[i + 1]));
      if (i == 0) {
        pstat.step_ms += ms;
        pstat.steps += 1;
      } else {
        pstat.kv_ms += ms;
        pstat.kv_launches += 1;
      }
    }
    pstat.kv_evals += pending_evals;
    pstat.kv_flops += pending_flops;
    pstat.kv_symmetric += pending_sym;
    pending_evals = pending_flops = 0.0;
    pending_sym = 0;
    evused = 0;
    return IGP_OK;
  }

  int set_profiling(int enable) override {
    prof = enable > 0;
    prof_every = enable > 0 ? enable : 1;
    prof_seq = 0;
    pstat = igp_profile{};
    evused = 0;
    pending_evals = pending_flops = 0.0;
    pending_sym = 0;
    return IGP_OK;
  }

  int get_profile(igp_profile* out) const override {
    *out = pstat;
    return IGP_OK;
  }

  bool prepared = false;

  KVProblem kv_problem(const T* X1, int64_t n1, const T* V, int64_t nb, int64_t ldv, T* Out,
                       int64_t ldo, const void* X1p = nullptr,
                       const float* norm1 = nullptr) const {
    KVProblem p{};
    if (prepared) {
      p.X1p = X1p ? X1p : L.Xp;
      p.norm1 = X1p ? norm1 : L.nrm;
      p.X2p = L.Xp;
      p.norm2 = L.nrm;
    }
    p.kp = kp;
    if (n_kp > 1) {
      p.kpc = kps.data();
      p.n_kp = n_kp;
    }
    p.precision = cfg.precision;
    p.X1 = X1;
    p.X2 = L.X;
    p.n1 = n1;
    p.n2 = N;
    p.d = D;
    p.V = V;
    p.C = C;
    p.nb = nb;
    p.ldv = ldv;
    p.Out = Out;
    p.ldo = ldo;
    p.beta = 0.0;
    return p;
  }

  bool recurrence() const { return cfg.residual_mode == IGP_RESIDUAL_RECURRENCE; }

  // Out = K V; with a gate, part of solver iteration `iter`, skipped once the gate closes
  // Out = K V (one vector); with zout (softmax): also zout = Out + W^+ V in the
  // product's reduction when its launch path takes that epilogue (*zdone = 1).
  // A product timed for the profile leaves z to the caller, so that the timed
  // unit is the product alone (kernel and reduction).
  int apply_K(const T* V, T* Out, const int* gate = nullptr, int iter = 0, T* zout = nullptr,
              int* zdone = nullptr) {
    hipEvent_t a = nullptr, b = nullptr;
    const bool timed = prof && (prof_seq++ % prof_every == 0);
    if (timed) {
      IGP_TRY(event_pair(&a, &b));
      IGP_CHECK_HIP(hipEventRecord(a, stream));
    }
    int sym = 0;
    KVProblem p = kv_problem(L.X, N, V, 1, n, Out, n);
    p.symmetric_out = &sym;
    p.skip = gate;
    if (zout && softmax() && !timed) {
      p.epi_pi = L.pi;
      p.epi_s = V;
      p.epi_z = zout;
      p.epi_applied = zdone;
    }
    IGP_TRY(kv_launch(p, L.kvws, L.kvws_bytes, stream));
    if (timed) {
      IGP_CHECK_HIP(hipEventRecord(b, stream));
      const double Nd = static_cast<double>(N);
      const double evals = sym ? Nd * (Nd + 1.0) / 2.0 : Nd * Nd;
      const double flops = sym ? Nd * (Nd + 1.0) * D + 2.0 * Nd * Nd * C
                               : 2.0 * Nd * Nd * (D + C);
      if (gate) {
        spec_products.push_back({evused / 2 - 1, evals, flops, sym != 0, iter});
      } else {
        pending_evals += evals;
        pending_flops += flops;
        pending_sym += sym;
      }
    }
    return IGP_OK;
  }

  // after a window of iterations: count the products of those that ran
  // (iteration number <= last_run), drop the rest from the profile
  // after iterations lo..hi were consumed: count the products of those that
  // ran (iteration <= last_run), drop the rest from the profile
  void settle_products(int lo, int hi, int last_run) {
    std::vector<SpecProduct> keep;
    for (const SpecProduct& sp : spec_products) {
      if (sp.iter < lo || sp.iter > hi) {
        keep.push_back(sp);
      } else if (sp.iter <= last_run) {
        pending_evals += sp.evals;
        pending_flops += sp.flops;
        pending_sym += sp.sym ? 1 : 0;
      } else {
        pair_skipped[sp.pair] = 1;
      }
    }
    spec_products.swap(keep);
  }

  int read_scalars(double* out) {
    IGP_CHECK_HIP(hipMemcpyAsync(out, L.scal, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                                 stream));
    IGP_CHECK_HIP(hipStreamSynchronize(stream));
    return IGP_OK;
  }

  // ---- one Newton step, in phases (a single model runs them back to back;
  // the batched driver interleaves the phases of many models) ----------------
  struct StepState {
    igp_step_info info{};
    double thresh = 0.0;
    int j = 0, kprod = 0;
    bool active = false;      // still taking actions
    bool next_r = false;      // the last iteration enqueued a residual
    hipEvent_t step_b = nullptr;
    int keep = 0, dropped = 0;
    bool chol = false;        // the virtual solver run took the Cholesky form
  } st;
  double sc[SC_COUNT];

  bool softmax() const { return cfg.likelihood == IGP_LIK_SOFTMAX; }
  bool block() const { return cfg.likelihood == IGP_LIK_BLOCK; }
  bool block_set = false;   // blocks given for the current f, not yet consumed

  // W at f (pi for softmax, the diagonal of W^{-1} for Poisson and Gaussian,
  // both kept in L.pi) and the pseudo-targets yhat - m = f + W^{-1} grad into
  // rhs; for the block likelihood both were formed by set_block_likelihood
  // (the blocks are consumed here)
  int likelihood_terms(T* rhs) {
    if (block()) {
      IGP_REQUIRE(block_set, "block likelihood: itergp_set_block_likelihood must give the "
                             "blocks at the current f before each Newton step or compress");
      block_set = false;
      return IGP_OK;
    }
    if (softmax()) {
      int nblk = 0;
      return softmax_pi_rhs<T>(L.f, static_cast<const int32_t*>(y), N, C, L.pi, rhs, L.part,
                               &nblk, stream);
    }
    return diag_begin<T>(cfg.likelihood, L.f, y, n, cfg.noise_var, L.pi, rhs, stream);
  }

  // Out[:, b] = W^+ V[:, b] (+ Add[:, b]) for b < nb
  int apply_winv(const T* V, int64_t nb, int64_t ldv, const T* Add, int64_t lda, T* Out,
                 int64_t ldo, const int* gate = nullptr) {
    if (softmax())
      return winv_apply<T>(L.pi, false, IGP_W_PINV, N, C, V, nb, ldv, Add, lda, Out, ldo, stream,
                           gate);
    if (block())
      return block_apply<T>(L.wblk, N, C, V, nb, ldv, Add, lda, Out, ldo, stream, gate);
    return diag_apply<T>(L.pi, n, V, nb, ldv, Add, lda, Out, ldo, stream, gate);
  }

  // pseudo-targets yhat - m = g + W^+ (onehot(y) - pi), m = 0 (softmax), or
  // f + W^{-1} grad (diagonal W)
  int phase_begin() {
    st = StepState{};
    st.info.eta_min = INFINITY;
    evused = 0;
    if (prof) {
      hipEvent_t a;
      IGP_TRY(event_pair(&a, &st.step_b));
      IGP_CHECK_HIP(hipEventRecord(a, stream));
    }
    spec_products.clear();
    IGP_TRY(likelihood_terms(L.rhs));
    IGP_TRY(dot_into<T>(L.rhs, L.rhs, n, L.part, L.scal + SC_RHS2, stream));
    const bool recycle = cfg.recycle && cfg.policy != IGP_POLICY_UNIT;
    if (!recycle) ncols = 0;
    return IGP_OK;
  }

  // Algorithm 3, device part 1: M = S^T (T + W^+ S) (FP64 accumulation)
  int phase_vsr_gram() {
    if (ncols == 0) return IGP_OK;
    const int B = ncols;
    IGP_TRY(apply_winv(L.S, B, ld, L.Tb, ld, L.S2, ld));
    return gram<T>(L.S, L.S2, ld, n, B, L.gram_part, L.gram_cap, L.M, stream);
  }

  int phase_vsr_fetch() {
    if (ncols == 0) return IGP_OK;
    hM.resize(static_cast<size_t>(ncols) * ncols);
    IGP_CHECK_HIP(hipMemcpyAsync(hM.data(), L.M, hM.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, stream));
    IGP_CHECK_HIP(hipStreamSynchronize(stream));
    return IGP_OK;
  }

  // Untruncated form of Algorithm 3.  Only Q_0 Q_0^T = S M^{-1} S^T enters C_0,
  // so when no direction would be dropped any factor F with F F^T = M^{-1}
  // serves: F = L^{-T} from the Cholesky factor M = L L^T (B^3/3 flops instead
  // of an eigendecomposition, and S, T keep their basis).  It is taken only
  // when it provably changes nothing: the rank limit keeps all B columns, and
  // lambda_max <= tr(M), lambda_min >= 1 / tr(M^{-1}) = 1 / ||L^{-1}||_F^2 put
  // every eigenvalue above the floor lambda_max B eps whenever
  // tr(M) tr(M^{-1}) B eps < 1.  On success hU holds F = L^{-T} in the layout
  // of an eigenvector block (column r of F at hU[r B ...]).
  static double dot4(const double* a, const double* b, int m) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int k = 0;
    for (; k + 4 <= m; k += 4) {
      s0 += a[k] * b[k];
      s1 += a[k + 1] * b[k + 1];
      s2 += a[k + 2] * b[k + 2];
      s3 += a[k + 3] * b[k + 3];
    }
    for (; k < m; ++k) s0 += a[k] * b[k];
    return (s0 + s1) + (s2 + s3);
  }

  bool chol_untruncated(int B) {
    if (cfg.rank_limit >= 0 && cfg.rank_limit < B) return false;
    // M = L L^T column by column (row-major L): the entries below the diagonal
    // of one column are independent dot products
    hL.assign(static_cast<size_t>(B) * B, 0.0);
    double trace = 0.0;
    for (int j = 0; j < B; ++j) {
      double* Lj = hL.data() + static_cast<size_t>(j) * B;
      const double* Mj = hMs.data() + static_cast<size_t>(j) * B;
      trace += Mj[j];
      const double dj = Mj[j] - dot4(Lj, Lj, j);
      if (!(dj > 0.0)) return false;
      Lj[j] = std::sqrt(dj);
      const double inv = 1.0 / Lj[j];
      for (int i = j + 1; i < B; ++i) {
        double* Li = hL.data() + static_cast<size_t>(i) * B;
        Li[j] = (hMs[static_cast<size_t>(i) * B + j] - dot4(Li, Lj, j)) * inv;
      }
    }
    // X = L^{-1} by rows, X_i = (e_i - sum_{k<i} L_ik X_k) / L_ii (contiguous
    // row updates).  F = L^{-T} has F[b][r] = X[r][b], so the row-major X is
    // already the eigenvector-block layout hU[r B + b].
    std::fill(hU.begin(), hU.end(), 0.0);
    double trinv = 0.0;
    for (int i = 0; i < B; ++i) {
      double* __restrict__ Xi = hU.data() + static_cast<size_t>(i) * B;
      const double* __restrict__ Li = hL.data() + static_cast<size_t>(i) * B;
      Xi[i] = 1.0;
      for (int k = 0; k < i; ++k) {
        const double a = Li[k];
        const double* __restrict__ Xk = hU.data() + static_cast<size_t>(k) * B;
        for (int c = 0; c <= k; ++c) Xi[c] -= a * Xk[c];
      }
      const double inv = 1.0 / Li[i];
      for (int c = 0; c <= i; ++c) {
        Xi[c] *= inv;
        trinv += Xi[c] * Xi[c];
      }
    }
    return std::isfinite(trinv) && trace * trinv * B * 2.220446049250313e-16 < 1.0;
  }

  // host part: M = U Lambda U^T (descending), tiny-eigenvalue floor, keep <= R.
  // Touches only this model's host buffers (safe to run concurrently).
  int phase_vsr_host() {
    const int B = ncols;
    if (B == 0) return IGP_OK;
    hMs.resize(hM.size());
    for (int i = 0; i < B; ++i)
      for (int k = 0; k < B; ++k)
        hMs[static_cast<size_t>(i) * B + k] =
            0.5 * (hM[static_cast<size_t>(i) * B + k] + hM[static_cast<size_t>(k) * B + i]);
    hU.resize(static_cast<size_t>(B) * B);
    st.chol = chol_untruncated(B);
    if (st.chol) {
      st.dropped = 0;
      st.keep = B;
      return IGP_OK;
    }
    hlam.resize(B);
    IGP_TRY(eigh_desc(B, hMs.data(), hlam.data(), hU.data()));
    int keep = 0;
    const double floor = hlam[0] > 0.0 ? hlam[0] * B * 2.220446049250313e-16 : INFINITY;
    while (keep < B && hlam[keep] > floor) ++keep;
    st.dropped = B - keep;
    if (cfg.rank_limit >= 0 && keep > cfg.rank_limit) keep = cfg.rank_limit;
    st.keep = keep;
    hscale.resize(std::max(keep, 1));
    for (int k = 0; k < keep; ++k) hscale[k] = 1.0 / std::sqrt(hlam[k]);
    return IGP_OK;
  }

  // device part 2: S <- S U, T <- T U, Q_0 = S U Lambda^{-1/2} (and K Q_0 = T U Lambda^{-1/2})
  int phase_vsr_apply() {
    const int B = ncols;
    if (B == 0) return IGP_OK;
    const int keep = st.keep;
    if (st.chol) {
      // Q_0 = S L^{-T}, K Q_0 = T L^{-T}; S and T stay as they are
      IGP_CHECK_HIP(hipMemcpyAsync(L.U, hU.data(), static_cast<size_t>(B) * B * sizeof(double),
                                   hipMemcpyHostToDevice, stream));
      IGP_TRY(right_mul<T>(L.S, ld, n, B, L.U, B, nullptr, L.Q, ld, stream));
      if (recurrence()) IGP_TRY(right_mul<T>(L.Tb, ld, n, B, L.U, B, nullptr, L.KQ, ld, stream));
    } else if (keep > 0) {
      IGP_CHECK_HIP(hipMemcpyAsync(L.U, hU.data(), static_cast<size_t>(B) * keep * sizeof(double),
                                   hipMemcpyHostToDevice, stream));
      IGP_CHECK_HIP(hipMemcpyAsync(L.lamscale, hscale.data(), keep * sizeof(double),
                                   hipMemcpyHostToDevice, stream));
      IGP_TRY(right_mul<T>(L.S, ld, n, B, L.U, keep, nullptr, L.S2, ld, stream));
      IGP_TRY(right_mul<T>(L.Tb, ld, n, B, L.U, keep, nullptr, L.T2, ld, stream));
      IGP_TRY(right_mul<T>(L.S, ld, n, B, L.U, keep, L.lamscale, L.Q, ld, stream));
      if (recurrence())
        IGP_TRY(right_mul<T>(L.Tb, ld, n, B, L.U, keep, L.lamscale, L.KQ, ld, stream));
      std::swap(L.S, L.S2);
      std::swap(L.Tb, L.T2);
    }
    ncols = keep;
    st.info.recycled_cols = keep;
    st.info.eig_dropped = st.dropped;
    return IGP_OK;
  }

  // v_0 = C_0 (yhat - m) = Q (Q^T (yhat - m)); then r_0 when j_max > 0
  int phase_v0() {
    if (ncols > 0) {
      IGP_TRY(gemv_t<T>(L.Q, ld, n, ncols, L.rhs, L.part, L.yb, stream));
      IGP_TRY(gemv_n<T>(L.Q, ld, n, ncols, L.yb, L.v, stream));
      if (recurrence()) IGP_TRY(gemv_n<T>(L.KQ, ld, n, ncols, L.yb, L.kv, stream));
    } else {
      IGP_TRY(fill_zero<T>(L.v, n, stream));
      if (recurrence()) IGP_TRY(fill_zero<T>(L.kv, n, stream));
    }
    if (cfg.j_max > 0) IGP_TRY(enqueue_residual());
    return IGP_OK;
  }

  // r = (yhat - m) - K v - W^+ v with K v formed (explicit) or carried (recurrence)
  // r = rhs - K v - W^+ v (K v from the recurrence or a product); within a
  // solver iteration (iter > 0) behind the gate, ending the iteration
  int enqueue_residual(int iter = 0) {
    int* gate = iter > 0 ? L.gate : nullptr;
    if (!recurrence()) {
      IGP_TRY(apply_K(L.v, L.kv, gate, iter));
      if (!gate) ++st.kprod;
    }
    if (gate && softmax()) {   // W^+ v and the residual in one pass over the points
      int g = 0;
      IGP_TRY(winv_residual<T>(L.pi, N, C, L.v, L.rhs, L.kv, L.wv, L.r, L.part, &g, stream,
                               gate));
      return rr_consume(L.part, g, L.scal, st.thresh, gate, L.rec, stream);
    }
    IGP_TRY(apply_winv(L.v, 1, n, nullptr, 0, L.wv, n, gate));
    if (gate)
      return residual_consume<T>(L.rhs, L.kv, L.wv, L.r, n, L.part, L.scal, st.thresh, gate,
                                 L.rec, stream);
    return residual<T>(L.rhs, L.kv, L.wv, L.r, n, L.part, L.scal + SC_RR, stream);
  }

  // after the scalars of phase_v0 are on the host
  void phase_start_iterations() {
    st.info.rhs_norm = std::sqrt(sc[SC_RHS2]);
    st.thresh = std::max(cfg.tol_abs, cfg.tol_rel * st.info.rhs_norm);
    st.active = false;
    if (cfg.j_max > 0) {
      st.info.res_norm = std::sqrt(sc[SC_RR]);
      if (!(st.info.res_norm >= st.thresh)) st.info.converged = 1;
      else st.active = true;
    }
  }

  // whether another action is taken (sets st.active = false otherwise)
  int phase_can_act() {
    if (!st.active) return IGP_OK;
    if (st.j >= cfg.j_max) {
      st.active = false;
      return IGP_OK;
    }
    if (ncols >= cfg.max_buffer) {
      set_error("buffer full: %d columns (max_buffer too small)", ncols);
      return IGP_ENOMEM;
    }
    if (cfg.policy == IGP_POLICY_USER && (!user || st.j >= user_cols)) st.active = false;
    return IGP_OK;
  }

  T* s_col() const { return L.S + static_cast<int64_t>(ncols) * ld; }
  T* t_col() const { return L.Tb + static_cast<int64_t>(ncols) * ld; }

  // host bookkeeping of an iteration (shared with the batched driver)
  void host_action() { ++st.j; }
  void host_after_product() {
    ++st.kprod;
    st.next_r = st.j < cfg.j_max;
  }

  // this model's part of a batched iteration (after host_action)
  BIter biter() const {
    BIter t{};
    t.r = L.r; t.s = s_col(); t.t = t_col(); t.z = L.z; t.d = L.d; t.v = L.v; t.kv = L.kv;
    t.kd = L.kd; t.rhs = L.rhs; t.wv = L.wv; t.Q = L.Q; t.KQ = L.KQ;
    t.qcol = L.Q + static_cast<int64_t>(ncols) * ld;
    t.kqcol = L.KQ + static_cast<int64_t>(ncols) * ld;
    t.pi = L.pi;
    t.user = cfg.policy == IGP_POLICY_USER && user
                 ? user + static_cast<int64_t>(st.j - 1) * user_ld : nullptr;
    t.scal = L.scal; t.part = L.part; t.epart = L.epart; t.yb = L.yb;
    t.n = n; t.N = N; t.ld = ld; t.unit_idx = st.j - 1;
    t.C = static_cast<int>(C); t.ncols = ncols; t.lik = cfg.likelihood; t.policy = cfg.policy;
    t.nchunks = static_cast<int>(ceil_div(n, QTZ_ROWS));
    t.next_r = st.next_r ? 1 : 0;
    return t;
  }

  // device-controlled batched window: iteration jj (1-based) with its action in
  // buffer column col, as biter() would describe it after jj - 1 appended
  // iterations; the gate and record end the iteration on the device
  BIter biter_at(int64_t jj, int col) const {
    BIter t = biter();
    const int64_t off = static_cast<int64_t>(col) * ld;
    t.s = L.S + off;
    t.t = L.Tb + off;
    t.qcol = L.Q + off;
    t.kqcol = L.KQ + off;
    t.user = cfg.policy == IGP_POLICY_USER && user ? user + (jj - 1) * user_ld : nullptr;
    t.unit_idx = jj - 1;
    t.ncols = col;
    t.next_r = jj < cfg.j_max ? 1 : 0;
    t.gate = L.gate;
    t.rec = L.rec;
    t.thresh = st.thresh;
    return t;
  }
  KVProblem product_action_at(int col) const {
    const int64_t off = static_cast<int64_t>(col) * ld;
    return kv_problem(L.X, N, L.S + off, 1, n, L.Tb + off, n);
  }
  // rounds a device-controlled window may give this model (iteration cap,
  // buffer, user actions); 0 when it cannot act
  int window_cap(int wmax) const {
    if (!st.active) return 0;
    int64_t c = std::min<int64_t>(wmax, cfg.j_max - st.j);
    c = std::min<int64_t>(c, cfg.max_buffer - ncols);
    if (cfg.policy == IGP_POLICY_USER) c = std::min<int64_t>(c, user ? user_cols - st.j : 0);
    return static_cast<int>(std::max<int64_t>(c, 0));
  }
  // after a device-controlled window of `cap` rounds: fold the device record
  // (rec, this model's REC_COUNT values) into the host state
  int consume_dc(const double* rec, int cap) {
    const int ran = static_cast<int>(rec[REC_EXEC] - rec_h[REC_EXEC]);
    const int appended = static_cast<int>(rec[REC_APPEND] - rec_h[REC_APPEND]);
    const bool stopped = rec[REC_BREAK] != 0.0 || rec[REC_CONV] != 0.0;
    IGP_REQUIRE(ran >= 0 && ran <= cap && appended <= ran && appended >= ran - 1 &&
                    (ran == cap || stopped) && (appended == ran || rec[REC_BREAK] != 0.0),
                "batched iteration record out of step with the host");
    const int64_t j0 = st.j;
    st.kprod += ran;
    st.j += appended;
    ncols += appended;
    st.next_r = st.j < cfg.j_max;
    if (ran > 0) st.info.eta_min = std::min(st.info.eta_min, rec[REC_ETAMIN]);
    if (appended > 0 && j0 + 1 < cfg.j_max) st.info.res_norm = std::sqrt(rec[REC_RR]);
    if (rec[REC_BREAK] != 0.0) {
      st.info.breakdown = 1;
      st.active = false;
    } else if (rec[REC_CONV] != 0.0) {
      st.info.converged = 1;
      st.active = false;
    }
    std::copy(rec, rec + REC_COUNT, rec_h);
    return IGP_OK;
  }

  // after the iteration's scalars are on the host (batched driver)
  void phase_consume() {
    const double eta = sc[SC_ETA];
    if (!(eta > 0.0)) {
      st.info.breakdown = 1;   // s_j and t_j are dropped: ncols is not advanced
      --st.j;
      st.active = false;
      return;
    }
    st.info.eta_min = std::min(st.info.eta_min, eta);
    ++ncols;
    if (st.next_r) {
      st.info.res_norm = std::sqrt(sc[SC_RR]);
      if (!(st.info.res_norm >= st.thresh)) {
        st.info.converged = 1;
        st.active = false;
      }
    }
  }

  // K v of the final iterate is on the device already when the solver carried it
  // (recurrence residual) or formed it for its last residual (explicit residual:
  // every iteration but iteration j_max forms one, and r_0 is formed when
  // j_max > 0); a breakdown leaves v, hence that K v, as they were
  bool kv_current() const { return recurrence() || (cfg.j_max > 0 && st.j < cfg.j_max); }

  // f_{i+1} = K v into fnew: that K v when it is current, else a product
  int phase_update() {
    if (kv_current()) return copy_vec<T>(L.kv, L.fnew, n, stream);
    ++st.kprod;
    return apply_K(L.v, L.fnew);
  }

  // after f_{i+1} = K v + m has been enqueued into fnew
  int phase_stats() {
    if (softmax())
      IGP_TRY(newton_stats<T>(L.fnew, L.f, L.v, static_cast<const int32_t*>(y), N, C, L.part,
                              L.scal, stream));
    else
      IGP_TRY(diag_stats<T>(cfg.likelihood, cfg.noise_var, L.fnew, L.f, L.v, y, n, L.part,
                            L.scal, stream));
    if (prof) IGP_CHECK_HIP(hipEventRecord(st.step_b, stream));
    return IGP_OK;
  }

  int phase_finish(igp_step_info* info_out) {
    IGP_TRY(collect_profile());
    std::swap(L.f, L.fnew);
    igp_step_info& info = st.info;
    info.iters = st.j;
    info.buffer_cols = ncols;
    info.k_products = st.kprod;
    info.rel_change = sc[SC_FNEW2] > 0.0 ? std::sqrt(sc[SC_DIFF2] / sc[SC_FNEW2]) : INFINITY;
    info.psi = sc[SC_LOGLIK] - 0.5 * sc[SC_GV];
    if (!std::isfinite(info.eta_min)) info.eta_min = 0.0;
    ++steps_done;
    if (info_out) *info_out = info;
    return IGP_OK;
  }

  KVProblem product_action() const { return kv_problem(L.X, N, s_col(), 1, n, t_col(), n); }
  KVProblem product_update() const { return kv_problem(L.X, N, L.v, 1, n, L.fnew, n); }

  // An iteration's end (the norm of its residual and iter_consume) left to
  // the next iteration's action kernel: the residual partials to finish.
  struct PendingEnd {
    const double* part = nullptr;
    int nblk = 0;
  };
  // whether an iteration's end may be left to the next iteration's action
  bool can_defer_end() const {
    return cfg.policy == IGP_POLICY_CG && recurrence() && softmax();
  }

  // Solver iteration jj (1-based) with its action in buffer column col, behind
  // the gate: the action, alpha, t = K s, z, Q^T z, d and eta, the guarded
  // append, the next residual when next_r, and iter_consume (Algorithm 2).
  // pend: the previous iteration's end when it was left to this action (then
  // cleared); defer_end: leave this iteration's end to the next one, which
  // the caller enqueues right after it.
  int enqueue_iteration(int jj, int col, bool next_r, PendingEnd* pend, bool defer_end) {
    int* gate = L.gate;
    T* sv = L.S + static_cast<int64_t>(col) * ld;
    T* tv = L.Tb + static_cast<int64_t>(col) * ld;
    // alpha and eta stay as partials (L.apart, L.part) until the append step
    // finishes them
    if (cfg.policy == IGP_POLICY_CG && pend->part) {
      IGP_TRY(consume_action_cg_dot<T>(L.r, pend->part, pend->nblk, L.scal, st.thresh, gate,
                                       L.rec, sv, n, L.apart, stream));
      *pend = PendingEnd{};
    } else if (cfg.policy == IGP_POLICY_CG) {
      IGP_TRY(action_cg_dot<T>(L.r, L.scal + SC_RR, sv, n, L.apart, nullptr, gate, stream));
    } else {
      if (cfg.policy == IGP_POLICY_UNIT)
        IGP_TRY(fill_unit<T>(sv, n, jj - 1, stream, gate));
      else
        IGP_TRY(copy_vec<T>(user + static_cast<int64_t>(jj - 1) * user_ld, sv, n, stream, gate));
      IGP_TRY(dot_into<T>(sv, L.r, n, L.apart, nullptr, stream, gate));
    }
    // t = K s, with z = t + W^+ s in the product's reduction where it can be
    int zdone = 0;
    IGP_TRY(apply_K(sv, tv, gate, jj, L.z, &zdone));
    if (!zdone) IGP_TRY(apply_winv(sv, 1, n, tv, n, L.z, n, gate));
    IGP_TRY(gemv_t<T>(L.Q, ld, n, col, L.z, L.part, L.yb, stream, gate));
    IGP_TRY(dir_update<T>(sv, L.Q, ld, n, col, L.yb, L.z, L.d, L.epart, nullptr, stream, tv,
                          recurrence() ? L.KQ : nullptr, L.kd, gate));
    if (next_r && recurrence() && softmax()) {
      // the append and the next residual in one pass over the points
      int g = 0;
      IGP_TRY(append_winv_residual<T>(L.d, L.apart, L.epart, L.scal,
                                      L.Q + static_cast<int64_t>(col) * ld, L.v, L.kd,
                                      L.KQ + static_cast<int64_t>(col) * ld, L.kv, L.pi, N, C,
                                      L.rhs, L.wv, L.r, L.part, &g, stream, gate));
      if (defer_end) {   // L.part is next written after the next action has read it
        *pend = PendingEnd{L.part, g};
        return IGP_OK;
      }
      return rr_consume(L.part, g, L.scal, st.thresh, gate, L.rec, stream);
    }
    IGP_TRY(append_and_step<T>(L.d, L.apart, L.epart, L.scal,
                               L.Q + static_cast<int64_t>(col) * ld, L.v, n,
                               stream, recurrence() ? L.kd : nullptr,
                               recurrence() ? L.KQ + static_cast<int64_t>(col) * ld : nullptr,
                               L.kv, gate));
    if (next_r) return enqueue_residual(jj);   // its last block ends the iteration
    return iter_consume(L.scal, st.thresh, 0, L.gate, L.rec, stream);
  }

  // Iterations go to the stream in windows of up to SPEC_WINDOW, each followed by
  // an asynchronous copy of the scalars and the iteration record to pinned host
  // memory and an event; the next window is enqueued (assuming every iteration
  // of this one appends) before the host waits for this one, so the device is
  // not left idle while the host reads and plans.
  static constexpr int64_t SPEC_WINDOW = 4;
  struct Window {
    int j0 = 0, col0 = 0, w = 0, slot = 0;
  };
  double rec_h[REC_COUNT] = {};     // record as of the last consumed window
  double* win_host = nullptr;       // pinned: 2 x (SC_COUNT + REC_COUNT) doubles
  hipEvent_t win_ev[2] = {nullptr, nullptr};

  int window_buffers() {
    if (!win_host) {
      IGP_CHECK_HIP(hipHostMalloc(reinterpret_cast<void**>(&win_host),
                                  2 * (SC_COUNT + REC_COUNT) * sizeof(double)));
    }
    for (hipEvent_t& e : win_ev)
      if (!e) IGP_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return IGP_OK;
  }

  // how many iterations may follow iteration j0 with ncols0 buffer columns
  int64_t window_size(int j0, int ncols0, int64_t budget) const {
    int64_t w = std::min<int64_t>(SPEC_WINDOW, budget);
    w = std::min<int64_t>(w, cfg.j_max - j0);
    w = std::min<int64_t>(w, cfg.max_buffer - ncols0);
    if (cfg.policy == IGP_POLICY_USER) w = std::min<int64_t>(w, user_cols - j0);
    return std::max<int64_t>(w, 0);
  }

  int enqueue_window(const Window& win) {
    // within the window each iteration's end goes into the next iteration's
    // action where that is possible; the last iteration ends on its own
    PendingEnd pend;
    for (int i = 0; i < win.w; ++i) {
      const int jj = win.j0 + i + 1;
      const bool next_r = jj < cfg.j_max;
      IGP_TRY(enqueue_iteration(jj, win.col0 + i, next_r, &pend,
                                next_r && i + 1 < win.w && can_defer_end()));
    }
    IGP_REQUIRE(!pend.part, "a solver iteration's end was left without a next iteration");
    double* h = win_host + win.slot * (SC_COUNT + REC_COUNT);
    // scalars and record (adjacent in the arena) in one copy
    IGP_CHECK_HIP(hipMemcpyAsync(h, L.scal, (SC_COUNT + REC_COUNT) * sizeof(double),
                                 hipMemcpyDeviceToHost, stream));
    IGP_CHECK_HIP(hipEventRecord(win_ev[win.slot], stream));
    return IGP_OK;
  }

  // wait for a window and fold its iterations into the host state; returns the
  // number of iterations that ran (0 when the solver had stopped before it)
  int consume_window(const Window& win, int* ran_out) {
    IGP_CHECK_HIP(hipEventSynchronize(win_ev[win.slot]));
    const double* h = win_host + win.slot * (SC_COUNT + REC_COUNT);
    const double* rec = h + SC_COUNT;
    std::copy(h, h + SC_COUNT, sc);
    const int ran = static_cast<int>(rec[REC_EXEC] - rec_h[REC_EXEC]);
    const int appended = static_cast<int>(rec[REC_APPEND] - rec_h[REC_APPEND]);
    std::copy(rec, rec + REC_COUNT, rec_h);
    IGP_REQUIRE(ran >= 0 && ran <= win.w && appended <= ran && appended >= ran - 1 &&
                    (ran == 0 || (win.j0 == st.j && win.col0 == ncols)),
                "solver iteration record out of step with the host");
    for (int i = 1; i <= ran; ++i)
      st.kprod += 1 + (!recurrence() && win.j0 + i < cfg.j_max ? 1 : 0);
    settle_products(win.j0 + 1, win.j0 + win.w, win.j0 + ran);
    *ran_out = ran;
    if (ran == 0) return IGP_OK;
    st.j = win.j0 + appended;
    ncols += appended;
    st.info.eta_min = std::min(st.info.eta_min, rec[REC_ETAMIN]);
    if (appended > 0 && win.j0 + 1 < cfg.j_max) st.info.res_norm = std::sqrt(rec[REC_RR]);
    if (rec[REC_BREAK] != 0.0) {   // s_j and t_j of the last iteration are dropped
      st.info.breakdown = 1;
      st.active = false;
    } else if (rec[REC_CONV] != 0.0) {
      st.info.converged = 1;
      st.active = false;
    }
    return IGP_OK;
  }

  // A Newton step in three parts, so that a caller can interleave other work
  // between solver iterations: begin (pseudo-targets, Algorithm 3, v_0, r_0),
  // iterate (up to max_iters iterations of Algorithm 2), end (f = K v + m and
  // the step's statistics).  newton_step runs the three back to back.
  bool in_step = false;

  int step_begin() override {
    clear_error();
    IGP_REQUIRE(!in_step, "a Newton step is already in progress");
    IGP_TRY(phase_begin());
    IGP_TRY(phase_vsr_gram());
    IGP_TRY(phase_vsr_fetch());
    IGP_TRY(phase_vsr_host());
    IGP_TRY(phase_vsr_apply());
    IGP_TRY(phase_v0());
    IGP_TRY(read_scalars(sc));
    phase_start_iterations();
    IGP_TRY(iter_gate_init(L.gate, L.rec, stream));
    for (double& x : rec_h) x = 0.0;
    in_step = true;
    return IGP_OK;
  }

  int step_iterate(int64_t max_iters, int32_t* done) override {
    clear_error();
    IGP_REQUIRE(in_step, "no Newton step in progress");
    IGP_REQUIRE(max_iters >= 0, "max_iters must be >= 0");
    IGP_TRY(window_buffers());
    int64_t k = 0;        // iterations run
    int64_t queued = 0;   // iterations enqueued, not yet consumed
    Window cur, nxt;
    bool have_cur = false;
    int slot = 0;
    while (k < max_iters) {
      if (!have_cur) {
        IGP_TRY(phase_can_act());
        if (!st.active) break;
        cur = Window{st.j, ncols, static_cast<int>(window_size(st.j, ncols, max_iters - k)), slot};
        IGP_TRY(enqueue_window(cur));
        queued = cur.w;
        have_cur = true;
      }
      // the following window, as if every iteration of this one appends
      const int64_t wn = window_size(cur.j0 + cur.w, cur.col0 + cur.w, max_iters - k - queued);
      const bool have_nxt = wn > 0;
      if (have_nxt) {
        nxt = Window{cur.j0 + cur.w, cur.col0 + cur.w, static_cast<int>(wn), cur.slot ^ 1};
        IGP_TRY(enqueue_window(nxt));
      }
      int ran = 0;
      IGP_TRY(consume_window(cur, &ran));
      k += ran;
      queued = have_nxt ? nxt.w : 0;
      if (!st.active) {
        if (have_nxt) IGP_TRY(consume_window(nxt, &ran));   // runs nothing: the gate is closed
        have_cur = false;
        break;
      }
      have_cur = have_nxt;
      if (have_nxt) cur = nxt;
      slot = cur.slot ^ (have_cur ? 0 : 1);
    }
    if (done) {
      IGP_TRY(phase_can_act());
      *done = st.active ? 0 : 1;
    }
    return IGP_OK;
  }

  int step_end(igp_step_info* info_out) override {
    clear_error();
    IGP_REQUIRE(in_step, "no Newton step in progress");
    IGP_TRY(phase_can_act());
    IGP_REQUIRE(!st.active, "the solver has not finished: iterate until done");
    in_step = false;
    IGP_TRY(phase_update());
    IGP_TRY(phase_stats());
    IGP_TRY(read_scalars(sc));
    return phase_finish(info_out);
  }

  int newton_step(igp_step_info* info_out) override {
    IGP_TRY(step_begin());
    IGP_TRY(step_iterate(INT64_MAX, nullptr));
    return step_end(info_out);
  }

  // Algorithm 3 on its own: the virtual solver run over the stored buffer with
  // W^+ taken at the current f (the point the predictive covariance is formed
  // at), keeping at most rank_limit directions; v and f are left as they are.
  int compress(int32_t rank_limit, int32_t* kept) override {
    clear_error();
    IGP_REQUIRE(!in_step, "compress during a Newton step");
    IGP_REQUIRE(rank_limit >= -1, "rank_limit must be >= -1");
    // W at f; the pseudo-targets it also forms go to scratch (rhs is kept)
    IGP_TRY(likelihood_terms(L.wv));
    st = StepState{};
    const int saved = cfg.rank_limit;
    cfg.rank_limit = rank_limit;
    int rc = phase_vsr_gram();
    if (rc == IGP_OK) rc = phase_vsr_fetch();
    if (rc == IGP_OK) rc = phase_vsr_host();
    if (rc == IGP_OK) rc = phase_vsr_apply();
    cfg.rank_limit = saved;
    IGP_TRY(rc);
    IGP_CHECK_HIP(hipStreamSynchronize(stream));
    if (kept) *kept = ncols;
    return IGP_OK;
  }

  // prediction launches split X2 independently of the number of test rows, so
  // a test row's result does not depend on which rows share its launch
  size_t kvws_for(int64_t n1, int64_t nb) const {
    return prepared ? kv_ws_bytes_prepared(n1, N, D, C, nb, cfg.precision, true)
                    : kv_ws_bytes(n1, N, D, C, nb, cfg.precision, true);
  }

  size_t predict_ws_bytes(int64_t Ns) const override {
    Carver cv(nullptr, 0);
    const int64_t B = std::max(ncols, 1);
    cv.take<T>(Ns * C * B);
    cv.take<char>(kvws_for(Ns, 1));
    cv.take<char>(kvws_for(Ns, B));
    if (prepared) cv.take<char>(prepared_rows_bytes(cfg.precision, Ns, D));
    return cv.used + 256;
  }

  int predict(const void* Xs_, int64_t Ns, void* mean_, void* var_, void* probs_, void* ws,
              size_t ws_bytes, hipStream_t s) const override {
    clear_error();
    if (Ns == 0) return IGP_OK;
    IGP_REQUIRE(Xs_ && mean_, "predict: NULL Xs or mean");
    IGP_REQUIRE(!probs_ || var_, "predict: probs requires var");
    IGP_REQUIRE(!probs_ || softmax(), "predict: class probabilities need the softmax likelihood");
    if (ws_bytes < predict_ws_bytes(Ns)) {
      set_error("predict workspace too small: need %zu bytes", predict_ws_bytes(Ns));
      return IGP_ENOMEM;
    }
    const T* Xs = static_cast<const T*>(Xs_);
    T* mean = static_cast<T*>(mean_);
    Carver cv(ws, ws_bytes);
    const int64_t B = std::max(ncols, 1);
    T* A = cv.take<T>(Ns * C * B);
    const size_t w1 = kvws_for(Ns, 1);
    void* ws1 = cv.take<char>(w1);
    const size_t w2 = kvws_for(Ns, B);
    void* ws2 = cv.take<char>(w2);
    void* xsp = nullptr;
    float* nsp = nullptr;
    if (prepared) {
      const size_t rb = prepared_rows_bytes(cfg.precision, Ns, D);
      char* base = cv.take<char>(rb);
      xsp = base;
      nsp = reinterpret_cast<float*>(base + rb - align_up(Ns * sizeof(float)));
      IGP_TRY(prep_rows_any(cfg.precision, reinterpret_cast<const float*>(Xs), Ns, D, L.centre,
                            xsp, nsp, s));
    }
    KVProblem pm = kv_problem(Xs, Ns, L.v, 1, n, mean, Ns * C, xsp, nsp);
    pm.fixed_split = true;
    IGP_TRY(kv_launch(pm, ws1, w1, s));
    if (var_) {
      if (ncols > 0) {
        KVProblem pv = kv_problem(Xs, Ns, L.Q, ncols, ld, A, Ns * C, xsp, nsp);
        pv.fixed_split = true;
        IGP_TRY(kv_launch(pv, ws2, w2, s));
      }
      IGP_TRY(predict_epilogue<T>(A, Ns * C, Ns * C, ncols, prior_var.data(), mean, Ns, C,
                                  static_cast<T*>(var_), static_cast<T*>(probs_), s));
    }
    return IGP_OK;
  }

  int view(int which, const void** ptr, int64_t* rows, int64_t* cols,
           int64_t* ldo) const override {
    int64_t r = n, c = 1, l = n;
    const void* p = nullptr;
    switch (which) {
      case IGP_VIEW_F: p = L.f; break;
      case IGP_VIEW_V: p = L.v; break;
      case IGP_VIEW_RHS: p = L.rhs; break;
      case IGP_VIEW_Q: p = L.Q; c = ncols; l = ld; break;
      case IGP_VIEW_S: p = L.S; c = ncols; l = ld; break;
      case IGP_VIEW_T: p = L.Tb; c = ncols; l = ld; break;
      case IGP_VIEW_X: p = L.X; r = N; c = D; l = D; break;
      default: set_error("unknown view %d", which); return IGP_EINVAL;
    }
    if (ptr) *ptr = p;
    if (rows) *rows = r;
    if (cols) *cols = c;
    if (ldo) *ldo = l;
    return IGP_OK;
  }

  int set_block_likelihood(const void* grad, const void* W) override {
    clear_error();
    IGP_REQUIRE(block(), "itergp_set_block_likelihood needs a model with IGP_LIK_BLOCK");
    IGP_REQUIRE(!in_step, "itergp_set_block_likelihood during a Newton step");
    IGP_REQUIRE(grad && W, "block likelihood: NULL gradient or blocks");
    IGP_CHECK_HIP(hipMemsetAsync(L.flags, 0, sizeof(int), stream));
    IGP_TRY(block_begin<T>(static_cast<const T*>(W), static_cast<const T*>(grad), L.f, N, C,
                           L.wblk, L.rhs, L.flags, stream));
    int bad = 0;
    IGP_CHECK_HIP(hipMemcpyAsync(&bad, L.flags, sizeof(int), hipMemcpyDeviceToHost, stream));
    IGP_CHECK_HIP(hipStreamSynchronize(stream));
    block_set = bad == 0;
    if (bad) {
      set_error("block likelihood: %d of %lld blocks are not positive definite", bad,
                (long long)N);
      return IGP_EINVAL;
    }
    return IGP_OK;
  }

  int set_user_actions(const void* a, int64_t nc, int64_t l) override {
    IGP_REQUIRE(nc >= 0 && (nc == 0 || (a && l >= n)), "user actions: bad pointer or stride");
    user = static_cast<const T*>(a);
    user_cols = nc;
    user_ld = l;
    return IGP_OK;
  }
};

// ---- batched form: many independent models advance together -------------------
__global__ void k_gather_scalars(const double* const* __restrict__ src, int n,
                                 double* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * SC_COUNT) return;
  dst[i] = src[i / SC_COUNT][i % SC_COUNT];
}

// the iteration records of the models (REC_COUNT doubles each), gathered
__global__ void k_gather_records(const double* const* __restrict__ src, int n,
                                 double* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * REC_COUNT) return;
  dst[i] = src[i / REC_COUNT][i % REC_COUNT];
}

// the virtual solver run's Gram matrices of a batch's models, gathered into one
// device buffer for a single copy to the host: entry k covers
// dst[off_k, off_{k+1}) from src_k (off of the last entry: the total)
struct GatherEnt {
  const double* src;
  int64_t off;
};
__global__ void k_gather_mats(const GatherEnt* __restrict__ ent, int n, double* __restrict__ dst) {
  const int64_t total = ent[n].off;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (ent[mid].off <= i) lo = mid;
      else hi = mid - 1;
    }
    dst[i] = ent[lo].src[i - ent[lo].off];
  }
}

struct TuneKey {
  int kind, dch, nbucket, bf16;
  bool operator<(const TuneKey& o) const {
    return std::tie(bf16, kind, dch, nbucket) < std::tie(o.bf16, o.kind, o.dch, o.nbucket);
  }
};
struct TuneVal {
  int ns;
  int64_t split_rows;
  double us;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
constexpr int64_t TUNE_SPLITS[] = {1024, 4096};
constexpr int TUNE_NS[] = {1, 2};

struct Batch {
  std::vector<Model<float>*> ms;
  hipStream_t stream = nullptr;
  int kind = 0, dch = 1;
  bool bf16 = false;        // BF16 models (the narrow BF16 tile)
  // workspace
  BatchProblem* dtab = nullptr;
  int* counter = nullptr;
  const double** dscal = nullptr;
  double* gathered = nullptr;
  float* partials = nullptr;
  std::vector<double> hgather;
  std::vector<BatchProblem> htab;
  BIter* dit = nullptr;            // iteration descriptors (device)
  int64_t* dpre = nullptr;         // per-operation block prefixes (device)
  std::vector<unsigned char> hitbuf;
  // device control: the tables of every round of a window, in slots of their
  // own ([DC_WINDOW][models] descriptors, [DC_WINDOW][BOP_COUNT][models + 1]
  // prefixes, [DC_WINDOW][models] product problems), uploaded in one copy
  static constexpr int DC_WINDOW = 8;
  BIter* dit_w = nullptr;
  int64_t* dpre_w = nullptr;
  BatchProblem* dtab_w = nullptr;
  char* dwin_end = nullptr;
  const double** drec = nullptr;   // record pointers of the models
  double* grec = nullptr;          // gathered records
  std::vector<double> hrec;
  std::vector<unsigned char> hwin;
  // the Gram matrices M of the virtual solver run, gathered for one copy
  GatherEnt* dgent = nullptr;
  double* gM = nullptr;
  std::vector<GatherEnt> hgent;
  std::vector<double> hgM;

  static size_t gram_doubles(const std::vector<Model<float>*>& ms) {
    size_t t = 0;
    for (auto* m : ms) t += static_cast<size_t>(m->cfg.max_buffer) * m->cfg.max_buffer;
    return std::max<size_t>(t, 1);
  }

  // partial slots of a model's product: the one-sided tiles' splits, or the
  // symmetric plan's super-blocks (FP32)
  static size_t partial_floats(const Model<float>* m) {
    size_t f = static_cast<size_t>(ceil_div(m->N, TUNE_SPLITS[0]) + 1) * m->N * m->C;
    BatchProblem bp{};
    if (m->cfg.precision == IGP_FP32 && batched_sym_plan(m->N, m->D, m->C, &bp))
      f = std::max(f, static_cast<size_t>(bp.sym_q) * m->N * m->C);
    return f;
  }

  // a product's partial slots must fit the model's partial area
  static int check_partials(const BatchProblem& bp, const Model<float>* m) {
    IGP_REQUIRE(static_cast<size_t>(bp.nsplit) * bp.n1 * bp.W <= partial_floats(m),
                "batched product partials exceed the model's partial area");
    return IGP_OK;
  }

  // the launch layout of one round's products: symmetric problems first,
  // sorted by output width and distance k-blocks (one group and launch each)
  struct Layout {
    std::vector<SymGroup> groups;
    int64_t tiles = 0, outs = 0;
  };
  Layout lay_out(BatchProblem* tb, size_t n) const {
    auto* mid = std::stable_partition(tb, tb + n, [](const BatchProblem& b) { return b.sym_q > 0; });
    std::stable_sort(tb, mid, [](const BatchProblem& a, const BatchProblem& b) {
      return a.W < b.W || (a.W == b.W && a.sym_kb < b.sym_kb);
    });
    Layout L;
    for (size_t q = 0; q < n; ++q) {
      BatchProblem& bp = tb[q];
      if (bp.sym_q > 0) {
        if (L.groups.empty() || L.groups.back().W != bp.W || L.groups.back().kb != bp.sym_kb)
          L.groups.push_back(SymGroup{static_cast<int>(q), 0, bp.W, bp.sym_kb, 0, 0});
        SymGroup& g = L.groups.back();
        bp.tile_begin = g.tiles;
        g.tiles += batched_tiles(bp);
        ++g.count;
        g.lds = std::max(g.lds, batched_sym_lds(bp, dch));
      } else {
        bp.tile_begin = L.tiles;
        L.tiles += batched_tiles(bp);
      }
      bp.out_begin = L.outs;
      L.outs += bp.n1 * bp.W;
    }
    return L;
  }

  static size_t ws_bytes(const std::vector<Model<float>*>& ms) {
    Carver cv(nullptr, 0);
    cv.take<BIter>(ms.size());
    cv.take<int64_t>(static_cast<size_t>(BOP_COUNT) * (ms.size() + 1));
    cv.take<BatchProblem>(ms.size());
    cv.take<int64_t>(BATCH_COUNTERS);
    cv.take<const double*>(ms.size());
    cv.take<double>(ms.size() * SC_COUNT);
    cv.take<BIter>(DC_WINDOW * ms.size());
    cv.take<int64_t>(static_cast<size_t>(DC_WINDOW) * BOP_COUNT * (ms.size() + 1));
    cv.take<BatchProblem>(DC_WINDOW * ms.size());
    cv.take<const double*>(ms.size());
    cv.take<double>(ms.size() * REC_COUNT);
    cv.take<GatherEnt>(ms.size() + 1);
    cv.take<double>(gram_doubles(ms));
    size_t pf = 0;
    for (auto* m : ms) pf += align_up(partial_floats(m) * sizeof(float)) / sizeof(float);
    cv.take<float>(pf);
    return cv.used + 256;
  }

  int carve_ws(void* ws, size_t bytes) {
    Carver cv(ws, bytes);
    dit = cv.take<BIter>(ms.size());
    dpre = cv.take<int64_t>(static_cast<size_t>(BOP_COUNT) * (ms.size() + 1));
    dtab = cv.take<BatchProblem>(ms.size());
    counter = reinterpret_cast<int*>(cv.take<int64_t>(BATCH_COUNTERS));
    dscal = cv.take<const double*>(ms.size());
    gathered = cv.take<double>(ms.size() * SC_COUNT);
    dit_w = cv.take<BIter>(DC_WINDOW * ms.size());
    dpre_w = cv.take<int64_t>(static_cast<size_t>(DC_WINDOW) * BOP_COUNT * (ms.size() + 1));
    dtab_w = cv.take<BatchProblem>(DC_WINDOW * ms.size());
    dwin_end = reinterpret_cast<char*>(dtab_w + DC_WINDOW * ms.size());
    drec = cv.take<const double*>(ms.size());
    grec = cv.take<double>(ms.size() * REC_COUNT);
    dgent = cv.take<GatherEnt>(ms.size() + 1);
    gM = cv.take<double>(gram_doubles(ms));
    size_t pf = 0;
    for (auto* m : ms) pf += align_up(partial_floats(m) * sizeof(float)) / sizeof(float);
    partials = cv.take<float>(pf);
    if (!cv.fits() || !ws) {
      set_error("batched workspace too small: need %zu bytes", ws_bytes(ms));
      return IGP_ENOMEM;
    }
    std::vector<const double*> hs(ms.size()), hr(ms.size());
    for (size_t i = 0; i < ms.size(); ++i) {
      hs[i] = ms[i]->L.scal;
      hr[i] = ms[i]->L.rec;
    }
    IGP_CHECK_HIP(hipMemcpyAsync(dscal, hs.data(), hs.size() * sizeof(double*),
                                 hipMemcpyHostToDevice, stream));
    IGP_CHECK_HIP(hipMemcpyAsync(drec, hr.data(), hr.size() * sizeof(double*),
                                 hipMemcpyHostToDevice, stream));
    IGP_CHECK_HIP(hipStreamSynchronize(stream));
    hgather.resize(ms.size() * SC_COUNT);
    hrec.resize(ms.size() * REC_COUNT);
    return IGP_OK;
  }

  // every model's M (ncols x ncols) to its host copy: one gather kernel and one
  // device-to-host copy for the batch, instead of a copy and a wait per model
  int fetch_grams() {
    hgent.clear();
    int64_t off = 0;
    std::vector<int> who;
    for (size_t i = 0; i < ms.size(); ++i) {
      const int B = ms[i]->ncols;
      if (B == 0) continue;
      hgent.push_back(GatherEnt{ms[i]->L.M, off});
      who.push_back(static_cast<int>(i));
      off += static_cast<int64_t>(B) * B;
    }
    if (who.empty()) return IGP_OK;
    IGP_REQUIRE(static_cast<size_t>(off) <= gram_doubles(ms), "batched Gram gather too large");
    hgent.push_back(GatherEnt{nullptr, off});
    IGP_CHECK_HIP(hipMemcpyAsync(dgent, hgent.data(), hgent.size() * sizeof(GatherEnt),
                                 hipMemcpyHostToDevice, stream));
    const int blocks = static_cast<int>(std::min<int64_t>(ceil_div(off, 256), 2048));
    k_gather_mats<<<blocks, 256, 0, stream>>>(dgent, static_cast<int>(who.size()), gM);
    IGP_CHECK_LAUNCH();
    hgM.resize(static_cast<size_t>(off));
    IGP_CHECK_HIP(hipMemcpyAsync(hgM.data(), gM, hgM.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, stream));
    IGP_CHECK_HIP(hipStreamSynchronize(stream));
    for (size_t k = 0; k < who.size(); ++k) {
      Model<float>* m = ms[who[k]];
      m->hM.assign(hgM.begin() + hgent[k].off, hgM.begin() + hgent[k + 1].off);
    }
    return IGP_OK;
  }

  int read_records() {
    const int n = static_cast<int>(ms.size());
    k_gather_records<<<static_cast<unsigned>(ceil_div(n * REC_COUNT, 256)), 256, 0, stream>>>(
        drec, n, grec);
    IGP_CHECK_LAUNCH();
    IGP_CHECK_HIP(hipMemcpyAsync(hrec.data(), grec, hrec.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, stream));
    IGP_CHECK_HIP(hipStreamSynchronize(stream));
    return IGP_OK;
  }

  // The tuned launch shape for the product of the models in idx, if known.
  bool tuned(const std::vector<int>& idx, TuneVal* out) const {
    int64_t total = 0;
    for (int i : idx) total += ms[i]->N;
    const TuneKey key{kind, dch, static_cast<int>(std::log2(std::max<int64_t>(total, 1))),
                      bf16 ? 1 : 0};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
  }

  // One device-controlled window: round k < rounds.size() runs iteration
  // jj = j + k + 1 at column ncols + k of every model listed for it (each
  // model's rounds are a prefix).  All rounds' tables are built on the host
  // and uploaded in one copy; every operation and product tile of a model
  // whose gate has closed returns at once.  Returns IGP_EUNSUPPORTED (nothing
  // enqueued) if a round's launch shape has not been tuned yet.
  int dc_window(const std::vector<std::vector<int>>& rounds) {
    const size_t nmod = ms.size(), pre_len = nmod + 1;
    const size_t R = rounds.size();
    std::vector<TuneVal> tv(R);
    for (size_t k = 0; k < R; ++k)
      if (!tuned(rounds[k], &tv[k])) return IGP_EUNSUPPORTED;
    char* base = reinterpret_cast<char*>(dit_w);
    const size_t bytes = static_cast<size_t>(dwin_end - base);
    hwin.assign(bytes, 0);
    auto hit = [&](size_t k) {
      return reinterpret_cast<BIter*>(hwin.data() + (reinterpret_cast<char*>(dit_w + k * nmod) - base));
    };
    auto hpre = [&](size_t k, int op) {
      return reinterpret_cast<int64_t*>(
          hwin.data() + (reinterpret_cast<char*>(dpre_w + (k * BOP_COUNT + op) * pre_len) - base));
    };
    auto htb = [&](size_t k) {
      return reinterpret_cast<BatchProblem*>(
          hwin.data() + (reinterpret_cast<char*>(dtab_w + k * nmod) - base));
    };
    std::vector<std::vector<int64_t>> totals(R, std::vector<int64_t>(BOP_COUNT, 0));
    std::vector<Layout> lay(R);
    for (size_t k = 0; k < R; ++k) {
      const auto& idx = rounds[k];
      BIter* ht = hit(k);
      for (size_t q = 0; q < idx.size(); ++q) {
        Model<float>* m = ms[idx[q]];
        ht[q] = m->biter_at(m->st.j + static_cast<int64_t>(k) + 1, m->ncols + static_cast<int>(k));
      }
      for (int op = 0; op < BOP_COUNT; ++op) {
        int64_t* pre = hpre(k, op);
        pre[0] = 0;
        for (size_t q = 0; q < idx.size(); ++q)
          pre[q + 1] = pre[q] + biter_blocks(op, ht[q], ht[q].next_r != 0);
        totals[k][op] = pre[idx.size()];
      }
      BatchProblem* tb = htb(k);
      size_t poff = 0;
      for (size_t q = 0; q < idx.size(); ++q) {
        Model<float>* m = ms[idx[q]];
        const KVProblem kp = m->product_action_at(m->ncols + static_cast<int>(k));
        BatchProblem& bp = tb[q];
        bp = problem_of(kp, tv[k].ns, tv[k].split_rows, !bf16);
        IGP_TRY(check_partials(bp, m));
        bp.P = partials + poff;
        poff += align_up(partial_floats(m) * sizeof(float)) / sizeof(float);
        bp.gate = m->L.gate;
      }
      lay[k] = lay_out(tb, idx.size());
    }
    IGP_CHECK_HIP(hipMemcpyAsync(base, hwin.data(), bytes, hipMemcpyHostToDevice, stream));
    for (size_t k = 0; k < R; ++k) {
      const int nm = static_cast<int>(rounds[k].size());
      if (nm == 0) continue;
      BIter* dt = dit_w + k * nmod;
      for (int op = BOP_ACTION; op <= BOP_FIN_ALPHA; ++op)
        IGP_TRY(biter_launch(op, dt, dpre_w + (k * BOP_COUNT + op) * pre_len, nm, totals[k][op],
                             stream));
      IGP_TRY(kv_batched_run(kind, dch, tv[k].ns, bf16, dtab_w + k * nmod, nm,
                             lay[k].groups.data(), static_cast<int>(lay[k].groups.size()),
                             lay[k].tiles, lay[k].outs, counter, stream));
      for (int op = BOP_WINV_Z; op < BOP_COUNT; ++op)
        IGP_TRY(biter_launch(op, dt, dpre_w + (k * BOP_COUNT + op) * pre_len, nm, totals[k][op],
                             stream));
    }
    return IGP_OK;
  }


  // copy every model's scalar block to its host array (one transfer)
  int read_all() {
    const int n = static_cast<int>(ms.size());
    k_gather_scalars<<<static_cast<unsigned>(ceil_div(n * SC_COUNT, 256)), 256, 0, stream>>>(
        dscal, n, gathered);
    IGP_CHECK_LAUNCH();
    IGP_CHECK_HIP(hipMemcpyAsync(hgather.data(), gathered, hgather.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, stream));
    IGP_CHECK_HIP(hipStreamSynchronize(stream));
    for (int i = 0; i < n; ++i)
      std::copy(&hgather[static_cast<size_t>(i) * SC_COUNT],
                &hgather[static_cast<size_t>(i) * SC_COUNT] + SC_COUNT, ms[i]->sc);
    return IGP_OK;
  }

  // operations [op_begin, op_end) of one iteration for the selected models,
  // one launch each (descriptors and block prefixes uploaded in one copy)
  int iter_group(const std::vector<int>& idx, int op_begin, int op_end) {
    const size_t nm = idx.size();
    if (nm == 0) return IGP_OK;
    const size_t tab_bytes = nm * sizeof(BIter);
    const size_t pre_len = nm + 1;
    hitbuf.resize(tab_bytes + static_cast<size_t>(BOP_COUNT) * pre_len * sizeof(int64_t));
    BIter* ht = reinterpret_cast<BIter*>(hitbuf.data());
    int64_t* hp = reinterpret_cast<int64_t*>(hitbuf.data() + tab_bytes);
    std::vector<char> resid(nm);
    for (size_t k = 0; k < nm; ++k) {
      ht[k] = ms[idx[k]]->biter();
      resid[k] = ms[idx[k]]->st.next_r ? 1 : 0;
    }
    std::vector<int64_t> total(BOP_COUNT, 0);
    for (int op = op_begin; op < op_end; ++op) {
      int64_t* pre = hp + static_cast<size_t>(op) * pre_len;
      pre[0] = 0;
      for (size_t k = 0; k < nm; ++k) pre[k + 1] = pre[k] + biter_blocks(op, ht[k], resid[k]);
      total[op] = pre[nm];
    }
    // the table goes to dit; the prefix block to the matching offset of dpre
    IGP_CHECK_HIP(hipMemcpyAsync(dit, ht, tab_bytes, hipMemcpyHostToDevice, stream));
    IGP_CHECK_HIP(hipMemcpyAsync(dpre + static_cast<size_t>(op_begin) * pre_len,
                                 hp + static_cast<size_t>(op_begin) * pre_len,
                                 static_cast<size_t>(op_end - op_begin) * pre_len * sizeof(int64_t),
                                 hipMemcpyHostToDevice, stream));
    for (int op = op_begin; op < op_end; ++op)
      IGP_TRY(biter_launch(op, dit, dpre + static_cast<size_t>(op) * pre_len,
                           static_cast<int>(nm), total[op], stream));
    return IGP_OK;
  }

  // one model's product in the batched launch (partials, tile and output
  // offsets and gate are set by the caller)
  // (sym: FP32, where the symmetric plan applies to K(X, X) V)
  static BatchProblem problem_of(const KVProblem& kp, int ns, int64_t split_rows, bool sym) {
    BatchProblem bp{};
    bp.X1p = kp.X1p;
    bp.nrm1 = kp.norm1;
    bp.X2p = kp.X2p;
    bp.nrm2 = kp.norm2;
    bp.n1 = kp.n1;
    bp.n2 = kp.n2;
    bp.V = static_cast<const float*>(kp.V);
    bp.ldv = kp.ldv;
    bp.C = static_cast<int>(kp.C);
    bp.W = static_cast<int>(kp.C * kp.nb);
    batched_plan(bp.n1, bp.n2, bp.W, ns, split_rows, &bp);
    if (sym && kp.X1p == kp.X2p && kp.norm1 == kp.norm2 && kp.n1 == kp.n2)
      batched_sym_plan(bp.n1, kp.d, bp.W, &bp);
    const double inv_l2 = 1.0 / (kp.kp.lengthscale * kp.kp.lengthscale);
    const float kap = kv_kappa(kp.kp.kind);
    bp.cnorm = static_cast<float>(kap * inv_l2);
    bp.cdot = static_cast<float>(-2.0 * kap * inv_l2);
    bp.os = static_cast<float>(kp.kp.outputscale);
    bp.Out = static_cast<float*>(kp.Out);
    bp.ldo = kp.ldo;
    return bp;
  }

  // one persistent launch for the products of the selected models
  int run_products(const std::vector<int>& idx, bool update, int ns, int64_t split_rows) {
    htab.clear();
    size_t poff = 0;
    for (int i : idx) {
      Model<float>* m = ms[i];
      const KVProblem kp = update ? m->product_update() : m->product_action();
      BatchProblem bp = problem_of(kp, ns, split_rows, !bf16);
      IGP_TRY(check_partials(bp, m));
      bp.P = partials + poff;
      poff += align_up(partial_floats(m) * sizeof(float)) / sizeof(float);
      htab.push_back(bp);
      if (m->prof) {
        m->pending_evals += static_cast<double>(bp.n1) * bp.n2;
        m->pending_flops += 2.0 * bp.n1 * bp.n2 * (m->D + bp.W);
      }
    }
    if (htab.empty()) return IGP_OK;
    const Layout L = lay_out(htab.data(), htab.size());
    IGP_CHECK_HIP(hipMemcpyAsync(dtab, htab.data(), htab.size() * sizeof(BatchProblem),
                                 hipMemcpyHostToDevice, stream));
    return kv_batched_run(kind, dch, ns, bf16, dtab, static_cast<int>(htab.size()),
                          L.groups.data(), static_cast<int>(L.groups.size()), L.tiles, L.outs,
                          counter, stream);
  }

  // the tuned launch shape for this batch (timed on first use, then cached)
  int products(const std::vector<int>& idx, bool update) {
    int64_t total = 0;
    for (int i : idx) total += ms[i]->N;
    const TuneKey key{kind, dch, static_cast<int>(std::log2(std::max<int64_t>(total, 1))),
                      bf16 ? 1 : 0};
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) return run_products(idx, update, it->second.ns, it->second.split_rows);
    }
    hipEvent_t a, b;
    IGP_CHECK_HIP(hipEventCreate(&a));
    IGP_CHECK_HIP(hipEventCreate(&b));
    TuneVal best{2, TUNE_SPLITS[1], INFINITY};
    for (int ns : TUNE_NS)
      for (int64_t sr : TUNE_SPLITS) {
        IGP_TRY(run_products(idx, update, ns, sr));   // warm
        IGP_CHECK_HIP(hipEventRecord(a, stream));
        IGP_TRY(run_products(idx, update, ns, sr));
        IGP_CHECK_HIP(hipEventRecord(b, stream));
        IGP_CHECK_HIP(hipEventSynchronize(b));
        float ms_ = 0.f;
        IGP_CHECK_HIP(hipEventElapsedTime(&ms_, a, b));
        if (ms_ * 1e3 < best.us) best = TuneVal{ns, sr, ms_ * 1e3};
      }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[key] = best;
    }
    // the last candidate ran last; run the chosen one so its result stands
    return run_products(idx, update, best.ns, best.split_rows);
  }
};

template <typename F>
int parallel_for(int n, F&& f) {
  const int nt = std::max(1, std::min<int>(n, static_cast<int>(std::thread::hardware_concurrency())));
  std::vector<int> rc(nt, IGP_OK);
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      for (int i; (i = next.fetch_add(1)) < n;) {
        const int r = f(i);
        if (r != IGP_OK) rc[t] = r;
      }
    });
  for (auto& x : th) x.join();
  for (int r : rc)
    if (r != IGP_OK) return r;
  return IGP_OK;
}

int batch_models(igp_model* const* models, int n, std::vector<Model<float>*>* out, int* kind,
                 int* dch, hipStream_t* stream, bool* bf16) {
  IGP_REQUIRE(models && n >= 1, "no models");
  out->clear();
  for (int i = 0; i < n; ++i) {
    auto* m = dynamic_cast<Model<float>*>(models[i]);
    IGP_REQUIRE(m, "batched steps need FP32 or BF16 models (model %d is FP64)", i);
    IGP_REQUIRE(m->prepared && (m->cfg.precision == IGP_FP32 || m->cfg.precision == IGP_BF16),
                "model %d: batched steps need the FP32 or BF16 matrix-core path", i);
    IGP_REQUIRE(m->n_kp == 1, "model %d: batched steps need one kernel shared by the classes",
                i);
    IGP_REQUIRE(m->recurrence(), "model %d: batched steps need the recurrence residual", i);
    IGP_REQUIRE(!m->block(), "model %d: batched steps do not take the block likelihood", i);
    IGP_REQUIRE(batched_supported(m->kp.kind, m->D, m->C), "model %d: kernel, D <= 32 and C <= 8 "
                "are required for the batched launch", i);
    if (i == 0) {
      *kind = m->kp.kind;
      *dch = static_cast<int>(ceil_div(m->D, 16));
      *stream = m->stream;
      *bf16 = m->cfg.precision == IGP_BF16;
    }
    IGP_REQUIRE(m->kp.kind == *kind && ceil_div(m->D, 16) == *dch && m->stream == *stream &&
                    (m->cfg.precision == IGP_BF16) == *bf16,
                "model %d: all models of a batch share kernel family, feature count class, "
                "precision and stream", i);
    for (auto* o : *out) IGP_REQUIRE(o != m, "model %d appears twice", i);
    IGP_REQUIRE(!m->in_step, "model %d is in the middle of a Newton step", i);
    out->push_back(m);
  }
  return IGP_OK;
}

}  // namespace

size_t batched_ws_bytes(igp_model* const* models, int n) {
  std::vector<Model<float>*> ms;
  int kind, dch;
  hipStream_t st;
  bool bf;
  if (batch_models(models, n, &ms, &kind, &dch, &st, &bf) != IGP_OK) return 0;
  return Batch::ws_bytes(ms);
}

int newton_step_batched(igp_model* const* models, int n, igp_step_info* infos, void* ws,
                        size_t ws_bytes, int flags) {
  IGP_REQUIRE((flags & ~IGP_BATCH_DEVICE_CONTROL) == 0, "unknown batched-step flags %d", flags);
  const bool dc = (flags & IGP_BATCH_DEVICE_CONTROL) != 0;
  Batch b;
  IGP_TRY(batch_models(models, n, &b.ms, &b.kind, &b.dch, &b.stream, &b.bf16));
  IGP_TRY(b.carve_ws(ws, ws_bytes));
  auto& ms = b.ms;
  for (auto* m : ms) IGP_TRY(m->phase_begin());
  for (auto* m : ms) IGP_TRY(m->phase_vsr_gram());
  IGP_TRY(b.fetch_grams());
  IGP_TRY(parallel_for(n, [&](int i) { return ms[i]->phase_vsr_host(); }));
  for (auto* m : ms) IGP_TRY(m->phase_vsr_apply());
  for (auto* m : ms) IGP_TRY(m->phase_v0());
  IGP_TRY(b.read_all());
  for (auto* m : ms) m->phase_start_iterations();
  if (dc) {
    for (auto* m : ms) {
      IGP_TRY(iter_gate_init(m->L.gate, m->L.rec, b.stream));
      for (double& x : m->rec_h) x = 0.0;
    }
  }
  std::vector<int> act;
  for (;;) {
    act.clear();
    for (int i = 0; i < n; ++i) {
      IGP_TRY(ms[i]->phase_can_act());
      if (ms[i]->st.active) act.push_back(i);
    }
    if (act.empty()) break;
    if (dc) {
      // a window of up to DC_WINDOW rounds, the host reading the records once:
      // model i takes rounds 0 .. cap_i - 1, its gate skips those after it stops
      std::vector<int> cap(n, 0);
      int R = 0;
      for (int i : act) {
        cap[i] = ms[i]->window_cap(Batch::DC_WINDOW);
        R = std::max(R, cap[i]);
      }
      std::vector<std::vector<int>> rounds(R);
      for (int k = 0; k < R; ++k)
        for (int i : act)
          if (k < cap[i]) rounds[k].push_back(i);
      const int rc = R > 0 ? b.dc_window(rounds) : IGP_EUNSUPPORTED;
      if (rc == IGP_OK) {
        IGP_TRY(b.read_records());
        for (int i : act)
          IGP_TRY(ms[i]->consume_dc(&b.hrec[static_cast<size_t>(i) * REC_COUNT], cap[i]));
        continue;
      }
      if (rc != IGP_EUNSUPPORTED) return rc;
      clear_error();
      // a launch shape not timed yet: one round under host control times it
    }
    for (int i : act) ms[i]->host_action();
    IGP_TRY(b.iter_group(act, BOP_ACTION, BOP_FIN_ALPHA + 1));   // s_j, alpha_j
    IGP_TRY(b.products(act, false));                    // t_j = K s_j for every active model
    for (int i : act) ms[i]->host_after_product();
    IGP_TRY(b.iter_group(act, BOP_WINV_Z, BOP_COUNT));  // z_j .. r_j for every active model
    IGP_TRY(b.read_all());
    for (int i : act) ms[i]->phase_consume();
  }
  // f_{i+1} = K v: the carried K v, or one launch for the models without it
  std::vector<int> need;
  for (int i = 0; i < n; ++i) {
    if (ms[i]->kv_current())
      IGP_TRY(ms[i]->phase_update());
    else
      need.push_back(i);
  }
  if (!need.empty()) {
    IGP_TRY(b.products(need, true));
    for (int i : need) ++ms[i]->st.kprod;
  }
  for (auto* m : ms) IGP_TRY(m->phase_stats());
  IGP_TRY(b.read_all());
  for (int i = 0; i < n; ++i) IGP_TRY(ms[i]->phase_finish(infos ? &infos[i] : nullptr));
  return IGP_OK;
}

std::string batched_tuning_json() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::string s = "[";
  for (auto& kv : g_tune) {
    char buf[256];
    snprintf(buf, sizeof(buf),
             "%s{\"precision\": \"%s\", \"kind\": %d, \"feature_chunks\": %d, "
             "\"log2_rows\": %d, \"strips\": %d, \"split_rows\": %lld, \"us\": %.2f}",
             s.size() > 1 ? ", " : "", kv.first.bf16 ? "bf16" : "fp32", kv.first.kind,
             kv.first.dch, kv.first.nbucket,
             kv.second.ns, (long long)kv.second.split_rows, kv.second.us);
    s += buf;
  }
  return s + "]";
}

namespace {
// the number after "key": inside the object text [b, e); false if absent
bool json_number(const std::string& js, size_t b, size_t e, const char* key, double* out) {
  const std::string pat = std::string("\"") + key + "\"";
  size_t k = js.find(pat, b);
  if (k == std::string::npos || k >= e) return false;
  k = js.find(':', k + pat.size());
  if (k == std::string::npos || k >= e) return false;
  const char* start = js.c_str() + k + 1;
  char* end = nullptr;
  const double v = std::strtod(start, &end);
  if (end == start || static_cast<size_t>(end - js.c_str()) > e) return false;
  *out = v;
  return true;
}
}  // namespace

// Seeds the tuner's table from the JSON that batched_tuning_json writes (an
// array of flat objects); entries already in the table are kept.
int batched_tuning_load(const char* json, int* loaded) {
  IGP_REQUIRE(json, "NULL tuning text");
  const std::string js(json);
  std::vector<std::pair<TuneKey, TuneVal>> entries;
  size_t pos = 0;
  while ((pos = js.find('{', pos)) != std::string::npos) {
    const size_t end = js.find('}', pos);
    IGP_REQUIRE(end != std::string::npos, "tuning text: unterminated object");
    double kind, dch, nb, ns, sr, us = 0.0;
    IGP_REQUIRE(json_number(js, pos, end, "kind", &kind) &&
                    json_number(js, pos, end, "feature_chunks", &dch) &&
                    json_number(js, pos, end, "log2_rows", &nb) &&
                    json_number(js, pos, end, "strips", &ns) &&
                    json_number(js, pos, end, "split_rows", &sr),
                "tuning text: an entry lacks kind, feature_chunks, log2_rows, strips or "
                "split_rows");
    json_number(js, pos, end, "us", &us);
    // precision: "fp32" (the default when absent) or "bf16"
    const size_t pk = js.find("\"precision\"", pos);
    int bf = 0;
    if (pk != std::string::npos && pk < end) {
      const bool is32 = js.find("\"fp32\"", pk) < end, is16 = js.find("\"bf16\"", pk) < end;
      IGP_REQUIRE(is32 || is16, "tuning text: precision must be \"fp32\" or \"bf16\"");
      bf = is16 && !is32 ? 1 : 0;
    }
    bool ns_ok = false, sr_ok = false;
    for (int c : TUNE_NS) ns_ok |= ns == c;
    for (int64_t c : TUNE_SPLITS) sr_ok |= sr == static_cast<double>(c);
    IGP_REQUIRE(ns_ok && sr_ok && kind >= IGP_RBF && kind <= IGP_MATERN52 && dch >= 1 &&
                    nb >= 0 && nb < 64,
                "tuning text: entry out of range (strips %g, split_rows %g, kind %g)", ns, sr,
                kind);
    entries.push_back({TuneKey{static_cast<int>(kind), static_cast<int>(dch),
                               static_cast<int>(nb), bf},
                       TuneVal{static_cast<int>(ns), static_cast<int64_t>(sr), us}});
    pos = end + 1;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int added = 0;
  for (auto& e : entries) added += g_tune.insert(e).second ? 1 : 0;
  if (loaded) *loaded = added;
  return IGP_OK;
}

namespace {

template <typename T>
__global__ void k_check_labels(const int32_t* y, int64_t N, int C, int* bad) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    if (y[i] < 0 || y[i] >= C) atomicAdd(bad, 1);
}

// counts the entries of X that are NaN or infinite
template <typename T>
__global__ void k_count_nonfinite(const T* X, int64_t n, int* bad) {
  int cnt = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    cnt += isfinite(X[i]) ? 0 : 1;
  if (cnt) atomicAdd(bad, cnt);
}

int validate_common(const igp_kernel_params* kp, int n_kp, const igp_solver_config* cfg,
                    int64_t N, int64_t D, int64_t C) {
  IGP_REQUIRE(kp && cfg, "NULL kernel params or config");
  IGP_REQUIRE(n_kp == 1 || n_kp == C, "n_kp must be 1 or C, got %d", n_kp);
  for (int c = 0; c < n_kp; ++c) {
    IGP_REQUIRE(kp[c].kind >= IGP_RBF && kp[c].kind <= IGP_MATERN52, "unknown kernel kind %d",
                kp[c].kind);
    IGP_REQUIRE(kp[c].kind == kp[0].kind, "per-class kernels must share one kernel family");
    IGP_REQUIRE(std::isfinite(kp[c].lengthscale) && kp[c].lengthscale > 0 &&
                    std::isfinite(kp[c].outputscale) && kp[c].outputscale > 0,
                "kernel hyperparameters must be finite and positive");
  }
  IGP_REQUIRE(n_kp == 1 || !is_bf16(cfg->precision),
              "one kernel per class is not supported in the BF16 modes");
  IGP_REQUIRE(N >= 1 && D >= 1 && C >= 1, "N, D, C must be >= 1");
  IGP_REQUIRE(C <= 64, "C must be <= 64");
  IGP_REQUIRE(cfg->policy >= IGP_POLICY_CG && cfg->policy <= IGP_POLICY_USER, "unknown policy");
  IGP_REQUIRE(cfg->j_max >= 0, "j_max must be >= 0");
  IGP_REQUIRE(cfg->max_buffer >= 1 && cfg->max_buffer <= 4096, "max_buffer must be in [1, 4096]");
  IGP_REQUIRE(cfg->max_buffer >= cfg->j_max, "max_buffer must be >= j_max");
  IGP_REQUIRE(cfg->precision >= IGP_FP64 && cfg->precision <= IGP_BF16X3, "unknown precision");
  IGP_REQUIRE(cfg->residual_mode == IGP_RESIDUAL_EXPLICIT ||
                  cfg->residual_mode == IGP_RESIDUAL_RECURRENCE,
              "unknown residual mode %d", cfg->residual_mode);
  IGP_REQUIRE(std::isfinite(cfg->tol_abs) && std::isfinite(cfg->tol_rel) && cfg->tol_abs >= 0 &&
                  cfg->tol_rel >= 0,
              "tolerances must be finite and >= 0");
  IGP_REQUIRE(cfg->likelihood >= IGP_LIK_SOFTMAX && cfg->likelihood <= IGP_LIK_BLOCK,
              "unknown likelihood %d", cfg->likelihood);
  IGP_REQUIRE(cfg->likelihood != IGP_LIK_GAUSSIAN ||
                  (std::isfinite(cfg->noise_var) && cfg->noise_var > 0),
              "the Gaussian likelihood needs a finite noise_var > 0");
  return IGP_OK;
}

// prepared (centred, padded) rows feed the matrix-core products; one kernel per
// class runs on the direct-difference kernel instead
// centred rows prepared once per model for the matrix-core products (also
// with one kernel per class: K(X, X) v then takes the symmetric kernel's
// per-class form)
bool model_prepared(int precision, int kind, int64_t D, int n_kp) {
  (void)n_kp;
  return kv_uses_prepared(precision, kind, D);
}

template <typename T>
size_t state_bytes_t(int64_t N, int64_t D, int64_t C, const igp_solver_config& cfg, int kind,
                     int n_kp = 1) {
  Carver cv(nullptr, 0);
  carve<T>(cv, N, D, C, cfg, model_prepared(cfg.precision, kind, D, n_kp));
  return cv.used + 256;
}

template <typename T>
int init_t(igp_model** out, const igp_kernel_params* kp, int n_kp, const igp_solver_config* cfg,
           const void* X, const void* y, int64_t N, int64_t D, int64_t C, void* arena,
           size_t arena_bytes, hipStream_t stream) {
  // the arena must hold what itergp_state_bytes reports (the query does not
  // know the kernel and sizes for the larger layout), whatever this kernel needs
  const size_t need = std::max(::igp::state_bytes(N, D, C, cfg),
                               state_bytes_t<T>(N, D, C, *cfg, kp->kind, n_kp));
  if (arena_bytes < need) {
    set_error("arena too small: need %zu bytes, have %zu", need, arena_bytes);
    return IGP_ENOMEM;
  }
  IGP_REQUIRE(reinterpret_cast<uintptr_t>(arena) % 256 == 0, "arena must be 256-byte aligned");
  auto m = std::make_unique<Model<T>>();
  m->kp = *kp;
  m->n_kp = n_kp;
  m->kps.assign(kp, kp + n_kp);
  for (int64_t c = 0; c < C; ++c) m->prior_var.push_back(kp[n_kp > 1 ? c : 0].outputscale);
  m->cfg = *cfg;
  m->N = N;
  m->D = D;
  m->C = C;
  m->n = N * C;
  m->ld = col_stride(m->n);
  m->y = y;
  m->stream = stream;
  Carver cv(arena, arena_bytes);
  m->prepared = model_prepared(cfg->precision, kp->kind, D, n_kp);
  m->L = carve<T>(cv, N, D, C, *cfg, m->prepared);
  IGP_CHECK_HIP(hipMemcpyAsync(m->L.X, X, N * D * sizeof(T), hipMemcpyDeviceToDevice, stream));
  if (m->prepared) {
    const float* Xf = reinterpret_cast<const float*>(m->L.X);
    IGP_TRY(column_mean_f32(Xf, N, D, m->L.centre, m->L.meanpart, MEAN_BLOCKS * D, stream));
    IGP_TRY(prep_rows_any(cfg->precision, Xf, N, D, m->L.centre, m->L.Xp, m->L.nrm, stream));
  }
  IGP_CHECK_HIP(hipMemsetAsync(m->L.f, 0, m->n * sizeof(T), stream));
  IGP_CHECK_HIP(hipMemsetAsync(m->L.v, 0, m->n * sizeof(T), stream));
  IGP_CHECK_HIP(hipMemsetAsync(m->L.flags, 0, 64 * sizeof(int), stream));
  if (cfg->likelihood == IGP_LIK_SOFTMAX) {
    k_check_labels<T><<<256, 256, 0, stream>>>(static_cast<const int32_t*>(y), N,
                                               static_cast<int>(C), m->L.flags);
    IGP_CHECK_LAUNCH();
  } else if (cfg->likelihood != IGP_LIK_BLOCK) {
    IGP_TRY(diag_check_targets<T>(cfg->likelihood, y, m->n, m->L.flags, stream));
  }
  k_count_nonfinite<T><<<256, 256, 0, stream>>>(static_cast<const T*>(m->L.X), N * D,
                                                 m->L.flags + 1);
  IGP_CHECK_LAUNCH();
  int bad2[2] = {0, 0};
  IGP_CHECK_HIP(hipMemcpyAsync(bad2, m->L.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, stream));
  IGP_CHECK_HIP(hipStreamSynchronize(stream));
  const int bad = bad2[0];
  if (bad2[1]) {
    set_error("%d non-finite entries in X", bad2[1]);
    return IGP_EINVAL;
  }
  if (bad) {
    set_error(cfg->likelihood == IGP_LIK_SOFTMAX ? "%d labels outside [0, C)"
              : cfg->likelihood == IGP_LIK_POISSON ? "%d negative counts"
                                                   : "%d non-finite targets",
              bad);
    return IGP_EINVAL;
  }
  *out = m.release();
  return IGP_OK;
}

}  // namespace

size_t state_bytes(int64_t N, int64_t D, int64_t C, const igp_solver_config* cfg) {
  if (!cfg || N < 1 || D < 1 || C < 1 || cfg->max_buffer < 1) return 0;
  if (cfg->precision == IGP_FP64) return state_bytes_t<double>(N, D, C, *cfg, IGP_RBF);
  // the query does not know the kernel: size for the larger of the two layouts
  return std::max(state_bytes_t<float>(N, D, C, *cfg, IGP_RBF),
                  state_bytes_t<float>(N, D, C, *cfg, IGP_MATERN12));
}

int model_init(igp_model** out, const igp_kernel_params* kp, int n_kp,
               const igp_solver_config* cfg, const void* X, const void* y, int64_t N, int64_t D,
               int64_t C, void* arena, size_t arena_bytes, hipStream_t stream) {
  IGP_REQUIRE(out, "NULL output handle");
  *out = nullptr;
  IGP_TRY(validate_common(kp, n_kp, cfg, N, D, C));
  IGP_REQUIRE(X && arena, "NULL X or arena");
  IGP_REQUIRE(y || cfg->likelihood == IGP_LIK_BLOCK, "NULL y");
  if (cfg->precision == IGP_FP64)
    return init_t<double>(out, kp, n_kp, cfg, X, y, N, D, C, arena, arena_bytes, stream);
  return init_t<float>(out, kp, n_kp, cfg, X, y, N, D, C, arena, arena_bytes, stream);
}

}  // namespace igp
