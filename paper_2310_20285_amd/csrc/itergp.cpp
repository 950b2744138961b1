// IterNCGP driver: Algorithm 1 (outer Newton loop), Algorithm 2 (IterGP) and
// Algorithm 3 (virtual solver run with compression), with every NC-sized
// operation running in the library's HIP kernels and only B x B algebra and
// scalar control on the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "ops.hpp"

namespace igp {

namespace {

constexpr int PARTIAL_DOUBLES = 1 << 16;

template <typename T>
struct Layout {
  T *X, *f, *fnew, *pi, *rhs, *v, *r, *z, *d, *kv, *wv;
  T *S, *Tb, *Q, *S2, *T2;
  T *KQ, *kd;   // recurrence mode: K Q and K d
  double *part, *scal, *yb, *M, *U, *lamscale, *gram_part;
  size_t gram_cap;
  void* kvws;
  size_t kvws_bytes;
  int* flags;
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
  int64_t npart = PARTIAL_DOUBLES;
  const int64_t gemv_need = (ceil_div(n, 2048) + 1) * std::max<int64_t>(B, 1);
  npart = std::max(npart, gemv_need);
  npart = std::max(npart, 4 * ceil_div(N, 256) + 64);
  L.part = cv.take<double>(npart);
  L.scal = cv.take<double>(SC_COUNT);
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
  if (prepared) {
    L.centre = cv.take<float>(D);
    L.Xp = cfg.precision == IGP_BF16 ? static_cast<void*>(cv.take<uint16_t>(N * bf16_padded_dim(D)))
                                     : static_cast<void*>(cv.take<float>(N * padded_dim(D)));
    L.nrm = cv.take<float>(N);
    L.meanpart = cv.take<double>(MEAN_BLOCKS * D);
  }
  return L;
}

template <typename T>
struct Model final : igp_model {
  igp_kernel_params kp{};
  igp_solver_config cfg{};
  int64_t N = 0, D = 0, C = 0, n = 0, ld = 0;
  const int32_t* y = nullptr;
  hipStream_t stream = nullptr;
  Layout<T> L{};
  int ncols = 0;                 // columns of S, T and Q
  const T* user = nullptr;
  int64_t user_cols = 0, user_ld = 0;
  int steps_done = 0;
  std::vector<double> hM, hMs, hU, hlam;
  // tracing
  bool prof = false;
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  igp_profile pstat{};
  double pending_evals = 0.0, pending_flops = 0.0;

  ~Model() override {
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
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
    return IGP_OK;
  }

  // after a stream synchronisation: fold the recorded pairs into the counters
  int collect_profile() {
    if (!prof) return IGP_OK;
    // pair 0 brackets the whole step; the rest bracket products with K
    for (size_t i = 0; i + 1 < evused; i += 2) {
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
    pending_evals = pending_flops = 0.0;
    evused = 0;
    return IGP_OK;
  }

  int set_profiling(int enable) override {
    prof = enable != 0;
    pstat = igp_profile{};
    evused = 0;
    pending_evals = pending_flops = 0.0;
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

  int apply_K(const T* V, T* Out) {
    hipEvent_t a = nullptr, b = nullptr;
    if (prof) {
      IGP_TRY(event_pair(&a, &b));
      IGP_CHECK_HIP(hipEventRecord(a, stream));
    }
    IGP_TRY(kv_launch(kv_problem(L.X, N, V, 1, n, Out, n), L.kvws, L.kvws_bytes, stream));
    if (prof) {
      IGP_CHECK_HIP(hipEventRecord(b, stream));
      pending_evals += static_cast<double>(N) * N;
      pending_flops += 2.0 * N * N * (D + C);
    }
    return IGP_OK;
  }

  int read_scalars(double* out) {
    IGP_CHECK_HIP(hipMemcpyAsync(out, L.scal, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                                 stream));
    IGP_CHECK_HIP(hipStreamSynchronize(stream));
    return IGP_OK;
  }

  // Algorithm 3: M = S^T (T + W^+ S); M = U Lambda U^T (descending);
  // keep eigenvalues above the floor and at most R of them; S <- S U,
  // T <- T U, Q_0 = S U Lambda^{-1/2}.
  int virtual_solver_run(igp_step_info* info) {
    const int B = ncols;
    if (B == 0) return IGP_OK;
    IGP_TRY(winv_apply<T>(L.pi, false, IGP_W_PINV, N, C, L.S, B, ld, L.Tb, ld, L.S2, ld, stream));
    IGP_TRY(gram<T>(L.S, L.S2, ld, n, B, L.gram_part, L.gram_cap, L.M, stream));
    hM.resize(static_cast<size_t>(B) * B);
    IGP_CHECK_HIP(hipMemcpyAsync(hM.data(), L.M, hM.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, stream));
    IGP_CHECK_HIP(hipStreamSynchronize(stream));
    hMs.resize(hM.size());
    for (int i = 0; i < B; ++i)
      for (int j = 0; j < B; ++j)
        hMs[static_cast<size_t>(i) * B + j] =
            0.5 * (hM[static_cast<size_t>(i) * B + j] + hM[static_cast<size_t>(j) * B + i]);
    hlam.resize(B);
    hU.resize(static_cast<size_t>(B) * B);
    IGP_TRY(eigh_desc(B, hMs.data(), hlam.data(), hU.data()));
    int keep = 0;
    const double floor = hlam[0] > 0.0 ? hlam[0] * B * 2.220446049250313e-16 : INFINITY;
    while (keep < B && hlam[keep] > floor) ++keep;
    const int dropped_floor = B - keep;
    if (cfg.rank_limit >= 0 && keep > cfg.rank_limit) keep = cfg.rank_limit;
    std::vector<double> scale(std::max(keep, 1));
    for (int k = 0; k < keep; ++k) scale[k] = 1.0 / std::sqrt(hlam[k]);
    if (keep > 0) {
      IGP_CHECK_HIP(hipMemcpyAsync(L.U, hU.data(), static_cast<size_t>(B) * keep * sizeof(double),
                                   hipMemcpyHostToDevice, stream));
      IGP_CHECK_HIP(hipMemcpyAsync(L.lamscale, scale.data(), keep * sizeof(double),
                                   hipMemcpyHostToDevice, stream));
      IGP_TRY(right_mul<T>(L.S, ld, n, B, L.U, keep, nullptr, L.S2, ld, stream));
      IGP_TRY(right_mul<T>(L.Tb, ld, n, B, L.U, keep, nullptr, L.T2, ld, stream));
      IGP_TRY(right_mul<T>(L.S, ld, n, B, L.U, keep, L.lamscale, L.Q, ld, stream));
      if (recurrence())   // K Q_0 = K S U Lambda^{-1/2} = T U Lambda^{-1/2}
        IGP_TRY(right_mul<T>(L.Tb, ld, n, B, L.U, keep, L.lamscale, L.KQ, ld, stream));
      std::swap(L.S, L.S2);
      std::swap(L.Tb, L.T2);
    }
    // host buffers must outlive the async copies
    IGP_CHECK_HIP(hipStreamSynchronize(stream));
    ncols = keep;
    if (info) {
      info->recycled_cols = keep;
      info->eig_dropped = dropped_floor;
    }
    return IGP_OK;
  }

  int newton_step(igp_step_info* info_out) override {
    clear_error();
    igp_step_info info{};
    info.eta_min = INFINITY;
    double sc[SC_COUNT];
    int nblk = 0;
    hipEvent_t step_a = nullptr, step_b = nullptr;
    evused = 0;
    if (prof) {
      IGP_TRY(event_pair(&step_a, &step_b));
      IGP_CHECK_HIP(hipEventRecord(step_a, stream));
    }
    // pseudo-targets yhat - m = g + W^+ (onehot(y) - pi), m = 0
    IGP_TRY(softmax_pi_rhs<T>(L.f, y, N, C, L.pi, L.rhs, L.part, &nblk, stream));
    IGP_TRY(dot_into<T>(L.rhs, L.rhs, n, L.part, L.scal + SC_RHS2, stream));
    const bool recycle = cfg.recycle && cfg.policy != IGP_POLICY_UNIT;
    if (!recycle) ncols = 0;
    IGP_TRY(virtual_solver_run(&info));
    // v_0 = C_0 (yhat - m) = Q (Q^T (yhat - m))
    if (ncols > 0) {
      IGP_TRY(gemv_t<T>(L.Q, ld, n, ncols, L.rhs, L.part, L.yb, stream));
      IGP_TRY(gemv_n<T>(L.Q, ld, n, ncols, L.yb, L.v, stream));
      if (recurrence()) IGP_TRY(gemv_n<T>(L.KQ, ld, n, ncols, L.yb, L.kv, stream));
    } else {
      IGP_CHECK_HIP(hipMemsetAsync(L.v, 0, n * sizeof(T), stream));
      if (recurrence()) IGP_CHECK_HIP(hipMemsetAsync(L.kv, 0, n * sizeof(T), stream));
    }
    IGP_TRY(read_scalars(sc));
    info.rhs_norm = std::sqrt(sc[SC_RHS2]);
    const double thresh = std::max(cfg.tol_abs, cfg.tol_rel * info.rhs_norm);
    int kprod = 0;
    int j = 0;
    // r = (yhat - m) - K v - W^+ v with K v formed (explicit) or carried (recurrence)
    auto enqueue_residual = [&]() -> int {
      if (!recurrence()) {
        IGP_TRY(apply_K(L.v, L.kv));
        ++kprod;
      }
      IGP_TRY(winv_apply<T>(L.pi, false, IGP_W_PINV, N, C, L.v, 1, n, nullptr, 0, L.wv, n,
                            stream));
      return residual<T>(L.rhs, L.kv, L.wv, L.r, n, L.part, L.scal + SC_RR, stream);
    };
    bool have_r = false;
    if (cfg.j_max > 0) {
      IGP_TRY(enqueue_residual());   // r_0
      IGP_TRY(read_scalars(sc));
      info.res_norm = std::sqrt(sc[SC_RR]);
      have_r = true;
      if (!(info.res_norm >= thresh)) info.converged = 1;
    }
    // One host synchronisation per iteration: the update of Q and v is guarded
    // on the device by eta_j > 0, and the next residual is enqueued before the
    // host reads eta_j and ||r_j|| together.
    while (have_r && !info.converged && j < cfg.j_max) {
      if (ncols >= cfg.max_buffer) {
        set_error("buffer full: %d columns (max_buffer too small)", ncols);
        return IGP_ENOMEM;
      }
      if (cfg.policy == IGP_POLICY_USER && (!user || j >= user_cols)) break;  // actions used up
      ++j;
      T* s_col = L.S + static_cast<int64_t>(ncols) * ld;
      T* t_col = L.Tb + static_cast<int64_t>(ncols) * ld;
      if (cfg.policy == IGP_POLICY_CG) {
        IGP_TRY(action_cg<T>(L.r, L.scal + SC_RR, s_col, n, stream));
      } else if (cfg.policy == IGP_POLICY_UNIT) {
        IGP_TRY(fill_unit<T>(s_col, n, j - 1, stream));
      } else {
        IGP_TRY(copy_vec<T>(user + static_cast<int64_t>(j - 1) * user_ld, s_col, n, stream));
      }
      IGP_TRY(dot_into<T>(s_col, L.r, n, L.part, L.scal + SC_ALPHA, stream));   // alpha_j
      IGP_TRY(apply_K(s_col, t_col));                                            // t_j = K s_j
      ++kprod;
      IGP_TRY(winv_apply<T>(L.pi, false, IGP_W_PINV, N, C, s_col, 1, n, t_col, n, L.z, n,
                            stream));                                            // z_j
      IGP_TRY(gemv_t<T>(L.Q, ld, n, ncols, L.z, L.part, L.yb, stream));          // Q^T z
      IGP_TRY(dir_update<T>(s_col, L.Q, ld, n, ncols, L.yb, L.z, L.d, L.part,
                            L.scal + SC_ETA, stream, t_col, recurrence() ? L.KQ : nullptr,
                            L.kd));                                              // d_j, eta_j
      IGP_TRY(append_and_step<T>(L.d, L.scal, L.Q + static_cast<int64_t>(ncols) * ld, L.v, n,
                                 stream, recurrence() ? L.kd : nullptr,
                                 recurrence() ? L.KQ + static_cast<int64_t>(ncols) * ld : nullptr,
                                 L.kv));                                         // eta > 0 only
      const bool next_r = j < cfg.j_max;
      if (next_r) IGP_TRY(enqueue_residual());                                   // r_j
      IGP_TRY(read_scalars(sc));
      const double eta = sc[SC_ETA];
      if (!(eta > 0.0)) {
        info.breakdown = 1;   // s_j and t_j are dropped: ncols is not advanced
        --j;
        break;
      }
      info.eta_min = std::min(info.eta_min, eta);
      ++ncols;
      if (next_r) {
        info.res_norm = std::sqrt(sc[SC_RR]);
        if (!(info.res_norm >= thresh)) info.converged = 1;
      }
    }
    info.iters = j;
    // f_{i+1} = K v + m
    IGP_TRY(apply_K(L.v, L.fnew));
    ++kprod;
    IGP_TRY(newton_stats<T>(L.fnew, L.f, L.v, y, N, C, L.part, L.scal, stream));
    if (prof) IGP_CHECK_HIP(hipEventRecord(step_b, stream));
    IGP_TRY(read_scalars(sc));
    IGP_TRY(collect_profile());
    std::swap(L.f, L.fnew);
    info.buffer_cols = ncols;
    info.k_products = kprod;
    info.rel_change = sc[SC_FNEW2] > 0.0 ? std::sqrt(sc[SC_DIFF2] / sc[SC_FNEW2]) : INFINITY;
    info.psi = sc[SC_LOGLIK] - 0.5 * sc[SC_GV];
    if (!std::isfinite(info.eta_min)) info.eta_min = 0.0;
    ++steps_done;
    if (info_out) *info_out = info;
    return IGP_OK;
  }

  size_t kvws_for(int64_t n1, int64_t nb) const {
    return prepared ? kv_ws_bytes_prepared(n1, N, D, C, nb, cfg.precision)
                    : kv_ws_bytes(n1, N, D, C, nb, cfg.precision);
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
    IGP_TRY(kv_launch(kv_problem(Xs, Ns, L.v, 1, n, mean, Ns * C, xsp, nsp), ws1, w1, s));
    if (var_) {
      if (ncols > 0) {
        IGP_TRY(kv_launch(kv_problem(Xs, Ns, L.Q, ncols, ld, A, Ns * C, xsp, nsp), ws2, w2, s));
      }
      IGP_TRY(predict_epilogue<T>(A, Ns * C, Ns * C, ncols, kp.outputscale, mean, Ns, C,
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

  int set_user_actions(const void* a, int64_t nc, int64_t l) override {
    IGP_REQUIRE(nc >= 0 && (nc == 0 || (a && l >= n)), "user actions: bad pointer or stride");
    user = static_cast<const T*>(a);
    user_cols = nc;
    user_ld = l;
    return IGP_OK;
  }
};

template <typename T>
__global__ void k_check_labels(const int32_t* y, int64_t N, int C, int* bad) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < N;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    if (y[i] < 0 || y[i] >= C) atomicAdd(bad, 1);
}

int validate_common(const igp_kernel_params* kp, const igp_solver_config* cfg, int64_t N,
                    int64_t D, int64_t C) {
  IGP_REQUIRE(kp && cfg, "NULL kernel params or config");
  IGP_REQUIRE(kp->kind >= IGP_RBF && kp->kind <= IGP_MATERN52, "unknown kernel kind %d", kp->kind);
  IGP_REQUIRE(std::isfinite(kp->lengthscale) && kp->lengthscale > 0 &&
                  std::isfinite(kp->outputscale) && kp->outputscale > 0,
              "kernel hyperparameters must be finite and positive");
  IGP_REQUIRE(N >= 1 && D >= 1 && C >= 1, "N, D, C must be >= 1");
  IGP_REQUIRE(C <= 64, "C must be <= 64");
  IGP_REQUIRE(cfg->policy >= IGP_POLICY_CG && cfg->policy <= IGP_POLICY_USER, "unknown policy");
  IGP_REQUIRE(cfg->j_max >= 0, "j_max must be >= 0");
  IGP_REQUIRE(cfg->max_buffer >= 1 && cfg->max_buffer <= 4096, "max_buffer must be in [1, 4096]");
  IGP_REQUIRE(cfg->max_buffer >= cfg->j_max, "max_buffer must be >= j_max");
  IGP_REQUIRE(cfg->precision >= IGP_FP64 && cfg->precision <= IGP_BF16, "unknown precision");
  IGP_REQUIRE(cfg->residual_mode == IGP_RESIDUAL_EXPLICIT ||
                  cfg->residual_mode == IGP_RESIDUAL_RECURRENCE,
              "unknown residual mode %d", cfg->residual_mode);
  IGP_REQUIRE(std::isfinite(cfg->tol_abs) && std::isfinite(cfg->tol_rel) && cfg->tol_abs >= 0 &&
                  cfg->tol_rel >= 0,
              "tolerances must be finite and >= 0");
  return IGP_OK;
}

template <typename T>
size_t state_bytes_t(int64_t N, int64_t D, int64_t C, const igp_solver_config& cfg, int kind) {
  Carver cv(nullptr, 0);
  carve<T>(cv, N, D, C, cfg, kv_uses_prepared(cfg.precision, kind, D));
  return cv.used + 256;
}

template <typename T>
int init_t(igp_model** out, const igp_kernel_params* kp, const igp_solver_config* cfg,
           const void* X, const int32_t* y, int64_t N, int64_t D, int64_t C, void* arena,
           size_t arena_bytes, hipStream_t stream) {
  const size_t need = state_bytes_t<T>(N, D, C, *cfg, kp->kind);
  if (arena_bytes < need) {
    set_error("arena too small: need %zu bytes, have %zu", need, arena_bytes);
    return IGP_ENOMEM;
  }
  IGP_REQUIRE(reinterpret_cast<uintptr_t>(arena) % 256 == 0, "arena must be 256-byte aligned");
  auto m = std::make_unique<Model<T>>();
  m->kp = *kp;
  m->cfg = *cfg;
  m->N = N;
  m->D = D;
  m->C = C;
  m->n = N * C;
  m->ld = col_stride(m->n);
  m->y = y;
  m->stream = stream;
  Carver cv(arena, arena_bytes);
  m->prepared = kv_uses_prepared(cfg->precision, kp->kind, D);
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
  k_check_labels<T><<<256, 256, 0, stream>>>(y, N, static_cast<int>(C), m->L.flags);
  IGP_CHECK_LAUNCH();
  int bad = 0;
  IGP_CHECK_HIP(hipMemcpyAsync(&bad, m->L.flags, sizeof(int), hipMemcpyDeviceToHost, stream));
  IGP_CHECK_HIP(hipStreamSynchronize(stream));
  if (bad) {
    set_error("%d labels outside [0, C)", bad);
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

int model_init(igp_model** out, const igp_kernel_params* kp, const igp_solver_config* cfg,
               const void* X, const int32_t* y, int64_t N, int64_t D, int64_t C, void* arena,
               size_t arena_bytes, hipStream_t stream) {
  IGP_REQUIRE(out, "NULL output handle");
  *out = nullptr;
  IGP_TRY(validate_common(kp, cfg, N, D, C));
  IGP_REQUIRE(X && y && arena, "NULL X, y or arena");
  if (cfg->precision == IGP_FP64)
    return init_t<double>(out, kp, cfg, X, y, N, D, C, arena, arena_bytes, stream);
  return init_t<float>(out, kp, cfg, X, y, N, D, C, arena, arena_bytes, stream);
}

}  // namespace igp
