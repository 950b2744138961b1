// extern "C" entry points declared in include/itergp.h.  Argument checking
// and dispatch only; the work runs in the HIP kernels behind ops.hpp.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <string>

#include "ops.hpp"

namespace igp {
size_t batched_ws_bytes(igp_model* const* models, int n);
int newton_step_batched(igp_model* const* models, int n, igp_step_info* infos, void* ws,
                        size_t ws_bytes, int flags);
std::string batched_tuning_json();
int batched_tuning_load(const char* json, int* loaded);
size_t state_bytes(int64_t N, int64_t D, int64_t C, const igp_solver_config* cfg);
int model_init(igp_model** out, const igp_kernel_params* kp, int n_kp,
               const igp_solver_config* cfg, const void* X, const void* y, int64_t N, int64_t D,
               int64_t C, void* arena, size_t arena_bytes, hipStream_t stream);

namespace {
thread_local std::string g_error;
}

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
}

void clear_error() { g_error.clear(); }

}  // namespace igp

using namespace igp;

namespace {
template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::exception& e) {
    set_error("internal error: %s", e.what());
    return IGP_EDEVICE;
  } catch (...) {
    set_error("internal error");
    return IGP_EDEVICE;
  }
}

int check_kp(const igp_kernel_params* kp) {
  IGP_REQUIRE(kp, "NULL kernel params");
  IGP_REQUIRE(kp->kind >= IGP_RBF && kp->kind <= IGP_MATERN52, "unknown kernel kind %d", kp->kind);
  IGP_REQUIRE(std::isfinite(kp->lengthscale) && kp->lengthscale > 0 &&
                  std::isfinite(kp->outputscale) && kp->outputscale > 0,
              "kernel hyperparameters must be finite and positive");
  return IGP_OK;
}
}  // namespace

extern "C" {

const char* igp_last_error(void) { return g_error.c_str(); }
const char* igp_version(void) { return "itergp-gfx950 0.1"; }

size_t glm_kernel_matmul_ws_bytes(int64_t n1, int64_t n2, int64_t d, int64_t C, int64_t nb,
                                  int32_t precision) {
  if (n1 < 0 || n2 < 0 || d < 1 || C < 1 || nb < 0) return 0;
  return kv_ws_bytes(n1, n2, d, C, nb, precision);
}

int glm_kernel_matmul(const igp_kernel_params* kp, int32_t n_kp, const void* X1, int64_t n1,
                      const void* X2, int64_t n2, int64_t d, const void* V, int64_t C,
                      int64_t nb, int64_t ldv, void* Out, int64_t ldo, double beta,
                      int32_t precision, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    clear_error();
    IGP_REQUIRE(n_kp == 1 || (n_kp == C && C <= 64), "n_kp must be 1 or C (<= 64), got %d",
                n_kp);
    for (int c = 0; c < n_kp; ++c) {
      IGP_TRY(check_kp(kp ? kp + c : nullptr));
      IGP_REQUIRE(kp[c].kind == kp[0].kind, "per-class kernels must share one kernel family");
    }
    IGP_REQUIRE(n1 >= 0 && n2 >= 0 && nb >= 0, "negative size");
    IGP_REQUIRE(d >= 1 && C >= 1, "d and C must be >= 1");
    IGP_REQUIRE(precision >= IGP_FP64 && precision <= IGP_BF16X3, "unknown precision %d", precision);
    IGP_REQUIRE(std::isfinite(beta), "beta must be finite");
    if (n1 == 0 || nb == 0) return IGP_OK;
    IGP_REQUIRE(X1 && Out, "NULL X1 or Out");
    IGP_REQUIRE(n2 == 0 || (X2 && V), "NULL X2 or V");
    IGP_REQUIRE(ldv >= n2 * C && ldo >= n1 * C, "ldv/ldo smaller than a vector");
    const size_t need = kv_ws_bytes(n1, n2, d, C, nb, precision);
    if (ws_bytes < need || (need > 0 && !ws)) {
      set_error("workspace too small: need %zu bytes, have %zu", need, ws_bytes);
      return IGP_ENOMEM;
    }
    KVProblem p{};
    p.kp = *kp;
    if (n_kp > 1) {
      p.kpc = kp;
      p.n_kp = n_kp;
    }
    p.precision = precision;
    p.X1 = X1;
    p.X2 = X2;
    p.n1 = n1;
    p.n2 = n2;
    p.d = d;
    p.V = V;
    p.C = C;
    p.nb = nb;
    p.ldv = ldv;
    p.Out = Out;
    p.ldo = ldo;
    p.beta = beta;
    return kv_launch(p, ws, ws_bytes, stream);
  });
}

int glm_softmax_hessian_apply(const void* F, int64_t N, int64_t C, const void* V, int64_t nb,
                              int64_t ldv, void* Out, int64_t ldo, int32_t mode,
                              int32_t precision, hipStream_t stream) {
  return guarded([&]() -> int {
    clear_error();
    IGP_REQUIRE(N >= 0 && nb >= 0 && C >= 1, "bad sizes");
    IGP_REQUIRE(mode == IGP_W || mode == IGP_W_PINV, "unknown mode %d", mode);
    IGP_REQUIRE(precision == IGP_FP64 || precision == IGP_FP32,
                "precision must be IGP_FP64 or IGP_FP32");
    if (N == 0 || nb == 0) return IGP_OK;
    IGP_REQUIRE(F && V && Out, "NULL pointer");
    IGP_REQUIRE(ldv >= N * C && ldo >= N * C, "ldv/ldo smaller than a vector");
    if (precision == IGP_FP64)
      return winv_apply<double>(static_cast<const double*>(F), true, mode, N, C,
                                static_cast<const double*>(V), nb, ldv, nullptr, 0,
                                static_cast<double*>(Out), ldo, stream);
    return winv_apply<float>(static_cast<const float*>(F), true, mode, N, C,
                             static_cast<const float*>(V), nb, ldv, nullptr, 0,
                             static_cast<float*>(Out), ldo, stream);
  });
}

size_t itergp_state_bytes(int64_t N, int64_t D, int64_t C, const igp_solver_config* cfg) {
  return state_bytes(N, D, C, cfg);
}

int itergp_init(igp_model** out, const igp_kernel_params* kp, int32_t n_kp,
                const igp_solver_config* cfg, const void* X, const void* y, int64_t N,
                int64_t D, int64_t C, void* arena, size_t arena_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    clear_error();
    return model_init(out, kp, n_kp, cfg, X, y, N, D, C, arena, arena_bytes, stream);
  });
}

int itergp_set_user_actions(igp_model* m, const void* actions, int64_t ncols, int64_t ld) {
  return guarded([&]() -> int {
    clear_error();
    IGP_REQUIRE(m, "NULL model");
    return m->set_user_actions(actions, ncols, ld);
  });
}

int itergp_newton_step(igp_model* m, igp_step_info* info) {
  return guarded([&]() -> int {
    IGP_REQUIRE(m, "NULL model");
    return m->newton_step(info);
  });
}

int itergp_newton_step_begin(igp_model* m) {
  return guarded([&]() -> int {
    IGP_REQUIRE(m, "NULL model");
    return m->step_begin();
  });
}

int itergp_newton_step_iterate(igp_model* m, int64_t max_iters, int32_t* done) {
  return guarded([&]() -> int {
    IGP_REQUIRE(m, "NULL model");
    return m->step_iterate(max_iters, done);
  });
}

int itergp_newton_step_end(igp_model* m, igp_step_info* info) {
  return guarded([&]() -> int {
    IGP_REQUIRE(m, "NULL model");
    return m->step_end(info);
  });
}

int itergp_compress(igp_model* m, int32_t rank_limit, int32_t* kept) {
  return guarded([&]() -> int {
    IGP_REQUIRE(m, "NULL model");
    return m->compress(rank_limit, kept);
  });
}

size_t itergp_predict_ws_bytes(const igp_model* m, int64_t Ns) {
  if (!m || Ns < 0) return 0;
  return m->predict_ws_bytes(Ns);
}

int itergp_predict(const igp_model* m, const void* Xs, int64_t Ns, void* mean, void* var,
                   void* probs, void* ws, size_t ws_bytes, hipStream_t stream) {
  return guarded([&]() -> int {
    clear_error();
    IGP_REQUIRE(m, "NULL model");
    IGP_REQUIRE(Ns >= 0, "negative Ns");
    return m->predict(Xs, Ns, mean, var, probs, ws, ws_bytes, stream);
  });
}

int itergp_get_view(const igp_model* m, int32_t which, const void** ptr, int64_t* rows,
                    int64_t* cols, int64_t* ld) {
  return guarded([&]() -> int {
    clear_error();
    IGP_REQUIRE(m, "NULL model");
    return m->view(which, ptr, rows, cols, ld);
  });
}

int igp_host_eigh(int32_t n, const double* A, double* w, double* Z) {
  return guarded([&]() -> int {
    clear_error();
    IGP_REQUIRE(n >= 0, "n must be >= 0");
    if (n == 0) return IGP_OK;
    IGP_REQUIRE(A && w && Z, "NULL pointer");
    return eigh_desc(n, A, w, Z);
  });
}

int itergp_set_block_likelihood(igp_model* m, const void* grad, const void* W) {
  return guarded([&]() -> int {
    clear_error();
    IGP_REQUIRE(m, "NULL model");
    return m->set_block_likelihood(grad, W);
  });
}

int itergp_set_profiling(igp_model* m, int32_t enable) {
  return guarded([&]() -> int {
    clear_error();
    IGP_REQUIRE(m, "NULL model");
    IGP_REQUIRE(enable >= 0, "profiling: enable must be 0 (off) or a sampling stride >= 1");
    return m->set_profiling(enable);
  });
}

int itergp_get_profile(const igp_model* m, igp_profile* out) {
  return guarded([&]() -> int {
    clear_error();
    IGP_REQUIRE(m && out, "NULL model or output");
    return m->get_profile(out);
  });
}

size_t itergp_batched_ws_bytes(igp_model* const* models, int32_t n) {
  try {
    return batched_ws_bytes(models, n);
  } catch (...) {
    return 0;
  }
}

int itergp_newton_step_batched(igp_model* const* models, int32_t n, igp_step_info* infos,
                               void* ws, size_t ws_bytes) {
  return guarded([&]() -> int {
    clear_error();
    return newton_step_batched(models, n, infos, ws, ws_bytes, 0);
  });
}

int itergp_newton_step_batched_ex(igp_model* const* models, int32_t n, igp_step_info* infos,
                                  void* ws, size_t ws_bytes, int32_t flags) {
  return guarded([&]() -> int {
    clear_error();
    return newton_step_batched(models, n, infos, ws, ws_bytes, flags);
  });
}

int itergp_batched_tuning(char* buf, size_t len) {
  return guarded([&]() -> int {
    clear_error();
    const std::string js = batched_tuning_json();
    IGP_REQUIRE(buf && len > js.size(), "buffer of %zu bytes too small (need %zu)", len,
                js.size() + 1);
    memcpy(buf, js.c_str(), js.size() + 1);
    return IGP_OK;
  });
}

int itergp_batched_tuning_load(const char* json, int32_t* loaded) {
  return guarded([&]() -> int {
    clear_error();
    int n = 0;
    IGP_TRY(batched_tuning_load(json, &n));
    if (loaded) *loaded = n;
    return IGP_OK;
  });
}

int itergp_destroy(igp_model* m) {
  delete m;
  return IGP_OK;
}

}  // extern "C"
