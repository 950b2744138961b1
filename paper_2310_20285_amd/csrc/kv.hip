// Matrix-free product with the prior covariance, K_X(X1, X2) V, with the
// kernel evaluated on the fly and never stored (the paper's lazily evaluated
// products with K, appendix on matrix-vector products).
//
// kv_valu: tiled VALU kernel, FP64 or FP32.  A workgroup owns 64 output rows
// and a contiguous range of X2 columns (split-N2 for occupancy); each of its
// four waves evaluates k on 64 rows x 16 columns of every 64-column X2 tile
// from explicit coordinate differences, then accumulates against the V tile
// staged in LDS.  Partial sums per split are reduced in a fixed order by
// kv_reduce, so results do not depend on scheduling.
#include <algorithm>
#include <type_traits>

#include "ops.hpp"

namespace igp {
namespace {

constexpr int TM = 64;    // rows of X1 per workgroup
constexpr int TN = 64;    // columns of X2 per tile
constexpr int DC = 32;    // feature chunk staged in LDS

// class-specific 1/l^2 and outputscale, passed by value (C <= 64)
template <typename T>
struct ClassParams {
  T il2[64];
  T os[64];
};

template <typename T, int KIND, int WC, bool PC = false>
__global__ void __launch_bounds__(256)
kv_valu(const T* __restrict__ X1, const T* __restrict__ X2, int64_t n1, int64_t n2, int d,
        const T* __restrict__ V, int C, int W, int64_t ldv, T* __restrict__ P,
        int64_t cols_per_split, T inv_l2, const int* skip, ClassParams<T> cp) {
  if (gate_closed(skip)) return;
  constexpr int TILE_BYTES = 2 * TM * (DC + 1) * sizeof(T);
  constexpr int RED_BYTES = 4 * TM * WC * sizeof(T);
  constexpr int U_BYTES = TILE_BYTES > RED_BYTES ? TILE_BYTES : RED_BYTES;
  __shared__ __align__(16) unsigned char smem[U_BYTES];
  __shared__ T sV[TN][WC];
  T(*sX1)[DC + 1] = reinterpret_cast<T(*)[DC + 1]>(smem);
  T(*sX2)[DC + 1] = reinterpret_cast<T(*)[DC + 1]>(smem + TM * (DC + 1) * sizeof(T));

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * TM;
  const int w0 = blockIdx.z * WC;
  const int64_t m_begin = static_cast<int64_t>(blockIdx.y) * cols_per_split;
  const int64_t m_end = m_begin + cols_per_split < n2 ? m_begin + cols_per_split : n2;

  T acc[WC];
#pragma unroll
  for (int w = 0; w < WC; ++w) acc[w] = T(0);
  // one kernel per class: column w belongs to class (w0 + w) % C
  T il2w[PC ? WC : 1], osw[PC ? WC : 1];
  if constexpr (PC) {
#pragma unroll
    for (int w = 0; w < WC; ++w) {
      const int c = (w0 + w) % C;
      il2w[w] = cp.il2[c];
      osw[w] = cp.os[c];
    }
  }

  for (int64_t m0 = m_begin; m0 < m_end; m0 += TN) {
    T r2[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) r2[c] = T(0);
    for (int k0 = 0; k0 < d; k0 += DC) {
      for (int e = tid; e < TM * DC; e += 256) {
        const int i = e / DC, k = e % DC, gk = k0 + k;
        const int64_t gi = r0 + i, gm = m0 + i;
        sX1[i][k] = (gi < n1 && gk < d) ? X1[gi * d + gk] : T(0);
        sX2[i][k] = (gm < m_end && gk < d) ? X2[gm * d + gk] : T(0);
      }
      __syncthreads();
      const int kmax = d - k0 < DC ? d - k0 : DC;
      for (int k = 0; k < kmax; ++k) {
        const T a = sX1[lane][k];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const T df = a - sX2[wv * 16 + c][k];
          r2[c] += df * df;
        }
      }
      __syncthreads();
    }
    for (int e = tid; e < TN * WC; e += 256) {
      const int m = e / WC, w = e % WC, gw = w0 + w;
      const int64_t gm = m0 + m;
      T val = T(0);
      if (gm < m_end && gw < W) val = V[(gw / C) * ldv + gm * C + (gw % C)];
      sV[m][w] = val;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      if constexpr (PC) {
#pragma unroll
        for (int w = 0; w < WC; ++w)
          acc[w] += osw[w] * kfun<KIND>(r2[c] * il2w[w]) * sV[wv * 16 + c][w];
      } else {
        const T kv = kfun<KIND>(r2[c] * inv_l2);
#pragma unroll
        for (int w = 0; w < WC; ++w) acc[w] += kv * sV[wv * 16 + c][w];
      }
    }
    __syncthreads();
  }

  T(*sRed)[TM][WC] = reinterpret_cast<T(*)[TM][WC]>(smem);
#pragma unroll
  for (int w = 0; w < WC; ++w) sRed[wv][lane][w] = acc[w];
  __syncthreads();
  for (int e = tid; e < TM * WC; e += 256) {
    const int i = e / WC, w = e % WC;
    const int64_t gi = r0 + i;
    if (gi < n1 && w0 + w < W) {
      const T s = sRed[0][i][w] + sRed[1][i][w] + sRed[2][i][w] + sRed[3][i][w];
      P[(static_cast<int64_t>(blockIdx.y) * n1 + gi) * W + w0 + w] = s;
    }
  }
}

// With epi_z (one vector, W == C, beta == 0): z = Out + W^+ s at point n,
// W^+ s in the order of iter::apply_block (class means summed in class order).
template <typename T>
__global__ void kv_reduce(const T* __restrict__ P, int nsplit, int64_t n1, int W, int C,
                          T* __restrict__ Out, int64_t ldo, T os, T beta, const int* skip,
                          const T* __restrict__ epi_pi, const T* __restrict__ epi_s,
                          T* __restrict__ epi_z) {
  if (gate_closed(skip)) return;
  const int64_t total = n1 * W;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t n = idx / W;
    const int w = static_cast<int>(idx % W);
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    const int64_t stride = n1 * W;
    const T* p = P + n * W + w;
    int sp = 0;
    // unrolled for loads in flight; each accumulator keeps its order (slots
    // 4k + j go to s_j in increasing k), so the sum does not change
#pragma unroll 4
    for (; sp + 4 <= nsplit; sp += 4) {
      s0 += p[sp * stride];
      s1 += p[(sp + 1) * stride];
      s2 += p[(sp + 2) * stride];
      s3 += p[(sp + 3) * stride];
    }
    for (; sp < nsplit; ++sp) s0 += p[sp * stride];
    const T s = (s0 + s1) + (s2 + s3);
    T* o = Out + (w / C) * ldo + n * C + (w % C);
    const T val = (beta != T(0)) ? os * s + beta * *o : os * s;
    *o = val;
    if (epi_z) {
      const T* sn = epi_s + n * C;
      const T* pn = epi_pi + n * C;
      T m = T(0);
      for (int c = 0; c < C; ++c) m += sn[c];
      m /= T(C);
      T m2 = T(0), uw = T(0);
      for (int c = 0; c < C; ++c) {
        const T u = (sn[c] - m) / pn[c];
        m2 += u;
        if (c == w) uw = u;
      }
      m2 /= T(C);
      epi_z[n * C + w] = (uw - m2) + val;
    }
  }
}

// whether the product's reduction can take the z = Out + W^+ s epilogue
bool epilogue_ok(const KVProblem& p) {
  return p.epi_z && p.epi_s && p.epi_pi && p.nb == 1 && p.beta == 0.0;
}

struct SplitPlan {
  int wc, gx, gz, nsplit;
  int64_t cols_per_split;
};

SplitPlan plan_valu(int64_t n1, int64_t n2, int64_t W, bool fixed = false) {
  SplitPlan p{};
  p.wc = W <= 4 ? 4 : (W <= 8 ? 8 : 16);
  p.gx = static_cast<int>(ceil_div(n1, TM));
  p.gz = static_cast<int>(ceil_div(W, p.wc));
  const int64_t tiles = ceil_div(n2, TN);
  int64_t want = ceil_div(2048, static_cast<int64_t>(p.gx) * p.gz);
  if (want < 1) want = 1;
  if (want > tiles) want = tiles;
  if (tiles == 0) {
    p.nsplit = 0;
    p.cols_per_split = TN;
    return p;
  }
  p.cols_per_split = fixed ? FIXED_SPLIT_ROWS : ceil_div(tiles, want) * TN;
  p.nsplit = static_cast<int>(ceil_div(n2, p.cols_per_split));
  return p;
}

template <typename T, int KIND>
void launch_valu_kind(const KVProblem& p, const SplitPlan& sp, T* P, hipStream_t s) {
  dim3 grid(sp.gx, sp.nsplit, sp.gz);
  const T inv_l2 = static_cast<T>(1.0 / (p.kp.lengthscale * p.kp.lengthscale));
  const int W = static_cast<int>(p.C * p.nb);
  const T* X1 = static_cast<const T*>(p.X1);
  const T* X2 = static_cast<const T*>(p.X2);
  const T* V = static_cast<const T*>(p.V);
  const int d = static_cast<int>(p.d), C = static_cast<int>(p.C);
  ClassParams<T> cp{};
  const bool pc = p.n_kp > 1;
  if (pc)
    for (int c = 0; c < C; ++c) {
      cp.il2[c] = static_cast<T>(1.0 / (p.kpc[c].lengthscale * p.kpc[c].lengthscale));
      cp.os[c] = static_cast<T>(p.kpc[c].outputscale);
    }
  auto go = [&](auto wc, auto pcv) {
    kv_valu<T, KIND, decltype(wc)::value, decltype(pcv)::value><<<grid, 256, 0, s>>>(
        X1, X2, p.n1, p.n2, d, V, C, W, p.ldv, P, sp.cols_per_split, inv_l2, p.skip, cp);
  };
  using F = std::false_type;
  using Tr = std::true_type;
  if (sp.wc == 4) {
    if (pc) go(std::integral_constant<int, 4>{}, Tr{}); else go(std::integral_constant<int, 4>{}, F{});
  } else if (sp.wc == 8) {
    if (pc) go(std::integral_constant<int, 8>{}, Tr{}); else go(std::integral_constant<int, 8>{}, F{});
  } else {
    if (pc) go(std::integral_constant<int, 16>{}, Tr{}); else go(std::integral_constant<int, 16>{}, F{});
  }
}

template <typename T>
int launch_valu(const KVProblem& p, void* ws, size_t ws_bytes, hipStream_t s) {
  const int64_t W = p.C * p.nb;
  SplitPlan sp = plan_valu(p.n1, p.n2, W, p.fixed_split);
  const size_t need = static_cast<size_t>(sp.nsplit) * p.n1 * W * sizeof(T);
  if (need > ws_bytes) {
    set_error("kernel-product workspace too small: need %zu bytes, have %zu", need, ws_bytes);
    return IGP_ENOMEM;
  }
  T* P = static_cast<T*>(ws);
  if (sp.nsplit > 0) {
    switch (p.kp.kind) {
      case IGP_RBF: launch_valu_kind<T, IGP_RBF>(p, sp, P, s); break;
      case IGP_MATERN12: launch_valu_kind<T, IGP_MATERN12>(p, sp, P, s); break;
      case IGP_MATERN32: launch_valu_kind<T, IGP_MATERN32>(p, sp, P, s); break;
      default: launch_valu_kind<T, IGP_MATERN52>(p, sp, P, s); break;
    }
    IGP_CHECK_LAUNCH();
  }
  const int64_t total = p.n1 * W;
  int blocks = static_cast<int>(ceil_div(total, 256));
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  // with one kernel per class the outputscales are applied inside the product
  const T os = p.n_kp > 1 ? T(1) : static_cast<T>(p.kp.outputscale);
  const bool epi = epilogue_ok(p);
  kv_reduce<T><<<blocks, 256, 0, s>>>(P, sp.nsplit, p.n1, static_cast<int>(W),
                                      static_cast<int>(p.C), static_cast<T*>(p.Out), p.ldo, os,
                                      static_cast<T>(p.beta), p.skip,
                                      epi ? static_cast<const T*>(p.epi_pi) : nullptr,
                                      epi ? static_cast<const T*>(p.epi_s) : nullptr,
                                      epi ? static_cast<T*>(p.epi_z) : nullptr);
  if (epi && p.epi_applied) *p.epi_applied = 1;
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

}  // namespace

bool kv_uses_prepared(int precision, int kind, int64_t d) {
  return is_bf16(precision) || (precision == IGP_FP32 && mfma_f32_supported(kind, d));
}

size_t prepared_rows_bytes(int precision, int64_t n, int64_t d) {
  Carver cv(nullptr, 0);
  if (is_bf16(precision)) cv.take<uint16_t>(bf16_rows_elems(precision, n, d));
  else cv.take<float>(n * padded_dim(d));
  cv.take<float>(n);
  return cv.used;
}

int prep_rows_any(int precision, const float* X, int64_t n, int64_t d, const float* centre,
                  void* rows, float* norms, hipStream_t s) {
  if (is_bf16(precision)) return prep_rows_bf16(precision, X, n, d, centre, rows, norms, s);
  return prep_rows_f32(X, n, d, centre, static_cast<float*>(rows), norms, s);
}

namespace {
constexpr int64_t MEAN_PART_BLOCKS = 1024;

size_t prep_bytes(int precision, int64_t n1, int64_t n2, int64_t d) {
  Carver cv(nullptr, 0);
  cv.take<float>(d);
  cv.take<double>(MEAN_PART_BLOCKS * d);
  cv.take<char>(prepared_rows_bytes(precision, n1, d));
  cv.take<char>(prepared_rows_bytes(precision, n2, d));
  return cv.used;
}
}  // namespace

size_t kv_ws_bytes_prepared(int64_t n1, int64_t n2, int64_t d, int64_t C, int64_t nb,
                            int precision, bool fixed) {
  const int64_t W = C * nb;
  SplitPlan sp = plan_valu(n1, n2, W, fixed);
  const size_t elt = precision == IGP_FP64 ? sizeof(double) : sizeof(float);
  size_t b = static_cast<size_t>(sp.nsplit) * n1 * W * elt;
  if (precision == IGP_FP32 && d <= 128)
    b = std::max(b, mfma_f32_partial_bytes(n1, n2, d, W, fixed));
  if (is_bf16(precision)) b = bf16_partial_bytes(n1, n2, W, fixed);
  return align_up(b + 256);
}

size_t kv_ws_bytes(int64_t n1, int64_t n2, int64_t d, int64_t C, int64_t nb, int precision,
                   bool fixed) {
  size_t b = kv_ws_bytes_prepared(n1, n2, d, C, nb, precision, fixed);
  if (is_bf16(precision) || (precision == IGP_FP32 && d <= 128))
    b += align_up(prep_bytes(precision, n1, n2, d) + 256);
  return b;
}

namespace {
int launch_mfma_path(const KVProblem& p, void* ws, size_t ws_bytes, hipStream_t s) {
  const int64_t W = p.C * p.nb;
  const bool bf = is_bf16(p.precision);
  Carver cv(ws, ws_bytes);
  const size_t pbytes = bf ? bf16_partial_bytes(p.n1, p.n2, W, p.fixed_split)
                           : mfma_f32_partial_bytes(p.n1, p.n2, p.d, W, p.fixed_split);
  float* P = cv.take<float>(pbytes / sizeof(float) + 1);
  const void *X1p = p.X1p, *X2p = p.X2p;
  const float *n1p = p.norm1, *n2p = p.norm2;
  if (!X1p || !X2p || !n1p || !n2p) {
    float* centre = cv.take<float>(p.d);
    double* part = cv.take<double>(MEAN_PART_BLOCKS * p.d);
    const size_t r1 = prepared_rows_bytes(p.precision, p.n1, p.d);
    const size_t r2 = prepared_rows_bytes(p.precision, p.n2, p.d);
    char* b1 = cv.take<char>(r1);
    char* b2 = cv.take<char>(r2);
    if (!cv.fits() || !ws) {
      set_error("kernel-product workspace too small: need %zu bytes, have %zu", cv.used, ws_bytes);
      return IGP_ENOMEM;
    }
    const size_t rows1 = r1 - align_up(p.n1 * sizeof(float));
    const size_t rows2 = r2 - align_up(p.n2 * sizeof(float));
    float* m1 = reinterpret_cast<float*>(b1 + rows1);
    float* m2 = reinterpret_cast<float*>(b2 + rows2);
    IGP_TRY(column_mean_f32(static_cast<const float*>(p.X2), p.n2, p.d, centre, part,
                            MEAN_PART_BLOCKS * p.d, s));
    IGP_TRY(prep_rows_any(p.precision, static_cast<const float*>(p.X1), p.n1, p.d, centre, b1, m1, s));
    if (p.X1 == p.X2 && p.n1 == p.n2) {
      // one point set on both sides: one prepared copy (the products may then
      // use the symmetric kernel)
      b2 = b1;
      m2 = m1;
    } else {
      IGP_TRY(prep_rows_any(p.precision, static_cast<const float*>(p.X2), p.n2, p.d, centre, b2, m2, s));
    }
    X1p = b1; n1p = m1; X2p = b2; n2p = m2;
  }
  if (!cv.fits() || !ws) {
    set_error("kernel-product workspace too small: need %zu bytes, have %zu", cv.used, ws_bytes);
    return IGP_ENOMEM;
  }
  int nsplit = 0;
  if (bf)
    IGP_TRY(kv_bf16_launch(p, X1p, n1p, X2p, n2p, P, pbytes, s, &nsplit));
  else
    IGP_TRY(kv_mfma_f32_launch(p, static_cast<const float*>(X1p), n1p,
                               static_cast<const float*>(X2p), n2p, P, pbytes, s, &nsplit));
  const int64_t total = p.n1 * W;
  int blocks = static_cast<int>(std::min<int64_t>(std::max<int64_t>(ceil_div(total, 256), 1), 4096));
  // with one kernel per class the outputscales are applied inside the product
  const float os = p.n_kp > 1 ? 1.0f : static_cast<float>(p.kp.outputscale);
  const bool epi = epilogue_ok(p);
  kv_reduce<float><<<blocks, 256, 0, s>>>(P, nsplit, p.n1, static_cast<int>(W),
                                          static_cast<int>(p.C), static_cast<float*>(p.Out), p.ldo,
                                          os, static_cast<float>(p.beta), p.skip,
                                          epi ? static_cast<const float*>(p.epi_pi) : nullptr,
                                          epi ? static_cast<const float*>(p.epi_s) : nullptr,
                                          epi ? static_cast<float*>(p.epi_z) : nullptr);
  if (epi && p.epi_applied) *p.epi_applied = 1;
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}
}  // namespace

int kv_launch(const KVProblem& p, void* ws, size_t ws_bytes, hipStream_t s) {
  if (p.n1 == 0 || p.nb == 0) return IGP_OK;
  if (p.n_kp > 1) {
    // one kernel per class: each class's kernel evaluated on the shared
    // distances
    IGP_REQUIRE(p.kpc && p.n_kp == p.C && p.C <= 64,
                "one kernel per class needs n_kp == C <= 64 parameter sets");
    for (int c = 0; c < p.n_kp; ++c)
      IGP_REQUIRE(p.kpc[c].kind == p.kp.kind, "per-class kernels must share one kernel family");
    if (is_bf16(p.precision)) {
      set_error("one kernel per class is not supported in the BF16 modes");
      return IGP_EUNSUPPORTED;
    }
    if (p.precision == IGP_FP64) return launch_valu<double>(p, ws, ws_bytes, s);
    // FP32 K(X, X) v (one vector, at most 8 classes): the symmetric matrix-core
    // kernel in its per-class form; otherwise the direct-difference kernel
    if (mfma_f32_perclass_ok(p)) return launch_mfma_path(p, ws, ws_bytes, s);
    return launch_valu<float>(p, ws, ws_bytes, s);
  }
  if (p.precision == IGP_FP64) return launch_valu<double>(p, ws, ws_bytes, s);
  if (kv_uses_prepared(p.precision, p.kp.kind, p.d)) return launch_mfma_path(p, ws, ws_bytes, s);
  return launch_valu<float>(p, ws, ws_bytes, s);
}

}  // namespace igp
