// Fused kernel-matrix product on the FP32 matrix cores of gfx950:
//
//   Out[n, w] = sum_m k(x1_n, x2_m) V[m, w]
//
// per 16 x 16 block of (m, n) and per wave:
//   1. D^T = X2_blk X1_blk^T with v_mfma_f32_16x16x4f32 (the distance term of
//      r^2 = |x1|^2 + |x2|^2 - 2 x1.x2, inputs centred on a common point);
//   2. the kernel function applied in registers to the 4 accumulator values;
//   3. Out_blk += K_blk V_blk with the same instruction.  Because step 1 is
//      computed transposed, lane l holds K[n = l%16][m = 4(l/16) + v] in its
//      accumulator register v -- exactly the A-operand lane layout of the
//      MFMA whose k-index v*4+l/16 enumerates m -- so K never leaves
//      registers and is never written to LDS or HBM.
// The contraction order over features inside step 1 is chosen so that every
// lane's four A (and B) values are one contiguous float4.
//
// A workgroup holds 64 rows of X1 (four waves x 16, kept in registers) and
// streams a contiguous range of X2 rows (split-N2) in tiles of 64 through
// LDS, double-buffered through registers: the next tile's global loads are in
// flight while the current tile is computed.  Partial sums per split are
// reduced in a fixed order (kv_reduce), so the product is deterministic.
#include <algorithm>

#include "ops.hpp"

namespace igp {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8x __attribute__((ext_vector_type(8)));
typedef unsigned int u4x __attribute__((ext_vector_type(4)));

namespace {

constexpr float LOG2E = 1.4426950408889634f;

// Scale kappa applied to r^2 = |x - x'|^2 / l^2 before the transform below.
template <int KIND>
constexpr float kappa() {
  if constexpr (KIND == IGP_RBF) return 0.5f * LOG2E;
  else if constexpr (KIND == IGP_MATERN12) return LOG2E * LOG2E;
  else if constexpr (KIND == IGP_MATERN32) return 3.0f * LOG2E * LOG2E;
  else return 5.0f * LOG2E * LOG2E;
}

// k as a function of t = kappa r^2 (outputscale applied later):
//   RBF  2^-t;  Matern-nu  poly(a) 2^-a with a = sqrt(t) = sqrt(c_nu) r log2(e)
template <int KIND>
__device__ inline float ktransform(float t) {
  if constexpr (KIND == IGP_RBF) {
    return __builtin_amdgcn_exp2f(-t);
  } else {
    // Matern-3/2 and -5/2 are flat at r = 0 (k = 1 - O(r^2)), so a slightly
    // negative t from rounding may enter through its magnitude (a free operand
    // modifier); Matern-1/2 has slope at 0 and clamps instead
    const float a = __builtin_amdgcn_sqrtf(KIND == IGP_MATERN12 ? fmaxf(t, 0.0f) : fabsf(t));
    const float e = __builtin_amdgcn_exp2f(-a);
    if constexpr (KIND == IGP_MATERN12) {
      return e;
    } else if constexpr (KIND == IGP_MATERN32) {
      return __builtin_fmaf(a, 1.0f / LOG2E, 1.0f) * e;
    } else {
      const float p = __builtin_fmaf(t, 1.0f / (3.0f * LOG2E * LOG2E), 1.0f);
      return __builtin_fmaf(a, 1.0f / LOG2E, p) * e;
    }
  }
}

constexpr int TN = 64;   // X2 rows per LDS tile

// D4: at most 4 features.  The prepared rows keep their 16 padded floats, but
// features 0..3 form the one k-block of a single distance MFMA per 16 x 16
// block (lane group g takes feature g) instead of four MFMAs over 16 mostly
// zero features.
template <int KIND, int DCH, int WCH, bool D4 = false>
__global__ void __launch_bounds__(256)
kv_mfma_f32(const float* __restrict__ X1p, const float* __restrict__ nrm1,
            const float* __restrict__ X2p, const float* __restrict__ nrm2, int64_t n1,
            int64_t n2, const float* __restrict__ V, int C, int W, int64_t ldv,
            float* __restrict__ P, int64_t cols_per_split, float cnorm, float cdot,
            const int* skip) {
  static_assert(!D4 || DCH == 1, "the 4-feature form pads to one chunk");
  if (gate_closed(skip)) return;
  constexpr int DP = DCH * 16;        // padded feature count
  constexpr int XS = DP + 4;          // LDS row stride of the X2 tile (floats)
  constexpr int WT = WCH * 16;        // output columns per workgroup
  constexpr int VS = TN + 4;          // LDS row stride of the transposed V tile
  constexpr int XQ = TN * DP / 4;     // float4 loads per X2 tile
  constexpr int XQT = XQ / 256;       // ... per thread (DCH)
  constexpr int VE = TN * WT / 256;   // V elements per thread (4*WCH)
  __shared__ __align__(16) float sX[2][TN * XS];
  __shared__ __align__(16) float sN[2][TN];
  __shared__ __align__(16) float sV[2][WT * VS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * 64 + wave * 16;
  const int w0 = blockIdx.z * WT;
  const int64_t m_begin = static_cast<int64_t>(blockIdx.y) * cols_per_split;
  const int64_t m_end = m_begin + cols_per_split < n2 ? m_begin + cols_per_split : n2;

  // this lane's X1 row (as B operand of the distance MFMA) and its norm
  const int64_t nrow = row0 + r;
  const bool nvalid = nrow < n1;
  f4 xb[DCH];
#pragma unroll
  for (int c = 0; c < DCH; ++c)
    xb[c] = nvalid ? *reinterpret_cast<const f4*>(X1p + nrow * DP + 16 * c + 4 * g) : f4{0, 0, 0, 0};
  const float xg = nvalid ? X1p[nrow * DP + g] : 0.0f;   // D4: feature g of the row
  const float n1v = nvalid ? nrm1[nrow] * cnorm : 0.0f;

  f4 out[WCH];
#pragma unroll
  for (int wc = 0; wc < WCH; ++wc) out[wc] = f4{0, 0, 0, 0};

  // register staging of one tile.  A thread stages one V column, w = w0 +
  // tid % WT, at rows tid / WT + q MSTEP, through one base pointer; a column
  // past W reads column W - 1 instead (it only feeds outputs that are not
  // stored).  Whole tiles skip the row checks.
  constexpr int MSTEP = 256 / WT;
  const int wl_t = tid % WT, m_t = tid / WT;
  const int w_t = w0 + wl_t < W ? w0 + wl_t : W - 1;
  const float* vbase = V + static_cast<int64_t>(w_t / C) * ldv + (w_t % C) +
                       static_cast<int64_t>(m_t) * C;
  f4 px[XQT];
  float pv[VE];
  float pn = 0.0f;
  auto fetch = [&](int64_t m0) {
    const float* vt = vbase + m0 * C;
    if (m0 + TN <= m_end) {
#pragma unroll
      for (int q = 0; q < XQT; ++q) {
        const int e = tid + q * 256;
        const int row = e / (DP / 4), col = e % (DP / 4);
        px[q] = *reinterpret_cast<const f4*>(X2p + (m0 + row) * DP + col * 4);
      }
      if (tid < TN) pn = nrm2[m0 + tid];   // scaled at the LDS store (no wait here)
#pragma unroll
      for (int q = 0; q < VE; ++q) pv[q] = vt[static_cast<int64_t>(q) * MSTEP * C];
    } else {
#pragma unroll
      for (int q = 0; q < XQT; ++q) {
        const int e = tid + q * 256;
        const int row = e / (DP / 4), col = e % (DP / 4);
        const int64_t m = m0 + row;
        px[q] = m < m_end ? *reinterpret_cast<const f4*>(X2p + m * DP + col * 4) : f4{0, 0, 0, 0};
      }
      if (tid < TN) {
        const int64_t m = m0 + tid;
        pn = m < m_end ? nrm2[m] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < VE; ++q)
        pv[q] = m0 + m_t + q * MSTEP < m_end ? vt[static_cast<int64_t>(q) * MSTEP * C] : 0.0f;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < XQT; ++q) {
      const int e = tid + q * 256;
      const int row = e / (DP / 4), col = e % (DP / 4);
      *reinterpret_cast<f4*>(&sX[buf][row * XS + col * 4]) = px[q];
    }
    if (tid < TN) sN[buf][tid] = pn * cnorm;
#pragma unroll
    for (int q = 0; q < VE; ++q) sV[buf][wl_t * VS + m_t + q * MSTEP] = pv[q];
  };

  if (m_begin < m_end) {
    fetch(m_begin);
    stash(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t m0 = m_begin; m0 < m_end; m0 += TN) {
    const bool more = m0 + TN < m_end;
    if (more) fetch(m0 + TN);
#pragma unroll
    for (int mb = 0; mb < TN / 16; ++mb) {
      f4 acc = {0, 0, 0, 0};
      if constexpr (D4) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(sX[buf][(mb * 16 + r) * XS + g], xg, acc, 0,
                                                   0, 0);
      } else {
#pragma unroll
        for (int c = 0; c < DCH; ++c) {
          const f4 a = *reinterpret_cast<const f4*>(&sX[buf][(mb * 16 + r) * XS + 16 * c + 4 * g]);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], xb[c][0], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], xb[c][1], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], xb[c][2], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], xb[c][3], acc, 0, 0, 0);
        }
      }
      const f4 n2v = *reinterpret_cast<const f4*>(&sN[buf][mb * 16 + 4 * g]);
      // this block's V fragments, read before the transform so that their
      // LDS latency hides behind it
      f4 vb[WCH];
#pragma unroll
      for (int wc = 0; wc < WCH; ++wc)
        vb[wc] = *reinterpret_cast<const f4*>(&sV[buf][(wc * 16 + r) * VS + mb * 16 + 4 * g]);
      f4 kv;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        kv[v] = ktransform<KIND>(__builtin_fmaf(acc[v], cdot, n1v + n2v[v]));
#pragma unroll
      for (int wc = 0; wc < WCH; ++wc) {
        out[wc] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv[0], vb[wc][0], out[wc], 0, 0, 0);
        out[wc] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv[1], vb[wc][1], out[wc], 0, 0, 0);
        out[wc] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv[2], vb[wc][2], out[wc], 0, 0, 0);
        out[wc] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv[3], vb[wc][3], out[wc], 0, 0, 0);
      }
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // out[wc][j] = Out[row0 + 4g + j][w0 + 16 wc + r]
#pragma unroll
  for (int wc = 0; wc < WCH; ++wc) {
    const int w = w0 + wc * 16 + r;
    if (w >= W) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t n = row0 + 4 * g + j;
      if (n < n1) P[(static_cast<int64_t>(blockIdx.y) * n1 + n) * W + w] = out[wc][j];
    }
  }
}

// Narrow-output variant (W <= 8, the solver products K s and K v): the
// contraction with V runs on VALU FMAs, which on gfx950 costs fewer issue
// cycles than four 16x16x4 MFMAs for W <= 8 (FP32 MFMA and VALU work do not
// overlap on a SIMD, so the kernel minimises their sum).  Each wave owns two
// 16-row strips of X1 (32 rows), so every X2 and V value read from LDS serves
// 32 output rows.  Lane l accumulates, for its rows r and 16 + r, the sum over
// the m assigned to its lane group g = l/16; the four group partials are
// added with cross-lane shuffles at the end.
constexpr int WV = 8;    // widest output of the narrow variant
#ifndef IGP_NARROW_NS
#define IGP_NARROW_NS 2
#endif
constexpr int NSTRIP = IGP_NARROW_NS;   // 16-row strips of X1 per wave

template <int DCH, int WX>
struct NarrowSmem {
  static constexpr int DP = DCH * 16;
  static constexpr int XS = DP + 4;
  static constexpr int VE = (TN * WX + 255) / 256;
  float sX[2][TN * XS];
  float sN[2][TN];
  float sV[2][VE * 256];
};

// One workgroup tile of the narrow variant: rows [row_base, row_base + 64 NS) of
// X1 against X2 rows [m_begin, m_end), partial outputs to P (row stride WX).
template <int KIND, int DCH, int WX, int NS>
__device__ inline void narrow_tile(NarrowSmem<DCH, WX>& sm, const float* __restrict__ X1p,
                                   const float* __restrict__ nrm1, const float* __restrict__ X2p,
                                   const float* __restrict__ nrm2, int64_t n1, int64_t row_base,
                                   int64_t m_begin, int64_t m_end, const float* __restrict__ V,
                                   int C, int64_t ldv, float* __restrict__ P, float cnorm,
                                   float cdot) {
  constexpr int DP = DCH * 16;
  constexpr int XS = DP + 4;
  constexpr int XQT = TN * DP / 4 / 256;   // float4 of X2 per thread per tile (= DCH)
  constexpr int VT = TN * WX;              // V values per tile, layout [m][WX]
  constexpr int VE = (VT + 255) / 256;     // V elements per thread per tile
  auto& sX = sm.sX;
  auto& sN = sm.sN;
  auto& sV = sm.sV;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int64_t row0 = row_base + wave * (16 * NS);
  f4 xb[NS][DCH];
  float n1v[NS];
#pragma unroll
  for (int st = 0; st < NS; ++st) {
    const int64_t nrow = row0 + st * 16 + r;
    const bool ok = nrow < n1;
#pragma unroll
    for (int c = 0; c < DCH; ++c)
      xb[st][c] = ok ? *reinterpret_cast<const f4*>(X1p + nrow * DP + 16 * c + 4 * g)
                     : f4{0, 0, 0, 0};
    n1v[st] = ok ? nrm1[nrow] * cnorm : 0.0f;
  }
  float acc[NS][WX];
#pragma unroll
  for (int st = 0; st < NS; ++st)
#pragma unroll
    for (int w = 0; w < WX; ++w) acc[st][w] = 0.0f;

  // V tile element e = tid + q*256 is (m = e / WX, w = e % WX); its global
  // offset from row m is (w / C) ldv + w % C, fixed per (tid, q): hoisted.
  int vm[VE];
  int64_t voff[VE];
#pragma unroll
  for (int q = 0; q < VE; ++q) {
    const int e = tid + q * 256;
    const int w = e % WX;
    vm[q] = e < VT ? e / WX : TN;   // TN marks an unused slot
    voff[q] = static_cast<int64_t>(w / C) * ldv + (w % C);
  }

  f4 px[XQT];
  float pv[VE];
  float pn = 0.0f;
  auto fetch = [&](int64_t m0) {
#pragma unroll
    for (int q = 0; q < XQT; ++q) {
      const int e = tid + q * 256;
      const int row = e / (DP / 4), col = e % (DP / 4);
      const int64_t m = m0 + row;
      px[q] = m < m_end ? *reinterpret_cast<const f4*>(X2p + m * DP + col * 4) : f4{0, 0, 0, 0};
    }
    if (tid < TN) {
      const int64_t m = m0 + tid;
      pn = m < m_end ? nrm2[m] : 0.0f;   // scaled at the LDS store (no wait here)
    }
#pragma unroll
    for (int q = 0; q < VE; ++q) {
      const int64_t gm = m0 + vm[q];
      pv[q] = (vm[q] < TN && gm < m_end) ? V[voff[q] + gm * C] : 0.0f;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < XQT; ++q) {
      const int e = tid + q * 256;
      const int row = e / (DP / 4), col = e % (DP / 4);
      *reinterpret_cast<f4*>(&sX[buf][row * XS + col * 4]) = px[q];
    }
    if (tid < TN) sN[buf][tid] = pn * cnorm;
#pragma unroll
    for (int q = 0; q < VE; ++q) sV[buf][tid + q * 256] = pv[q];
  };

  if (m_begin < m_end) {
    fetch(m_begin);
    stash(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t m0 = m_begin; m0 < m_end; m0 += TN) {
    const bool more = m0 + TN < m_end;
    if (more) fetch(m0 + TN);
#pragma unroll 2
    for (int mb = 0; mb < TN / 16; ++mb) {
      f4 dd[NS];
#pragma unroll
      for (int st = 0; st < NS; ++st) dd[st] = f4{0, 0, 0, 0};
#pragma unroll
      for (int c = 0; c < DCH; ++c) {
        const f4 a = *reinterpret_cast<const f4*>(&sX[buf][(mb * 16 + r) * XS + 16 * c + 4 * g]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int st = 0; st < NS; ++st)
            dd[st] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k], xb[st][c][k], dd[st], 0, 0, 0);
      }
      const f4 n2v = *reinterpret_cast<const f4*>(&sN[buf][mb * 16 + 4 * g]);
      // V rows m = mb*16 + 4g .. +3 are 4*WX contiguous floats (16-byte aligned)
      f4 vv[WX];
      const f4* vsrc = reinterpret_cast<const f4*>(&sV[buf][(mb * 16 + 4 * g) * WX]);
#pragma unroll
      for (int q = 0; q < WX; ++q) vv[q] = vsrc[q];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
#pragma unroll
        for (int st = 0; st < NS; ++st) {
          const float kk = ktransform<KIND>(__builtin_fmaf(dd[st][v], cdot, n1v[st] + n2v[v]));
#pragma unroll
          for (int w = 0; w < WX; ++w) {
            const int idx = v * WX + w;
            acc[st][w] = __builtin_fmaf(kk, vv[idx / 4][idx % 4], acc[st][w]);
          }
        }
      }
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // add the four lane-group partials (lanes r, r+16, r+32, r+48)
#pragma unroll
  for (int st = 0; st < NS; ++st)
#pragma unroll
    for (int w = 0; w < WX; ++w) {
      float x = acc[st][w];
      x += __shfl_xor(x, 16, 64);
      x += __shfl_xor(x, 32, 64);
      acc[st][w] = x;
    }
  if (g == 0) {
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int64_t n = row0 + st * 16 + r;
      if (n < n1) {
        float* dst = P + n * WX;
#pragma unroll
        for (int w = 0; w < WX; ++w) dst[w] = acc[st][w];
      }
    }
  }
}

// BF16 form of the narrow tile (inputs of at most 32 features): the X rows are
// the model's centred rows rounded to BF16 and zero-padded to 32 features, so
// one v_mfma_f32_16x16x32_bf16 forms a 16 x 16 block of distances where the
// FP32 tile issues four (D <= 16) or eight 16x16x4 instructions; norms, kernel
// transform and the VALU contraction are those of the FP32 tile.
template <int WX>
struct NarrowSmemB {
  static constexpr int XS = 40;    // bf16 per LDS row: 32 features + 16 bytes of padding
  static constexpr int VE = (TN * WX + 255) / 256;
  __bf16 sX[2][TN * XS];
  float sN[2][TN];
  float sV[2][VE * 256];
};

template <int KIND, int WX, int NS>
__device__ inline void narrow_tile_bf16(NarrowSmemB<WX>& sm, const __bf16* __restrict__ X1p,
                                        const float* __restrict__ nrm1,
                                        const __bf16* __restrict__ X2p,
                                        const float* __restrict__ nrm2, int64_t n1,
                                        int64_t row_base, int64_t m_begin, int64_t m_end,
                                        const float* __restrict__ V, int C, int64_t ldv,
                                        float* __restrict__ P, float cnorm, float cdot) {
  constexpr int DPB = 32;
  constexpr int XS = NarrowSmemB<WX>::XS;
  constexpr int XQT = TN * DPB / 8 / 256;  // 16-byte pieces of X2 per thread per tile
  static_assert(XQT >= 1, "one X2 tile covers at least one piece per thread");
  constexpr int VT = TN * WX;
  constexpr int VE = (VT + 255) / 256;
  auto& sX = sm.sX;
  auto& sN = sm.sN;
  auto& sV = sm.sV;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int64_t row0 = row_base + wave * (16 * NS);
  bf8x xb[NS];
  float n1v[NS];
#pragma unroll
  for (int st = 0; st < NS; ++st) {
    const int64_t nrow = row0 + st * 16 + r;
    const bool ok = nrow < n1;
    const u4x q = ok ? *reinterpret_cast<const u4x*>(X1p + nrow * DPB + 8 * g) : u4x{0, 0, 0, 0};
    xb[st] = *reinterpret_cast<const bf8x*>(&q);
    n1v[st] = ok ? nrm1[nrow] * cnorm : 0.0f;
  }
  float acc[NS][WX];
#pragma unroll
  for (int st = 0; st < NS; ++st)
#pragma unroll
    for (int w = 0; w < WX; ++w) acc[st][w] = 0.0f;
  int vm[VE];
  int64_t voff[VE];
#pragma unroll
  for (int q = 0; q < VE; ++q) {
    const int e = tid + q * 256;
    const int w = e % WX;
    vm[q] = e < VT ? e / WX : TN;
    voff[q] = static_cast<int64_t>(w / C) * ldv + (w % C);
  }
  u4x px[XQT];
  float pv[VE];
  float pn = 0.0f;
  auto fetch = [&](int64_t m0) {
#pragma unroll
    for (int q = 0; q < XQT; ++q) {
      const int e = tid + q * 256;
      const int row = e / (DPB / 8), col = e % (DPB / 8);
      const int64_t m = m0 + row;
      px[q] = m < m_end ? *reinterpret_cast<const u4x*>(X2p + m * DPB + col * 8)
                        : u4x{0, 0, 0, 0};
    }
    if (tid < TN) {
      const int64_t m = m0 + tid;
      pn = m < m_end ? nrm2[m] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < VE; ++q) {
      const int64_t gm = m0 + vm[q];
      pv[q] = (vm[q] < TN && gm < m_end) ? V[voff[q] + gm * C] : 0.0f;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < XQT; ++q) {
      const int e = tid + q * 256;
      const int row = e / (DPB / 8), col = e % (DPB / 8);
      *reinterpret_cast<u4x*>(&sX[buf][row * XS + col * 8]) = px[q];
    }
    if (tid < TN) sN[buf][tid] = pn * cnorm;
#pragma unroll
    for (int q = 0; q < VE; ++q) sV[buf][tid + q * 256] = pv[q];
  };

  if (m_begin < m_end) {
    fetch(m_begin);
    stash(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t m0 = m_begin; m0 < m_end; m0 += TN) {
    const bool more = m0 + TN < m_end;
    if (more) fetch(m0 + TN);
#pragma unroll 2
    for (int mb = 0; mb < TN / 16; ++mb) {
      const bf8x a = *reinterpret_cast<const bf8x*>(&sX[buf][(mb * 16 + r) * XS + 8 * g]);
      f4 dd[NS];
#pragma unroll
      for (int st = 0; st < NS; ++st)
        dd[st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, xb[st], f4{0, 0, 0, 0}, 0, 0, 0);
      const f4 n2v = *reinterpret_cast<const f4*>(&sN[buf][mb * 16 + 4 * g]);
      f4 vv[WX];
      const f4* vsrc = reinterpret_cast<const f4*>(&sV[buf][(mb * 16 + 4 * g) * WX]);
#pragma unroll
      for (int q = 0; q < WX; ++q) vv[q] = vsrc[q];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
#pragma unroll
        for (int st = 0; st < NS; ++st) {
          const float kk = ktransform<KIND>(__builtin_fmaf(dd[st][v], cdot, n1v[st] + n2v[v]));
#pragma unroll
          for (int w = 0; w < WX; ++w) {
            const int idx = v * WX + w;
            acc[st][w] = __builtin_fmaf(kk, vv[idx / 4][idx % 4], acc[st][w]);
          }
        }
      }
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int st = 0; st < NS; ++st)
#pragma unroll
    for (int w = 0; w < WX; ++w) {
      float x = acc[st][w];
      x += __shfl_xor(x, 16, 64);
      x += __shfl_xor(x, 32, 64);
      acc[st][w] = x;
    }
  if (g == 0) {
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int64_t n = row0 + st * 16 + r;
      if (n < n1) {
        float* dst = P + n * WX;
#pragma unroll
        for (int w = 0; w < WX; ++w) dst[w] = acc[st][w];
      }
    }
  }
}

template <int KIND, int DCH, int WX, int NS>
__global__ void __launch_bounds__(256)
kv_mfma_f32_narrow(const float* __restrict__ X1p, const float* __restrict__ nrm1,
                   const float* __restrict__ X2p, const float* __restrict__ nrm2, int64_t n1,
                   int64_t n2, const float* __restrict__ V, int C, int64_t ldv,
                   float* __restrict__ P, int64_t cols_per_split, float cnorm, float cdot,
                   const int* skip) {
  if (gate_closed(skip)) return;
  __shared__ __align__(16) NarrowSmem<DCH, WX> sm;
  const int64_t m_begin = static_cast<int64_t>(blockIdx.y) * cols_per_split;
  const int64_t m_end = m_begin + cols_per_split < n2 ? m_begin + cols_per_split : n2;
  narrow_tile<KIND, DCH, WX, NS>(sm, X1p, nrm1, X2p, nrm2, n1,
                                 static_cast<int64_t>(blockIdx.x) * (64 * NS), m_begin, m_end, V,
                                 C, ldv, P + static_cast<int64_t>(blockIdx.y) * n1 * WX, cnorm,
                                 cdot);
}

// ---- symmetric product K(X, X) V ----------------------------------------------
// When both row sets are the same points, each kernel value k(x_n, x_m) serves
// two outputs, Out[n] += k V[m] and Out[m] += k V[n], so every unordered pair
// of rows is evaluated once.  The rows are cut into I-blocks of 64 NS rows (one
// workgroup pass: four waves x NS strips of 16) and super-blocks of G I-blocks;
// the workgroups take the pairs (s, u), u >= s, of super-blocks.  A workgroup
// runs one pass per I-block of super-block s, streaming the rows of super-block
// u through LDS (on the pair u == s only the rows from the I-block itself on,
// and inside the I-block -- the 128 x 128 diagonal tile -- only the direct sum).
//
// The distance MFMA is issued with the register rows as A, so lane (r, g) holds
// k(n = 16 st + 4g + v, m = r) in accumulator register v of strip st -- the
// B-operand layout of an MFMA whose k-index runs over n:
//   direct      acc[st][v][w] += k V[m][w] on VALU FMAs (summed over the 16
//               lanes r of a lane row once per pass);
//   transposed  D[w][m] += V[n][w] k(n, m) on v_mfma_f32_16x16x4f32, one per
//               (st, v), with lane (r, g) supplying V[16 st + 4g + v][w = r] as
//               A; lanes (r, g < WX / 4) add their four D values (w = 4g ..
//               4g + 3, m = r) to this wave's slice of an LDS slab [m][w] with
//               one 128-bit read and write (the four slices are added in wave
//               order when the slab is written out).
// Partials: slot u of row n in super-block s holds the direct sum of the pair
// (s, u); slot s of row m in super-block u > s holds the transposed sum of the
// pair (s, u); on the pair (s, s) the slab is added to the direct sum of each
// I-block when it is written.  Every row thus has exactly Q slots, each written
// once, and kv_reduce adds them in slot order: the product is deterministic.
constexpr int SYM_NS = 2;                 // strips per wave: I-blocks of 128 rows
constexpr int SYM_MAX_Q = 128;            // super-blocks (partial slots per row)
constexpr size_t SYM_MAX_LDS = 48 * 1024;

__device__ inline float row16_sum(float x) {
  // sum over the 16 lanes of a lane row (rotations by 8, 4, 2, 1, each one
  // v_add_f32 with a DPP source); every lane holds the sum, each lane always
  // in the same order
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xF, 0xF, true));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xF, 0xF, true));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x122, 0xF, 0xF, true));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x121, 0xF, 0xF, true));
  return x;
}

template <int DCH, int WX>
struct SymLayout {
  static constexpr int DP = DCH * 16;
  static constexpr int XS = DP + 4;       // LDS row stride of the X2 tile
  static constexpr int VS = TN + 1;       // LDS row stride of the V tile, stored [w][m]
  static constexpr int FIXED = 2 * TN * XS + 2 * TN + 2 * WX * VS;   // floats before the slab
  static constexpr int SW = WX <= 4 ? 4 : 8;   // slab row: the output columns, padded
};

// One kernel per class (PC): the products of the solver (one vector, W = C
// columns, column w of class w) with per-class lengthscales and outputscales.
// The distance is formed once with the kernel constant alone (cnorm = kappa,
// cdot = -2 kappa) and column w takes os_w k(t il2_w); the transposed sums
// run on VALU FMAs per lane (one MFMA cannot serve columns with different
// kernel values) and are added over the four lane rows of a 16-row tile
// before they go to the slab.
struct ClassScale {
  float il2[8];   // 1 / lengthscale^2 of class w
  float os[8];    // outputscale of class w
};

// Item t of a symmetric plan with Q super-blocks -> pair (s, u): the
// Q (Q - 1) / 2 pairs u > s first (those of super-blocks before s number
// s (Q - 1) - s (s - 1) / 2), then the Q diagonal pairs, which take about half
// the work, at the end.
__device__ inline void sym_pair(int t, int Q, int& s, int& u) {
  const int noff = Q * (Q - 1) / 2;
  if (t >= noff) {
    s = u = t - noff;
    return;
  }
  int lo = 0, hi = Q - 2;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (mid * (Q - 1) - mid * (mid - 1) / 2 <= t) lo = mid;
    else hi = mid - 1;
  }
  s = lo;
  u = s + 1 + (t - (s * (Q - 1) - s * (s - 1) / 2));
}

// One item (super-block pair (s, u)) of the symmetric product on a workgroup of
// 256 threads; smem holds sym_lds_bytes(DCH, WX, G) bytes of LDS.  Every
// thread takes the same path (the barriers inside are workgroup-uniform).
// KB < 4 (at most 4 KB features, one padded chunk): the distance takes the
// features in KB k-blocks of four, lane group g holding feature 4 kb + g, so
// KB MFMAs per strip instead of four over mostly zero features.
template <int KIND, int DCH, int WX, bool PC, int KB = 4>
__device__ __forceinline__ void sym_item(float* smem, const float* __restrict__ Xp,
                                         const float* __restrict__ nrm, int64_t n,
                                         const float* __restrict__ V, int C, int64_t ldv,
                                         float* __restrict__ P, int G, int s, int u,
                                         float cnorm, float cdot, const ClassScale& cs) {
  static_assert(!PC || WX <= 8, "per-class columns are at most 8");
  static_assert(KB == 4 || (DCH == 1 && KB >= 1 && KB <= 3), "k-blocks of one feature chunk");
  using L = SymLayout<DCH, WX>;
  constexpr int NS = SYM_NS;
  constexpr int DP = L::DP, XS = L::XS, VS = L::VS;
  constexpr int XQT = TN * DP / 4 / 256;   // float4 of X2 per thread per tile (= DCH)
  constexpr int VT = TN * WX;
  constexpr int VE = (VT + 255) / 256;
  constexpr int IB = 64 * NS;
  float* sX = smem;                        // [2][TN * XS]
  float* sN = sX + 2 * TN * XS;            // [2][TN]
  float* sV = sN + 2 * TN;                 // [2][WX * VS]
  constexpr int SW = L::SW;
  const int64_t ST = static_cast<int64_t>(G) * IB;
  float* slab = smem + L::FIXED;           // [4 waves][ST][SW]
  const int SLICE = static_cast<int>(ST) * SW;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r = lane & 15;

  const bool diag_item = u == s;
  const int64_t j_lo = u * ST;
  const int64_t j_hi = (u + 1) * ST < n ? (u + 1) * ST : n;

  for (int e = tid; e < 4 * SLICE; e += 256) slab[e] = 0.0f;
  float* myslab = slab + wave * SLICE;

  int vm[VE], vdst[VE];
  int64_t voff[VE];
#pragma unroll
  for (int q = 0; q < VE; ++q) {
    const int e = tid + q * 256;
    const int w = e % WX;
    vm[q] = e < VT ? e / WX : TN;   // TN marks an unused slot
    vdst[q] = w * VS + (e < VT ? e / WX : 0);
    voff[q] = static_cast<int64_t>(w / C) * ldv + (w % C);
  }

  f4 px[XQT];
  float pv[VE];
  float pn = 0.0f;
  auto fetch = [&](int64_t m0, int64_t m_end) {
#pragma unroll
    for (int q = 0; q < XQT; ++q) {
      const int e = tid + q * 256;
      const int row = e / (DP / 4), col = e % (DP / 4);
      const int64_t m = m0 + row;
      px[q] = m < m_end ? *reinterpret_cast<const f4*>(Xp + m * DP + col * 4) : f4{0, 0, 0, 0};
    }
    if (tid < TN) {
      const int64_t m = m0 + tid;
      pn = m < m_end ? nrm[m] : 0.0f;   // scaled at the LDS store (no wait here)
    }
#pragma unroll
    for (int q = 0; q < VE; ++q) {
      const int64_t gm = m0 + vm[q];
      pv[q] = (vm[q] < TN && gm < m_end) ? V[voff[q] + gm * C] : 0.0f;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < XQT; ++q) {
      const int e = tid + q * 256;
      const int row = e / (DP / 4), col = e % (DP / 4);
      *reinterpret_cast<f4*>(&sX[buf * TN * XS + row * XS + col * 4]) = px[q];
    }
    if (tid < TN) sN[buf * TN + tid] = pn * cnorm;
#pragma unroll
    for (int q = 0; q < VE; ++q)
      if (vm[q] < TN) sV[buf * WX * VS + vdst[q]] = pv[q];
  };

  for (int k = 0; k < G; ++k) {
    const int64_t ib0 = s * ST + static_cast<int64_t>(k) * IB;
    if (ib0 >= n) break;
    const int64_t row0 = ib0 + wave * (16 * NS);
    // this wave's rows: A operand (row 16 st + r), norms and V of rows 16 st + 4g + v
    f4 xa[NS][DCH];
    float xk[NS][KB < 4 ? KB : 1];   // KB < 4: feature 4 kb + g of row 16 st + r
    float n1v[NS][4];
    float a1[NS][4];   // V[16 st + 4g + v][w = r]: A operand of the transposed MFMA
    // PC: V[16 st + 4g + v][w] for every column w (the transposed sums on VALU)
    float a1w[PC ? NS : 1][4][PC ? WX : 1];
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int64_t na = row0 + st * 16 + r;
      if constexpr (KB < 4) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) xk[st][kb] = na < n ? Xp[na * DP + 4 * kb + g] : 0.0f;
      } else {
#pragma unroll
        for (int c = 0; c < DCH; ++c)
          xa[st][c] = na < n ? *reinterpret_cast<const f4*>(Xp + na * DP + 16 * c + 4 * g)
                             : f4{0, 0, 0, 0};
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t nb = row0 + st * 16 + 4 * g + v;
        const bool ok = nb < n;
        n1v[st][v] = ok ? nrm[nb] * cnorm : 0.0f;
        if constexpr (PC) {
          a1[st][v] = 0.0f;
#pragma unroll
          for (int w = 0; w < WX; ++w)
            a1w[st][v][w] = ok ? V[static_cast<int64_t>(w / C) * ldv + (w % C) + nb * C] : 0.0f;
        } else {
          a1[st][v] = (ok && r < WX) ? V[static_cast<int64_t>(r / C) * ldv + (r % C) + nb * C]
                                     : 0.0f;
        }
      }
    }
    float acc[NS][4][WX];
#pragma unroll
    for (int st = 0; st < NS; ++st)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int w = 0; w < WX; ++w) acc[st][v][w] = 0.0f;

    const int64_t m_begin = diag_item ? ib0 : j_lo;
    const int64_t m_end = j_hi;
    const int64_t direct_only_end = diag_item ? ib0 + IB : m_begin;
    fetch(m_begin, m_end);
    stash(0);
    __syncthreads();
    int buf = 0;
    for (int64_t m0 = m_begin; m0 < m_end; m0 += TN) {
      const bool more = m0 + TN < m_end;
      if (more) fetch(m0 + TN, m_end);
      const bool both = m0 >= direct_only_end;
      const float* bX = sX + buf * TN * XS;
      const float* bN = sN + buf * TN;
      const float* bV = sV + buf * WX * VS;
#pragma unroll 1
      for (int mb = 0; mb < TN / 16; ++mb) {
        f4 dd[NS];
#pragma unroll
        for (int st = 0; st < NS; ++st) dd[st] = f4{0, 0, 0, 0};
        if constexpr (KB < 4) {
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) {
            const float b = bX[(mb * 16 + r) * XS + 4 * kb + g];
#pragma unroll
            for (int st = 0; st < NS; ++st)
              dd[st] = __builtin_amdgcn_mfma_f32_16x16x4f32(xk[st][kb], b, dd[st], 0, 0, 0);
          }
        } else {
#pragma unroll
          for (int c = 0; c < DCH; ++c) {
            const f4 b = *reinterpret_cast<const f4*>(&bX[(mb * 16 + r) * XS + 16 * c + 4 * g]);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
              for (int st = 0; st < NS; ++st)
                dd[st] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[st][c][kk], b[kk], dd[st], 0, 0,
                                                              0);
          }
        }
        const float n2v = bN[mb * 16 + r];
        float vm2[WX];
#pragma unroll
        for (int w = 0; w < WX; ++w) vm2[w] = bV[w * VS + mb * 16 + r];
        if constexpr (PC) {
          // column w: os_w k(t il2_w), t = kappa |x_n - x_m|^2; tr2[w] = this
          // lane's part of the transposed sum for m = mb 16 + r
          float tr2[WX];
#pragma unroll
          for (int w = 0; w < WX; ++w) tr2[w] = 0.0f;
#pragma unroll
          for (int st = 0; st < NS; ++st)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const float t = __builtin_fmaf(dd[st][v], cdot, n1v[st][v] + n2v);
#pragma unroll
              for (int w = 0; w < WX; ++w) {
                const float kw = cs.os[w] * ktransform<KIND>(t * cs.il2[w]);
                acc[st][v][w] = __builtin_fmaf(kw, vm2[w], acc[st][v][w]);
                tr2[w] = __builtin_fmaf(kw, a1w[st][v][w], tr2[w]);
              }
            }
          if (both) {
            // add over the lane rows g (the same m), then lane (r, g) adds
            // columns 4g .. 4g + 3 to the slab row m
#pragma unroll
            for (int w = 0; w < WX; ++w) {
              tr2[w] += __shfl_xor(tr2[w], 16, 64);
              tr2[w] += __shfl_xor(tr2[w], 32, 64);
            }
            f4* dst = reinterpret_cast<f4*>(myslab + ((m0 - j_lo) + mb * 16 + r) * SW + 4 * g);
            if (4 * g < SW) {
              f4 add = {0, 0, 0, 0};
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                float x = 0.0f;
#pragma unroll
                for (int q = 0; q < SW / 4; ++q)
                  if (4 * q + j < WX && g == q) x = tr2[4 * q + j];
                add[j] = x;
              }
              *dst = *dst + add;
            }
          }
          continue;
        }
        f4 kk[NS];
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            kk[st][v] = ktransform<KIND>(__builtin_fmaf(dd[st][v], cdot, n1v[st][v] + n2v));
#pragma unroll
            for (int w = 0; w < WX; ++w)
              acc[st][v][w] = __builtin_fmaf(kk[st][v], vm2[w], acc[st][v][w]);
          }
        if (both) {
          // lane (r, g) receives D[w = 4g + j][m = r], j < 4
          f4* dst = reinterpret_cast<f4*>(myslab + ((m0 - j_lo) + mb * 16 + r) * SW + 4 * g);
          const bool mine = 4 * g < SW;
          f4 old = {0, 0, 0, 0};
          if (mine) old = *dst;
          f4 tr = {0, 0, 0, 0};
#pragma unroll
          for (int st = 0; st < NS; ++st)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              tr = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[st][v], kk[st][v], tr, 0, 0, 0);
          if (mine) *dst = old + tr;
        }
      }
      if (more) stash(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
    // direct sums of this I-block -> slot u (plus, on the diagonal pair, the
    // transposed sums its rows received from the earlier I-blocks)
#pragma unroll
    for (int st = 0; st < NS; ++st)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int w = 0; w < WX; ++w) acc[st][v][w] = row16_sum(acc[st][v][w]);
    // lane r of the row writes output column w = r
#pragma unroll
    for (int st = 0; st < NS; ++st)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float x = acc[st][v][0];
#pragma unroll
        for (int w = 1; w < WX; ++w) x = r == w ? acc[st][v][w] : x;
        const int64_t nb = row0 + st * 16 + 4 * g + v;
        if (r < WX && nb < n) {
          if (diag_item) {
            const int o = static_cast<int>(nb - j_lo) * SW + r;
            x += (slab[o] + slab[SLICE + o]) + (slab[2 * SLICE + o] + slab[3 * SLICE + o]);
          }
          P[(static_cast<int64_t>(u) * n + nb) * WX + r] = x;
        }
      }
  }
  if (!diag_item) {
    // transposed sums of super-block u -> slot s (every pass ended with a barrier)
    const int64_t rows = j_hi - j_lo;
    for (int64_t e = tid; e < rows * WX; e += 256) {
      const int ml = static_cast<int>(e / WX), w = static_cast<int>(e % WX);
      const int o = ml * SW + w;
      P[(static_cast<int64_t>(s) * n + j_lo + ml) * WX + w] =
          (slab[o] + slab[SLICE + o]) + (slab[2 * SLICE + o] + slab[3 * SLICE + o]);
    }
  }
}

template <int KIND, int DCH, int WX, bool PC = false, int KB = 4>
__global__ void __launch_bounds__(256)
kv_mfma_f32_sym(const float* __restrict__ Xp, const float* __restrict__ nrm, int64_t n,
                const float* __restrict__ V, int C, int64_t ldv, float* __restrict__ P, int G,
                int Q, float cnorm, float cdot, ClassScale cs, const int* skip) {
  if (gate_closed(skip)) return;
  extern __shared__ __align__(16) float smem[];
  int s, u;
  sym_pair(static_cast<int>(blockIdx.x), Q, s, u);
  sym_item<KIND, DCH, WX, PC, KB>(smem, Xp, nrm, n, V, C, ldv, P, G, s, u, cnorm, cdot, cs);
}

// ---- persistent batched launch -------------------------------------------------
// Every product of a batch (independent problems of different sizes, output
// widths and hyperparameters; same kernel family and feature count) is cut
// into workgroup tiles (problem, 64*NS-row block, X2 split); a fixed grid of
// workgroups takes tiles from an atomic counter until none are left, so one
// launch covers all problems x classes and keeps every CU busy while small
// problems finish.  The counter is cleared by a kernel before each launch.
// One product of a BF16 model with at most 32 features on the narrow BF16 tile
// (grid: X1 row blocks x X2 splits), partial sums per split.
template <int KIND, int WX, int NS>
__global__ void __launch_bounds__(256)
kv_bf16_narrow(const __bf16* __restrict__ X1p, const float* __restrict__ nrm1,
               const __bf16* __restrict__ X2p, const float* __restrict__ nrm2, int64_t n1,
               int64_t n2, const float* __restrict__ V, int C, int64_t ldv,
               float* __restrict__ P, int64_t cols_per_split, float cnorm, float cdot,
               const int* skip) {
  if (gate_closed(skip)) return;
  __shared__ __align__(16) NarrowSmemB<WX> sm;
  const int64_t m_begin = static_cast<int64_t>(blockIdx.y) * cols_per_split;
  const int64_t m_end = m_begin + cols_per_split < n2 ? m_begin + cols_per_split : n2;
  narrow_tile_bf16<KIND, WX, NS>(sm, X1p, nrm1, X2p, nrm2, n1,
                                 static_cast<int64_t>(blockIdx.x) * (64 * NS), m_begin, m_end,
                                 V, C, ldv, P + static_cast<int64_t>(blockIdx.y) * n1 * WX,
                                 cnorm, cdot);
}

template <int KIND, int DCH, int NS, bool BF>
__global__ void __launch_bounds__(256)
kv_batched_persistent(const BatchProblem* __restrict__ probs, int np, int64_t ntiles,
                      int* __restrict__ counter) {
  constexpr size_t SMEM = BF ? sizeof(NarrowSmemB<WV>) : sizeof(NarrowSmem<DCH, WV>);
  __shared__ __align__(16) unsigned char smem_raw[SMEM];
  __shared__ int64_t s_tile;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(reinterpret_cast<unsigned long long*>(counter), 1ull);
    __syncthreads();
    const int64_t t = s_tile;
    __syncthreads();
    if (t >= ntiles) break;
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (probs[mid].tile_begin <= t) lo = mid;
      else hi = mid - 1;
    }
    const BatchProblem& pb = probs[lo];
    if (pb.gate && gate_closed(pb.gate)) continue;   // the problem's solver has stopped
    const int64_t local = t - pb.tile_begin;
    const int64_t rb = local % pb.gx, sp = local / pb.gx;
    const int64_t m_begin = sp * pb.cols_per_split;
    const int64_t m_end = m_begin + pb.cols_per_split < pb.n2 ? m_begin + pb.cols_per_split : pb.n2;
    float* P = pb.P + sp * pb.n1 * pb.W;
    switch (pb.W) {
#define IGP_BW(K)                                                                              \
  case K:                                                                                      \
    if constexpr (BF)                                                                          \
      narrow_tile_bf16<KIND, K, NS>(*reinterpret_cast<NarrowSmemB<K>*>(smem_raw),              \
                                    static_cast<const __bf16*>(pb.X1p), pb.nrm1,               \
                                    static_cast<const __bf16*>(pb.X2p), pb.nrm2, pb.n1,        \
                                    rb * (64 * NS), m_begin, m_end, pb.V, pb.C, pb.ldv, P,     \
                                    pb.cnorm, pb.cdot);                                        \
    else                                                                                       \
      narrow_tile<KIND, DCH, K, NS>(*reinterpret_cast<NarrowSmem<DCH, K>*>(smem_raw),          \
                                    static_cast<const float*>(pb.X1p), pb.nrm1,                \
                                    static_cast<const float*>(pb.X2p), pb.nrm2, pb.n1,         \
                                    rb * (64 * NS), m_begin, m_end, pb.V, pb.C, pb.ldv, P,     \
                                    pb.cnorm, pb.cdot);                                        \
    break;
      IGP_BW(1) IGP_BW(2) IGP_BW(3) IGP_BW(4) IGP_BW(5) IGP_BW(6) IGP_BW(7) IGP_BW(8)
#undef IGP_BW
      default: break;
    }
    __syncthreads();
  }
}

__global__ void k_zero_counter(int* c) {
  // the queue counters of a batched launch
  if (threadIdx.x < BATCH_COUNTERS && blockIdx.x == 0)
    reinterpret_cast<unsigned long long*>(c)[threadIdx.x] = 0ull;
}

__global__ void kv_reduce_batched(const BatchProblem* __restrict__ probs, int np,
                                  int64_t total) {
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (probs[mid].out_begin <= idx) lo = mid;
      else hi = mid - 1;
    }
    const BatchProblem& pb = probs[lo];
    if (pb.gate && gate_closed(pb.gate)) continue;
    const int64_t e = idx - pb.out_begin;
    const int64_t n = e / pb.W;
    const int w = static_cast<int>(e % pb.W);
    const int64_t stride = pb.n1 * pb.W;
    const float* q = pb.P + n * pb.W + w;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int sp = 0;
    for (; sp + 4 <= pb.nsplit; sp += 4) {
      s0 += q[sp * stride];
      s1 += q[(sp + 1) * stride];
      s2 += q[(sp + 2) * stride];
      s3 += q[(sp + 3) * stride];
    }
    for (; sp < pb.nsplit; ++sp) s0 += q[sp * stride];
    pb.Out[(w / pb.C) * pb.ldo + n * pb.C + (w % pb.C)] = pb.os * ((s0 + s1) + (s2 + s3));
  }
}

// The symmetric FP32 products of a batch with W output columns (problems whose
// plan admits the symmetric kernel): items (problem, super-block pair) from
// one queue, each run by sym_item with the problem's own plan (G, Q), so the
// partial slots -- and after kv_reduce_batched the product -- are those of the
// single-problem launch, bit for bit.  One instantiation per W keeps the
// single kernel's register budget.  Dynamic LDS: the largest plan's bytes.
template <int KIND, int DCH, int WX, int KB>
__global__ void __launch_bounds__(256)
kv_batched_sym(const BatchProblem* __restrict__ probs, int np, int64_t ntiles,
               int* __restrict__ counter) {
  extern __shared__ __align__(16) float smem[];
  __shared__ int64_t s_tile;
  const ClassScale none{};
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(reinterpret_cast<unsigned long long*>(counter), 1ull);
    __syncthreads();
    const int64_t t = s_tile;
    __syncthreads();
    if (t >= ntiles) break;
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (probs[mid].tile_begin <= t) lo = mid;
      else hi = mid - 1;
    }
    const BatchProblem& pb = probs[lo];
    if (pb.gate && gate_closed(pb.gate)) continue;   // the problem's solver has stopped
    int su, uu;
    sym_pair(static_cast<int>(t - pb.tile_begin), pb.sym_q, su, uu);
    sym_item<KIND, DCH, WX, false, KB>(smem, static_cast<const float*>(pb.X1p), pb.nrm1, pb.n1, pb.V,
                                   pb.C, pb.ldv, pb.P, pb.sym_g, su, uu, pb.cnorm, pb.cdot,
                                   none);
  }
}

// Centred, zero-padded copies of rows (DP floats each) and their squared norms.
__global__ void k_prep_rows(const float* __restrict__ X, int64_t n, int d, int DP,
                            const float* __restrict__ centre, float* __restrict__ Xp,
                            float* __restrict__ norms) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < DP; ++k) {
    float v = 0.0f;
    if (k < d) v = X[i * d + k] - (centre ? centre[k] : 0.0f);
    Xp[i * DP + k] = v;
    s += static_cast<double>(v) * v;
  }
  norms[i] = static_cast<float>(s);
}

__global__ void k_col_partial(const float* __restrict__ X, int64_t n, int d, int64_t rows_per,
                              double* __restrict__ part) {
  const int64_t r0 = blockIdx.x * rows_per;
  const int64_t r1 = r0 + rows_per < n ? r0 + rows_per : n;
  for (int k = threadIdx.x; k < d; k += blockDim.x) {
    double s = 0.0;
    for (int64_t i = r0; i < r1; ++i) s += X[i * d + k];
    part[blockIdx.x * static_cast<int64_t>(d) + k] = s;
  }
}

// one block per column: fixed-order sum of the block partials
__global__ void __launch_bounds__(256)
k_col_finish(const double* __restrict__ part, int nblk, int d, int64_t n,
             float* __restrict__ mean) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += part[static_cast<int64_t>(b) * d + k];
  s = block_sum(s, red);
  if (threadIdx.x == 0) mean[k] = static_cast<float>(n > 0 ? s / n : 0.0);
}

struct Plan {
  int dch, wch, gx, gz, nsplit;
  bool narrow;
  bool d4;          // at most 4 features (the wide kernel's one-MFMA distance)
  int64_t cols_per_split;
};

Plan plan_mfma(int64_t n1, int64_t n2, int64_t d, int64_t W, bool fixed = false) {
  Plan p{};
  p.dch = static_cast<int>(ceil_div(d, 16));
  p.d4 = d <= 4;
  p.narrow = W <= WV && p.dch <= 2;
  p.wch = W <= 16 ? 1 : (W <= 32 ? 2 : 4);
  p.gx = static_cast<int>(ceil_div(n1, p.narrow ? 64 * NSTRIP : 64));
  p.gz = p.narrow ? 1 : static_cast<int>(ceil_div(W, 16 * p.wch));
  const int64_t tiles = ceil_div(n2, TN);
  if (tiles == 0) {
    p.nsplit = 0;
    p.cols_per_split = TN;
    return p;
  }
  // about 8192 workgroups (several rounds over 256 CUs, small tail)
  int64_t want = ceil_div(8192, static_cast<int64_t>(p.gx) * p.gz);
  if (want < 1) want = 1;
  if (want > tiles) want = tiles;
  // a fixed split depends on n2 and the output width only, never on n1:
  // narrow outputs (a predictive mean) split at 512 rows, widths up to 512
  // into about 20 ranges of at least 1024 rows (enough workgroups for a few
  // thousand test rows, partial sums bounded by 20 outputs), wider at 4096
  int64_t fixed_rows = FIXED_SPLIT_ROWS;
  if (W <= 16) fixed_rows = FIXED_SPLIT_ROWS_NARROW;
  else if (W <= 512) fixed_rows = std::max<int64_t>(1024, ceil_div(ceil_div(n2, 20), TN) * TN);
  p.cols_per_split = fixed ? fixed_rows : ceil_div(tiles, want) * TN;
  p.nsplit = static_cast<int>(ceil_div(n2, p.cols_per_split));
  return p;
}

// Symmetric plan: G I-blocks per super-block, Q super-blocks, Q (Q + 1) / 2
// workgroups.  G grows with n so that there are about 4000 workgroups, within
// 48 KB of LDS for the slab; beyond SYM_MAX_Q super-blocks the partial slots
// would outgrow the plain plan's and the plain kernel is used.
struct SymPlan {
  bool ok;
  int G, Q;
  int kb;           // feature k-blocks of the distance (sym_item's KB)
  size_t lds;
};

// sym_item's KB for d features: 1 or 2 k-blocks of four within one padded chunk
int sym_kblocks(int64_t d) { return d <= 4 ? 1 : (d <= 8 ? 2 : 4); }

size_t sym_lds_bytes(int dch, int64_t W, int G) {
  const int64_t fixed = 2 * TN * (dch * 16 + 4) + 2 * TN + 2 * W * (TN + 1);
  const int64_t sw = W <= 4 ? 4 : 8;
  return sizeof(float) *
         static_cast<size_t>(fixed + 4 * static_cast<int64_t>(G) * 64 * SYM_NS * sw);
}

SymPlan plan_sym(int64_t n, int64_t d, int64_t W) {
  SymPlan sp{};
  const int dch = static_cast<int>(ceil_div(d, 16));
  if (n < 1 || W < 1 || W > WV || dch > 2) return sp;
  const int64_t IB = 64 * SYM_NS;
  int G = static_cast<int>(std::min<int64_t>(std::max<int64_t>(ceil_div(n, IB * 90), 1), 4));
  while (G > 1 && sym_lds_bytes(dch, W, G) > SYM_MAX_LDS) --G;
  sp.G = G;
  sp.kb = sym_kblocks(d);
  sp.Q = static_cast<int>(ceil_div(n, G * IB));
  sp.lds = sym_lds_bytes(dch, W, G);
  sp.ok = sp.Q <= SYM_MAX_Q && sp.lds <= SYM_MAX_LDS;
  return sp;
}

template <int KIND, int DCH, bool PC, int KB>
int launch_sym_kb(const SymPlan& sp, const float* Xp, const float* np_, int64_t n,
                  const float* V, int C, int W, int64_t ldv, float* P, float cnorm, float cdot,
                  const ClassScale& cs, const int* skip, hipStream_t s) {
  const unsigned items = static_cast<unsigned>(sp.Q * (sp.Q + 1) / 2);
  switch (W) {
#define IGP_SW(K)                                                                              \
  case K:                                                                                      \
    kv_mfma_f32_sym<KIND, DCH, K, PC, KB><<<items, 256, sp.lds, s>>>(Xp, np_, n, V, C, ldv, P, \
                                                                     sp.G, sp.Q, cnorm, cdot,  \
                                                                     cs, skip);                \
    break;
    IGP_SW(1) IGP_SW(2) IGP_SW(3) IGP_SW(4) IGP_SW(5) IGP_SW(6) IGP_SW(7) IGP_SW(8)
#undef IGP_SW
    default: break;
  }
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

// the per-class form keeps four k-blocks (its registers are spent on the classes)
template <int KIND, int DCH, bool PC>
int launch_sym_dch(const SymPlan& sp, const float* Xp, const float* np_, int64_t n,
                   const float* V, int C, int W, int64_t ldv, float* P, float cnorm, float cdot,
                   const ClassScale& cs, const int* skip, hipStream_t s) {
  if constexpr (DCH == 1 && !PC) {
    if (sp.kb == 1)
      return launch_sym_kb<KIND, 1, false, 1>(sp, Xp, np_, n, V, C, W, ldv, P, cnorm, cdot, cs,
                                              skip, s);
    if (sp.kb == 2)
      return launch_sym_kb<KIND, 1, false, 2>(sp, Xp, np_, n, V, C, W, ldv, P, cnorm, cdot, cs,
                                              skip, s);
  }
  return launch_sym_kb<KIND, DCH, PC, 4>(sp, Xp, np_, n, V, C, W, ldv, P, cnorm, cdot, cs, skip,
                                         s);
}

template <int KIND, bool PC = false>
int launch_sym(const SymPlan& sp, int dch, const float* Xp, const float* np_, int64_t n,
               const float* V, int C, int W, int64_t ldv, float* P, float cnorm, float cdot,
               const int* skip, hipStream_t s, const ClassScale& cs = ClassScale{}) {
  if (dch == 1)
    return launch_sym_dch<KIND, 1, PC>(sp, Xp, np_, n, V, C, W, ldv, P, cnorm, cdot, cs, skip, s);
  return launch_sym_dch<KIND, 2, PC>(sp, Xp, np_, n, V, C, W, ldv, P, cnorm, cdot, cs, skip, s);
}

template <int KIND, int DCH>
int launch_kind_dch(const Plan& pl, const float* X1p, const float* n1p, const float* X2p,
                    const float* n2p, int64_t n1, int64_t n2, const float* V, int C, int W,
                    int64_t ldv, float* P, float cnorm, float cdot, const int* skip,
                    hipStream_t s) {
  dim3 grid(pl.gx, pl.nsplit, pl.gz);
  if (pl.narrow) {
    if constexpr (DCH <= 2) {
      switch (W) {
#define IGP_NW(K) \
  case K: kv_mfma_f32_narrow<KIND, DCH, K, NSTRIP><<<grid, 256, 0, s>>>(X1p, n1p, X2p, n2p, n1, n2, V, C, ldv, P, pl.cols_per_split, cnorm, cdot, skip); break;
        IGP_NW(1) IGP_NW(2) IGP_NW(3) IGP_NW(4) IGP_NW(5) IGP_NW(6) IGP_NW(7) IGP_NW(8)
#undef IGP_NW
        default: break;
      }
    }
  } else if (DCH == 1 && pl.d4) {
    if constexpr (DCH == 1) {
      if (pl.wch == 1)
        kv_mfma_f32<KIND, 1, 1, true><<<grid, 256, 0, s>>>(X1p, n1p, X2p, n2p, n1, n2, V, C, W,
                                                           ldv, P, pl.cols_per_split, cnorm,
                                                           cdot, skip);
      else if (pl.wch == 2)
        kv_mfma_f32<KIND, 1, 2, true><<<grid, 256, 0, s>>>(X1p, n1p, X2p, n2p, n1, n2, V, C, W,
                                                           ldv, P, pl.cols_per_split, cnorm,
                                                           cdot, skip);
      else
        kv_mfma_f32<KIND, 1, 4, true><<<grid, 256, 0, s>>>(X1p, n1p, X2p, n2p, n1, n2, V, C, W,
                                                           ldv, P, pl.cols_per_split, cnorm,
                                                           cdot, skip);
    }
  } else if (pl.wch == 1)
    kv_mfma_f32<KIND, DCH, 1><<<grid, 256, 0, s>>>(X1p, n1p, X2p, n2p, n1, n2, V, C, W, ldv, P,
                                                   pl.cols_per_split, cnorm, cdot, skip);
  else if (pl.wch == 2)
    kv_mfma_f32<KIND, DCH, 2><<<grid, 256, 0, s>>>(X1p, n1p, X2p, n2p, n1, n2, V, C, W, ldv, P,
                                                   pl.cols_per_split, cnorm, cdot, skip);
  else
    kv_mfma_f32<KIND, DCH, 4><<<grid, 256, 0, s>>>(X1p, n1p, X2p, n2p, n1, n2, V, C, W, ldv, P,
                                                   pl.cols_per_split, cnorm, cdot, skip);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

template <int KIND>
int launch_kind(const Plan& pl, const float* X1p, const float* n1p, const float* X2p,
                const float* n2p, int64_t n1, int64_t n2, const float* V, int C, int W,
                int64_t ldv, float* P, float cnorm, float cdot, const int* skip, hipStream_t s) {
  switch (pl.dch) {
#define IGP_DCH(K) \
  case K: return launch_kind_dch<KIND, K>(pl, X1p, n1p, X2p, n2p, n1, n2, V, C, W, ldv, P, cnorm, cdot, skip, s);
    IGP_DCH(1) IGP_DCH(2) IGP_DCH(3) IGP_DCH(4) IGP_DCH(5) IGP_DCH(6) IGP_DCH(7) IGP_DCH(8)
#undef IGP_DCH
    default:
      set_error("feature count outside the FP32 matrix-core kernel's range");
      return IGP_EUNSUPPORTED;
  }
}

}  // namespace

float kv_kappa(int kind) {
  switch (kind) {
    case IGP_RBF: return kappa<IGP_RBF>();
    case IGP_MATERN12: return kappa<IGP_MATERN12>();
    case IGP_MATERN32: return kappa<IGP_MATERN32>();
    default: return kappa<IGP_MATERN52>();
  }
}

bool bf16_narrow_supported(int kind, int64_t d, int64_t W) {
  return kind != IGP_MATERN12 && d >= 1 && d <= 32 && W >= 1 && W <= WV;
}

size_t bf16_narrow_partial_bytes(int64_t n1, int64_t n2, int64_t W, bool fixed) {
  const Plan pl = plan_mfma(n1, n2, 32, W, fixed);
  return static_cast<size_t>(pl.nsplit) * n1 * W * sizeof(float);
}

namespace {
template <int KIND>
void launch_bf16_narrow_kind(const Plan& pl, const __bf16* X1, const float* n1p,
                             const __bf16* X2, const float* n2p, int64_t n1, int64_t n2,
                             const float* V, int C, int W, int64_t ldv, float* P, float cnorm,
                             float cdot, const int* skip, hipStream_t s) {
  const dim3 grid(pl.gx, pl.nsplit);
  switch (W) {
#define IGP_BNW(K)                                                                             \
  case K:                                                                                      \
    kv_bf16_narrow<KIND, K, NSTRIP><<<grid, 256, 0, s>>>(X1, n1p, X2, n2p, n1, n2, V, C, ldv,   \
                                                         P, pl.cols_per_split, cnorm, cdot,    \
                                                         skip);                                \
    break;
    IGP_BNW(1) IGP_BNW(2) IGP_BNW(3) IGP_BNW(4) IGP_BNW(5) IGP_BNW(6) IGP_BNW(7) IGP_BNW(8)
#undef IGP_BNW
    default: break;
  }
}
}  // namespace

// Out partials of a BF16 product with at most 32 features and 8 output columns
// on the narrow BF16 tile (rows prepared as for the wide BF16 kernel).
int kv_bf16_narrow_launch(const KVProblem& p, const void* X1b, const float* n1p,
                          const void* X2b, const float* n2p, float* P, size_t P_bytes,
                          hipStream_t s, int* nsplit_out) {
  const int64_t W = p.C * p.nb;
  const Plan pl = plan_mfma(p.n1, p.n2, 32, W, p.fixed_split);
  *nsplit_out = pl.nsplit;
  if (p.symmetric_out) *p.symmetric_out = 0;
  if (static_cast<size_t>(pl.nsplit) * p.n1 * W * sizeof(float) > P_bytes) {
    set_error("kernel-product workspace too small for the split partials");
    return IGP_ENOMEM;
  }
  if (pl.nsplit == 0 || pl.gx == 0) return IGP_OK;
  const double inv_l2 = 1.0 / (p.kp.lengthscale * p.kp.lengthscale);
  const float k = kv_kappa(p.kp.kind);
  const float cnorm = static_cast<float>(k * inv_l2), cdot = static_cast<float>(-2.0 * k * inv_l2);
  const __bf16* A1 = static_cast<const __bf16*>(X1b);
  const __bf16* A2 = static_cast<const __bf16*>(X2b);
  const float* V = static_cast<const float*>(p.V);
  const int C = static_cast<int>(p.C), Wi = static_cast<int>(W);
  switch (p.kp.kind) {
    case IGP_RBF:
      launch_bf16_narrow_kind<IGP_RBF>(pl, A1, n1p, A2, n2p, p.n1, p.n2, V, C, Wi, p.ldv, P,
                                       cnorm, cdot, p.skip, s);
      break;
    case IGP_MATERN32:
      launch_bf16_narrow_kind<IGP_MATERN32>(pl, A1, n1p, A2, n2p, p.n1, p.n2, V, C, Wi, p.ldv,
                                            P, cnorm, cdot, p.skip, s);
      break;
    default:
      launch_bf16_narrow_kind<IGP_MATERN52>(pl, A1, n1p, A2, n2p, p.n1, p.n2, V, C, Wi, p.ldv,
                                            P, cnorm, cdot, p.skip, s);
      break;
  }
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

bool mfma_f32_supported(int kind, int64_t d) {
  return kind != IGP_MATERN12 && d >= 1 && d <= 128;
}

size_t mfma_f32_partial_bytes(int64_t n1, int64_t n2, int64_t d, int64_t W, bool fixed) {
  Plan pl = plan_mfma(n1, n2, d, W, fixed);
  size_t b = static_cast<size_t>(pl.nsplit) * n1 * W * sizeof(float);
  if (!fixed && n1 == n2) {
    const SymPlan sp = plan_sym(n1, d, W);
    if (sp.ok) b = std::max(b, static_cast<size_t>(sp.Q) * n1 * W * sizeof(float));
  }
  return b;
}

int64_t padded_dim(int64_t d) { return ceil_div(d, 16) * 16; }

int column_mean_f32(const float* X, int64_t n, int64_t d, float* mean, double* part,
                    int64_t part_cap, hipStream_t s) {
  if (n == 0) {
    // a fill kernel, not a memset node, so that the call can be graph-captured
    IGP_TRY(fill_zero<float>(mean, d, s));
    return IGP_OK;
  }
  // ~64 rows per block and 256 threads across the columns: short FP64 chains
  int64_t nblk = std::min<int64_t>(ceil_div(n, 64), std::max<int64_t>(part_cap / d, 1));
  const int64_t rows_per = ceil_div(n, nblk);
  nblk = ceil_div(n, rows_per);
  k_col_partial<<<static_cast<unsigned>(nblk), 256, 0, s>>>(X, n, static_cast<int>(d), rows_per, part);
  k_col_finish<<<static_cast<unsigned>(d), 256, 0, s>>>(part, static_cast<int>(nblk),
                                                         static_cast<int>(d), n, mean);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

int prep_rows_f32(const float* X, int64_t n, int64_t d, const float* centre, float* Xp,
                  float* norms, hipStream_t s) {
  if (n == 0) return IGP_OK;
  k_prep_rows<<<static_cast<unsigned>(ceil_div(n, 256)), 256, 0, s>>>(
      X, n, static_cast<int>(d), static_cast<int>(padded_dim(d)), centre, Xp, norms);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

// Out = os * K(X1, X2) V from prepared (centred, padded) rows; partials in ws.
// whether a per-class FP32 product (n_kp == C) can take the symmetric
// matrix-core kernel: one vector (W = C <= 8), the same point set on both
// sides, a symmetric plan, and a kernel family that path supports
bool mfma_f32_perclass_ok(const KVProblem& p) {
  const int64_t W = p.C * p.nb;
  const bool same = p.X1p ? (p.X1p == p.X2p && p.norm1 == p.norm2) : (p.X1 == p.X2);
  return p.precision == IGP_FP32 && p.n_kp > 1 && p.n_kp == p.C && p.nb == 1 && W <= 8 &&
         same && p.n1 == p.n2 && !p.fixed_split && mfma_f32_supported(p.kp.kind, p.d) &&
         (p.kp.kind == IGP_RBF || p.kp.kind == IGP_MATERN32 || p.kp.kind == IGP_MATERN52) &&
         plan_sym(p.n1, p.d, W).ok;
}

int kv_mfma_f32_launch(const KVProblem& p, const float* X1p, const float* n1p,
                       const float* X2p, const float* n2p, float* P, size_t P_bytes,
                       hipStream_t s, int* nsplit_out) {
  const int64_t W = p.C * p.nb;
  Plan pl = plan_mfma(p.n1, p.n2, p.d, W, p.fixed_split);
  *nsplit_out = pl.nsplit;
  if (static_cast<size_t>(pl.nsplit) * p.n1 * W * sizeof(float) > P_bytes) {
    set_error("kernel-product workspace too small for the split partials");
    return IGP_ENOMEM;
  }
  if (pl.nsplit == 0) return IGP_OK;
  const double inv_l2 = 1.0 / (p.kp.lengthscale * p.kp.lengthscale);
  const float* V = static_cast<const float*>(p.V);
  const int C = static_cast<int>(p.C), Wi = static_cast<int>(W);
  // the same prepared rows on both sides: each pair of rows evaluated once
  const SymPlan sp = (X1p == X2p && n1p == n2p && p.n1 == p.n2 && !p.fixed_split)
                         ? plan_sym(p.n1, p.d, W) : SymPlan{};
  if (p.symmetric_out) *p.symmetric_out = sp.ok ? 1 : 0;
  if (p.n_kp > 1) {
    // one kernel per class: the symmetric kernel's per-class form only
    if (!(sp.ok && p.nb == 1 && p.n_kp == p.C && W <= 8)) {
      set_error("per-class product not supported on the matrix-core path");
      return IGP_EUNSUPPORTED;
    }
    if (static_cast<size_t>(sp.Q) * p.n1 * W * sizeof(float) > P_bytes) {
      set_error("kernel-product workspace too small for the symmetric partials");
      return IGP_ENOMEM;
    }
    *nsplit_out = sp.Q;
    ClassScale cs{};
    for (int w = 0; w < Wi; ++w) {
      cs.il2[w] = static_cast<float>(1.0 / (p.kpc[w].lengthscale * p.kpc[w].lengthscale));
      cs.os[w] = static_cast<float>(p.kpc[w].outputscale);
    }
    const int dch = static_cast<int>(ceil_div(p.d, 16));
    const float k = kv_kappa(p.kp.kind);
    switch (p.kp.kind) {
      case IGP_RBF:
        return launch_sym<IGP_RBF, true>(sp, dch, X1p, n1p, p.n1, V, C, Wi, p.ldv, P, k, -2.0f * k,
                                         p.skip, s, cs);
      case IGP_MATERN32:
        return launch_sym<IGP_MATERN32, true>(sp, dch, X1p, n1p, p.n1, V, C, Wi, p.ldv, P, k,
                                              -2.0f * k, p.skip, s, cs);
      case IGP_MATERN52:
        return launch_sym<IGP_MATERN52, true>(sp, dch, X1p, n1p, p.n1, V, C, Wi, p.ldv, P, k,
                                              -2.0f * k, p.skip, s, cs);
      default:
        set_error("per-class product not supported on the matrix-core path");
        return IGP_EUNSUPPORTED;
    }
  }
  if (sp.ok) {
    if (static_cast<size_t>(sp.Q) * p.n1 * W * sizeof(float) > P_bytes) {
      set_error("kernel-product workspace too small for the symmetric partials");
      return IGP_ENOMEM;
    }
    *nsplit_out = sp.Q;
    const int dch = static_cast<int>(ceil_div(p.d, 16));
    const float k = kv_kappa(p.kp.kind);
    const float cn = static_cast<float>(k * inv_l2), cd = static_cast<float>(-2.0 * k * inv_l2);
    switch (p.kp.kind) {
      case IGP_RBF:
        return launch_sym<IGP_RBF>(sp, dch, X1p, n1p, p.n1, V, C, Wi, p.ldv, P, cn, cd, p.skip, s);
      case IGP_MATERN32:
        return launch_sym<IGP_MATERN32>(sp, dch, X1p, n1p, p.n1, V, C, Wi, p.ldv, P, cn, cd,
                                        p.skip, s);
      case IGP_MATERN52:
        return launch_sym<IGP_MATERN52>(sp, dch, X1p, n1p, p.n1, V, C, Wi, p.ldv, P, cn, cd,
                                        p.skip, s);
      default:
        break;
    }
  }
  switch (p.kp.kind) {
    case IGP_RBF: {
      const float k = kappa<IGP_RBF>();
      return launch_kind<IGP_RBF>(pl, X1p, n1p, X2p, n2p, p.n1, p.n2, V, C, Wi, p.ldv, P,
                                  static_cast<float>(k * inv_l2), static_cast<float>(-2.0 * k * inv_l2),
                                  p.skip, s);
    }
    case IGP_MATERN32: {
      const float k = kappa<IGP_MATERN32>();
      return launch_kind<IGP_MATERN32>(pl, X1p, n1p, X2p, n2p, p.n1, p.n2, V, C, Wi, p.ldv, P,
                                       static_cast<float>(k * inv_l2),
                                       static_cast<float>(-2.0 * k * inv_l2), p.skip, s);
    }
    case IGP_MATERN52: {
      const float k = kappa<IGP_MATERN52>();
      return launch_kind<IGP_MATERN52>(pl, X1p, n1p, X2p, n2p, p.n1, p.n2, V, C, Wi, p.ldv, P,
                                       static_cast<float>(k * inv_l2),
                                       static_cast<float>(-2.0 * k * inv_l2), p.skip, s);
    }
    default:
      set_error("Matern-1/2 runs on the direct-difference kernel");
      return IGP_EUNSUPPORTED;
  }
}

namespace {
template <int KIND, int NS>
void launch_batched_kind(int dch, bool bf, const BatchProblem* dprobs, int np, int64_t ntiles,
                         int* counter, int grid, hipStream_t s) {
  if (bf) {
    kv_batched_persistent<KIND, 1, NS, true><<<grid, 256, 0, s>>>(dprobs, np, ntiles, counter);
    return;
  }
  switch (dch) {
    case 1: kv_batched_persistent<KIND, 1, NS, false><<<grid, 256, 0, s>>>(dprobs, np, ntiles, counter); break;
    default: kv_batched_persistent<KIND, 2, NS, false><<<grid, 256, 0, s>>>(dprobs, np, ntiles, counter); break;
  }
}
}  // namespace

bool batched_supported(int kind, int64_t d, int64_t W) {
  return kind != IGP_MATERN12 && d >= 1 && d <= 32 && W >= 1 && W <= WV;
}

void batched_plan(int64_t n1, int64_t n2, int64_t W, int ns, int64_t split_rows,
                  BatchProblem* bp) {
  const int64_t tiles = ceil_div(n2, TN);
  bp->gx = static_cast<int>(ceil_div(n1, 64 * ns));
  int64_t per = std::max<int64_t>(1, ceil_div(split_rows, TN));
  if (tiles == 0) per = 1;
  bp->cols_per_split = per * TN;
  bp->nsplit = tiles == 0 ? 0 : static_cast<int>(ceil_div(n2, bp->cols_per_split));
  (void)W;
}

bool batched_sym_plan(int64_t n, int64_t d, int64_t W, BatchProblem* bp) {
  const SymPlan sp = plan_sym(n, d, W);
  if (!sp.ok) return false;
  bp->sym_g = sp.G;
  bp->sym_q = sp.Q;
  bp->sym_kb = sp.kb;
  bp->nsplit = sp.Q;
  bp->gx = 0;
  bp->cols_per_split = 0;
  return true;
}

size_t batched_sym_lds(const BatchProblem& bp, int dch) {
  return sym_lds_bytes(dch, bp.W, bp.sym_g);
}

int64_t batched_tiles(const BatchProblem& bp) {
  if (bp.sym_q > 0) return static_cast<int64_t>(bp.sym_q) * (bp.sym_q + 1) / 2;
  return static_cast<int64_t>(bp.gx) * bp.nsplit;
}

namespace {
template <int KIND, int DCH, int KB>
void launch_batched_sym_kb(const SymGroup& g, const BatchProblem* dprobs, int* counter,
                           hipStream_t s) {
  const int grid = static_cast<int>(std::min<int64_t>(g.tiles, 256 * 4));
  const BatchProblem* pr = dprobs + g.first;
  switch (g.W) {
#define IGP_BS(K)                                                                              \
  case K:                                                                                      \
    kv_batched_sym<KIND, DCH, K, KB><<<grid, 256, g.lds, s>>>(pr, g.count, g.tiles, counter);  \
    break;
    IGP_BS(1) IGP_BS(2) IGP_BS(3) IGP_BS(4) IGP_BS(5) IGP_BS(6) IGP_BS(7) IGP_BS(8)
#undef IGP_BS
    default: break;
  }
}

template <int KIND, int DCH>
void launch_batched_sym(const SymGroup& g, const BatchProblem* dprobs, int* counter,
                        hipStream_t s) {
  if constexpr (DCH == 1) {
    if (g.kb == 1) return launch_batched_sym_kb<KIND, 1, 1>(g, dprobs, counter, s);
    if (g.kb == 2) return launch_batched_sym_kb<KIND, 1, 2>(g, dprobs, counter, s);
  }
  launch_batched_sym_kb<KIND, DCH, 4>(g, dprobs, counter, s);
}
}  // namespace

int kv_batched_run(int kind, int dch, int ns, bool bf16, const BatchProblem* dprobs, int np,
                   const SymGroup* groups, int ngroups, int64_t ntiles, int64_t total_out,
                   int* counter, hipStream_t s) {
  // validate the symmetric groups against the table (contiguous from 0)
  int nsym = 0;
  if (ngroups < 0 || ngroups > BATCH_COUNTERS - 1 || (ngroups > 0 && (bf16 || dch > 2))) {
    set_error("batched launch: bad symmetric groups");
    return IGP_EINVAL;
  }
  for (int k = 0; k < ngroups; ++k) {
    const SymGroup& g = groups[k];
    if (g.first != nsym || g.count < 1 || g.W < 1 || g.W > 8 || g.tiles < 1 ||
        g.lds > SYM_MAX_LDS || !(g.kb == 4 || (dch == 1 && (g.kb == 1 || g.kb == 2)))) {
      set_error("batched launch: bad symmetric groups");
      return IGP_EINVAL;
    }
    nsym += g.count;
  }
  if (nsym > np) {
    set_error("batched launch: bad symmetric groups");
    return IGP_EINVAL;
  }
  k_zero_counter<<<1, 64, 0, s>>>(counter);
  for (int k = 0; k < ngroups; ++k) {
    int* ck = counter + 2 * k;
    switch (kind) {
      case IGP_RBF:
        if (dch == 1) launch_batched_sym<IGP_RBF, 1>(groups[k], dprobs, ck, s);
        else launch_batched_sym<IGP_RBF, 2>(groups[k], dprobs, ck, s);
        break;
      case IGP_MATERN32:
        if (dch == 1) launch_batched_sym<IGP_MATERN32, 1>(groups[k], dprobs, ck, s);
        else launch_batched_sym<IGP_MATERN32, 2>(groups[k], dprobs, ck, s);
        break;
      default:
        if (dch == 1) launch_batched_sym<IGP_MATERN52, 1>(groups[k], dprobs, ck, s);
        else launch_batched_sym<IGP_MATERN52, 2>(groups[k], dprobs, ck, s);
        break;
    }
  }
  // the one-sided problems: their own queue counter (the last) and tile prefixes
  const BatchProblem* oprobs = dprobs + nsym;
  const int onp = np - nsym;
  int* c1 = counter + 2 * (BATCH_COUNTERS - 1);
  if (ntiles > 0 && onp > 0) {
    const int grid = static_cast<int>(std::min<int64_t>(ntiles, 256 * 4));
    if (ns == 1) {
      switch (kind) {
        case IGP_RBF: launch_batched_kind<IGP_RBF, 1>(dch, bf16, oprobs, onp, ntiles, c1, grid, s); break;
        case IGP_MATERN32: launch_batched_kind<IGP_MATERN32, 1>(dch, bf16, oprobs, onp, ntiles, c1, grid, s); break;
        default: launch_batched_kind<IGP_MATERN52, 1>(dch, bf16, oprobs, onp, ntiles, c1, grid, s); break;
      }
    } else {
      switch (kind) {
        case IGP_RBF: launch_batched_kind<IGP_RBF, 2>(dch, bf16, oprobs, onp, ntiles, c1, grid, s); break;
        case IGP_MATERN32: launch_batched_kind<IGP_MATERN32, 2>(dch, bf16, oprobs, onp, ntiles, c1, grid, s); break;
        default: launch_batched_kind<IGP_MATERN52, 2>(dch, bf16, oprobs, onp, ntiles, c1, grid, s); break;
      }
    }
  }
  if (total_out > 0) {
    const int blocks = static_cast<int>(std::min<int64_t>(ceil_div(total_out, 256), 4096));
    kv_reduce_batched<<<blocks, 256, 0, s>>>(dprobs, np, total_out);
  }
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

}  // namespace igp
