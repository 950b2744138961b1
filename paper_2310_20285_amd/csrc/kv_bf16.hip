// Fused kernel-matrix product with the distance GEMM on the BF16 matrix cores
// of gfx950 (v_mfma_f32_16x16x32_bf16, FP32 accumulation), for wide inputs
// (hundreds of features).
//
// Inputs are rows centred on a common point and rounded to BF16; their squared
// norms are taken from the rounded values in FP32, so r^2 = |x1|^2 + |x2|^2 -
// 2 x1.x2 is the distance of the rounded points up to FP32 accumulation and the
// kernel matrix stays the (PSD) kernel matrix of those points.
//
// Workgroup tile: 256 rows of X1 (n) x 256 rows of X2 (m), eight waves in a
// 2 (m) x 4 (n) arrangement, each holding a 128 x 64 block of D^T = X2 X1^T in
// 32 accumulators of 16 x 16.  Feature chunks of 32 stream through LDS (rows
// padded to 80 bytes: conflict-free 128-bit fragment reads), double-buffered,
// each chunk loaded into registers one iteration ahead and written to LDS
// while the previous chunk is multiplied; the loads are branch-free (rows past the end are clamped
// to the last row: their products meet V = 0 or are never stored).  After the
// feature loop the kernel function is applied to the accumulators and the
// contraction with V runs on the same matrix cores: the accumulator of block
// (m, n) already holds K[n][m] in the A-operand lane layout (the
// transposed-tile arrangement), and a pair of m-blocks gives the 8 k-values of
// one 16x16x32 instruction.  K and V are split into BF16 high and low parts
// and the contraction takes hi*hi + hi*lo + lo*hi, which keeps about 16
// significant bits of each factor.  In the split-input mode (X3) the distance
// loop runs three phases (see dist_tile) and K and V are split into three BF16
// parts h + m + l (about 24 bits, the FP32 significand); the contraction takes
// the six products of combined order up to two, hh + hm + mh + hl + mm + lh.
//
// The grid is one-dimensional and remapped so that the workgroups the hardware
// deals to one XCD (ids congruent mod 8) take consecutive tiles: the same X2
// range with neighbouring X1 blocks, which then share that XCD's L2.
#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "ops.hpp"

namespace igp {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

namespace {

constexpr float LOG2E_B = 1.4426950408889634f;
constexpr int KC = 32;       // features per chunk
constexpr int RS = 40;       // LDS row stride in bf16 (80 bytes)
constexpr int VT = 16;       // output columns per workgroup

template <int KIND>
__device__ inline float kt_bf(float t) {
  if constexpr (KIND == IGP_RBF) {
    return __builtin_amdgcn_exp2f(-t);
  } else {
    const float a = __builtin_amdgcn_sqrtf(fmaxf(t, 0.0f));
    const float e = __builtin_amdgcn_exp2f(-a);
    if constexpr (KIND == IGP_MATERN12) {
      return e;
    } else if constexpr (KIND == IGP_MATERN32) {
      return __builtin_fmaf(a, 1.0f / LOG2E_B, 1.0f) * e;
    } else {
      const float p = __builtin_fmaf(t, 1.0f / (3.0f * LOG2E_B * LOG2E_B), 1.0f);
      return __builtin_fmaf(a, 1.0f / LOG2E_B, p) * e;
    }
  }
}

__device__ inline __bf16 to_bf(float x) { return static_cast<__bf16>(x); }
__device__ inline float from_bf(__bf16 x) { return static_cast<float>(x); }

typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));
typedef unsigned u4w __attribute__((ext_vector_type(4)));
// BF16 high and low parts of two values, each pair packed in one 32-bit word
// (element 0 in the low half): hi = RNE(x), lo = RNE(x - hi), where x - hi is
// exact (hi lies within a factor of two of x).  One packed conversion per pair
// for each part; the high parts are widened back by shift and mask.
__device__ inline void split2_pk(float a, float b, unsigned& hi, unsigned& lo) {
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector(f2v{a, b}, b2v));
  const float ha = __builtin_bit_cast(float, hi << 16);
  const float hb = __builtin_bit_cast(float, hi & 0xffff0000u);
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(f2v{a - ha, b - hb}, b2v));
}

// x = h + m + l to about 2^-24 |x| (three BF16 parts)
__device__ inline void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = to_bf(x);
  const float r = x - from_bf(h);
  m = to_bf(r);
  l = to_bf(r - from_bf(m));
}
// the same into element i of three register vectors
__device__ inline void split3_at(float x, bf8& h, bf8& m, bf8& l, int i) {
  const __bf16 a = to_bf(x);
  const float r = x - from_bf(a);
  const __bf16 b = to_bf(r);
  h[i] = a;
  m[i] = b;
  l[i] = to_bf(r - from_bf(b));
}

// out += the product of (kh, km, kl) and (vh, vm, vl) to combined order two;
// with X3 false only hh + hl + lh of the two-part splits (k*, v* with * = h, l)
template <bool X3>
__device__ inline f4 contract(const bf8& kh, const bf8& km, const bf8& kl, const bf8& vh,
                              const bf8& vm, const bf8& vl, f4 out) {
  if constexpr (X3) {
    out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, vl, out, 0, 0, 0);
    out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(km, vm, out, 0, 0, 0);
    out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kl, vh, out, 0, 0, 0);
    out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, vm, out, 0, 0, 0);
    out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(km, vh, out, 0, 0, 0);
    out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, vh, out, 0, 0, 0);
  } else {
    out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, vh, out, 0, 0, 0);
    out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, vl, out, 0, 0, 0);
    out = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kl, vh, out, 0, 0, 0);
  }
  return out;
}

constexpr int WM = 2, WN = 4;          // waves along m and n
constexpr int TMW = 128, TNW = 64;     // rows of m and n per wave
constexpr int BM = WM * TMW;           // X2 rows per tile (256)
constexpr int BN = WN * TNW;           // X1 rows per workgroup (256)
constexpr int NT = 64 * WM * WN;       // threads per workgroup (512)
constexpr int MB = TMW / 16, NB = TNW / 16;
constexpr int VS = BM + 8;             // LDS row stride of the transposed V tile (bf16)
constexpr int QA = BM * 4 / NT, QB = BN * 4 / NT;   // 16-byte pieces staged per thread
static_assert(NT % VT == 0 && BM % (NT / VT) == 0 && NT >= BM,
              "each thread stages one fixed column of the V^T tiles and one X2 norm");

// D^T of one (X2 tile, X1 block) pair for this wave: acc[mb][nb][v] =
// sum_k X2[m0 + wm TMW + mb 16 + 4g + v][k] X1[n0 + wn TNW + nb 16 + r][k].
// With nph = 3 (inputs split into BF16 high and low parts, X = H + L) the
// feature loop runs three phases, H2.H1 + H2.L1 + L2.H1: the chunk index
// selects the phase's pair of row arrays, so the same pipeline streams 3 DPB
// features.
// Feature chunks of KC stream through the double-buffered LDS tiles sA / sB
// ([2][BM RS] and [2][BN RS]); chunk ks+1 (loaded during the previous
// iteration) goes to the other buffer before the products of chunk ks, so its
// LDS writes overlap them, and the loads of chunk ks+2 are issued right after.
// Rows past the end are clamped to the last row (their products meet V = 0 or
// are never stored).  Ends with a barrier: the buffers may be reused.
__device__ __forceinline__ void dist_tile(f4 (&acc)[MB][NB], __bf16* __restrict__ sA,
                                          __bf16* __restrict__ sB,
                                          const __bf16* __restrict__ X1b,
                                          const __bf16* __restrict__ X2b,
                                          const __bf16* __restrict__ X1l,
                                          const __bf16* __restrict__ X2l, int nph, int64_t n0,
                                          int64_t n1, int64_t m0, int64_t m_end, int DPB, int tid,
                                          int wm, int wn, int g, int r) {
  u4 pa[QA], pb[QB];
  const int cpp = DPB / KC;   // chunks per phase
  auto fetch = [&](int kc) {
    const int ph = kc / cpp;
    const int k0 = (kc - ph * cpp) * KC;
    const __bf16* A2 = ph == 2 ? X2l : X2b;   // phase 0: H2.H1, 1: H2.L1, 2: L2.H1
    const __bf16* B1 = ph == 1 ? X1l : X1b;
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * NT;
      const int64_t m = m0 + (e >> 2) < m_end ? m0 + (e >> 2) : m_end - 1;
      pa[q] = *reinterpret_cast<const u4*>(A2 + m * DPB + k0 + (e & 3) * 8);
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * NT;
      const int64_t n = n0 + (e >> 2) < n1 ? n0 + (e >> 2) : n1 - 1;
      pb[q] = *reinterpret_cast<const u4*>(B1 + n * DPB + k0 + (e & 3) * 8);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = tid + q * NT;
      *reinterpret_cast<u4*>(&sA[buf * BM * RS + (e >> 2) * RS + (e & 3) * 8]) = pa[q];
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int e = tid + q * NT;
      *reinterpret_cast<u4*>(&sB[buf * BN * RS + (e >> 2) * RS + (e & 3) * 8]) = pb[q];
    }
  };
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4{0, 0, 0, 0};
  const int nks = cpp * nph;
  fetch(0);
  stash(0);
  __syncthreads();
  if (nks > 1) fetch(1);
  int buf = 0;
  for (int ks = 0; ks < nks; ++ks) {
    if (ks + 1 < nks) stash(buf ^ 1);
    if (ks + 2 < nks) fetch(ks + 2);
    bf8 b[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      b[nb] = *reinterpret_cast<const bf8*>(&sB[buf * BN * RS + (wn * TNW + nb * 16 + r) * RS + g * 8]);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const bf8 a = *reinterpret_cast<const bf8*>(&sA[buf * BM * RS + (wm * TMW + mb * 16 + r) * RS + g * 8]);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nb], acc[mb][nb], 0, 0, 0);
    }
    __syncthreads();
    buf ^= 1;
  }
}

template <int KIND, bool X3>
__global__ void __launch_bounds__(NT)
kv_bf16_kernel(const __bf16* __restrict__ X1b, const float* __restrict__ nrm1,
               const __bf16* __restrict__ X2b, const float* __restrict__ nrm2,
               const __bf16* __restrict__ X1l, const __bf16* __restrict__ X2l, int nph,
               int64_t n1, int64_t n2, int DPB, const float* __restrict__ V, int C, int W,
               int64_t ldv,
               float* __restrict__ P, int64_t cols_per_split, int gx, int nsplit, float cnorm,
               float cdot, const int* skip) {
  if (gate_closed(skip)) return;
  __shared__ __align__(16) __bf16 sA[2][BM * RS];   // X2 chunk (m rows)
  __shared__ __align__(16) __bf16 sB[2][BN * RS];   // X1 chunk (n rows)
  __shared__ __align__(16) __bf16 sVh[VT * VS];     // V^T tile, high part
  __shared__ __align__(16) __bf16 sVl[VT * VS];     // V^T tile, low part
  __shared__ __align__(16) __bf16 sVm[X3 ? VT * VS : 8];   // middle part (X3)
  __shared__ __align__(16) float sN2[BM];

  // ids congruent mod 8 run on one XCD: give each XCD a contiguous tile range
  const int nwg = gridDim.x, bid = blockIdx.x;
  const int xcd = bid & 7, loc = bid >> 3;
  const int per = (nwg + 7) >> 3, rem = nwg & 7;
  const int lin = (rem == 0 || xcd < rem) ? xcd * per + loc
                                          : rem * per + (xcd - rem) * (per - 1) + loc;
  const int bx = lin % gx;
  const int by = (lin / gx) % nsplit;
  const int bz = lin / gx / nsplit;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int wn = wave % WN, wm = wave / WN;
  const int64_t n0 = static_cast<int64_t>(bx) * BN;
  const int w0 = bz * VT;
  const int64_t m_begin = static_cast<int64_t>(by) * cols_per_split;
  const int64_t m_end = m_begin + cols_per_split < n2 ? m_begin + cols_per_split : n2;
  // this lane's X1 norms: n = n0 + wn*TNW + nb*16 + r
  float n1v[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int64_t n = n0 + wn * TNW + nb * 16 + r;
    n1v[nb] = n < n1 ? nrm1[n] * cnorm : 0.0f;
  }
  f4 out[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) out[nb] = f4{0, 0, 0, 0};

  // this thread stages column wl = tid % VT of V^T at every step (NT is a
  // multiple of VT): its offset in V, (w / C) ldv + w % C, is computed once
  const int wl = tid % VT, w = w0 + wl;
  const int64_t voff = w < W ? static_cast<int64_t>(w / C) * ldv + (w % C) : -1;
  for (int64_t m0 = m_begin; m0 < m_end; m0 += BM) {
    // V^T tile (hi / lo) and X2 norms of this m tile; V = 0 past the end
    for (int m = tid / VT; m < BM; m += NT / VT) {
      const int64_t gm = m0 + m;
      float v = 0.0f;
      if (gm < m_end && voff >= 0) v = V[voff + gm * C];
      if constexpr (X3) {
        split3(v, sVh[wl * VS + m], sVm[wl * VS + m], sVl[wl * VS + m]);
      } else {
        const __bf16 hi = to_bf(v);
        sVh[wl * VS + m] = hi;
        sVl[wl * VS + m] = to_bf(v - from_bf(hi));
      }
    }
    for (int e = tid; e < BM; e += NT) {
      const int64_t gm = m0 + e;
      sN2[e] = gm < m_end ? nrm2[gm] * cnorm : 0.0f;
    }
    f4 acc[MB][NB];
    dist_tile(acc, &sA[0][0], &sB[0][0], X1b, X2b, X1l, X2l, nph, n0, n1, m0, m_end, DPB, tid,
              wm, wn, g, r);
    // kernel transform + contraction: acc[mb][nb][v] = D^T[m = wm*TMW + mb*16 + 4g + v][n = .. + r]
#pragma unroll
    for (int p = 0; p < MB / 2; ++p) {
      const int mba = 2 * p, mbb = 2 * p + 1;
      const int ma = wm * TMW + mba * 16 + 4 * g, mbm = wm * TMW + mbb * 16 + 4 * g;
      const f4 na = *reinterpret_cast<const f4*>(&sN2[ma]);
      const f4 nbv = *reinterpret_cast<const f4*>(&sN2[mbm]);
      bf8 vh, vl, vm;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        vh[t] = sVh[r * VS + ma + t];
        vl[t] = sVl[r * VS + ma + t];
        vh[4 + t] = sVh[r * VS + mbm + t];
        vl[4 + t] = sVl[r * VS + mbm + t];
        if constexpr (X3) {
          vm[t] = sVm[r * VS + ma + t];
          vm[4 + t] = sVm[r * VS + mbm + t];
        }
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        bf8 kh, kl, km;
        float ka[4], kb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          ka[t] = kt_bf<KIND>(__builtin_fmaf(acc[mba][nb][t], cdot, n1v[nb] + na[t]));
          kb[t] = kt_bf<KIND>(__builtin_fmaf(acc[mbb][nb][t], cdot, n1v[nb] + nbv[t]));
          if constexpr (X3) {
            split3_at(ka[t], kh, km, kl, t);
            split3_at(kb[t], kh, km, kl, 4 + t);
          }
        }
        if constexpr (!X3) {
          unsigned h[4], l[4];
          split2_pk(ka[0], ka[1], h[0], l[0]);
          split2_pk(ka[2], ka[3], h[1], l[1]);
          split2_pk(kb[0], kb[1], h[2], l[2]);
          split2_pk(kb[2], kb[3], h[3], l[3]);
          kh = __builtin_bit_cast(bf8, u4w{h[0], h[1], h[2], h[3]});
          kl = __builtin_bit_cast(bf8, u4w{l[0], l[1], l[2], l[3]});
        }
        out[nb] = contract<X3>(kh, km, kl, vh, vm, vl, out[nb]);
      }
    }
    __syncthreads();   // sV* / sN2 / sA / sB are rewritten by the next m tile
  }
  // out[nb][j] = Out[n = n0 + wn*TNW + nb*16 + 4g + j][w = w0 + r]; add the WM wave rows
  // in LDS (sA is free after the last m tile)
  f4* red = reinterpret_cast<f4*>(&sA[0][0]);
  static_assert(WN * NB * 64 * sizeof(f4) <= sizeof(sA[0]), "reduction fits in one A buffer");
#pragma unroll
  for (int s = 1; s < WM; ++s) {
    if (wm == s) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) red[(wn * NB + nb) * 64 + lane] = out[nb];
    }
    __syncthreads();
    if (wm == 0) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) out[nb] += red[(wn * NB + nb) * 64 + lane];
    }
    __syncthreads();
  }
  if (wm == 0) {
    const int w = w0 + r;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t n = n0 + wn * TNW + nb * 16 + 4 * g + j;
        if (n < n1 && w < W) P[(static_cast<int64_t>(by) * n1 + n) * W + w] = out[nb][j];
      }
  }
}

// ---- symmetric product K(X, X) V -------------------------------------------
// With the same rows on both sides every kernel value serves Out[n] += k V[m]
// and Out[m] += k V[n], so each unordered pair (s, u >= s) of 256-row blocks is
// one workgroup and the distance tile -- the bulk of the work at hundreds of
// features -- is computed once.  After the tile and the kernel transform:
//   direct      as in kv_bf16_kernel (K in the A-operand layout, V of the
//               u rows as B), partial of rows in block s -> slot u;
//   transposed  Out[m][w] = sum_n V[n][w] K[n][m]: the MFMA needs 8
//               consecutive n per lane at fixed m, the transpose of the
//               accumulator layout, so each wave writes the hi / lo parts of
//               its K values for one pair of m-blocks to a private LDS scratch
//               [m][n] and reads them back as the B operand (V of the s rows,
//               stored [w][n], is A); the four waves that share the m rows
//               are added in wave order; partial of rows in block u -> slot s.
// The pair (s, s) takes only the direct sum.  Every row thus has exactly Q
// slots, each written once, reduced in slot order by kv_reduce.
constexpr int TS = TNW + 8;               // row stride (bf16) of the transpose scratch [m][n]
constexpr int TWAVE = 2 * 32 * TS;        // scratch per wave: hi and lo of 32 m rows
constexpr int TSF = TNW + 4;              // row stride of the FP32 scratch of the X3 mode
static_assert(32 * TSF * 2 <= TWAVE, "the FP32 transpose scratch fits in a wave's share");
// plain mode: the scratch holds K as [n][m] (64 n rows of 32 m + 4 padding),
// written 4 consecutive m at a time and read back transposed
constexpr int TRS = 36;
static_assert(TNW * TRS == 32 * TS, "the [n][m] scratch takes the hi part's share");
typedef __bf16 bf4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

// B operand of a 16x16x32 MFMA from a [n][m] BF16 scratch: lane (g, r) gets
// S[n0 + 8g + k][m0 + r] for k < 8.  ds_read_b64_tr_b16 hands output lane j of
// each 16-lane group element (j mod 4) of the 8-byte piece that lane
// 4k + j/4 addressed, for k < 4; so lane i of the group addresses
// S[nbase + i/4][m0 + 4 (i mod 4)], nbase = n0 + 8g (then + 4).
__device__ inline bf8 read_tr_b(const __bf16* S, int n0, int m0, int g, int r) {
  const __bf16* p0 = S + (n0 + 8 * g + (r >> 2)) * TRS + m0 + 4 * (r & 3);
  const s4v lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (__attribute__((address_space(3))) s4v*)(p0));
  const s4v hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (__attribute__((address_space(3))) s4v*)(p0 + 4 * TRS));
  const bf4v blo = __builtin_bit_cast(bf4v, lo), bhi = __builtin_bit_cast(bf4v, hi);
  return bf8{blo[0], blo[1], blo[2], blo[3], bhi[0], bhi[1], bhi[2], bhi[3]};
}
// Pair index -> block pair (s <= u) in bands of SYM_BAND s-blocks: inside a
// band the triangle u < s0 + SYM_BAND first, then u ascending with s the
// fastest index.  The ~32 workgroups an XCD runs at once then share a few s
// and u blocks in its L2 (in row order they would share one s block and each
// bring its own u block).  A bijection onto the pairs s <= u.
constexpr int SYM_BAND = 16;
__device__ inline void band_pair(int Q, int lin, int* sb, int* ub) {
  int s0 = 0, Sb = 1;
  for (;;) {
    Sb = SYM_BAND < Q - s0 ? SYM_BAND : Q - s0;
    if (Sb <= 0) {   // lin beyond the Q (Q + 1) / 2 pairs: no pair
      *sb = *ub = -1;
      return;
    }
    const int cnt = Sb * (Q - s0) - Sb * (Sb - 1) / 2;
    if (lin < cnt) break;
    lin -= cnt;
    s0 += Sb;
  }
  const int tri = Sb * (Sb + 1) / 2;
  if (lin < tri) {
    int k = 0;
    while ((k + 1) * (k + 2) / 2 <= lin) ++k;
    *sb = s0 + lin - k * (k + 1) / 2;
    *ub = s0 + k;
  } else {
    const int t = lin - tri;
    *sb = s0 + t % Sb;
    *ub = s0 + Sb + t / Sb;
  }
}

static_assert(WM == 2, "the direct reduction adds the second wave row to the first");
static_assert(WM * WN * TWAVE <= 2 * (BM + BN) * RS, "transpose scratch fits in the chunk buffers");
static_assert(WM * WN * MB * 64 * 16 + WN * NB * 64 * 16 <= 2 * (BM + BN) * RS * 2,
              "reduction buffers fit in the chunk buffers");

template <int KIND, bool X3>
__global__ void __launch_bounds__(NT)
kv_bf16_sym(const __bf16* __restrict__ Xb, const float* __restrict__ nrm,
            const __bf16* __restrict__ Xl, int nph, int64_t n, int DPB,
            const float* __restrict__ V, int C, int W, int64_t ldv, float* __restrict__ P, int Q,
            float cnorm, float cdot, const int* skip) {
  if (gate_closed(skip)) return;
  __shared__ __align__(16) __bf16 sAB[2 * (BM + BN) * RS];   // chunks, then scratch
  __shared__ __align__(16) __bf16 sVh[VT * VS];     // V^T of the u rows (m), high part
  __shared__ __align__(16) __bf16 sVl[VT * VS];     // ... low part
  __shared__ __align__(16) __bf16 sUh[VT * VS];     // V^T of the s rows (n), high part
  __shared__ __align__(16) __bf16 sUl[VT * VS];     // ... low part
  __shared__ __align__(16) __bf16 sVm[X3 ? VT * VS : 8];   // middle parts (X3)
  __shared__ __align__(16) __bf16 sUm[X3 ? VT * VS : 8];
  __shared__ __align__(16) float sN2[BM];

  // ids congruent mod 8 run on one XCD: give each XCD a contiguous range of pairs
  const int nwg = gridDim.x, bid = blockIdx.x;
  const int xcd = bid & 7, loc = bid >> 3;
  const int per = (nwg + 7) >> 3, rem = nwg & 7;
  const int lin = (rem == 0 || xcd < rem) ? xcd * per + loc
                                          : rem * per + (xcd - rem) * (per - 1) + loc;
  int sb, ub;
  band_pair(Q, lin, &sb, &ub);
  if (sb < 0) return;
  const bool diag = ub == sb;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int wn = wave % WN, wm = wave / WN;
  const int64_t n0 = static_cast<int64_t>(sb) * BN;
  const int64_t m0 = static_cast<int64_t>(ub) * BM;
  const int64_t m_end = m0 + BM < n ? m0 + BM : n;

  float n1v[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int64_t row = n0 + wn * TNW + nb * 16 + r;
    n1v[nb] = row < n ? nrm[row] * cnorm : 0.0f;
  }
  // V of the u rows and, off the diagonal, of the s rows (V = 0 past the end),
  // and the X2 norms of the u rows: loaded before the feature loop, so that
  // their latency overlaps its first chunks, and split into the V^T tiles
  // (hi / lo, or three parts) in LDS after it.  This thread stages column
  // w = tid % VT at every step (NT is a multiple of VT): its offset in V is
  // computed once.
  constexpr int VROWS = BM / (NT / VT);   // V rows per thread
  const int w = tid % VT;
  const int64_t voff = w < W ? static_cast<int64_t>(w / C) * ldv + (w % C) : -1;
  float vreg[VROWS], xreg[VROWS];
#pragma unroll
  for (int k = 0; k < VROWS; ++k) {
    const int m = tid / VT + k * (NT / VT);
    vreg[k] = (m0 + m < n && voff >= 0) ? V[voff + (m0 + m) * C] : 0.0f;
    xreg[k] = (!diag && n0 + m < n && voff >= 0) ? V[voff + (n0 + m) * C] : 0.0f;
  }
  const float nreg = (tid < BM && m0 + tid < n) ? nrm[m0 + tid] * cnorm : 0.0f;

  f4 acc[MB][NB];
  dist_tile(acc, sAB, sAB + 2 * BM * RS, Xb, Xb, Xl, Xl, nph, n0, n, m0, m_end, DPB, tid, wm,
            wn, g, r);
#pragma unroll
  for (int k = 0; k < VROWS; ++k) {
    const int m = tid / VT + k * (NT / VT);
    const float v = vreg[k], x = xreg[k];
    if constexpr (X3) {
      split3(v, sVh[w * VS + m], sVm[w * VS + m], sVl[w * VS + m]);
      split3(x, sUh[w * VS + m], sUm[w * VS + m], sUl[w * VS + m]);
    } else {
      const __bf16 vh = to_bf(v), xh = to_bf(x);
      sVh[w * VS + m] = vh;
      sVl[w * VS + m] = to_bf(v - from_bf(vh));
      sUh[w * VS + m] = xh;
      sUl[w * VS + m] = to_bf(x - from_bf(xh));
    }
  }
  if (tid < BM) sN2[tid] = nreg;
  __syncthreads();

  __bf16* Th = sAB + wave * TWAVE;     // this wave's transpose scratch, [32 m][TS]
  __bf16* Tl = Th + 32 * TS;
  float* Tf = reinterpret_cast<float*>(Th);   // X3: K values in FP32, [32 m][TSF]
  f4 out[NB], out2[MB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) out[nb] = f4{0, 0, 0, 0};
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) out2[mb] = f4{0, 0, 0, 0};
  // acc[mb][nb][v] = D^T[m = wm*TMW + mb*16 + 4g + v][n = wn*TNW + nb*16 + r]
#pragma unroll
  for (int p = 0; p < MB / 2; ++p) {
    const int mba = 2 * p, mbb = 2 * p + 1;
    const int ma = wm * TMW + mba * 16 + 4 * g, mbm = wm * TMW + mbb * 16 + 4 * g;
    const f4 na = *reinterpret_cast<const f4*>(&sN2[ma]);
    const f4 nbv = *reinterpret_cast<const f4*>(&sN2[mbm]);
    bf8 vh, vl, vm;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      vh[t] = sVh[r * VS + ma + t];
      vl[t] = sVl[r * VS + ma + t];
      vh[4 + t] = sVh[r * VS + mbm + t];
      vl[4 + t] = sVl[r * VS + mbm + t];
      if constexpr (X3) {
        vm[t] = sVm[r * VS + ma + t];
        vm[4 + t] = sVm[r * VS + mbm + t];
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      bf8 kh, kl, km;
      float kf[8];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float ka = kt_bf<KIND>(__builtin_fmaf(acc[mba][nb][t], cdot, n1v[nb] + na[t]));
        const float kb = kt_bf<KIND>(__builtin_fmaf(acc[mbb][nb][t], cdot, n1v[nb] + nbv[t]));
        kf[t] = ka;
        kf[4 + t] = kb;
        if constexpr (X3) {
          split3_at(ka, kh, km, kl, t);
          split3_at(kb, kh, km, kl, 4 + t);
        }
      }
      if constexpr (!X3) {
        unsigned h[4], l[4];
        split2_pk(kf[0], kf[1], h[0], l[0]);
        split2_pk(kf[2], kf[3], h[1], l[1]);
        split2_pk(kf[4], kf[5], h[2], l[2]);
        split2_pk(kf[6], kf[7], h[3], l[3]);
        kh = __builtin_bit_cast(bf8, u4w{h[0], h[1], h[2], h[3]});
        kl = __builtin_bit_cast(bf8, u4w{l[0], l[1], l[2], l[3]});
      }
      out[nb] = contract<X3>(kh, km, kl, vh, vm, vl, out[nb]);
      if (!diag) {
        if constexpr (X3) {
          // K[n = nb*16 + r][m = sub*16 + 4g + t] -> FP32 scratch row m, column n
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int row = (t >> 2) * 16 + 4 * g + (t & 3);
            Tf[row * TSF + nb * 16 + r] = kf[t];
          }
        } else {
          // row n = nb*16 + r of the [n][m] scratch, m = 4g..4g+3 and 16+4g..16+4g+3
          __bf16* rh = Th + (nb * 16 + r) * TRS + 4 * g;
          __bf16* rl = Tl + (nb * 16 + r) * TRS + 4 * g;
          *reinterpret_cast<bf4v*>(rh) = bf4v{kh[0], kh[1], kh[2], kh[3]};
          *reinterpret_cast<bf4v*>(rh + 16) = bf4v{kh[4], kh[5], kh[6], kh[7]};
          *reinterpret_cast<bf4v*>(rl) = bf4v{kl[0], kl[1], kl[2], kl[3]};
          *reinterpret_cast<bf4v*>(rl + 16) = bf4v{kl[4], kl[5], kl[6], kl[7]};
        }
      }
    }
    if (!diag) {
#pragma unroll
      for (int sub = 0; sub < 2; ++sub)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const int col = ks * 32 + 8 * g;
          f4& o = out2[2 * p + sub];
          const bf8 ah = *reinterpret_cast<const bf8*>(&sUh[r * VS + wn * TNW + col]);
          const bf8 al = *reinterpret_cast<const bf8*>(&sUl[r * VS + wn * TNW + col]);
          if constexpr (X3) {
            const bf8 am = *reinterpret_cast<const bf8*>(&sUm[r * VS + wn * TNW + col]);
            const f4 k0 = *reinterpret_cast<const f4*>(&Tf[(sub * 16 + r) * TSF + col]);
            const f4 k1 = *reinterpret_cast<const f4*>(&Tf[(sub * 16 + r) * TSF + col + 4]);
            bf8 bh, bm, bl;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              split3_at(k0[t], bh, bm, bl, t);
              split3_at(k1[t], bh, bm, bl, 4 + t);
            }
            o = contract<true>(ah, am, al, bh, bm, bl, o);
          } else {
            const bf8 bh = read_tr_b(Th, ks * 32, sub * 16, g, r);
            const bf8 bl = read_tr_b(Tl, ks * 32, sub * 16, g, r);
            o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, o, 0, 0, 0);
            o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, o, 0, 0, 0);
            o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, o, 0, 0, 0);
          }
        }
    }
  }
  // out[nb][j]  = direct sum for n = n0 + wn*TNW + nb*16 + 4g + j, w = r (add the WM wave rows);
  // out2[mb][j] = transposed sum for w = 4g + j, m = m0 + wm*TMW + mb*16 + r (add the WN wave
  // columns).  Both reductions go through the chunk buffers.
  f4* red2 = reinterpret_cast<f4*>(sAB);                       // [wave][mb][lane]
  f4* red1 = red2 + WM * WN * MB * 64;                         // [wn][nb][lane]
  __syncthreads();
  if (!diag) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) red2[(wave * MB + mb) * 64 + lane] = out2[mb];
  }
  if (wm == 1) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) red1[(wn * NB + nb) * 64 + lane] = out[nb];
  }
  __syncthreads();
  if (!diag) {
    // wave (wm, wn) writes m-blocks 2 wn and 2 wn + 1 of its wm rows
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int mb = 2 * wn + q;
      f4 x = red2[((wm * WN + 0) * MB + mb) * 64 + lane];
#pragma unroll
      for (int k = 1; k < WN; ++k) x += red2[((wm * WN + k) * MB + mb) * 64 + lane];
      const int64_t m = m0 + wm * TMW + mb * 16 + r;
      if (m < n) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int w = 4 * g + j;
          if (w < W) P[(static_cast<int64_t>(sb) * n + m) * W + w] = x[j];
        }
      }
    }
  }
  if (wm == 0) {
    const int w = r;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const f4 x = out[nb] + red1[(wn * NB + nb) * 64 + lane];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t row = n0 + wn * TNW + nb * 16 + 4 * g + j;
        if (row < n && w < W) P[(static_cast<int64_t>(ub) * n + row) * W + w] = x[j];
      }
    }
  }
}

// Centred rows rounded to BF16 (zero-padded to DPB features) and the squared
// norms of the rounded rows.  With Xl (split mode) the low parts
// l = bf16(x - h) go to Xl and the norms are those of h + l.
__global__ void k_prep_rows_bf16(const float* __restrict__ X, int64_t n, int d, int DPB,
                                 const float* __restrict__ centre, __bf16* __restrict__ Xb,
                                 __bf16* __restrict__ Xl, float* __restrict__ norms) {
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  __shared__ float red[4];
  float s = 0.0f;
  for (int k = threadIdx.x; k < DPB; k += blockDim.x) {
    float v = 0.0f;
    if (k < d) v = X[i * d + k] - (centre ? centre[k] : 0.0f);
    const __bf16 b = static_cast<__bf16>(v);
    Xb[i * DPB + k] = b;
    float fb = static_cast<float>(b);
    if (Xl) {
      const __bf16 l = static_cast<__bf16>(v - fb);
      Xl[i * DPB + k] = l;
      fb += static_cast<float>(l);
    }
    s += fb * fb;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) norms[i] = s;
}

struct PlanB {
  int gx, gz, nsplit;
  int64_t cols_per_split;
};

PlanB plan_bf16(int64_t n1, int64_t n2, int64_t W, bool fixed = false) {
  static_assert(FIXED_SPLIT_ROWS % BM == 0, "fixed split is a whole number of tiles");
  PlanB p{};
  p.gx = static_cast<int>(ceil_div(n1, BN));
  p.gz = static_cast<int>(ceil_div(W, VT));
  const int64_t tiles = ceil_div(n2, BM);
  if (tiles == 0) {
    p.nsplit = 0;
    p.cols_per_split = BM;
    return p;
  }
  // about 16 workgroups per CU (one resident at a time), without splitting
  // below 4 tiles
  int64_t want = ceil_div(4096, static_cast<int64_t>(p.gx) * p.gz);
  want = std::max<int64_t>(1, std::min<int64_t>(want, ceil_div(tiles, 4)));
  p.cols_per_split = fixed ? FIXED_SPLIT_ROWS : ceil_div(tiles, want) * BM;
  p.nsplit = static_cast<int>(ceil_div(n2, p.cols_per_split));
  return p;
}

}  // namespace

int64_t bf16_padded_dim(int64_t d) { return ceil_div(d, KC) * KC; }

namespace {
// blocks of the symmetric launch (partial slots per row); beyond the cap the
// slots would take several times the one-sided plan's memory and that plan runs
constexpr int64_t SYM_BF_MAX_Q = 256;

int64_t sym_blocks(int64_t n, int64_t W) {
  const int64_t q = ceil_div(n, BN);
  return (W >= 1 && W <= VT && q >= 1 && q <= SYM_BF_MAX_Q) ? q : 0;
}
}  // namespace

size_t bf16_partial_bytes(int64_t n1, int64_t n2, int64_t W, bool fixed) {
  PlanB pl = plan_bf16(n1, n2, W, fixed);
  size_t b = static_cast<size_t>(pl.nsplit) * n1 * W * sizeof(float);
  if (!fixed && n1 == n2)
    b = std::max(b, static_cast<size_t>(sym_blocks(n1, W)) * n1 * W * sizeof(float));
  // the narrow tile's plan (taken for few features; sized whatever the kernel)
  if (W <= 8) b = std::max(b, bf16_narrow_partial_bytes(n1, n2, W, fixed));
  return b;
}

int prep_rows_bf16(int precision, const float* X, int64_t n, int64_t d, const float* centre,
                   void* Xb, float* norms, hipStream_t s) {
  if (n == 0) return IGP_OK;
  __bf16* H = static_cast<__bf16*>(Xb);
  __bf16* Lo = precision == IGP_BF16X3 ? H + n * bf16_padded_dim(d) : nullptr;
  k_prep_rows_bf16<<<static_cast<unsigned>(n), 256, 0, s>>>(
      X, n, static_cast<int>(d), static_cast<int>(bf16_padded_dim(d)), centre, H, Lo, norms);
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

int kv_bf16_launch(const KVProblem& p, const void* X1b, const float* n1p, const void* X2b,
                   const float* n2p, float* P, size_t P_bytes, hipStream_t s, int* nsplit_out) {
  const int64_t W = p.C * p.nb;
  // few features and a narrow output: the narrow BF16 tile (one 16x16x32 MFMA
  // per block of distances, the contraction on VALU); the 256 x 256 tiles
  // below are built for hundreds of features
  if (p.precision == IGP_BF16 && bf16_narrow_supported(p.kp.kind, p.d, W))
    return kv_bf16_narrow_launch(p, X1b, n1p, X2b, n2p, P, P_bytes, s, nsplit_out);
  // the same prepared rows on both sides: each pair of 256-row blocks once
  const int64_t Q = (X1b == X2b && n1p == n2p && p.n1 == p.n2 && !p.fixed_split)
                        ? sym_blocks(p.n1, W) : 0;
  PlanB pl = plan_bf16(p.n1, p.n2, W, p.fixed_split);
  *nsplit_out = Q > 0 ? static_cast<int>(Q) : pl.nsplit;
  if (p.symmetric_out) *p.symmetric_out = Q > 0 ? 1 : 0;
  if (Q > 0 && static_cast<size_t>(Q) * p.n1 * W * sizeof(float) > P_bytes) {
    set_error("kernel-product workspace too small for the symmetric partials");
    return IGP_ENOMEM;
  }
  if (Q == 0 && static_cast<size_t>(pl.nsplit) * p.n1 * W * sizeof(float) > P_bytes) {
    set_error("kernel-product workspace too small for the split partials");
    return IGP_ENOMEM;
  }
  if (Q == 0 && (pl.nsplit == 0 || pl.gx == 0 || pl.gz == 0)) return IGP_OK;
  const double inv_l2 = 1.0 / (p.kp.lengthscale * p.kp.lengthscale);
  float kap;
  switch (p.kp.kind) {
    case IGP_RBF: kap = 0.5f * LOG2E_B; break;
    case IGP_MATERN12: kap = LOG2E_B * LOG2E_B; break;
    case IGP_MATERN32: kap = 3.0f * LOG2E_B * LOG2E_B; break;
    default: kap = 5.0f * LOG2E_B * LOG2E_B; break;
  }
  const float cnorm = static_cast<float>(kap * inv_l2);
  const float cdot = static_cast<float>(-2.0 * kap * inv_l2);
  const int64_t nwg = static_cast<int64_t>(pl.gx) * pl.nsplit * pl.gz;
  if (nwg > INT32_MAX) {
    set_error("kernel product too large for one launch");
    return IGP_EINVAL;
  }
  const dim3 grid(static_cast<unsigned>(nwg));
  const int DPB = static_cast<int>(bf16_padded_dim(p.d));
  const __bf16* A1 = static_cast<const __bf16*>(X1b);
  const __bf16* A2 = static_cast<const __bf16*>(X2b);
  // split mode: the low parts follow the high parts of each prepared set
  const int nph = p.precision == IGP_BF16X3 ? 3 : 1;
  const __bf16* L1 = nph == 3 ? A1 + p.n1 * DPB : A1;
  const __bf16* L2 = nph == 3 ? A2 + p.n2 * DPB : A2;
  const float* V = static_cast<const float*>(p.V);
  const int C = static_cast<int>(p.C), Wi = static_cast<int>(W);
  const unsigned sym_grid = static_cast<unsigned>(Q * (Q + 1) / 2);
  auto go = [&](auto kind) {
    constexpr int K_ = decltype(kind)::value;
    if (Q > 0 && nph == 3)
      kv_bf16_sym<K_, true><<<sym_grid, NT, 0, s>>>(
          A1, n1p, L1, nph, p.n1, DPB, V, C, Wi, p.ldv, P, static_cast<int>(Q), cnorm, cdot,
          p.skip);
    else if (Q > 0)
      kv_bf16_sym<K_, false><<<sym_grid, NT, 0, s>>>(
          A1, n1p, L1, nph, p.n1, DPB, V, C, Wi, p.ldv, P, static_cast<int>(Q), cnorm, cdot,
          p.skip);
    else if (nph == 3)
      kv_bf16_kernel<K_, true><<<grid, NT, 0, s>>>(
          A1, n1p, A2, n2p, L1, L2, nph, p.n1, p.n2, DPB, V, C, Wi, p.ldv, P, pl.cols_per_split,
          pl.gx, pl.nsplit, cnorm, cdot, p.skip);
    else
      kv_bf16_kernel<K_, false><<<grid, NT, 0, s>>>(
          A1, n1p, A2, n2p, L1, L2, nph, p.n1, p.n2, DPB, V, C, Wi, p.ldv, P, pl.cols_per_split,
          pl.gx,
          pl.nsplit, cnorm, cdot, p.skip);
  };
  switch (p.kp.kind) {
    case IGP_RBF: go(std::integral_constant<int, IGP_RBF>{}); break;
    case IGP_MATERN12: go(std::integral_constant<int, IGP_MATERN12>{}); break;
    case IGP_MATERN32: go(std::integral_constant<int, IGP_MATERN32>{}); break;
    default: go(std::integral_constant<int, IGP_MATERN52>{}); break;
  }
  IGP_CHECK_LAUNCH();
  return IGP_OK;
}

}  // namespace igp
