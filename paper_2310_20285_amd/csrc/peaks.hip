// Issue-rate microbenchmarks of gfx950 behind the ALU roofline of the fused
// FP32 product (a separate library, libitergp_peaks.so; not part of the
// solver).  Each kernel runs `iters` loop trips of independent dependency
// chains of one instruction kind, so that the issue rate, not the latency,
// bounds it; the host divides wave-instructions by time.
//   0  v_fma_f32                 8 chains x 8 per trip
//   1  v_exp_f32                 8 chains x 8 per trip
//   2  v_sqrt_f32                8 chains x 8 per trip
//   3  v_mfma_f32_16x16x4f32     4 accumulators x 4 per trip
//   4  v_mfma_f32_16x16x32_bf16  4 accumulators x 4 per trip
//   5  mixed: kind 3's 16 MFMAs + nvalu (multiple of 8) FMAs per trip, to see
//      whether FP32 MFMA and VALU work overlap on a SIMD
//   6  ds_read_b128              8 per trip feeding nvalu (4, 12 or 24) BF16 MFMAs
//                                (LDS read bandwidth, and its overlap with MFMA)
//   7  ds_write_b128             8 per trip (LDS write bandwidth)
//   8  v_mfma_f32_16x16x32_bf16  as kind 4 with random operands (random signs and
//                                mantissas, 8 operand registers cycled): the
//                                matrix rate on data like the product's, which
//                                draws more power than the constant operands of 4
//   9  FP32 MFMA and FMA in different waves of one SIMD: 512-thread workgroups,
//      waves 0-3 run kind 3's MFMA loop and waves 4-7 an FMA loop of nvalu FMAs
//      per trip (one wave of each kind per SIMD); nvalu = -1: only the MFMA
//      waves run, -2: only the FMA waves (64 FMAs per trip)
// The LDS kinds use 64 KB of LDS per workgroup (two workgroups per CU); every
// lane reads or writes its own 16 bytes, lanes contiguous (no bank conflicts).
// Every chain's result is stored, so nothing is dead code.
#include <hip/hip_runtime.h>

#include <cstdint>

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int NT = 256;

__global__ void __launch_bounds__(NT) k_fma(float* out, int iters, float b, float c) {
  float a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = threadIdx.x * 1e-3f + i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = __builtin_fmaf(a[i], b, c);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += a[i];
  out[blockIdx.x * NT + threadIdx.x] = s;
}

__global__ void __launch_bounds__(NT) k_exp(float* out, int iters) {
  float a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = (threadIdx.x & 7) * 0.1f + i * 0.01f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = __builtin_amdgcn_exp2f(-a[i]);   // stays in (0.5, 1]
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += a[i];
  out[blockIdx.x * NT + threadIdx.x] = s;
}

__global__ void __launch_bounds__(NT) k_sqrt(float* out, int iters) {
  float a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = 2.0f + (threadIdx.x & 7) + i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = __builtin_amdgcn_sqrtf(a[i]);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += a[i];
  out[blockIdx.x * NT + threadIdx.x] = s;
}

template <bool BF16, int NVALU>
__global__ void __launch_bounds__(NT) k_mfma(float* out, int iters, float b, float c) {
  f4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = f4{0, 0, 0, 0};
  const float x = 1e-3f * (threadIdx.x & 63), y = 1e-3f;
  bf8 xa, xb;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    xa[t] = static_cast<__bf16>(x + t);
    xb[t] = static_cast<__bf16>(y * t);
  }
  float v[NVALU > 0 ? 8 : 1];
#pragma unroll
  for (int i = 0; i < (NVALU > 0 ? 8 : 1); ++i) v[i] = threadIdx.x * 1e-3f + i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if constexpr (BF16)
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa, xb, acc[i], 0, 0, 0);
        else
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc[i], 0, 0, 0);
      }
      if constexpr (NVALU > 0) {
#pragma unroll
        for (int k = 0; k < NVALU / 32; ++k)
#pragma unroll
          for (int i = 0; i < 8; ++i) v[i] = __builtin_fmaf(v[i], b, c);
      }
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  if constexpr (NVALU > 0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) s += v[i];
  }
  out[blockIdx.x * NT + threadIdx.x] = s;
}

// random BF16 of magnitude in [0.5, 1) from a hash of (thread, index)
__device__ inline __bf16 rand_bf16(unsigned t, unsigned i) {
  unsigned h = t * 0x9E3779B1u ^ (i + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  const unsigned short bits = static_cast<unsigned short>((h & 0x807Fu) | 0x3F00u);
  return __builtin_bit_cast(__bf16, bits);
}

// 16 accumulators, each updated once per trip (a chain of several updates per
// trip makes the compiler rotate accumulators through extra moves)
__global__ void __launch_bounds__(NT) k_mfma_rand(float* out, int iters) {
  const unsigned t = blockIdx.x * NT + threadIdx.x;
  bf8 a[4], b[4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[u][e] = rand_bf16(t, u * 8 + e);
      b[u][e] = rand_bf16(t, 64 + u * 8 + e);
    }
  f4 acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = f4{0, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i)
      acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i & 3], b[i >> 2], acc[i], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[t] = s;
}

// kind 9: waves 0-3 MFMA, waves 4-7 FMA (wave w runs on SIMD w mod 4)
template <int NV>
__global__ void __launch_bounds__(512) k_split_waves(float* out, int iters, int which, float b,
                                                     float c) {
  const int wave = threadIdx.x >> 6;
  float s = 0.0f;
  if (wave < 4) {
    if (which == 2) return;
    f4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = f4{0, 0, 0, 0};
    const float x = 1e-3f * (threadIdx.x & 63), y = 1e-3f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc[i], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  } else {
    if (which == 1) return;
    float a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = threadIdx.x * 1e-3f + i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int u = 0; u < NV / 8; ++u)
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = __builtin_fmaf(a[i], b, c);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) s += a[i];
  }
  out[blockIdx.x * 512 + threadIdx.x] = s;
}

constexpr int LDS_Q = 4096;   // 16-byte pieces per workgroup (64 KB)

// 8 ds_read_b128 per trip feed NMF BF16 MFMAs (4: each pair of reads once, as
// A and B operands); with NMF = 4 the LDS, not the matrix unit, bounds the
// loop, and larger NMF show whether LDS reads and MFMAs overlap
template <int NMF>
__global__ void __launch_bounds__(NT) k_lds_read(float* out, int iters) {
  __shared__ __align__(16) bf8 buf[LDS_Q];
  for (int i = threadIdx.x; i < LDS_Q; i += NT) {
    bf8 v;
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = static_cast<__bf16>(1e-3f * ((i + t) & 7));
    buf[i] = v;
  }
  __syncthreads();
  f4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = f4{0, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
    int base = (it & 1) * (LDS_Q / 2) + threadIdx.x;   // 8 x 256 pieces = half the buffer
    asm volatile("" : "+v"(base));   // opaque address: the reads stay inside the loop
    bf8 a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = buf[base + u * NT];
#pragma unroll
    for (int k = 0; k < NMF; ++k)
      acc[k & 3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[(2 * k) & 7], a[(2 * k + 1) & 7],
                                                           acc[k & 3], 0, 0, 0);
  }
  float sum = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) sum += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * NT + threadIdx.x] = sum;
}

__global__ void __launch_bounds__(NT) k_lds_write(float* out, int iters) {
  __shared__ __align__(16) u4 buf[LDS_Q];
  u4 val = u4{threadIdx.x, blockIdx.x, 0u, 0u};
  for (int it = 0; it < iters; ++it) {
    val.z += 1u;
    int base = (it & 1) * (LDS_Q / 2) + threadIdx.x;
    asm volatile("" : "+v"(base));
#pragma unroll
    for (int u = 0; u < 8; ++u) buf[base + u * NT] = val;
  }
  __syncthreads();
  const u4 a = buf[(threadIdx.x * 7) & (LDS_Q - 1)];
  out[blockIdx.x * NT + threadIdx.x] = static_cast<float>((a.x ^ a.z) & 0xffff);
}

}  // namespace

extern "C" {

// Launch microbenchmark `which` (see above) with `blocks` workgroups of 256
// threads; out holds blocks * 256 floats (device).  nvalu (kind 5): FMAs
// per trip, one of 32, 64, 128; kind 6: MFMAs per trip, one of 4, 12, 24;
// kind 9: FMAs per trip of the FMA waves (32, 64, 128), or -1 / -2 (see above).
// Returns 0, or -1 for an unknown kind.
int igp_peaks_run(int which, int blocks, int iters, int nvalu, float* out, hipStream_t s) {
  const dim3 g(static_cast<unsigned>(blocks)), b(NT);
  switch (which) {
    case 0: k_fma<<<g, b, 0, s>>>(out, iters, 0.999f, 1e-4f); break;
    case 1: k_exp<<<g, b, 0, s>>>(out, iters); break;
    case 2: k_sqrt<<<g, b, 0, s>>>(out, iters); break;
    case 3: k_mfma<false, 0><<<g, b, 0, s>>>(out, iters, 0.999f, 1e-4f); break;
    case 4: k_mfma<true, 0><<<g, b, 0, s>>>(out, iters, 0.999f, 1e-4f); break;
    case 5:
      if (nvalu == 32) k_mfma<false, 32><<<g, b, 0, s>>>(out, iters, 0.999f, 1e-4f);
      else if (nvalu == 64) k_mfma<false, 64><<<g, b, 0, s>>>(out, iters, 0.999f, 1e-4f);
      else if (nvalu == 128) k_mfma<false, 128><<<g, b, 0, s>>>(out, iters, 0.999f, 1e-4f);
      else return -1;
      break;
    case 6:
      if (nvalu == 4) k_lds_read<4><<<g, b, 0, s>>>(out, iters);
      else if (nvalu == 12) k_lds_read<12><<<g, b, 0, s>>>(out, iters);
      else if (nvalu == 24) k_lds_read<24><<<g, b, 0, s>>>(out, iters);
      else return -1;
      break;
    case 7: k_lds_write<<<g, b, 0, s>>>(out, iters); break;
    case 8: k_mfma_rand<<<g, b, 0, s>>>(out, iters); break;
    case 9: {
      // blocks counts 256-thread units of out: half as many 512-thread workgroups
      const dim3 g2(static_cast<unsigned>(blocks / 2)), b2(512);
      const float bb = 0.999f, cc = 1e-4f;
      if (nvalu == -1) k_split_waves<64><<<g2, b2, 0, s>>>(out, iters, 1, bb, cc);
      else if (nvalu == -2) k_split_waves<64><<<g2, b2, 0, s>>>(out, iters, 2, bb, cc);
      else if (nvalu == 32) k_split_waves<32><<<g2, b2, 0, s>>>(out, iters, 0, bb, cc);
      else if (nvalu == 64) k_split_waves<64><<<g2, b2, 0, s>>>(out, iters, 0, bb, cc);
      else if (nvalu == 128) k_split_waves<128><<<g2, b2, 0, s>>>(out, iters, 0, bb, cc);
      else return -1;
      break;
    }
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
