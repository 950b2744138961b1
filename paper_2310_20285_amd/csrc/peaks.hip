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
// Every chain's result is stored, so nothing is dead code.
#include <hip/hip_runtime.h>

#include <cstdint>

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

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

}  // namespace

extern "C" {

// Launch microbenchmark `which` (see above) with `blocks` workgroups of 256
// threads; out holds blocks * 256 floats (device).  nvalu (kind 5 only): FMAs
// per trip, one of 32, 64, 128.  Returns 0, or -1 for an unknown kind.
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
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
