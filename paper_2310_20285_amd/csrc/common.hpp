// Shared helpers for the gfx950 IterNCGP library: status handling, wave64
// reductions and the kernel functions evaluated in registers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/itergp.h"

namespace igp {

// ---- error handling ------------------------------------------------------
void set_error(const char* fmt, ...);
void clear_error();

struct Status {
  int code = IGP_OK;
  bool ok() const { return code == IGP_OK; }
};

#define IGP_CHECK_HIP(expr)                                                    \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::igp::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),  \
                       __FILE__, __LINE__);                                    \
      return IGP_EDEVICE;                                                      \
    }                                                                          \
  } while (0)

#define IGP_CHECK_LAUNCH()                                                     \
  do {                                                                         \
    hipError_t e_ = hipGetLastError();                                         \
    if (e_ != hipSuccess) {                                                    \
      ::igp::set_error("kernel launch failed: %s (%s:%d)",                     \
                       hipGetErrorString(e_), __FILE__, __LINE__);             \
      return IGP_EDEVICE;                                                      \
    }                                                                          \
  } while (0)

#define IGP_TRY(expr)                                                          \
  do {                                                                         \
    int s_ = (expr);                                                           \
    if (s_ != IGP_OK) return s_;                                               \
  } while (0)

#define IGP_REQUIRE(cond, ...)                                                 \
  do {                                                                         \
    if (!(cond)) {                                                             \
      ::igp::set_error(__VA_ARGS__);                                           \
      return IGP_EINVAL;                                                       \
    }                                                                          \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Bump allocator over a caller-provided device region; never allocates.
struct Carver {
  char* base;
  size_t cap;
  size_t used = 0;
  Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    size_t off = align_up(used);
    used = off + align_up(count * sizeof(T));
    return (base && used <= cap) ? reinterpret_cast<T*>(base + off) : nullptr;
  }
  bool fits() const { return used <= cap; }
};

// ---- device helpers --------------------------------------------------------
// The solver's gate (and its iteration record) are written by kernels and read
// by later kernels of the same stream: read them with device-coherent vector
// loads, never through the scalar cache.
__device__ inline int coherent_load(const int* p) {
  return __hip_atomic_load(const_cast<int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double coherent_load(const double* p) {
  const unsigned long long u = __hip_atomic_load(
      reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED,
      __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double(static_cast<long long>(u));
}
__device__ inline bool gate_closed(const int* g) { return g && coherent_load(g) != 0; }

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a block of `nthreads` (multiple of 64, <= 1024).  Result valid in
// every thread.  `red` must hold nthreads/64 values.
template <typename T>
__device__ inline T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// Kernel function of the scaled squared distance r2 = ||x-x'||^2 / l^2,
// without the outputscale (applied once to the accumulated sums).
template <int KIND>
__device__ inline double kfun(double r2) {
  if constexpr (KIND == IGP_RBF) {
    return exp(-0.5 * r2);
  } else if constexpr (KIND == IGP_MATERN12) {
    return exp(-sqrt(r2));
  } else if constexpr (KIND == IGP_MATERN32) {
    double a = sqrt(3.0 * r2);
    return (1.0 + a) * exp(-a);
  } else {
    double a = sqrt(5.0 * r2);
    return (1.0 + a + (5.0 / 3.0) * r2) * exp(-a);
  }
}

// FP32 variant on the hardware transcendental units (v_exp_f32 = 2^x,
// v_sqrt_f32), both within ~1 ulp.
template <int KIND>
__device__ inline float kfun(float r2) {
  constexpr float LOG2E = 1.4426950408889634f;
  if constexpr (KIND == IGP_RBF) {
    return __builtin_amdgcn_exp2f(-0.5f * LOG2E * r2);
  } else if constexpr (KIND == IGP_MATERN12) {
    return __builtin_amdgcn_exp2f(-LOG2E * __builtin_amdgcn_sqrtf(r2));
  } else if constexpr (KIND == IGP_MATERN32) {
    float a = __builtin_amdgcn_sqrtf(3.0f * r2);
    return (1.0f + a) * __builtin_amdgcn_exp2f(-LOG2E * a);
  } else {
    float a = __builtin_amdgcn_sqrtf(5.0f * r2);
    return (1.0f + a + (5.0f / 3.0f) * r2) * __builtin_amdgcn_exp2f(-LOG2E * a);
  }
}

}  // namespace igp
