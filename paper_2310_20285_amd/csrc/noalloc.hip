// glm_kernel_matmul_noalloc: the kernel-matrix product with its scratch space
// (split partials, centred rows and their norms) taken from a file-scope
// device array instead of a caller workspace, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops).  Same kernels,
// same split plan and therefore bitwise the same result as glm_kernel_matmul.
#include <mutex>

#include "ops.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  In host code `scratch` is a
// host-side stand-in: its device address comes from hipGetSymbolAddress, once
// per device, and only that address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (the current device's).
int scratch_address(void** out) {
  int dev = -1;
  IGP_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    igp::set_error("device ordinal %d beyond the %d supported", dev, kMaxDevices);
    return IGP_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    IGP_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      igp::set_error("hipGetSymbolAddress returned a null scratch address");
      return IGP_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return IGP_OK;
}

}  // namespace

extern "C" {

size_t glm_kernel_matmul_noalloc_max_bytes(void) { return kScratchBytes; }

int glm_kernel_matmul_noalloc(const igp_kernel_params* kp, int32_t n_kp, const void* X1,
                              int64_t n1, const void* X2, int64_t n2, int64_t d, const void* V,
                              int64_t C, int64_t nb, int64_t ldv, void* Out, int64_t ldo,
                              double beta, int32_t precision, hipStream_t stream) {
  try {
    igp::clear_error();
    // invalid shapes give 0 here and are rejected by glm_kernel_matmul below
    const size_t need = glm_kernel_matmul_ws_bytes(n1, n2, d, C, nb, precision);
    if (need > kScratchBytes) {
      igp::set_error("product of %lld x %lld rows (d = %lld, %lld output columns) needs %zu "
                     "bytes of scratch, beyond the %zu bytes of the no-allocation entry point; "
                     "use glm_kernel_matmul with a workspace",
                     static_cast<long long>(n1), static_cast<long long>(n2),
                     static_cast<long long>(d), static_cast<long long>(C * nb), need,
                     kScratchBytes);
      return IGP_ENOMEM;
    }
    void* ws = nullptr;
    IGP_TRY(scratch_address(&ws));
    return glm_kernel_matmul(kp, n_kp, X1, n1, X2, n2, d, V, C, nb, ldv, Out, ldo, beta,
                             precision, ws, kScratchBytes, stream);
  } catch (const std::exception& e) {
    igp::set_error("internal error: %s", e.what());
    return IGP_EDEVICE;
  } catch (...) {
    igp::set_error("internal error");
    return IGP_EDEVICE;
  }
}

}  // extern "C"
