// noalloc.hip -- the image loss (Appendix "Losses") for callers that cannot
// allocate device memory: the same kernels as sssgs_image_loss, with their
// scratch (three derivative maps and the per-tile partial sums) in a
// file-scope device array instead of a caller workspace.
#include <mutex>

#include "launch.hpp"
#include "sssgs.h"

namespace sssgs {
sssgs_status noalloc_fail(sssgs_status s, const char *msg);
}

namespace {

constexpr size_t kScratchBytes = SSSGS_NOALLOC_SCRATCH_BYTES;

// Device-side scratch; each GPU holds its own copy until the process ends.
// Host code never passes this name to a kernel: it is a host-side stand-in,
// not a device address.  The device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
sssgs_status scratch_ptr(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return sssgs::noalloc_fail(SSSGS_ERR_HIP, "hipGetDevice failed or device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return sssgs::noalloc_fail(SSSGS_ERR_HIP, hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return SSSGS_OK;
}

}  // namespace

extern "C" sssgs_status sssgs_image_loss_noalloc(const float *pred, const float *target, int32_t channels,
                                                 int32_t height, int32_t width, float lambda_dssim,
                                                 float *loss_out, float *dL_dpred, void *stream) {
  if (channels <= 0 || height <= 0 || width <= 0)
    return sssgs::noalloc_fail(SSSGS_ERR_INVALID_ARG, "bad image size");
  if (!pred || !target || !loss_out) return sssgs::noalloc_fail(SSSGS_ERR_INVALID_ARG, "null pointer");
  if (sssgs::image_loss_workspace_bytes(channels, height, width) > kScratchBytes)
    return sssgs::noalloc_fail(SSSGS_ERR_INVALID_ARG,
                               "image too large for the fixed scratch (SSSGS_NOALLOC_SCRATCH_BYTES)");
  void *ws = nullptr;
  const sssgs_status s = scratch_ptr(&ws);
  if (s != SSSGS_OK) return s;
  sssgs::launch_image_loss(pred, target, channels, height, width, lambda_dssim, ws, loss_out, dL_dpred,
                           (hipStream_t)stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return sssgs::noalloc_fail(SSSGS_ERR_HIP, hipGetErrorString(e));
  return SSSGS_OK;
}
