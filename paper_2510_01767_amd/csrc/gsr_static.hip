// The allocation-free form of the fused training step, for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid it): the workspace is a file-scope device
// array of GSR_STATIC_SCRATCH_BYTES instead of a caller buffer.  Each GPU the
// library runs on holds its own copy of the array until the process ends;
// calls on one GPU share it, so calls that overlap on one GPU race.  The step
// itself clears everything that must start at zero (its set-up kernel resets
// the counters and tile counts), so no call depends on what the last one
// left in the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gsr_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)GSR_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The array's name is a host-side stand-in in host code: kernels receive the
// device address looked up below, never the name.
__device__ __align__(256) uint8_t scratch[kScratchBytes];

void *g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of the current device's copy of `scratch`, looked up once
// per device (on that device's first call) and kept.
gsr_status scratch_of_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GSR_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return GSR_ERR_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GSR_OK;
}

}  // namespace

extern "C" gsr_status gsr_forward_backward_l1_static(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams,
                                                      const float *targets, float *images, float *loss,
                                                      const gsr_grads *grads, const gsr_stats *stats, void *stream) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  size_t need = 0;
  if (gsr_workspace_size(plan, &need) != GSR_OK) return GSR_ERR_INVALID_ARG;
  if (need > kScratchBytes)
    return gsr::plan_error(plan, GSR_ERR_WORKSPACE_TOO_SMALL,
                           "the plan's workspace exceeds GSR_STATIC_SCRATCH_BYTES: use gsr_forward_backward_l1 "
                           "with a caller workspace");
  void *ws = nullptr;
  if (scratch_of_current_device(&ws) != GSR_OK)
    return gsr::plan_error(plan, GSR_ERR_HIP, "could not look up the device address of the static scratch array");
  return gsr::fused_l1_no_events(plan, g, cams, targets, images, loss, grads, stats, ws, kScratchBytes, stream);
}
