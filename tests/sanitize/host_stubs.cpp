// Stand-ins for the device launchers, for a host-only build of the library
// (plan creation, argument validation, workspace layout, the host partition)
// under AddressSanitizer and UndefinedBehaviorSanitizer.  Every launcher
// reports that no device is present; the host-side checks the tests exercise
// run before any launch, so they never reach these.
#include <hip/hip_runtime.h>

#include "gsr.h"
#include "gsr_internal.h"
#include "gsr_stages.h"

namespace gsr {

static int no_device() { return (int)hipErrorNoDevice; }

int launch_setup(const ViewTable &, const KWs &, int64_t, int64_t, int, int64_t, void *) { return no_device(); }
int launch_fill_u32(uint32_t *, uint32_t, int64_t, void *) { return no_device(); }
int launch_fill_f32(float *, float, int64_t, void *) { return no_device(); }
int launch_project(const KParams &, const gsr_camera *, const KOpts &, const KWs &, int, int, int, int, void *) {
  return no_device();
}
int launch_scan(const KWs &, int64_t, int64_t, int64_t, int, int, void *) { return no_device(); }
int launch_emit(const KWs &, int64_t, int, int, void *) { return no_device(); }
int launch_sort(const KWs &, int64_t, int64_t, void *) { return no_device(); }
int launch_raster_fwd(const KWs &, const KOpts &, int64_t, int64_t, float *, int, int, int, float *, uint32_t *,
                      void *) {
  return no_device();
}
int launch_l1(const KWs &, const KOpts &, int64_t, int64_t, const float *, const float *, int, void *) {
  return no_device();
}
int launch_raster_bwd(const KWs &, const KOpts &, int64_t, int64_t, const float *, int, int, int, int, void *) {
  return no_device();
}
int launch_fused(const KWs &, const KOpts &, const float *, float *, int, int, int, int, int, void *) {
  return no_device();
}
int launch_project_bwd(const KParams &, const gsr_camera *, const KOpts &, const KWs &, const KGrads &, float *,
                       uint32_t *, int, void *) {
  return no_device();
}
int launch_loss(const KWs &, int, float *, void *) { return no_device(); }
int launch_visibility(const KParams &, const gsr_camera *, const KOpts &, const KWs &, const float *, uint32_t *,
                      uint8_t *, uint8_t *, void *) {
  return no_device();
}
int launch_copy_pixels(const KWs &, float *, uint32_t *, void *) { return no_device(); }
int launch_count_visible(const KWs &, int64_t, int, void *) { return no_device(); }
int launch_tile_order(const KWs &, void *) { return no_device(); }
int launch_adam(const KAdam &, int, void *) { return no_device(); }
int launch_count_points(const float *, int64_t, const PartitionView *, int, int64_t, const float *, int, uint32_t *,
                        void *) {
  return no_device();
}
int launch_back_project(const ViewTable &, const gsr_camera *, const float *, float *, void *) { return no_device(); }
int launch_coverage(const ViewTable &, const gsr_camera *, const float *, const float *, int, float, uint32_t *,
                    float *, uint8_t *, void *) {
  return no_device();
}

}  // namespace gsr

// The densification and allocation-free entry points live with their device
// code; this host-only build carries placeholders so that the binding's
// declarations resolve (the sanitized suites do not call them).
extern "C" gsr_status gsr_densify_workspace_size(int64_t, size_t *) { return GSR_ERR_HIP; }
extern "C" gsr_status gsr_densify_count(int64_t, int32_t, const gsr_densify_opts *, const gsr_gaussians *,
                                        const gsr_stats *, const uint8_t *, void *, size_t, void *, int64_t *) {
  return GSR_ERR_HIP;
}
extern "C" gsr_status gsr_densify_apply(int64_t, int32_t, const gsr_densify_opts *, const gsr_gaussians *,
                                        const gsr_grads *, const gsr_grads *, const gsr_stats *, const uint8_t *,
                                        const float *, int64_t, const gsr_grads *, const gsr_grads *,
                                        const gsr_grads *, int64_t *, void *, size_t, void *) {
  return GSR_ERR_HIP;
}
extern "C" gsr_status gsr_forward_backward_l1_static(gsr_plan *, const gsr_gaussians *, const gsr_camera *,
                                                      const float *, float *, float *, const gsr_grads *,
                                                      const gsr_stats *, void *) {
  return GSR_ERR_HIP;
}
