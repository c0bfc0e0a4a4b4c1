// Optimizer step over the Gaussian parameter planes (gfx950): bias-corrected
// Adam, dense or restricted to the Gaussians visible in the last step (the
// optimizer is where unseen Gaussians cost time, Sec. 3.3; Sparse Adam,
// App. A.1).  A pure HBM stream: per element 4 loads (param, grad, two
// moments) and 3 stores.  One thread per element, the grid's y index is the
// plane (59 planes at SH degree 3), so every wavefront reads 256 consecutive
// bytes of each array (measured faster than four elements per thread with
// 16-byte accesses).
#include <hip/hip_runtime.h>

#include "gsr_device.h"
#include "gsr_stages.h"

namespace gsr {

__device__ __forceinline__ float adam_elem(const KAdam &a, int slot, float p, float g, float &m, float &v) {
  m = a.beta1 * m + (1.0f - a.beta1) * g;
  v = a.beta2 * v + (1.0f - a.beta2) * (g * g);
  const float denom = sqrtf(v) / a.bc2_sqrt + a.eps;
  return p - a.step_size[slot] * (m / denom);
}

__global__ __launch_bounds__(kBlock) void k_adam(KAdam a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  if (a.visible && a.visible[i] == 0u) return;
  // plane -> group and row
  int plane = blockIdx.y, grp = 0;
  while (grp < 4 && plane >= a.rows[grp]) {
    plane -= a.rows[grp];
    grp++;
  }
  const int lr_slot = grp < 4 ? grp : (plane < 3 ? 4 : 5);  // SH band 0 holds planes 0..2
  const int64_t e = (int64_t)plane * a.n + i;
  float m = a.m[grp][e], v = a.v[grp][e];
  a.p[grp][e] = adam_elem(a, lr_slot, a.p[grp][e], a.g[grp][e], m, v);
  a.m[grp][e] = m;
  a.v[grp][e] = v;
}

int launch_adam(const KAdam &a, int planes, void *stream) {
  if (a.n <= 0) return 0;
  const dim3 grid((unsigned)((a.n + kBlock - 1) / kBlock), (unsigned)planes), block(kBlock);
  hipLaunchKernelGGL(k_adam, grid, block, 0, (hipStream_t)stream, a);
  return last_err();
}

}  // namespace gsr
