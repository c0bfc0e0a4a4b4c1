// Fast camera selection (Sec. 3.2) on gfx950: every pixel's composited
// depth is back-projected through its pixel centre into world space and
// counted into the block boxes that hold it; the ratio V_{c,b} = count / N_p
// (N_p = the view's pixels) selects the cameras with V_{c,b} >= tau.
//
// Grid: x strides over a view's pixels, y is the view.  The boxes sit in
// LDS, each workgroup counts in LDS and adds its counts to the global ones
// with one atomic per (workgroup, block).  A second kernel turns counts into
// ratios and the selection.
#include <hip/hip_runtime.h>

#include "gsr_device.h"
#include "gsr_stages.h"

namespace gsr {

// World point of pixel pix of a view with composited depth D, through the
// pixel's centre: R^T (D ((u + 1/2 - cx) / fx, (v + 1/2 - cy) / fy, 1) - t).
__device__ __forceinline__ void back_project_pixel(const gsr_camera &c, int W, int64_t pix, double D, double w[3]) {
  const int px = (int)(pix % W), py = (int)(pix / W);
  const double q[3] = {D * (((double)px + 0.5 - (double)c.cx) / (double)c.fx) - (double)c.t[0],
                       D * (((double)py + 0.5 - (double)c.cy) / (double)c.fy) - (double)c.t[1],
                       D - (double)c.t[2]};
#pragma unroll
  for (int a = 0; a < 3; a++) w[a] = (double)c.R[a] * q[0] + (double)c.R[3 + a] * q[1] + (double)c.R[6 + a] * q[2];
}

__global__ __launch_bounds__(kBlock) void k_back_project(ViewTable tbl, const gsr_camera *cams, const float *depth,
                                                         float *points, int64_t total) {
  const int v = blockIdx.y;
  const ViewInfo vi = tbl.v[v];
  const gsr_camera c = cams[v];
  const int64_t P = (int64_t)vi.W * vi.H;
  for (int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pix < P; pix += (int64_t)gridDim.x * blockDim.x) {
    double w[3];
    back_project_pixel(c, vi.W, pix, (double)depth[vi.pix_base + pix], w);
#pragma unroll
    for (int a = 0; a < 3; a++) points[a * total + vi.pix_base + pix] = (float)w[a];
  }
}

__global__ __launch_bounds__(kBlock) void k_coverage(ViewTable tbl, const gsr_camera *cams, const float *depth,
                                                     const float *blocks, int n_blocks, uint32_t *counts) {
  __shared__ float s_box[GSR_MAX_COVERAGE_BLOCKS * 6];
  __shared__ uint32_t s_cnt[GSR_MAX_COVERAGE_BLOCKS];
  for (int k = threadIdx.x; k < n_blocks * 6; k += blockDim.x) s_box[k] = blocks[k];
  for (int k = threadIdx.x; k < n_blocks; k += blockDim.x) s_cnt[k] = 0u;
  __syncthreads();
  const int v = blockIdx.y;
  const ViewInfo vi = tbl.v[v];
  const gsr_camera c = cams[v];
  const int64_t P = (int64_t)vi.W * vi.H;
  for (int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pix < P; pix += (int64_t)gridDim.x * blockDim.x) {
    double wd[3];
    back_project_pixel(c, vi.W, pix, (double)depth[vi.pix_base + pix], wd);
    // the float32 point gsr_back_project stores, so that both count alike
    const float w[3] = {(float)wd[0], (float)wd[1], (float)wd[2]};
    for (int b = 0; b < n_blocks; b++) {
      const float *bx = s_box + 6 * b;
      const bool in = w[0] >= bx[0] && w[0] < bx[3] && w[1] >= bx[1] && w[1] < bx[4] && w[2] >= bx[2] && w[2] < bx[5];
      // one LDS atomic per wavefront and block: the ballot's population
      const uint64_t m = __ballot(in);
      if (m && (uint64_t)(__ffsll((unsigned long long)__ballot(true)) - 1) == (uint64_t)lane_id())
        atomicAdd(&s_cnt[b], (uint32_t)__popcll(m));
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < n_blocks; b += blockDim.x)
    if (s_cnt[b]) atomicAdd(&counts[(int64_t)v * n_blocks + b], s_cnt[b]);
}

__global__ __launch_bounds__(kBlock) void k_count_points(const float *points, int64_t total,
                                                         const PartitionView *views, const float *boxes, int nb,
                                                         uint32_t *counts) {
  __shared__ float s_box[GSR_MAX_COVERAGE_BLOCKS * 6];
  __shared__ uint32_t s_cnt[GSR_MAX_COVERAGE_BLOCKS];
  for (int k = threadIdx.x; k < nb * 6; k += blockDim.x) s_box[k] = boxes[k];
  for (int k = threadIdx.x; k < nb; k += blockDim.x) s_cnt[k] = 0u;
  __syncthreads();
  const int j = blockIdx.y;
  const int64_t first = views[j].first, count = views[j].count;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const float x = points[first + i], y = points[total + first + i], z = points[2 * total + first + i];
    for (int b = 0; b < nb; b++) {
      const float *bx = s_box + 6 * b;
      const bool in = x >= bx[0] && x < bx[3] && y >= bx[1] && y < bx[4] && z >= bx[2] && z < bx[5];
      const uint64_t m = __ballot(in);
      if (m && (uint64_t)(__ffsll((unsigned long long)__ballot(true)) - 1) == (uint64_t)lane_id())
        atomicAdd(&s_cnt[b], (uint32_t)__popcll(m));
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    if (s_cnt[b]) atomicAdd(&counts[(int64_t)j * nb + b], s_cnt[b]);
}

__global__ void k_coverage_ratio(ViewTable tbl, int n_blocks, float tau, const uint32_t *counts, float *ratio,
                                 uint8_t *selected) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)tbl.n_views * n_blocks) return;
  const ViewInfo vi = tbl.v[k / n_blocks];
  const double np = (double)vi.W * (double)vi.H;
  if (ratio) ratio[k] = (float)((double)counts[k] / np);
  // count / N_p >= tau exactly: tau N_p is exact in double
  if (selected) selected[k] = (double)counts[k] >= (double)tau * np ? 1 : 0;
}

__global__ void k_zero_u32(uint32_t *p, int64_t count) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
    p[k] = 0u;
}

int launch_back_project(const ViewTable &views, const gsr_camera *cams, const float *depth, float *points,
                        void *stream) {
  int64_t pmax = 1, total = 0;
  for (int v = 0; v < views.n_views; v++) {
    pmax = std::max(pmax, (int64_t)views.v[v].W * views.v[v].H);
    total += (int64_t)views.v[v].W * views.v[v].H;
  }
  const unsigned gx = (unsigned)std::min((pmax + kBlock - 1) / kBlock, (int64_t)1024);
  hipLaunchKernelGGL(k_back_project, dim3(gx, (unsigned)views.n_views), dim3(kBlock), 0, (hipStream_t)stream, views,
                     cams, depth, points, total);
  return last_err();
}

int launch_count_points(const float *points, int64_t total, const PartitionView *views, int n_sel, int64_t pmax,
                        const float *boxes, int nb, uint32_t *counts, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const int64_t nc = (int64_t)n_sel * nb;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::min((nc + kBlock - 1) / kBlock, (int64_t)4096)), dim3(kBlock),
                     0, s, counts, nc);
  const unsigned gx = (unsigned)std::min((pmax + kBlock - 1) / kBlock, (int64_t)1024);
  hipLaunchKernelGGL(k_count_points, dim3(gx, (unsigned)n_sel), dim3(kBlock), 0, s, points, total, views, boxes, nb,
                     counts);
  return last_err();
}

int launch_coverage(const ViewTable &views, const gsr_camera *cams, const float *depth, const float *blocks,
                    int n_blocks, float tau, uint32_t *counts, float *ratio, uint8_t *selected, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const int64_t nc = (int64_t)views.n_views * n_blocks;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((nc + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, counts, nc);
  int64_t pmax = 1;
  for (int v = 0; v < views.n_views; v++) pmax = std::max(pmax, (int64_t)views.v[v].W * views.v[v].H);
  const unsigned gx = (unsigned)std::min((pmax + kBlock - 1) / kBlock, (int64_t)1024);
  hipLaunchKernelGGL(k_coverage, dim3(gx, (unsigned)views.n_views), dim3(kBlock), 0, s, views, cams, depth, blocks,
                     n_blocks, counts);
  if (ratio || selected)
    hipLaunchKernelGGL(k_coverage_ratio, dim3((unsigned)((nc + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, views,
                       n_blocks, tau, counts, ratio, selected);
  return last_err();
}

}  // namespace gsr
