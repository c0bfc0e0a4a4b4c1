// Declarations of the stages after the training step: the optimizer
// (gsr_optim.hip), densification (gsr_densify.hip), fast camera selection
// (gsr_fcs.hip) and the scene partition's counting (gsr_partition.cpp).
#pragma once

#include "gsr_internal.h"

namespace gsr {

// Adam over the parameter planes (gsr_optim.hip).  Groups: means (3 rows),
// log_scales (3), quats (4), opacity_logits (1), sh (3K); step_size per
// learning-rate slot = lr / (1 - beta1^t), bc2_sqrt = sqrt(1 - beta2^t).
struct KAdam {
  float *p[5];
  const float *g[5];
  float *m[5];
  float *v[5];
  int rows[5];
  float step_size[6];
  float bc2_sqrt, beta1, beta2, eps;
  int64_t n;
  const uint32_t *visible;
};
int launch_adam(const KAdam &a, int planes, void *stream);

// Densification (gsr_densify.hip): inputs, decision thresholds and outputs.
struct KDensify {
  const float *mean, *ls, *quat, *opa, *sh;
  const uint8_t *keep;
  const float *m[5], *v[5];  // moments in, by group (means, log_scales, quats, opacity, sh)
  const float *S;
  const uint32_t *cnt;
  const uint8_t *in_block;
  const float *samples;  // [2][3][n]
  int64_t n, n_out;
  int sh_planes;
  int opa_on, world_on, selective;
  double grad_thr, log_clone_max, logit_min, log_world_max;
  float child_dlog;  // ln(1.6) rounded to float
  float *o_mean, *o_ls, *o_quat, *o_opa, *o_sh;
  float *om[5], *ov[5];
  int64_t *parent;
  uint64_t *block_sums;  // [blocks + 1]
};
int64_t densify_blocks(int64_t n);
int launch_densify_count(const KDensify &k, void *stream);
int launch_densify_apply(const KDensify &k, void *stream);

// Device workspace of the partition's pixel counting: the selected views'
// pixel ranges, the candidate boxes and their counts.
struct PartitionView {
  int64_t first, count;
};
struct PartitionWs {
  PartitionView *views;
  float *boxes;
  uint32_t *counts;
};
inline size_t partition_ws_bytes(int n_views) {
  return 256 + (size_t)n_views * sizeof(PartitionView) + (size_t)GSR_MAX_COVERAGE_BLOCKS * 6 * sizeof(float) +
         (size_t)n_views * GSR_MAX_COVERAGE_BLOCKS * sizeof(uint32_t);
}
inline PartitionWs partition_ws(char *ws, int n_views) {
  char *p = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  PartitionWs w;
  w.views = (PartitionView *)p;
  w.boxes = (float *)(p + (size_t)n_views * sizeof(PartitionView));
  w.counts = (uint32_t *)((char *)w.boxes + (size_t)GSR_MAX_COVERAGE_BLOCKS * 6 * sizeof(float));
  return w;
}
// counts[j][b] = number of points of view j (points [3][total], the view's
// range in views[j]) inside box b, for j < n_sel and b < nb <= 1024
int launch_count_points(const float *points, int64_t total, const PartitionView *views, int n_sel, int64_t pmax,
                        const float *boxes, int nb, uint32_t *counts, void *stream);
// Fast camera selection (gsr_fcs.hip): back-projected depth pixels counted
// per (view, block) box, the ratio to the view's pixel count and tau.
int launch_back_project(const ViewTable &views, const gsr_camera *cams, const float *depth, float *points,
                        void *stream);
int launch_coverage(const ViewTable &views, const gsr_camera *cams, const float *depth, const float *blocks,
                    int n_blocks, float tau, uint32_t *counts, float *ratio, uint8_t *selected, void *stream);
}  // namespace gsr
