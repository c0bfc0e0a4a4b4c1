/*
 * gsr.h - C ABI of the MI355X differentiable Gaussian rasterizer.
 *
 * The operation.  One fine-training step of a LoBE-GS block (arXiv
 * 2510.01767) renders every camera assigned to the block from the block's
 * Gaussians and back-propagates an image loss to the Gaussian parameters
 * (Sec. 3, Fig. 1 "parallel fine-tuning"; the per-block training follows
 * vanilla 3DGS, App. A.1).  The library computes, for n Gaussians and
 * n_views cameras:
 *   - per-view visibility (frustum culling during rasterization, Sec. 3.3)
 *     and the visibility-cropping mask over a block's cameras (Sec. 3.3, VC);
 *   - EWA projection with scale/quaternion covariance and SH colour;
 *   - tile binning and per-tile ordering by (depth, Gaussian index);
 *   - front-to-back alpha compositing (Sec. 3.2, blending equation);
 *   - the L1 image loss, the hand-written reverse pass to every parameter,
 *     and the per-Gaussian view-space gradient statistic plus visible count
 *     that selective densification reads (Sec. 3.3, SD).
 *
 * Conventions (all fields of gsr_options, defaults from gsr_default_options):
 *   pinhole camera, OpenCV axes (x right, y down, z forward), world->camera
 *   [R | t]; pixel centres at (px + 1/2, py + 1/2); near 0.01, far 1e10;
 *   2D covariance J W Sigma W^T J^T + 0.3 I with x/z, y/z clamped to 1.3
 *   half fields of view inside J; radius ceil(3 sqrt(lambda_max)); tile
 *   rectangle floor((mean +- r) / tile) clamped to the grid; alpha =
 *   min(0.99, o exp(p)), entries below 1/255 skipped, compositing stops
 *   before an entry that would drop T below 1e-4; background bg (black);
 *   colour = max(0, sum_k sh_k Y_k(dir) + 1/2) with the real orthonormal SH
 *   basis (Condon-Shortley phase, l-major, m = -l..l), dir from the camera
 *   centre to the mean; opacity = sigmoid(logit); scale = exp(log_scale);
 *   rotation = unit quaternion q / |q| in (w, x, y, z) order.
 *
 * Memory.  The caller owns every device buffer (parameters, gradients,
 * statistics, images, targets, cameras, workspace).  The library never
 * allocates device memory; it enqueues work on the caller's stream.  A plan
 * holds only host metadata and, after gsr_graph_capture, a graph.
 *
 * Errors.  Every call returns a gsr_status; nothing is printed and no call
 * aborts.  Argument errors are detected on the host before anything is
 * enqueued.  GSR_ERR_CAPACITY comes from a sticky device flag (the
 * intersection capacity was exceeded; outputs are invalid - grow
 * capacity_intersections and retry) and is reported by gsr_query_counts, or
 * directly by plain-mode calls, which read the per-view counts back.
 * GSR_ERR_HIP carries the runtime's message in gsr_last_error.  A plan is not
 * thread-safe; distinct plans are independent.
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gsr_status;
#define GSR_OK 0
#define GSR_ERR_INVALID_ARG 1
#define GSR_ERR_WORKSPACE_TOO_SMALL 2
#define GSR_ERR_CAPACITY 3
#define GSR_ERR_NONFINITE 4
#define GSR_ERR_HIP 5
#define GSR_ERR_STATE 6 /* call order: backward before forward, launch before capture */

#define GSR_MAX_VIEWS 32
/* Largest Gaussian count a plan accepts: the per-Gaussian kernels run one
 * thread per Gaussian on grids of at most 2^20 workgroups of 256 threads. */
#define GSR_MAX_GAUSSIANS ((int64_t)1 << 28)
#define GSR_MAX_IMAGE_SIDE 16384

/* Execution form. */
#define GSR_MODE_PLAIN 0   /* one launch chain per view, per-view count read-back */
#define GSR_MODE_BATCHED 1 /* all views in one chain, persistent fused raster, capturable */

/* Reverse pass of the blending sum (Sec. 3.2): how the transmittance in front
 * of each entry is obtained while walking a pixel's list back to front.  The
 * paper fixes only the sum; both forms give the same gradients (the choice
 * is a memory / time trade-off of this implementation). */
#define GSR_BWD_AUTO 0      /* stored history if it fits history_budget_bytes, else recompute */
#define GSR_BWD_RECOMPUTE 1 /* recover T_i = T_{i+1} / (1 - alpha_i) walking back */
#define GSR_BWD_STORED 2    /* read the per-(entry, pixel) transmittance saved by the forward */

/* One camera; the array lives in device memory so graph replays may take new
 * poses.  64 bytes. */
typedef struct gsr_camera {
  float R[9]; /* world -> camera rotation, row major */
  float t[3]; /* world -> camera translation */
  float fx, fy, cx, cy;
} gsr_camera;

typedef struct gsr_options {
  int32_t mode;          /* GSR_MODE_* */
  int32_t tile_w;        /* 16x16, 32x8 or 8x32 (width x height), 256 pixels */
  int32_t tile_h;
  int32_t bwd_variant;   /* GSR_BWD_* */
  int32_t lds_batch;     /* list entries staged in LDS per round: 64, 128 or 256 */
  int32_t grid_per_cu;   /* persistent raster grid = grid_per_cu * compute units (1..32) */
  int32_t accumulate_grads; /* 0: gradients are overwritten; 1: added to */
  int32_t check_finite;  /* 1: flag non-finite parameters (GSR_ERR_NONFINITE via query) */
  int32_t profile_stages; /* 1: time every stage of eager calls with device events */
  int32_t bwd_reduce;     /* reverse-pass reduction (each 16-lane row of a wavefront walks its own
                             entry list): 0 = a reduce-scatter over the row + one device atomic per
                             (row, record, component); 1 = per-lane LDS float atomics into a
                             per-batch accumulator + one device atomic per (tile, record,
                             component); 2 = as 1 after DPP sums over lane quads; 3 = as 1 after
                             DPP sums over 16-lane rows, one LDS atomic instruction per entry;
                             4 = as 3 with a reduce-scatter over the rows */
  int32_t project_table;  /* projection's tile counting: 0 = per-wavefront grouping of lanes that
                             share a tile, then device atomics; 1 = a per-workgroup table of tiles
                             in LDS, one device atomic per (workgroup, tile) (pays where wide
                             footprints make the device atomics' throughput the limit) */
  float near_plane, far_plane;
  float eps2d;           /* low-pass dilation of the 2D covariance */
  float sigma_extent;    /* footprint radius in standard deviations */
  float jac_clamp;       /* x/z, y/z clamp inside J, in half fields of view */
  float alpha_min, alpha_max, T_min;
  float bg[3];
  float stat_scale;      /* densification statistic scale; <= 0 means n_views */
  int64_t capacity_intersections; /* static capacity of (tile, Gaussian) entries;
                                     0: 4 n n_views (at least 65536, at most 2^31) */
  int64_t history_budget_bytes;   /* device bytes the stored history may use (AUTO/STORED) */
} gsr_options;

/* Static shape of a problem; widths/heights are host arrays [n_views]. */
typedef struct gsr_problem {
  int64_t n;         /* 1..GSR_MAX_GAUSSIANS, and n * n_views < 2^32 */
  int32_t sh_degree; /* 0..3; K = (sh_degree + 1)^2 coefficients per channel */
  int32_t n_views;   /* 1..GSR_MAX_VIEWS */
  const int32_t *widths;
  const int32_t *heights;
} gsr_problem;

/* Device pointers to structure-of-arrays float32 planes of length n. */
typedef struct gsr_gaussians {
  const float *means;          /* [3][n] */
  const float *log_scales;     /* [3][n] */
  const float *quats;          /* [4][n], (w, x, y, z), need not be unit */
  const float *opacity_logits; /* [n] */
  const float *sh;             /* [3K][n], plane k*3 + channel */
  const uint8_t *keep;         /* [n] or NULL: Gaussians with keep = 0 are culled */
} gsr_gaussians;

/* Gradient planes, same layout as gsr_gaussians (device). */
typedef struct gsr_grads {
  float *means, *log_scales, *quats, *opacity_logits, *sh;
} gsr_grads;

/* Densification statistics (device, accumulated across calls; the caller
 * resets them).  Either pointer may be NULL to skip it. */
typedef struct gsr_stats {
  float *grad2d_norm_sum;  /* [n] += stat_scale * |dL/dmean2d|_2 per visible view */
  uint32_t *visible_count; /* [n] += 1 per view in which the Gaussian is visible */
} gsr_stats;

typedef struct gsr_counts {
  int64_t visible[GSR_MAX_VIEWS];       /* visible Gaussians per view */
  int64_t intersections[GSR_MAX_VIEWS]; /* (tile, Gaussian) entries per view */
  int64_t visible_total, intersections_total;
  int64_t visible_union; /* Gaussians visible in at least one view */
  int32_t overflow;      /* 1 when capacity_intersections was exceeded */
  int32_t nonfinite;     /* 1 when check_finite found a non-finite parameter */
  int32_t tile_w, tile_h, bwd_variant, lds_batch, grid_per_cu, mode;
} gsr_counts;

/* Internal byte offsets of the workspace (for tests and profiling).  grad2d
 * holds one slot of GSR_SLOT_FLOATS 32-bit words per record: in words 0..8
 * what the reverse raster pass sums for the record, the moments of dL/dp over
 * the pixel offsets d = pixel - mean2d (gp dx, gp dy, gp dx^2, gp dx dy,
 * gp dy^2, with p = -d^T Q d / 2 the exponent of the Gaussian's alpha), then
 * dL/dopacity and dL/dcolour (3); its 2D gradient is dL/dmean2d = Q (m0, m1),
 * dL/d(A, B, C) = -(m2 / 2, m3, m4 / 2).  Then its in-tile ranks (4 x u32),
 * tile rectangle (2 x u32) and depth bits. */
#define GSR_SLOT_FLOATS 16
typedef struct gsr_layout {
  size_t header, view_table, view_bits, records, grad2d, tile_count, tile_start, tile_fill,
      tile_loss, tile_order, keys, keys_alt, pix_T, pix_last, pix_dLdC, history, total;
  int64_t vn;              /* n_views * n record slots (record of (v, i) at v * n + i) */
  int64_t tiles_total;     /* tiles over all views for the plan's tile shape */
  int64_t pixels_total;
  int64_t capacity;        /* intersection capacity */
  int64_t history_entries; /* stored-history capacity in (entry, pixel) pairs, 0 if none */
} gsr_layout;

typedef struct gsr_plan gsr_plan;

/* Fills *opt with the defaults above (plain mode, 16x16 tiles, recompute backward,
 * LDS batch 128, 4 persistent workgroups per compute unit, reverse reduction 0). */
void gsr_default_options(gsr_options *opt);

/* Creates a plan for a static problem shape.  Host only (no device call).
 * INVALID_ARG: null pointers, n <= 0, n * n_views >= 2^32, sh_degree outside
 * 0..3, n_views outside 1..32, a side outside 1..16384, an unsupported tile
 * shape, lds_batch or grid_per_cu out of range, non-positive thresholds. */
gsr_status gsr_plan_create(gsr_plan **plan, const gsr_problem *problem, const gsr_options *opt);
gsr_status gsr_plan_destroy(gsr_plan *plan);

/* Workspace bytes for this plan: large enough for every tile shape, so the
 * autotuner may switch shapes within one workspace.  Host only. */
gsr_status gsr_workspace_size(const gsr_plan *plan, size_t *bytes);
gsr_status gsr_workspace_layout(const gsr_plan *plan, gsr_layout *layout);

/* Pixel offset of view v inside the packed image/target buffers
 * (images are [3][H_v][W_v] per view, back to back; offset in floats). */
gsr_status gsr_image_offset(const gsr_plan *plan, int32_t view, int64_t *offset_floats);

/* Forward render of every view (Sec. 3.2 blending; frustum culling Sec. 3.3).
 * images: packed [3][H][W] per view (device, written).  Keeps what the
 * reverse pass needs in the workspace.  T_final/last may be NULL. */
gsr_status gsr_forward(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams,
                       float *images, float *T_final, uint32_t *last, void *ws, size_t ws_bytes,
                       void *stream);

/* Reverse pass for an arbitrary image gradient dL_dimages (packed like
 * images) after gsr_forward on the same plan and workspace: the exact
 * derivative of the blending sum (Sec. 3.2) through the projection to every
 * raw parameter, and the view-space gradient statistic and visible count
 * that selective densification reads (Sec. 3.3).  Writes grads (or adds,
 * with accumulate_grads) and accumulates stats (may be NULL).
 * GSR_ERR_STATE when no gsr_forward precedes it on this plan (each forward
 * allows one reverse pass). */
gsr_status gsr_backward(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams,
                        const float *dL_dimages, const gsr_grads *grads, const gsr_stats *stats,
                        void *ws, size_t ws_bytes, void *stream);

/* One fused training step of a block (Sec. 3, per-block fine training; its
 * image loss is the L1 term of vanilla 3DGS, App. A.1): forward, L = mean over
 * views of the per-view mean |image - target|, reverse pass (dL/dimage =
 * sign(image - target) / (3 H W n_views), sign(0) = 0), statistics (Sec. 3.3).
 * loss: one device float.  Inputs, outputs and errors as gsr_forward and
 * gsr_backward. */
gsr_status gsr_forward_backward_l1(gsr_plan *plan, const gsr_gaussians *g,
                                   const gsr_camera *cams, const float *targets, float *images,
                                   float *loss, const gsr_grads *grads, const gsr_stats *stats,
                                   void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): the fused step of
 * gsr_forward_backward_l1, same arguments and results, with the workspace
 * taken from a static device array of GSR_STATIC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends.  No device
 * memory is allocated or freed; no stage timing (profile_stages is ignored).
 * GSR_ERR_WORKSPACE_TOO_SMALL when gsr_workspace_size exceeds the array.
 * Calls on one GPU share the array: calls that overlap on one GPU race.  The
 * stream must belong to the current device. */
#define GSR_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
gsr_status gsr_forward_backward_l1_static(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams,
                                          const float *targets, float *images, float *loss,
                                          const gsr_grads *grads, const gsr_stats *stats, void *stream);

/* Visibility cropping over the plan's views (Sec. 3.3): view_bits[i] has bit
 * v set when Gaussian i is visible in view v; keep_out[i] = (view_bits != 0);
 * in_block[i] = 1 when the mean lies in the half-open box aabb = (xmin, ymin,
 * zmin, xmax, ymax, zmax) (host array).  Any output pointer may be NULL. */
gsr_status gsr_visibility_mask(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams,
                               const float *aabb, uint32_t *view_bits, uint8_t *keep_out,
                               uint8_t *in_block, void *ws, size_t ws_bytes, void *stream);

/* Graph form of the training step (Sec. 3: each block trains on its
 * assigned cameras, all of them per step here).  Records the batched fused
 * step (same arguments as gsr_forward_backward_l1) into a graph owned by the
 * plan; gsr_graph_launch replays it on a stream.
 * The stream must be capturable (not the legacy null stream).  Requires
 * GSR_MODE_BATCHED.  Replays read the same buffers, so new parameters or
 * poses are taken by writing into them. */
gsr_status gsr_graph_capture(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams,
                             const float *targets, float *images, float *loss,
                             const gsr_grads *grads, const gsr_stats *stats, void *ws,
                             size_t ws_bytes, void *stream);
gsr_status gsr_graph_launch(gsr_plan *plan, void *stream);

/* Counts of the last step: enqueues a small kernel that derives the visible
 * counts from the view masks in the workspace (writing the workspace header),
 * synchronises the stream and reads the header.  Returns GSR_ERR_CAPACITY /
 * GSR_ERR_NONFINITE when the corresponding flag is set (counts are still
 * filled in). */
gsr_status gsr_query_counts(gsr_plan *plan, const void *ws, gsr_counts *counts, void *stream);

/* Times the batched fused step for each candidate (tile shape 16x16, 32x8,
 * 8x32; lds_batch; grid_per_cu; backward variant within the history budget;
 * reverse reduction 0, 2, 3, 4) with device events, `reps` steps each after
 * one warm-up step, a candidate scoring its fastest step; the three fastest
 * are timed again over 2 reps + 3 steps, then the fastest of those with the
 * other project_table setting; the fastest is stored in the plan.  Steps
 * write images, loss and grads like gsr_forward_backward_l1.  *best receives
 * the choice (fields tile_w/tile_h/bwd_variant/lds_batch/grid_per_cu/
 * bwd_reduce/project_table); best_ms the time of one step (may be NULL). */
gsr_status gsr_autotune(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams,
                        const float *targets, float *images, float *loss, const gsr_grads *grads,
                        void *ws, size_t ws_bytes, int32_t reps, gsr_options *best,
                        float *best_ms, void *stream);

/* Per-stage device time of the last eager call made with profile_stages = 1
 * (graph replays are not timed).  Synchronises on the recorded events.
 * Stages with the same name (one per view in the plain form) are summed;
 * launches counts them. */
#define GSR_MAX_STAGES 16
typedef struct gsr_stage_times {
  int32_t count;
  int32_t launches[GSR_MAX_STAGES];
  float ms[GSR_MAX_STAGES];
  char name[GSR_MAX_STAGES][32];
} gsr_stage_times;
gsr_status gsr_last_stage_times(gsr_plan *plan, gsr_stage_times *out);

/* Current options of a plan (after autotuning). */
gsr_status gsr_plan_options(const gsr_plan *plan, gsr_options *opt);
/* Changes the tuning fields (tile_w, tile_h, bwd_variant, lds_batch,
 * grid_per_cu, bwd_reduce, project_table) of a plan; drops a captured graph. */
gsr_status gsr_plan_set_tuning(gsr_plan *plan, const gsr_options *opt);

/* ---- Fast camera selection (Sec. 3.2) -----------------------------------
 * gsr_render_depth: gsr_forward (same images) plus the per-pixel depth of
 * the blending sum, D = sum_i d_i alpha_i T_i with d_i the camera-space depth
 * of Gaussian i's mean, under the same skip and stop rules as the colour
 * (the depth form of the blending equation, Sec. 3.2; not normalised by the
 * accumulated opacity).  depth: device [sum_v H_v W_v] floats, packed by view
 * in input order, row-major.
 *
 * gsr_camera_coverage: the visibility ratio V_{c,b} of Sec. 3.2.  Each pixel
 * (u, v) of each view is back-projected with its depth through its centre,
 * p = R^T (D ((u + 1/2 - cx) / fx, (v + 1/2 - cy) / fy, 1) - t) (float64),
 * and counted into every block that holds it; a block is the half-open box
 * [min, max) of blocks[b] = (xmin, ymin, zmin, xmax, ymax, zmax) (device
 * [n_blocks][6] floats, 1 <= n_blocks <= GSR_MAX_COVERAGE_BLOCKS).  Outputs
 * (device, [n_views][n_blocks]): counts (cleared by the call), ratio =
 * counts / (W H) (N_p = all pixels of the view) and selected = (ratio >= tau),
 * the camera assignment C^(b) = {c | V_{c,b} >= tau}; ratio and selected may
 * be NULL.  Uses no workspace; the plan gives the views' sizes. */
#define GSR_MAX_COVERAGE_BLOCKS 1024

gsr_status gsr_render_depth(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, float *images,
                            float *depth, void *ws, size_t ws_bytes, void *stream);

/* Profiling: the forward render of gsr_forward (same images) that also
 * counts, per pixel, the (pixel, list entry) pairs of the blending sum
 * (Sec. 3.2): counts[p] = pairs blended into pixel p (alpha >= alpha_min
 * before the stop), counts[P + p] = pairs whose alpha the pixel's lane
 * evaluated after the per-sub-block culling (P = sum_v H_v W_v, pixels packed
 * by view in input order, row-major).  counts: device [2 P] u32, written.
 * The reverse pass cannot follow this call (GSR_ERR_STATE until the next
 * gsr_forward).  Errors as gsr_forward. */
gsr_status gsr_pair_counts(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, float *images,
                           uint32_t *counts, void *ws, size_t ws_bytes, void *stream);

gsr_status gsr_camera_coverage(gsr_plan *plan, const gsr_camera *cams, const float *depth, const float *blocks,
                               int32_t n_blocks, float tau, uint32_t *counts, float *ratio, uint8_t *selected,
                               void *stream);

/* ---- Load-balanced KD-tree partition (Sec. 3.1, App. A.5) ---------------
 * The tree is grown on the host; gsr_partition_blocks also counts the pixels
 * on the host, gsr_partition_blocks_device counts them on the GPU.  Both give
 * identical results for the same points. */
#define GSR_MAX_REFINE_STEPS 16

/*
 * Splits the scene box (scene_aabb: xmin, ymin, zmin, xmax, ymax, zmax,
 * half-open) into n_blocks leaves, best-first: while fewer than n_blocks
 * leaves, the leaf with the most cameras (the earliest created among equals)
 * is split orthogonally to the longer of its x / y extents (x on a tie).  The
 * cut at percentile q is the order statistic of index floor(q (m - 1)) of the
 * m Gaussian centres in the leaf along that axis (the extent's middle when
 * m = 0); left child [min, cut), right [cut, max).  Each child receives the
 * parent's cameras whose back-projected pixels fall into it with ratio >= tau
 * (fast camera selection, Sec. 3.2).  Cutline refinement: q starts at 0.5
 * (the median), q_low = q_min, q_high = q_max; for refine_steps evaluations
 * (the paper uses 3, with q_min 0.1 and q_max 0.9): if the left child has more
 * cameras, q_high = q and q = (q_low + q) / 2; if the right one has more,
 * q_low = q and q = (q_high + q) / 2; on a tie stop.  The children of the last
 * evaluated split are kept.  All on host memory, float comparisons:
 * centers [3][n]; points [3][total] (x plane, y plane, z plane), the pixels of
 * view v at [view_offsets[v], view_offsets[v + 1]) (view_offsets[0] = 0, all
 * W H pixels of the view, e.g. from gsr_back_project); outputs blocks_out
 * [n_blocks][6], assign_out [n_blocks][n_views] (1 = camera assigned; may be
 * NULL), workload_out [n_blocks] (camera counts; may be NULL), leaves in
 * creation order.  Needs no GPU and no plan; all buffers are the caller's.
 * GSR_ERR_INVALID_ARG for a null required pointer, n < 0, n_views < 1,
 * n_blocks < 1, refine_steps < 1, not 0 < q_min < q_max < 1, a non-finite
 * tau, refine_steps > GSR_MAX_REFINE_STEPS, view_offsets[0] != 0 or
 * decreasing offsets; outputs then untouched. */
gsr_status gsr_partition_blocks(const float *scene_aabb, const float *centers, int64_t n, const float *points,
                                const int64_t *view_offsets, int32_t n_views, int32_t n_blocks, float tau,
                                int32_t refine_steps, float q_min, float q_max, float *blocks_out,
                                uint8_t *assign_out, int32_t *workload_out);

/* Bytes of device workspace gsr_partition_blocks_device needs for n_views
 * cameras (about 4 KiB per camera).  GSR_ERR_INVALID_ARG for n_views < 1. */
gsr_status gsr_partition_workspace_size(int32_t n_views, size_t *bytes);

/* gsr_partition_blocks with the pixel counting on the GPU: `points` is
 * DEVICE memory [3][total] (e.g. gsr_back_project's output, left resident);
 * scene_aabb, centers, view_offsets and the three outputs are host memory.
 * Per split, one kernel counts the parent's cameras' pixels into both
 * children of every percentile the bisection can reach (when those
 * 2 (2^refine_steps - 1) boxes fit in GSR_MAX_COVERAGE_BLOCKS, else of each
 * evaluated split in turn), then the host walks the bisection.  Works on
 * `stream` and synchronizes it once per split; ws is caller-owned device
 * memory of gsr_partition_workspace_size bytes.  Errors as
 * gsr_partition_blocks, plus GSR_ERR_WORKSPACE_TOO_SMALL and GSR_ERR_HIP. */
gsr_status gsr_partition_blocks_device(const float *scene_aabb, const float *centers, int64_t n,
                                       const float *points, const int64_t *view_offsets, int32_t n_views,
                                       int32_t n_blocks, float tau, int32_t refine_steps, float q_min, float q_max,
                                       void *ws, size_t ws_bytes, void *stream, float *blocks_out,
                                       uint8_t *assign_out, int32_t *workload_out);

/* The back-projected pixels of gsr_camera_coverage as points: points [3][P]
 * (device, P = sum_v H_v W_v, view-major, row-major pixels; x plane, then y,
 * then z), float64 arithmetic rounded to float32; depth is the [V][H][W]
 * output of gsr_render_depth.  Enqueued on `stream`; GSR_ERR_INVALID_ARG for a
 * null pointer, GSR_ERR_HIP if the launch fails. */
gsr_status gsr_back_project(gsr_plan *plan, const gsr_camera *cams, const float *depth, float *points,
                            void *stream);

/* ---- Selective densification and pruning (Sec. 3.3) -------------------
 * The fine stage densifies like vanilla 3DGS (App. A.1) except that only
 * Gaussians inside the block may densify (selective densification).  Per
 * Gaussian i, with S_i and n_i the statistics of gsr_stats:
 *   - keep[i] = 0 (gsr_gaussians.keep, e.g. the in-block mask when the
 *     blocks are merged, Fig. 1): no output;
 *   - candidate when n_i > 0, S_i / n_i >= grad_threshold and, with
 *     selective = 1, in_block[i] = 1;
 *   - a candidate whose largest exp(log_scale) is <= clone_max_scale is
 *     cloned: the original (keeping its optimizer moments) and a copy (zero
 *     moments);
 *   - any other candidate is split into two children that replace it:
 *     child j's mean is mean + R(q/|q|) (exp(log_scale) * eps_j) with eps_j
 *     = samples[j][0..2][i] (standard normal draws the caller makes), its
 *     log scales are log_scale - ln(1.6) rounded to float (the scale divided
 *     by 0.8 times two children), quaternion, opacity and SH copied, zero
 *     moments;
 *   - every output is pruned when sigmoid(opacity logit) < min_opacity
 *     (min_opacity > 0) or its largest exp(log_scale) > max_world_scale
 *     (max_world_scale > 0).
 * The S_i / n_i, scale and opacity tests are made exactly on the float
 * inputs (S_i >= threshold n_i in double; log scale and logit against the
 * double logarithms of the thresholds).  Outputs of Gaussian i are written
 * at the prefix sum of the output counts of Gaussians 0..i-1 (input order
 * kept, a clone or the children next to their parent). */
typedef struct gsr_densify_opts {
  float grad_threshold;  /* densify when S / n >= this; +inf turns densification off */
  float clone_max_scale; /* > 0: clone at or below this largest scale, split above */
  float min_opacity;     /* in [0, 1); 0 turns the opacity pruning off */
  float max_world_scale; /* <= 0 turns the size pruning off */
  int32_t selective;     /* 1: only in_block Gaussians densify; 0: every Gaussian may */
  int32_t reserved;      /* 0 */
} gsr_densify_opts;

/* Device workspace bytes of the densification of n Gaussians (8 bytes per
 * 1024 Gaussians plus 16). */
gsr_status gsr_densify_workspace_size(int64_t n, size_t *bytes);

/* First half: decides every Gaussian and counts the outputs.  g (device
 * planes of n Gaussians, keep optional), stats (both pointers required) and
 * in_block (device [n] u8, required when selective = 1) are read on
 * `stream` (with n = 0 they may be null); the stream is synchronized and
 * *n_out (host) receives the output count.  The workspace keeps the per-block offsets for
 * gsr_densify_apply.  GSR_ERR_INVALID_ARG for n < 0, sh_degree outside
 * 0..3, a null required pointer, clone_max_scale <= 0, min_opacity outside
 * [0, 1) or a NaN threshold; GSR_ERR_WORKSPACE_TOO_SMALL; GSR_ERR_HIP. */
gsr_status gsr_densify_count(int64_t n, int32_t sh_degree, const gsr_densify_opts *opts, const gsr_gaussians *g,
                             const gsr_stats *stats, const uint8_t *in_block, void *ws, size_t ws_bytes,
                             void *stream, int64_t *n_out);

/* Second half: writes the n_out outputs counted by gsr_densify_count, whose
 * workspace and inputs it must be given unchanged, on the same stream.
 * out: writable device planes of n_out Gaussians (gsr_grads layout: means
 * [3][n_out], log_scales, quats, opacity_logits, sh [3K][n_out]).  m_in /
 * v_in and m_out / v_out (Adam moments, same layouts over n and n_out) are
 * optional together (NULL: no moments); parent_out (device [n_out] int64,
 * optional) receives each output's input index.  samples: device
 * [2][3][n] float.  Outputs beyond n_out are never written.  The caller
 * resets the statistics afterwards.  Errors as gsr_densify_count. */
gsr_status gsr_densify_apply(int64_t n, int32_t sh_degree, const gsr_densify_opts *opts, const gsr_gaussians *g,
                             const gsr_grads *m_in, const gsr_grads *v_in, const gsr_stats *stats,
                             const uint8_t *in_block, const float *samples, int64_t n_out, const gsr_grads *out,
                             const gsr_grads *m_out, const gsr_grads *v_out, int64_t *parent_out, void *ws,
                             size_t ws_bytes, void *stream);

/* ---- Optimizer step (the NEXT stage after the reverse projection) ------
 * The paper locates the cost of Gaussians that no assigned camera sees in the
 * optimizer rather than in rendering (Sec. 3.3) and uses Sparse Adam in the
 * coarse stage (App. A.1).  One Adam step (Kingma & Ba, bias-corrected) over
 * every parameter plane of the plan's n Gaussians:
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   p -= lr / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps)
 * with one learning rate per group.  params, grads, m, v: device planes in
 * the gsr_gaussians layout (grads as written by the reverse pass); updated in
 * place.  visible_bits: NULL for the dense step, else [n] u32 (e.g. the
 * workspace's view_bits of the last step): Gaussians whose word is 0 keep
 * their parameters and moments untouched (visible-only Adam).  float32
 * arithmetic; bias corrections in float64 on the host. */
typedef struct gsr_adam {
  float lr[6];  /* means, log_scales, quats, opacity_logits, SH band 0, SH bands >= 1 */
  float beta1, beta2, eps;
  int32_t step; /* t >= 1 */
} gsr_adam;

gsr_status gsr_adam_step(gsr_plan *plan, const gsr_adam *hp, const gsr_grads *params, const gsr_grads *grads,
                         const gsr_grads *m, const gsr_grads *v, const uint32_t *visible_bits, void *stream);

const char *gsr_status_string(gsr_status s);
const char *gsr_last_error(const gsr_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */
