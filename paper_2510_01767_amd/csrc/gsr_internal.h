// Internal types shared by the host orchestration and the HIP kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "gsr.h"

namespace gsr {

// One view of the plan as the kernels see it (copied into the workspace by
// the set-up kernel of every step).
struct ViewInfo {
  int32_t W, H, tiles_x, tiles_y;
  int64_t tile_base;  // first global tile id of the view
  int64_t pix_base;   // first pixel of the view in the packed [3][H][W] images (in floats / 3)
  float loss_scale;   // 1 / (3 H W n_views)
  int32_t pad[3];
};

struct ViewTable {
  ViewInfo v[GSR_MAX_VIEWS];
  int32_t n_views;
  int32_t pad[3];
};

// Device-side header at the start of the workspace.
struct WsHeader {
  uint32_t overflow;
  uint32_t nonfinite;
  uint32_t union_count;   // Gaussians visible in >= 1 view
  uint32_t isect_total;
  // the per-tile sort's lists, collected per sort call: runs of 2048 keys
  // (tiles of 1025..2048 entries), of 4096 (2049..4096), of 8192 (the runs
  // of longer tiles), and the tiles longer than one run (merged in global
  // memory, taken from the work counter big_next)
  uint32_t run2_count, run_count, run8_count;
  uint32_t big_count, big_next;
  uint32_t isect[GSR_MAX_VIEWS];
  uint32_t visible[GSR_MAX_VIEWS];
  // longest-list-first schedule of the persistent raster: tiles per length
  // bin (descending) and the bins' fill cursors
  uint32_t order_bins[1024];
  uint32_t order_cursor[1024];
  // persistent raster work counters, one per workgroup class (blockIdx mod
  // 8), each in a 128-byte line of its own
  uint32_t queue[8][32];
  // per-view loss sums (scaled), added up in view order for the loss
  double view_loss[GSR_MAX_VIEWS];
};
constexpr int kOrderBins = 1024;

// Rasterizer constants as kernel arguments.
struct KOpts {
  float near_plane, far_plane, eps2d, sigma, jac_clamp, alpha_min, alpha_max, T_min;
  float bg[3];
  float stat_scale;
  int32_t tile_w, tile_h;
  int32_t check_finite;
  int32_t accumulate;
};

struct KParams {
  const float *means, *log_scales, *quats, *logits, *sh;
  const uint8_t *keep;
  int64_t n;
  int32_t sh_degree;
  int32_t n_views;
};

struct KGrads {
  float *means, *log_scales, *quats, *logits, *sh;
};

// Record of one (view, Gaussian) pair, 64 bytes (4 x float4):
//   r0 = mean2d as float pairs (hi x, hi y, lo x, lo y): mean = hi + lo
//   r1 = the exponent's coefficients in base 2, (a, b, c) = log2(e) (-A/2,
//        -B, -C/2) for the conic (A, B, C), so that the exponent is
//        p log2(e) = a dx^2 + b dx dy + c dy^2; opacity
//   r2 = colour (r, g, b), pmin log2(e) (pmin: exponent below which
//        alpha < alpha_min)
//   r3 = rect (x0 | y0 << 16, x1 | y1 << 16), depth (camera z, float bits),
//        reach of the alpha >= alpha_min ellipse in pixels (float bits)
constexpr int kRecordFloat4 = 4;
// Slot of one record, 64 bytes (16 x 32 bit, one memory segment):
//   [0, 9)   summed by the reverse raster pass (cleared by the projection):
//            moments of dL/dp over the pixel offsets d (gp dx, gp dy,
//            gp dx^2, gp dx dy, gp dy^2), dopacity, dcolour (3); the reverse
//            projection turns the moments into dmean and dconic
//   [9, 13)  in-tile ranks of the record's first four tiles (u32)
//   [13, 15) tile rectangle (x0 | y0 << 16, x1 | y1 << 16)
//   [15]     depth (camera z, float bits: the sort key's high word)
// The projection writes the slot whole; the scatter reads its upper half.
constexpr int kGrad2dStride = GSR_SLOT_FLOATS;

struct KWs {
  WsHeader *hdr;
  ViewInfo *views;
  uint32_t *view_bits;
  float *records;   // [vn][16]
  float *grad2d;    // [vn][16] record slots
  uint32_t *tile_count, *tile_start, *tile_fill;
  float *tile_loss;
  uint32_t *tile_order;
  uint64_t *keys, *keys_alt;
  float *pix_T;
  uint32_t *pix_last;
  float *pix_dLdC;
  float *history;
  int64_t vn, tiles_total, pixels_total, capacity, history_entries;
};

// ---------------------------------------------------------------- launchers
// Defined in gsr_kernels.hip; every launcher enqueues on `stream` and returns
// the launch's hipError_t as int.

int launch_setup(const ViewTable &table, const KWs &ws, int64_t zero_tiles_from, int64_t zero_tiles_count,
                 int zero_view_bits, int64_t n, void *stream);
int launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, void *stream);
int launch_fill_f32(float *p, float value, int64_t count, void *stream);
int launch_project(const KParams &p, const gsr_camera *cams, const KOpts &o, const KWs &ws, int view_lo,
                   int view_hi, int or_bits, int table, void *stream);
int launch_scan(const KWs &ws, int64_t tile_lo, int64_t tile_hi, int64_t base, int view_lo, int view_hi,
                void *stream);
int launch_emit(const KWs &ws, int64_t n, int n_views, int view_only, void *stream);
int launch_sort(const KWs &ws, int64_t tile_lo, int64_t tile_count, void *stream);
int launch_raster_fwd(const KWs &ws, const KOpts &o, int64_t tile_lo, int64_t tile_count, float *images,
                      int n_views, int store_history, int lds_batch, float *depth, uint32_t *pair_counts,
                      void *stream);
int launch_l1(const KWs &ws, const KOpts &o, int64_t tile_lo, int64_t tile_count, const float *images,
              const float *targets, int n_views, void *stream);
int launch_raster_bwd(const KWs &ws, const KOpts &o, int64_t tile_lo, int64_t tile_count, const float *dLdC,
                      int n_views, int use_history, int lds_batch, int red, void *stream);
int launch_fused(const KWs &ws, const KOpts &o, const float *targets, float *images, int n_views,
                 int use_history, int lds_batch, int red, int grid, void *stream);
int launch_project_bwd(const KParams &p, const gsr_camera *cams, const KOpts &o, const KWs &ws,
                       const KGrads &g, float *stat_S, uint32_t *stat_n, int view_only, void *stream);
int launch_loss(const KWs &ws, int n_views, float *loss, void *stream);
int launch_visibility(const KParams &p, const gsr_camera *cams, const KOpts &o, const KWs &ws,
                      const float *aabb6, uint32_t *bits, uint8_t *keep_out, uint8_t *in_block,
                      void *stream);
int launch_copy_pixels(const KWs &ws, float *T_out, uint32_t *last_out, void *stream);

int launch_count_visible(const KWs &ws, int64_t n, int n_views, void *stream);
int launch_tile_order(const KWs &ws, void *stream);

// ------------------------------------------------------- host entry helpers
// Defined in gsr_api.cpp.  fused_l1_no_events: gsr_forward_backward_l1
// without stage timing (creates no event).  plan_error: records msg as the
// plan's last error and returns s.
gsr_status fused_l1_no_events(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, const float *targets,
                              float *images, float *loss, const gsr_grads *grads, const gsr_stats *stats, void *ws,
                              size_t ws_bytes, void *stream);
gsr_status plan_error(gsr_plan *plan, gsr_status s, const char *msg);

}  // namespace gsr
