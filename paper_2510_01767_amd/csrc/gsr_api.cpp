// Host side of the C ABI: argument validation, workspace layout, the launch
// sequences of the plain and batched forms, graph capture, counts and the
// autotuner.  Plan creation, validation and layout never touch the device,
// so they run (and are tested) on machines without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gsr_internal.h"
#include "gsr_stages.h"

struct gsr_plan {
  gsr_problem prob;
  std::vector<int32_t> W, H;
  gsr_options opt;
  gsr_layout layout;  // for the current tile shape
  size_t ws_bytes;    // required workspace (all tile shapes)
  std::string err;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool forward_ready = false;
  bool capturing = false;
  int n_cus = 0;
  struct Stage {
    std::string name;
    int a, b;
  };
  std::vector<hipEvent_t> ev_pool;
  std::vector<Stage> stages;
  int ev_used = 0;
};

namespace {

using namespace gsr;

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool tile_shape_ok(int tw, int th) {
  return (tw == 16 && th == 16) || (tw == 32 && th == 8) || (tw == 8 && th == 32);
}

int64_t tiles_for(const gsr_plan &p, int tw, int th) {
  int64_t t = 0;
  for (size_t v = 0; v < p.W.size(); v++) t += (int64_t)((p.W[v] + tw - 1) / tw) * ((p.H[v] + th - 1) / th);
  return t;
}

int64_t pixels_of(const gsr_plan &p) {
  int64_t s = 0;
  for (size_t v = 0; v < p.W.size(); v++) s += (int64_t)p.W[v] * p.H[v];
  return s;
}

int64_t default_capacity(const gsr_problem &pr) {
  int64_t c = 4 * pr.n * (int64_t)pr.n_views;
  if (c < 65536) c = 65536;
  if (c > ((int64_t)1 << 31)) c = (int64_t)1 << 31;
  return c;
}

bool history_allowed(const gsr_options &o, int64_t capacity) {
  if (o.bwd_variant == GSR_BWD_RECOMPUTE) return false;
  const double bytes = (double)capacity * 256.0 * 4.0;
  return bytes <= (double)o.history_budget_bytes;
}

void compute_layout(gsr_plan &p) {
  gsr_layout L;
  memset(&L, 0, sizeof L);
  const int64_t n = p.prob.n, V = p.prob.n_views;
  const int64_t tmax = std::max({tiles_for(p, 16, 16), tiles_for(p, 32, 8), tiles_for(p, 8, 32)});
  L.vn = n * V;
  L.tiles_total = tiles_for(p, p.opt.tile_w, p.opt.tile_h);
  L.pixels_total = pixels_of(p);
  L.capacity = p.opt.capacity_intersections > 0 ? p.opt.capacity_intersections : default_capacity(p.prob);
  L.history_entries = history_allowed(p.opt, L.capacity) ? L.capacity * 256 : 0;
  size_t off = 0;
  auto take = [&](size_t &field, size_t bytes) {
    field = off;
    off = align_up(off + bytes);
  };
  take(L.header, sizeof(WsHeader));
  take(L.view_table, sizeof(ViewInfo) * GSR_MAX_VIEWS);
  take(L.view_bits, sizeof(uint32_t) * (size_t)n);
  take(L.records, sizeof(float) * 16 * (size_t)L.vn);
  take(L.grad2d, sizeof(float) * kGrad2dStride * (size_t)L.vn);
  take(L.tile_count, sizeof(uint32_t) * (size_t)tmax);
  take(L.tile_start, sizeof(uint32_t) * (size_t)(tmax + 1));
  take(L.tile_fill, sizeof(uint32_t) * (size_t)tmax);
  take(L.tile_loss, sizeof(float) * (size_t)tmax);
  // the schedule order; before the sort, the scan's chunk sums (8 bytes per 4096 tiles)
  take(L.tile_order, std::max(sizeof(uint32_t) * (size_t)tmax, sizeof(uint64_t) * (size_t)(tmax / 4096 + 2)));
  take(L.keys, sizeof(uint64_t) * (size_t)L.capacity);
  take(L.keys_alt, sizeof(uint64_t) * (size_t)L.capacity);
  take(L.pix_T, sizeof(float) * (size_t)L.pixels_total);
  take(L.pix_last, sizeof(uint32_t) * (size_t)L.pixels_total);
  take(L.pix_dLdC, sizeof(float) * 3 * (size_t)L.pixels_total);
  take(L.history, sizeof(float) * (size_t)L.history_entries);
  L.total = off;
  p.layout = L;
  p.ws_bytes = off;
}

gsr_status validate_options(const gsr_options &o) {
  if (o.mode != GSR_MODE_PLAIN && o.mode != GSR_MODE_BATCHED) return GSR_ERR_INVALID_ARG;
  if (!tile_shape_ok(o.tile_w, o.tile_h)) return GSR_ERR_INVALID_ARG;
  if (o.bwd_variant < GSR_BWD_AUTO || o.bwd_variant > GSR_BWD_STORED) return GSR_ERR_INVALID_ARG;
  if (o.lds_batch != 64 && o.lds_batch != 128 && o.lds_batch != 256) return GSR_ERR_INVALID_ARG;
  if (o.grid_per_cu < 1 || o.grid_per_cu > 32) return GSR_ERR_INVALID_ARG;
  if (o.bwd_reduce < 0 || o.bwd_reduce > 4) return GSR_ERR_INVALID_ARG;
  if (o.project_table != 0 && o.project_table != 1) return GSR_ERR_INVALID_ARG;
  if (!(o.near_plane > 0.0f) || !(o.far_plane > o.near_plane)) return GSR_ERR_INVALID_ARG;
  if (!(o.eps2d >= 0.0f) || !(o.sigma_extent > 0.0f) || !(o.jac_clamp > 0.0f)) return GSR_ERR_INVALID_ARG;
  if (!(o.alpha_min > 0.0f) || !(o.alpha_max > o.alpha_min) || !(o.alpha_max < 1.0f)) return GSR_ERR_INVALID_ARG;
  if (!(o.T_min > 0.0f) || !(o.T_min < 1.0f)) return GSR_ERR_INVALID_ARG;
  if (o.capacity_intersections < 0 || o.capacity_intersections > (int64_t)0xffffffffLL) return GSR_ERR_INVALID_ARG;
  if (o.history_budget_bytes < 0) return GSR_ERR_INVALID_ARG;
  for (int c = 0; c < 3; c++)
    if (!std::isfinite(o.bg[c])) return GSR_ERR_INVALID_ARG;
  return GSR_OK;
}

gsr_status validate_problem(const gsr_problem *pr) {
  if (!pr || !pr->widths || !pr->heights) return GSR_ERR_INVALID_ARG;
  if (pr->n <= 0 || pr->n > GSR_MAX_GAUSSIANS || pr->sh_degree < 0 || pr->sh_degree > 3) return GSR_ERR_INVALID_ARG;
  if (pr->n_views < 1 || pr->n_views > GSR_MAX_VIEWS) return GSR_ERR_INVALID_ARG;
  if (pr->n * (int64_t)pr->n_views >= ((int64_t)1 << 32)) return GSR_ERR_INVALID_ARG;
  for (int v = 0; v < pr->n_views; v++)
    if (pr->widths[v] < 1 || pr->widths[v] > GSR_MAX_IMAGE_SIDE || pr->heights[v] < 1 ||
        pr->heights[v] > GSR_MAX_IMAGE_SIDE)
      return GSR_ERR_INVALID_ARG;
  return GSR_OK;
}

gsr_status fail(gsr_plan *p, gsr_status s, const std::string &msg) {
  if (p) p->err = msg;
  return s;
}

gsr_status hip_check(gsr_plan *p, int e, const char *what) {
  if (e == (int)hipSuccess) return GSR_OK;
  return fail(p, GSR_ERR_HIP, std::string(what) + ": " + hipGetErrorString((hipError_t)e));
}

#define HIPCHK(expr, what)                        \
  do {                                            \
    gsr_status _s = hip_check(plan, (int)(expr), what); \
    if (_s != GSR_OK) return _s;                  \
  } while (0)

// Stage timing (profile_stages): a pair of device events around a launch.
int stage_begin(gsr_plan *p, const char *name, void *stream) {
  if (!p->opt.profile_stages || p->capturing) return -1;
  while ((int)p->ev_pool.size() < p->ev_used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    p->ev_pool.push_back(e);
  }
  gsr_plan::Stage st{name, p->ev_used, p->ev_used + 1};
  p->ev_used += 2;
  if (hipEventRecord(p->ev_pool[st.a], (hipStream_t)stream) != hipSuccess) return -1;
  p->stages.push_back(st);
  return (int)p->stages.size() - 1;
}

void stage_end(gsr_plan *p, int k, void *stream) {
  if (k >= 0) (void)hipEventRecord(p->ev_pool[p->stages[k].b], (hipStream_t)stream);
}

void stage_reset(gsr_plan *p) {
  p->stages.clear();
  p->ev_used = 0;
}

#define STAGE(expr, what)                          \
  do {                                             \
    int _k = stage_begin(plan, what, stream);      \
    HIPCHK(expr, what);                            \
    stage_end(plan, _k, stream);                   \
  } while (0)

gsr_status check_gaussians(const gsr_gaussians *g) {
  if (!g || !g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh) return GSR_ERR_INVALID_ARG;
  return GSR_OK;
}

gsr_status check_grads(const gsr_grads *g) {
  if (!g || !g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh) return GSR_ERR_INVALID_ARG;
  return GSR_OK;
}

gsr_status check_ws(gsr_plan *plan, const void *ws, size_t ws_bytes) {
  if (!ws) return fail(plan, GSR_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws) % kAlign != 0) return fail(plan, GSR_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < plan->ws_bytes) return fail(plan, GSR_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
  return GSR_OK;
}

ViewTable view_table(const gsr_plan &p) {
  ViewTable t;
  memset(&t, 0, sizeof t);
  const int tw = p.opt.tile_w, th = p.opt.tile_h;
  int64_t tb = 0, pb = 0;
  t.n_views = p.prob.n_views;
  for (int v = 0; v < p.prob.n_views; v++) {
    ViewInfo &vi = t.v[v];
    vi.W = p.W[v];
    vi.H = p.H[v];
    vi.tiles_x = (vi.W + tw - 1) / tw;
    vi.tiles_y = (vi.H + th - 1) / th;
    vi.tile_base = tb;
    vi.pix_base = pb;
    vi.loss_scale = (float)(1.0 / (3.0 * (double)vi.W * vi.H * p.prob.n_views));
    tb += (int64_t)vi.tiles_x * vi.tiles_y;
    pb += (int64_t)vi.W * vi.H;
  }
  return t;
}

KWs ws_view(const gsr_plan &p, void *ws) {
  char *b = (char *)ws;
  const gsr_layout &L = p.layout;
  KWs k;
  k.hdr = (WsHeader *)(b + L.header);
  k.views = (ViewInfo *)(b + L.view_table);
  k.view_bits = (uint32_t *)(b + L.view_bits);
  k.records = (float *)(b + L.records);
  k.grad2d = (float *)(b + L.grad2d);
  k.tile_count = (uint32_t *)(b + L.tile_count);
  k.tile_start = (uint32_t *)(b + L.tile_start);
  k.tile_fill = (uint32_t *)(b + L.tile_fill);
  k.tile_loss = (float *)(b + L.tile_loss);
  k.tile_order = (uint32_t *)(b + L.tile_order);
  k.keys = (uint64_t *)(b + L.keys);
  k.keys_alt = (uint64_t *)(b + L.keys_alt);
  k.pix_T = (float *)(b + L.pix_T);
  k.pix_last = (uint32_t *)(b + L.pix_last);
  k.pix_dLdC = (float *)(b + L.pix_dLdC);
  k.history = L.history_entries ? (float *)(b + L.history) : nullptr;
  k.vn = L.vn;
  k.tiles_total = L.tiles_total;
  k.pixels_total = L.pixels_total;
  k.capacity = L.capacity;
  k.history_entries = L.history_entries;
  return k;
}

KParams kparams(const gsr_plan &p, const gsr_gaussians *g) {
  KParams k;
  k.means = g->means;
  k.log_scales = g->log_scales;
  k.quats = g->quats;
  k.logits = g->opacity_logits;
  k.sh = g->sh;
  k.keep = g->keep;
  k.n = p.prob.n;
  k.sh_degree = p.prob.sh_degree;
  k.n_views = p.prob.n_views;
  return k;
}

KOpts kopts(const gsr_plan &p) {
  KOpts k;
  const gsr_options &o = p.opt;
  k.near_plane = o.near_plane;
  k.far_plane = o.far_plane;
  k.eps2d = o.eps2d;
  k.sigma = o.sigma_extent;
  k.jac_clamp = o.jac_clamp;
  k.alpha_min = o.alpha_min;
  k.alpha_max = o.alpha_max;
  k.T_min = o.T_min;
  for (int c = 0; c < 3; c++) k.bg[c] = o.bg[c];
  k.stat_scale = o.stat_scale > 0.0f ? o.stat_scale : (float)p.prob.n_views;
  k.tile_w = o.tile_w;
  k.tile_h = o.tile_h;
  k.check_finite = o.check_finite;
  k.accumulate = o.accumulate_grads;
  return k;
}

KGrads kgrads(const gsr_grads *g) {
  KGrads k;
  k.means = g->means;
  k.log_scales = g->log_scales;
  k.quats = g->quats;
  k.logits = g->opacity_logits;
  k.sh = g->sh;
  return k;
}

bool use_history(const gsr_plan &p) {
  if (p.layout.history_entries == 0) return false;
  return p.opt.bwd_variant == GSR_BWD_STORED || p.opt.bwd_variant == GSR_BWD_AUTO;
}

int n_cus(gsr_plan *p) {
  if (p->n_cus == 0) {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
      p->n_cus = c;
    else
      p->n_cus = 256;
  }
  return p->n_cus;
}

gsr_status zero_grads(gsr_plan *plan, const gsr_grads *g, void *stream) {
  const int64_t n = plan->prob.n;
  const int K = (plan->prob.sh_degree + 1) * (plan->prob.sh_degree + 1);
  STAGE(launch_fill_f32(g->means, 0.f, 3 * n, stream), "fill");
  STAGE(launch_fill_f32(g->log_scales, 0.f, 3 * n, stream), "fill");
  STAGE(launch_fill_f32(g->quats, 0.f, 4 * n, stream), "fill");
  STAGE(launch_fill_f32(g->opacity_logits, 0.f, n, stream), "fill");
  STAGE(launch_fill_f32(g->sh, 0.f, (int64_t)3 * K * n, stream), "fill");
  return GSR_OK;
}

// Project, bin and order every view.  Plain: one chain per view with a
// read-back of each view's intersection count (the plain form's only sync).
// Batched: one chain for all views, no host synchronisation.
gsr_status enqueue_front(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, const KWs &ws,
                         void *stream, bool plain_raster_fwd, float *images, float *depth = nullptr,
                         uint32_t *pair_counts = nullptr) {
  const ViewTable tbl = view_table(*plan);
  const KParams kp = kparams(*plan, g);
  const KOpts ko = kopts(*plan);
  const int V = plan->prob.n_views;
  STAGE(launch_setup(tbl, ws, 0, ws.tiles_total, plan->opt.mode == GSR_MODE_PLAIN ? 1 : 0, plan->prob.n, stream),
         "setup");
  if (plan->opt.mode == GSR_MODE_BATCHED) {
    STAGE(launch_project(kp, cams, ko, ws, 0, V, 0, plan->opt.project_table, stream), "project");
    STAGE(launch_scan(ws, 0, ws.tiles_total, 0, 0, V, stream), "scan");
    STAGE(launch_emit(ws, plan->prob.n, V, -1, stream), "emit");
    STAGE(launch_sort(ws, 0, ws.tiles_total, stream), "sort");
    return GSR_OK;
  }
  int64_t base = 0;
  for (int v = 0; v < V; v++) {
    const ViewInfo &vi = tbl.v[v];
    const int64_t nt = (int64_t)vi.tiles_x * vi.tiles_y;
    STAGE(launch_project(kp, cams, ko, ws, v, v + 1, 1, plan->opt.project_table, stream), "project");
    STAGE(launch_scan(ws, vi.tile_base, vi.tile_base + nt, base, v, v + 1, stream), "scan");
    uint32_t iv = 0;
    HIPCHK(hipMemcpyAsync(&iv, &ws.hdr->isect[v], sizeof iv, hipMemcpyDeviceToHost, (hipStream_t)stream), "count read-back");
    HIPCHK(hipStreamSynchronize((hipStream_t)stream), "count read-back");
    if (base + (int64_t)iv > ws.capacity)
      return fail(plan, GSR_ERR_CAPACITY, "intersection capacity exceeded in view " + std::to_string(v));
    STAGE(launch_emit(ws, plan->prob.n, V, v, stream), "emit");
    STAGE(launch_sort(ws, vi.tile_base, nt, stream), "sort");
    if (plain_raster_fwd)
      STAGE(launch_raster_fwd(ws, ko, vi.tile_base, nt, images, V, use_history(*plan) ? 1 : 0, plan->opt.lds_batch,
                              depth, pair_counts, stream),
             "raster_fwd");
    base += iv;
  }
  return GSR_OK;
}

gsr_status enqueue_batched_l1(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, const float *targets,
                              float *images, float *loss, const gsr_grads *grads, const gsr_stats *stats,
                              const KWs &ws, void *stream) {
  gsr_status s = enqueue_front(plan, g, cams, ws, stream, false, nullptr);
  if (s != GSR_OK) return s;
  const KOpts ko = kopts(*plan);
  const int V = plan->prob.n_views;
  const int grid = n_cus(plan) * plan->opt.grid_per_cu;
  STAGE(launch_tile_order(ws, stream), "order");
  STAGE(launch_fused(ws, ko, targets, images, V, use_history(*plan) ? 1 : 0, plan->opt.lds_batch,
                     plan->opt.bwd_reduce, grid, stream),
         "fused raster");
  STAGE(launch_project_bwd(kparams(*plan, g), cams, ko, ws, kgrads(grads), stats ? stats->grad2d_norm_sum : nullptr,
                            stats ? stats->visible_count : nullptr, -1, stream),
         "project_bwd");
  STAGE(launch_loss(ws, V, loss, stream), "loss");
  return GSR_OK;
}

gsr_status enqueue_plain_l1(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, const float *targets,
                            float *images, float *loss, const gsr_grads *grads, const gsr_stats *stats,
                            const KWs &ws, void *stream) {
  const ViewTable tbl = view_table(*plan);
  const KParams kp = kparams(*plan, g);
  const KOpts ko = kopts(*plan);
  const int V = plan->prob.n_views;
  const int hist = use_history(*plan) ? 1 : 0;
  if (!plan->opt.accumulate_grads) {
    gsr_status s = zero_grads(plan, grads, stream);
    if (s != GSR_OK) return s;
  }
  STAGE(launch_setup(tbl, ws, 0, ws.tiles_total, 1, plan->prob.n, stream), "setup");
  int64_t base = 0;
  for (int v = 0; v < V; v++) {
    const ViewInfo &vi = tbl.v[v];
    const int64_t nt = (int64_t)vi.tiles_x * vi.tiles_y;
    STAGE(launch_project(kp, cams, ko, ws, v, v + 1, 1, plan->opt.project_table, stream), "project");
    STAGE(launch_scan(ws, vi.tile_base, vi.tile_base + nt, base, v, v + 1, stream), "scan");
    uint32_t iv = 0;
    HIPCHK(hipMemcpyAsync(&iv, &ws.hdr->isect[v], sizeof iv, hipMemcpyDeviceToHost, (hipStream_t)stream), "count read-back");
    HIPCHK(hipStreamSynchronize((hipStream_t)stream), "count read-back");
    if (base + (int64_t)iv > ws.capacity)
      return fail(plan, GSR_ERR_CAPACITY, "intersection capacity exceeded in view " + std::to_string(v));
    STAGE(launch_emit(ws, plan->prob.n, V, v, stream), "emit");
    STAGE(launch_sort(ws, vi.tile_base, nt, stream), "sort");
    STAGE(launch_raster_fwd(ws, ko, vi.tile_base, nt, images, V, hist, plan->opt.lds_batch, nullptr, nullptr,
                            stream),
          "raster_fwd");
    STAGE(launch_l1(ws, ko, vi.tile_base, nt, images, targets, V, stream), "l1");
    STAGE(launch_raster_bwd(ws, ko, vi.tile_base, nt, ws.pix_dLdC, V, hist, plan->opt.lds_batch,
                            plan->opt.bwd_reduce, stream), "raster_bwd");
    STAGE(launch_project_bwd(kp, cams, ko, ws, kgrads(grads), stats ? stats->grad2d_norm_sum : nullptr,
                              stats ? stats->visible_count : nullptr, v, stream),
           "project_bwd");
    base += iv;
  }
  STAGE(launch_loss(ws, V, loss, stream), "loss");
  return GSR_OK;
}

void drop_graph(gsr_plan *p) {
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
}

}  // namespace

extern "C" {

void gsr_default_options(gsr_options *o) {
  if (!o) return;
  memset(o, 0, sizeof *o);
  o->mode = GSR_MODE_PLAIN;
  o->tile_w = 16;
  o->tile_h = 16;
  o->bwd_variant = GSR_BWD_RECOMPUTE;
  o->lds_batch = 128;
  o->grid_per_cu = 4;
  o->bwd_reduce = 0;
  o->project_table = 0;
  o->accumulate_grads = 0;
  o->check_finite = 0;
  o->near_plane = 0.01f;
  o->far_plane = 1e10f;
  o->eps2d = 0.3f;
  o->sigma_extent = 3.0f;
  o->jac_clamp = 1.3f;
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->T_min = 1e-4f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.0f;
  o->stat_scale = 0.0f;
  o->capacity_intersections = 0;
  o->history_budget_bytes = (int64_t)16 << 30;
}

gsr_status gsr_plan_create(gsr_plan **out, const gsr_problem *pr, const gsr_options *opt) {
  if (!out) return GSR_ERR_INVALID_ARG;
  *out = nullptr;
  gsr_status s = validate_problem(pr);
  if (s != GSR_OK) return s;
  gsr_options o;
  if (opt) o = *opt;
  else gsr_default_options(&o);
  s = validate_options(o);
  if (s != GSR_OK) return s;
  gsr_plan *p = new gsr_plan();
  p->prob = *pr;
  p->W.assign(pr->widths, pr->widths + pr->n_views);
  p->H.assign(pr->heights, pr->heights + pr->n_views);
  p->prob.widths = p->W.data();
  p->prob.heights = p->H.data();
  p->opt = o;
  compute_layout(*p);
  if (p->layout.capacity * 8.0 > 1e15) {
    delete p;
    return GSR_ERR_INVALID_ARG;
  }
  *out = p;
  return GSR_OK;
}

gsr_status gsr_plan_destroy(gsr_plan *plan) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  drop_graph(plan);
  for (hipEvent_t e : plan->ev_pool) (void)hipEventDestroy(e);
  delete plan;
  return GSR_OK;
}

gsr_status gsr_workspace_size(const gsr_plan *plan, size_t *bytes) {
  if (!plan || !bytes) return GSR_ERR_INVALID_ARG;
  *bytes = plan->ws_bytes;
  return GSR_OK;
}

gsr_status gsr_workspace_layout(const gsr_plan *plan, gsr_layout *layout) {
  if (!plan || !layout) return GSR_ERR_INVALID_ARG;
  *layout = plan->layout;
  return GSR_OK;
}

gsr_status gsr_image_offset(const gsr_plan *plan, int32_t view, int64_t *offset) {
  if (!plan || !offset || view < 0 || view >= plan->prob.n_views) return GSR_ERR_INVALID_ARG;
  int64_t o = 0;
  for (int v = 0; v < view; v++) o += 3 * (int64_t)plan->W[v] * plan->H[v];
  *offset = o;
  return GSR_OK;
}

gsr_status gsr_plan_options(const gsr_plan *plan, gsr_options *opt) {
  if (!plan || !opt) return GSR_ERR_INVALID_ARG;
  *opt = plan->opt;
  return GSR_OK;
}

gsr_status gsr_plan_set_tuning(gsr_plan *plan, const gsr_options *t) {
  if (!plan || !t) return GSR_ERR_INVALID_ARG;
  gsr_options o = plan->opt;
  o.tile_w = t->tile_w;
  o.tile_h = t->tile_h;
  o.bwd_variant = t->bwd_variant;
  o.lds_batch = t->lds_batch;
  o.grid_per_cu = t->grid_per_cu;
  o.bwd_reduce = t->bwd_reduce;
  o.project_table = t->project_table;
  if (validate_options(o) != GSR_OK) return GSR_ERR_INVALID_ARG;
  const size_t old_bytes = plan->ws_bytes;
  const int64_t old_hist = plan->layout.history_entries;
  const gsr_options old = plan->opt;
  plan->opt = o;
  compute_layout(*plan);
  if (plan->ws_bytes > old_bytes || plan->layout.history_entries != old_hist) {
    // the workspace layout may not grow after the caller sized it
    plan->opt = old;
    compute_layout(*plan);
    return GSR_ERR_INVALID_ARG;
  }
  drop_graph(plan);
  plan->forward_ready = false;
  return GSR_OK;
}

static gsr_status forward_impl(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, float *images,
                               float *depth, float *T_final, uint32_t *last, void *ws, size_t ws_bytes,
                               void *stream, uint32_t *pair_counts = nullptr) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  if (check_gaussians(g) != GSR_OK || !cams || !images) return fail(plan, GSR_ERR_INVALID_ARG, "null argument");
  gsr_status s = check_ws(plan, ws, ws_bytes);
  if (s != GSR_OK) return s;
  const KWs k = ws_view(*plan, ws);
  plan->forward_ready = false;
  stage_reset(plan);
  if (plan->opt.mode == GSR_MODE_PLAIN) {
    s = enqueue_front(plan, g, cams, k, stream, true, images, depth, pair_counts);
    if (s != GSR_OK) return s;
  } else {
    s = enqueue_front(plan, g, cams, k, stream, false, nullptr);
    if (s != GSR_OK) return s;
    STAGE(launch_raster_fwd(k, kopts(*plan), 0, k.tiles_total, images, plan->prob.n_views, use_history(*plan) ? 1 : 0,
                             plan->opt.lds_batch, depth, pair_counts, stream),
           "raster_fwd");
  }
  if (T_final || last) STAGE(launch_copy_pixels(k, T_final, last, stream), "copy");
  plan->forward_ready = true;
  return GSR_OK;
}

gsr_status gsr_forward(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, float *images,
                       float *T_final, uint32_t *last, void *ws, size_t ws_bytes, void *stream) {
  return forward_impl(plan, g, cams, images, nullptr, T_final, last, ws, ws_bytes, stream);
}

gsr_status gsr_render_depth(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, float *images,
                            float *depth, void *ws, size_t ws_bytes, void *stream) {
  if (!depth) return plan ? fail(plan, GSR_ERR_INVALID_ARG, "null argument") : GSR_ERR_INVALID_ARG;
  return forward_impl(plan, g, cams, images, depth, nullptr, nullptr, ws, ws_bytes, stream);
}

gsr_status gsr_pair_counts(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, float *images,
                           uint32_t *counts, void *ws, size_t ws_bytes, void *stream) {
  if (!counts) return plan ? fail(plan, GSR_ERR_INVALID_ARG, "null argument") : GSR_ERR_INVALID_ARG;
  gsr_status s = forward_impl(plan, g, cams, images, nullptr, nullptr, nullptr, ws, ws_bytes, stream, counts);
  // the stored history (if any) was not written: no reverse pass may follow
  if (plan) plan->forward_ready = false;
  return s;
}

gsr_status gsr_back_project(gsr_plan *plan, const gsr_camera *cams, const float *depth, float *points,
                            void *stream) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  if (!cams || !depth || !points) return fail(plan, GSR_ERR_INVALID_ARG, "null argument");
  HIPCHK(launch_back_project(view_table(*plan), cams, depth, points, stream), "back-projection");
  return GSR_OK;
}

gsr_status gsr_camera_coverage(gsr_plan *plan, const gsr_camera *cams, const float *depth, const float *blocks,
                               int32_t n_blocks, float tau, uint32_t *counts, float *ratio, uint8_t *selected,
                               void *stream) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  if (!cams || !depth || !blocks || !counts) return fail(plan, GSR_ERR_INVALID_ARG, "null argument");
  if (n_blocks < 1 || n_blocks > GSR_MAX_COVERAGE_BLOCKS)
    return fail(plan, GSR_ERR_INVALID_ARG, "n_blocks must be in [1, GSR_MAX_COVERAGE_BLOCKS]");
  if (!std::isfinite(tau)) return fail(plan, GSR_ERR_INVALID_ARG, "tau must be finite");
  HIPCHK(launch_coverage(view_table(*plan), cams, depth, blocks, n_blocks, tau, counts, ratio, selected, stream),
         "coverage");
  return GSR_OK;
}

gsr_status gsr_backward(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, const float *dL_dimages,
                        const gsr_grads *grads, const gsr_stats *stats, void *ws, size_t ws_bytes, void *stream) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  if (check_gaussians(g) != GSR_OK || check_grads(grads) != GSR_OK || !cams || !dL_dimages)
    return fail(plan, GSR_ERR_INVALID_ARG, "null argument");
  gsr_status s = check_ws(plan, ws, ws_bytes);
  if (s != GSR_OK) return s;
  if (!plan->forward_ready) return fail(plan, GSR_ERR_STATE, "gsr_backward needs a preceding gsr_forward");
  stage_reset(plan);
  const KWs k = ws_view(*plan, ws);
  const KOpts ko = kopts(*plan);
  const KParams kp = kparams(*plan, g);
  const int hist = use_history(*plan) ? 1 : 0;
  const int V = plan->prob.n_views;
  float *sS = stats ? stats->grad2d_norm_sum : nullptr;
  uint32_t *sN = stats ? stats->visible_count : nullptr;
  if (plan->opt.mode == GSR_MODE_PLAIN) {
    if (!plan->opt.accumulate_grads) {
      s = zero_grads(plan, grads, stream);
      if (s != GSR_OK) return s;
    }
    const ViewTable tbl = view_table(*plan);
    for (int v = 0; v < V; v++) {
      const int64_t nt = (int64_t)tbl.v[v].tiles_x * tbl.v[v].tiles_y;
      STAGE(launch_raster_bwd(k, ko, tbl.v[v].tile_base, nt, dL_dimages, V, hist, plan->opt.lds_batch,
                              plan->opt.bwd_reduce, stream), "raster_bwd");
      STAGE(launch_project_bwd(kp, cams, ko, k, kgrads(grads), sS, sN, v, stream), "project_bwd");
    }
  } else {
    STAGE(launch_raster_bwd(k, ko, 0, k.tiles_total, dL_dimages, V, hist, plan->opt.lds_batch,
                            plan->opt.bwd_reduce, stream), "raster_bwd");
    STAGE(launch_project_bwd(kp, cams, ko, k, kgrads(grads), sS, sN, -1, stream), "project_bwd");
  }
  plan->forward_ready = false;
  return GSR_OK;
}

gsr_status gsr_forward_backward_l1(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams,
                                   const float *targets, float *images, float *loss, const gsr_grads *grads,
                                   const gsr_stats *stats, void *ws, size_t ws_bytes, void *stream) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  if (check_gaussians(g) != GSR_OK || check_grads(grads) != GSR_OK || !cams || !targets || !images || !loss)
    return fail(plan, GSR_ERR_INVALID_ARG, "null argument");
  gsr_status s = check_ws(plan, ws, ws_bytes);
  if (s != GSR_OK) return s;
  const KWs k = ws_view(*plan, ws);
  plan->forward_ready = false;
  stage_reset(plan);
  if (plan->opt.mode == GSR_MODE_PLAIN) return enqueue_plain_l1(plan, g, cams, targets, images, loss, grads, stats, k, stream);
  return enqueue_batched_l1(plan, g, cams, targets, images, loss, grads, stats, k, stream);
}

}  // extern "C"

namespace gsr {

gsr_status fused_l1_no_events(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, const float *targets,
                              float *images, float *loss, const gsr_grads *grads, const gsr_stats *stats, void *ws,
                              size_t ws_bytes, void *stream) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  const bool was = plan->capturing;
  plan->capturing = true;  // suppresses stage timing, which would create events
  const gsr_status s = gsr_forward_backward_l1(plan, g, cams, targets, images, loss, grads, stats, ws, ws_bytes,
                                               stream);
  plan->capturing = was;
  return s;
}

gsr_status plan_error(gsr_plan *plan, gsr_status s, const char *msg) { return fail(plan, s, msg); }

}  // namespace gsr

extern "C" {

gsr_status gsr_visibility_mask(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, const float *aabb,
                               uint32_t *view_bits, uint8_t *keep_out, uint8_t *in_block, void *ws, size_t ws_bytes,
                               void *stream) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  if (check_gaussians(g) != GSR_OK || !cams) return fail(plan, GSR_ERR_INVALID_ARG, "null argument");
  if (in_block && !aabb) return fail(plan, GSR_ERR_INVALID_ARG, "in_block needs an aabb");
  gsr_status s = check_ws(plan, ws, ws_bytes);
  if (s != GSR_OK) return s;
  const KWs k = ws_view(*plan, ws);
  const float box[6] = {aabb ? aabb[0] : 0.f, aabb ? aabb[1] : 0.f, aabb ? aabb[2] : 0.f,
                        aabb ? aabb[3] : 0.f, aabb ? aabb[4] : 0.f, aabb ? aabb[5] : 0.f};
  STAGE(launch_setup(view_table(*plan), k, 0, 0, 0, plan->prob.n, stream), "setup");
  STAGE(launch_visibility(kparams(*plan, g), cams, kopts(*plan), k, box, view_bits, keep_out, in_block, stream),
         "visibility");
  return GSR_OK;
}

gsr_status gsr_graph_capture(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, const float *targets,
                             float *images, float *loss, const gsr_grads *grads, const gsr_stats *stats, void *ws,
                             size_t ws_bytes, void *stream) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  if (plan->opt.mode != GSR_MODE_BATCHED) return fail(plan, GSR_ERR_STATE, "graph capture needs GSR_MODE_BATCHED");
  if (!stream) return fail(plan, GSR_ERR_INVALID_ARG, "the legacy null stream cannot be captured");
  if (check_gaussians(g) != GSR_OK || check_grads(grads) != GSR_OK || !cams || !targets || !images || !loss)
    return fail(plan, GSR_ERR_INVALID_ARG, "null argument");
  gsr_status s = check_ws(plan, ws, ws_bytes);
  if (s != GSR_OK) return s;
  drop_graph(plan);
  n_cus(plan);  // query the device before capture
  const KWs k = ws_view(*plan, ws);
  HIPCHK(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeRelaxed), "begin capture");
  plan->capturing = true;
  s = enqueue_batched_l1(plan, g, cams, targets, images, loss, grads, stats, k, stream);
  plan->capturing = false;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture((hipStream_t)stream, &graph);
  if (s != GSR_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return hip_check(plan, (int)e, "end capture");
  plan->graph = graph;
  HIPCHK(hipGraphInstantiate(&plan->graph_exec, graph, nullptr, nullptr, 0), "instantiate");
  return GSR_OK;
}

gsr_status gsr_graph_launch(gsr_plan *plan, void *stream) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  if (!plan->graph_exec) return fail(plan, GSR_ERR_STATE, "no captured graph");
  HIPCHK(hipGraphLaunch(plan->graph_exec, (hipStream_t)stream), "graph launch");
  return GSR_OK;
}

gsr_status gsr_query_counts(gsr_plan *plan, const void *ws, gsr_counts *c, void *stream) {
  if (!plan || !ws || !c) return GSR_ERR_INVALID_ARG;
  // visible counts are derived from the view masks on demand (see k_count_visible)
  HIPCHK(launch_count_visible(ws_view(*plan, const_cast<void *>(ws)), plan->prob.n, plan->prob.n_views, stream),
         "count visible");
  HIPCHK(hipStreamSynchronize((hipStream_t)stream), "sync");
  WsHeader h;
  HIPCHK(hipMemcpy(&h, (const char *)ws + plan->layout.header, sizeof h, hipMemcpyDeviceToHost), "read counts");
  memset(c, 0, sizeof *c);
  for (int v = 0; v < plan->prob.n_views; v++) {
    c->visible[v] = h.visible[v];
    c->intersections[v] = h.isect[v];
    c->visible_total += h.visible[v];
    c->intersections_total += h.isect[v];
  }
  c->visible_union = h.union_count;
  c->overflow = h.overflow ? 1 : 0;
  c->nonfinite = h.nonfinite ? 1 : 0;
  c->tile_w = plan->opt.tile_w;
  c->tile_h = plan->opt.tile_h;
  c->bwd_variant = use_history(*plan) ? GSR_BWD_STORED : GSR_BWD_RECOMPUTE;
  c->lds_batch = plan->opt.lds_batch;
  c->grid_per_cu = plan->opt.grid_per_cu;
  c->mode = plan->opt.mode;
  if (c->overflow) return fail(plan, GSR_ERR_CAPACITY, "intersection capacity exceeded");
  if (c->nonfinite) return fail(plan, GSR_ERR_NONFINITE, "non-finite parameter");
  return GSR_OK;
}

gsr_status gsr_autotune(gsr_plan *plan, const gsr_gaussians *g, const gsr_camera *cams, const float *targets,
                        float *images, float *loss, const gsr_grads *grads, void *ws, size_t ws_bytes, int32_t reps,
                        gsr_options *best, float *best_ms, void *stream) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  if (plan->opt.mode != GSR_MODE_BATCHED) return fail(plan, GSR_ERR_STATE, "autotuning needs GSR_MODE_BATCHED");
  if (check_gaussians(g) != GSR_OK || check_grads(grads) != GSR_OK || !cams || !targets || !images || !loss)
    return fail(plan, GSR_ERR_INVALID_ARG, "null argument");
  gsr_status s = check_ws(plan, ws, ws_bytes);
  if (s != GSR_OK) return s;
  if (reps < 1) reps = 1;
  drop_graph(plan);
  const gsr_options start = plan->opt;
  plan->capturing = true;  // no stage timing while tuning
  const int shapes[3][2] = {{16, 16}, {32, 8}, {8, 32}};
  const int batches[3] = {64, 128, 256};
  const int grids[2] = {4, 8};
  std::vector<int> variants = {GSR_BWD_RECOMPUTE};
  if (plan->layout.history_entries > 0) variants.push_back(GSR_BWD_STORED);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0), "event");
  HIPCHK(hipEventCreate(&e1), "event");
  // One step per repetition, each timed alone; a candidate's time is its
  // fastest repetition (robust to interference).  The three fastest
  // candidates are then timed again with more repetitions.
  auto time_candidate = [&](const gsr_options &o, int nrep, float &ms_out) -> gsr_status {
    plan->opt = o;
    compute_layout(*plan);
    const KWs k = ws_view(*plan, ws);
    gsr_status st = enqueue_batched_l1(plan, g, cams, targets, images, loss, grads, nullptr, k, stream);
    ms_out = 1e30f;
    for (int r = 0; r < nrep && st == GSR_OK; r++) {
      HIPCHK(hipEventRecord(e0, (hipStream_t)stream), "event");
      st = enqueue_batched_l1(plan, g, cams, targets, images, loss, grads, nullptr, k, stream);
      HIPCHK(hipEventRecord(e1, (hipStream_t)stream), "event");
      HIPCHK(hipEventSynchronize(e1), "event");
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1), "event");
      ms_out = std::min(ms_out, ms);
    }
    if (st != GSR_OK) return st;
    WsHeader h;
    HIPCHK(hipMemcpy(&h, (const char *)ws + plan->layout.header, sizeof h, hipMemcpyDeviceToHost), "read counts");
    if (h.overflow) ms_out = 1e30f;  // this shape needs more capacity: not a candidate
    return GSR_OK;
  };
  std::vector<std::pair<float, gsr_options>> timed;
  for (auto &sh : shapes)
    for (int b : batches)
      for (int gpc : grids)
        for (int var : variants)
          for (int red : {0, 2, 3, 4}) {  // 1 (per-lane LDS atomics) is dominated by 2
            gsr_options o = start;
            o.tile_w = sh[0];
            o.tile_h = sh[1];
            o.lds_batch = b;
            o.grid_per_cu = gpc;
            o.bwd_variant = var;
            o.bwd_reduce = red;
            plan->opt = o;
            compute_layout(*plan);
            if (var == GSR_BWD_STORED && plan->layout.history_entries == 0) continue;
            float ms = 0.f;
            s = time_candidate(o, reps, ms);
            if (s != GSR_OK) break;
            if (ms < 1e29f) timed.push_back({ms, o});
          }
  std::sort(timed.begin(), timed.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
  float best_t = 1e30f;
  gsr_options best_o = start;
  for (size_t c = 0; c < timed.size() && c < 3 && s == GSR_OK; c++) {
    float ms = 0.f;
    s = time_candidate(timed[c].second, 2 * reps + 3, ms);
    if (s == GSR_OK && ms < best_t) {
      best_t = ms;
      best_o = timed[c].second;
    }
  }
  // the projection's tile counting, on the chosen raster tuning
  if (s == GSR_OK && best_t < 1e29f) {
    gsr_options alt = best_o;
    alt.project_table = 1 - best_o.project_table;
    float ms = 0.f;
    s = time_candidate(alt, 2 * reps + 3, ms);
    if (s == GSR_OK && ms < best_t) {
      best_t = ms;
      best_o = alt;
    }
  }
  plan->capturing = false;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  plan->opt = best_t < 1e29f ? best_o : start;
  compute_layout(*plan);
  if (s != GSR_OK) return s;
  if (best_t >= 1e29f) return fail(plan, GSR_ERR_CAPACITY, "no candidate fits the intersection capacity");
  if (best) *best = plan->opt;
  if (best_ms) *best_ms = best_t;
  return GSR_OK;
}

gsr_status gsr_adam_step(gsr_plan *plan, const gsr_adam *hp, const gsr_grads *params, const gsr_grads *grads,
                         const gsr_grads *m, const gsr_grads *v, const uint32_t *visible_bits, void *stream) {
  if (!plan) return GSR_ERR_INVALID_ARG;
  if (!hp || check_grads(params) != GSR_OK || check_grads(grads) != GSR_OK || check_grads(m) != GSR_OK ||
      check_grads(v) != GSR_OK)
    return fail(plan, GSR_ERR_INVALID_ARG, "null argument");
  if (hp->step < 1) return fail(plan, GSR_ERR_INVALID_ARG, "step must be >= 1");
  if (!(hp->beta1 >= 0.0f && hp->beta1 < 1.0f && hp->beta2 >= 0.0f && hp->beta2 < 1.0f && hp->eps > 0.0f))
    return fail(plan, GSR_ERR_INVALID_ARG, "need 0 <= beta1, beta2 < 1 and eps > 0");
  for (int k = 0; k < 6; k++)
    if (!std::isfinite(hp->lr[k])) return fail(plan, GSR_ERR_INVALID_ARG, "learning rates must be finite");
  const int K = (plan->prob.sh_degree + 1) * (plan->prob.sh_degree + 1);
  KAdam a;
  float *const ps[5] = {params->means, params->log_scales, params->quats, params->opacity_logits, params->sh};
  const float *const gs[5] = {grads->means, grads->log_scales, grads->quats, grads->opacity_logits, grads->sh};
  float *const ms[5] = {m->means, m->log_scales, m->quats, m->opacity_logits, m->sh};
  float *const vs[5] = {v->means, v->log_scales, v->quats, v->opacity_logits, v->sh};
  const int rows[5] = {3, 3, 4, 1, 3 * K};
  for (int k = 0; k < 5; k++) {
    a.p[k] = ps[k];
    a.g[k] = gs[k];
    a.m[k] = ms[k];
    a.v[k] = vs[k];
    a.rows[k] = rows[k];
  }
  const double bc1 = 1.0 - std::pow((double)hp->beta1, (double)hp->step);
  const double bc2 = 1.0 - std::pow((double)hp->beta2, (double)hp->step);
  for (int k = 0; k < 6; k++) a.step_size[k] = (float)((double)hp->lr[k] / bc1);
  a.bc2_sqrt = (float)std::sqrt(bc2);
  a.beta1 = hp->beta1;
  a.beta2 = hp->beta2;
  a.eps = hp->eps;
  a.n = plan->prob.n;
  a.visible = visible_bits;
  HIPCHK(launch_adam(a, 11 + 3 * K, stream), "adam");
  return GSR_OK;
}

gsr_status gsr_last_stage_times(gsr_plan *plan, gsr_stage_times *out) {
  if (!plan || !out) return GSR_ERR_INVALID_ARG;
  memset(out, 0, sizeof *out);
  if (plan->stages.empty()) return GSR_OK;
  HIPCHK(hipEventSynchronize(plan->ev_pool[plan->stages.back().b]), "stage events");
  for (const auto &st : plan->stages) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, plan->ev_pool[st.a], plan->ev_pool[st.b]), "stage events");
    int k = 0;
    while (k < out->count && strncmp(out->name[k], st.name.c_str(), 31) != 0) k++;
    if (k == out->count) {
      if (out->count == GSR_MAX_STAGES) continue;
      strncpy(out->name[k], st.name.c_str(), 31);
      out->count++;
    }
    out->ms[k] += ms;
    out->launches[k] += 1;
  }
  return GSR_OK;
}

const char *gsr_status_string(gsr_status s) {
  switch (s) {
    case GSR_OK: return "ok";
    case GSR_ERR_INVALID_ARG: return "invalid argument";
    case GSR_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case GSR_ERR_CAPACITY: return "intersection capacity exceeded";
    case GSR_ERR_NONFINITE: return "non-finite parameter";
    case GSR_ERR_HIP: return "HIP runtime error";
    case GSR_ERR_STATE: return "invalid call order";
    default: return "unknown status";
  }
}

const char *gsr_last_error(const gsr_plan *plan) { return plan ? plan->err.c_str() : ""; }

}  // extern "C"
