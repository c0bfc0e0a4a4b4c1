/*
 * FP64 CPU oracle for the differentiable Gaussian rasterizer (test
 * infrastructure only: the library never links or calls this file).
 *
 * What is computed.  LoBE-GS (arXiv 2510.01767) fine-trains each block with
 * the vanilla 3DGS rasterizer (App. A.1, "3DGS Training"); the paper fixes the
 * alpha-compositing sum (Sec. 3.2, the depth form of the blending equation),
 * frustum culling during rasterization (Sec. 3.3), visibility cropping and
 * selective densification (Sec. 3.3).  Everything else follows the 3DGS prior
 * art the paper builds on, with the conventions stated at each function.  For
 * these conventions the rendered image is exactly a per-pixel definition:
 *
 *   for every pixel, take the Gaussians whose 3-sigma tile rectangle covers
 *   the pixel's tile, order them by (fp32 depth bits, Gaussian index) and
 *   composite them front to back.
 *
 * The oracle writes that definition out in double precision, one Gaussian,
 * one pixel and one list entry at a time.  Gradients are the exact reverse
 * mode of the same forward, with the subgradients stated in ora_render_bwd
 * and ora_project_bwd.  OpenMP only runs independent pixels / Gaussians
 * concurrently; it does not change any arithmetic.
 *
 * Guard band.  Every discrete decision (near/far, det > 0, the ceil of the
 * radius, the floors of the tile rectangle, the float32 rounding of the depth
 * that orders a tile's list, the colour clamp, alpha >= alpha_min,
 * o*G >= alpha_max, T*(1-alpha) < T_min, and the order of two entries whose
 * depths nearly coincide) records its relative margin; a float32
 * implementation may legitimately decide the other way when the margin is
 * tiny, so callers exclude such Gaussians and pixels from strict comparison.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_MAX_SH 16

typedef struct {
  double near_plane, far_plane;
  double eps2d;        /* dilation added to the diagonal of the 2D covariance */
  double sigma_extent; /* footprint radius in standard deviations */
  double jac_clamp;    /* off-screen clamp of x/z, y/z as a multiple of the half field of view */
  double alpha_min, alpha_max, T_min;
  double bg[3];
  int32_t tile_w, tile_h;
} ora_opts;

typedef struct {
  double R[9]; /* world -> camera rotation, row major */
  double t[3];
  double fx, fy, cx, cy;
  int32_t W, H;
} ora_cam;

static double rel_margin(double value, double threshold) {
  double s = fabs(threshold) > 0 ? fabs(threshold) : 1.0;
  return fabs(value - threshold) / s;
}

static double frac_margin(double v) { /* distance to the nearest integer, relative */
  double d = fabs(v - nearbyint(v));
  double s = fabs(v) > 1.0 ? fabs(v) : 1.0;
  return d / s;
}

/* ------------------------------------------------------------------------
 * Real spherical harmonics up to degree 3: orthonormal on the unit sphere,
 * Condon-Shortley phase, index k = l*l + l + m with m = -l..l.  Each function
 * is a polynomial in the unit direction (x, y, z) with the textbook
 * normalisation sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (times sqrt 2 if m != 0).
 * dY (optional) receives the gradient of each polynomial w.r.t. (x, y, z)
 * treated as free variables.
 */
void ora_sh_basis(int degree, const double dir[3], double *Y, double *dY) {
  const double pi = 3.14159265358979323846;
  const double x = dir[0], y = dir[1], z = dir[2];
  const double c0 = 0.5 * sqrt(1.0 / pi);
  const double c1 = sqrt(3.0 / (4.0 * pi));
  const double c2a = 0.5 * sqrt(15.0 / pi);
  const double c20 = 0.25 * sqrt(5.0 / pi);
  const double c22 = 0.25 * sqrt(15.0 / pi);
  const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi));
  const double c3b = 0.5 * sqrt(105.0 / pi);
  const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi));
  const double c30 = 0.25 * sqrt(7.0 / pi);
  const double c3d = 0.25 * sqrt(105.0 / pi);
  double g[ORA_MAX_SH][3];
  memset(g, 0, sizeof g);
  Y[0] = c0;
  if (degree >= 1) {
    Y[1] = -c1 * y;  g[1][1] = -c1;
    Y[2] = c1 * z;   g[2][2] = c1;
    Y[3] = -c1 * x;  g[3][0] = -c1;
  }
  if (degree >= 2) {
    Y[4] = c2a * x * y;          g[4][0] = c2a * y; g[4][1] = c2a * x;
    Y[5] = -c2a * y * z;         g[5][1] = -c2a * z; g[5][2] = -c2a * y;
    Y[6] = c20 * (3 * z * z - 1); g[6][2] = 6 * c20 * z;
    Y[7] = -c2a * x * z;         g[7][0] = -c2a * z; g[7][2] = -c2a * x;
    Y[8] = c22 * (x * x - y * y); g[8][0] = 2 * c22 * x; g[8][1] = -2 * c22 * y;
  }
  if (degree >= 3) {
    Y[9] = -c3a * y * (3 * x * x - y * y);
    g[9][0] = -c3a * 6 * x * y; g[9][1] = -c3a * (3 * x * x - 3 * y * y);
    Y[10] = c3b * x * y * z;
    g[10][0] = c3b * y * z; g[10][1] = c3b * x * z; g[10][2] = c3b * x * y;
    Y[11] = -c3c * y * (5 * z * z - 1);
    g[11][1] = -c3c * (5 * z * z - 1); g[11][2] = -c3c * 10 * y * z;
    Y[12] = c30 * z * (5 * z * z - 3);
    g[12][2] = c30 * (15 * z * z - 3);
    Y[13] = -c3c * x * (5 * z * z - 1);
    g[13][0] = -c3c * (5 * z * z - 1); g[13][2] = -c3c * 10 * x * z;
    Y[14] = c3d * z * (x * x - y * y);
    g[14][0] = 2 * c3d * x * z; g[14][1] = -2 * c3d * y * z; g[14][2] = c3d * (x * x - y * y);
    Y[15] = -c3a * x * (x * x - 3 * y * y);
    g[15][0] = -c3a * (3 * x * x - 3 * y * y); g[15][1] = c3a * 6 * x * y;
  }
  if (dY) {
    int K = (degree + 1) * (degree + 1);
    for (int k = 0; k < K; k++)
      for (int a = 0; a < 3; a++) dY[k * 3 + a] = g[k][a];
  }
}

/* Rotation matrix of the unit quaternion (w, x, y, z), row major. */
static void quat_to_rot(const double q[4], double Rq[9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  Rq[0] = 1 - 2 * (y * y + z * z); Rq[1] = 2 * (x * y - w * z);     Rq[2] = 2 * (x * z + w * y);
  Rq[3] = 2 * (x * y + w * z);     Rq[4] = 1 - 2 * (x * x + z * z); Rq[5] = 2 * (y * z - w * x);
  Rq[6] = 2 * (x * z - w * y);     Rq[7] = 2 * (y * z + w * x);     Rq[8] = 1 - 2 * (x * x + y * y);
}

/* Everything the forward derives for one Gaussian in one view. */
typedef struct {
  int culled_depth, culled_det;
  double s[3], qn, qh[4], Rq[9], M[9], Sigma[9];
  double tc[3], u, v; /* u, v: the clamped x/z and y/z used inside J */
  int clamp_u, clamp_v;
  double J[6], Wc[9];   /* J and the camera rotation */
  double a, b, c, det;  /* 2D covariance after dilation */
  double conic[3], mean2d[2], lam, radius_f;
  int radius, rect[4], visible, ntiles;
  double opacity, dirn[3], dnorm, Y[ORA_MAX_SH], color_raw[3], color[3];
  double margin, grad_margin;
  double depth_margin; /* distance of the depth to a float32 rounding boundary, relative */
  double color_margin; /* distance of the raw colour to the clamp at 0, relative */
} ora_fwd;

/* Relative distance of v to the nearest point where its rounding to float32
 * changes: the midpoints between the float32 value nearest v and its two
 * neighbours. */
static double f32_round_margin(double v) {
  float f = (float)v;
  double up = 0.5 * ((double)f + (double)nextafterf(f, INFINITY));
  double dn = 0.5 * ((double)f + (double)nextafterf(f, -INFINITY));
  double d = fmin(fabs(v - up), fabs(v - dn));
  return d / fmax(fabs(v), 1e-300);
}

static void project_one(const ora_opts *o, const ora_cam *cam, int sh_degree, const double mu[3],
                        const double ls[3], const double qr[4], double logit,
                        const double *shv /* [3K], plane k*3+c */, int keep, ora_fwd *f) {
  memset(f, 0, sizeof *f);
  f->margin = INFINITY;
  f->grad_margin = INFINITY;
  f->depth_margin = INFINITY;
  f->color_margin = INFINITY;
  /* activations */
  for (int a = 0; a < 3; a++) f->s[a] = exp(ls[a]);
  f->qn = sqrt(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
  for (int a = 0; a < 4; a++) f->qh[a] = qr[a] / f->qn;
  f->opacity = 1.0 / (1.0 + exp(-logit));
  /* 3D covariance Sigma = M M^T with M = R(q) diag(s) */
  quat_to_rot(f->qh, f->Rq);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) f->M[i * 3 + j] = f->Rq[i * 3 + j] * f->s[j];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0;
      for (int k = 0; k < 3; k++) acc += f->M[i * 3 + k] * f->M[j * 3 + k];
      f->Sigma[i * 3 + j] = acc;
    }
  /* camera-space mean */
  for (int i = 0; i < 3; i++) {
    f->tc[i] = cam->t[i];
    for (int k = 0; k < 3; k++) f->tc[i] += cam->R[i * 3 + k] * mu[k];
  }
  memcpy(f->Wc, cam->R, sizeof f->Wc);
  double tz = f->tc[2];
  /* the list order compares depths as float32 bit patterns */
  f->depth_margin = f32_round_margin(tz);
  f->margin = fmin(f->margin, fabs(tz - o->near_plane) / fmax(fabs(tz), 1e-300));
  f->margin = fmin(f->margin, rel_margin(tz, o->far_plane));
  if (!(tz > o->near_plane && tz < o->far_plane)) {
    f->culled_depth = 1;
    return;
  }
  /* perspective projection of the mean (pixel centres at integer + 1/2) */
  f->mean2d[0] = cam->fx * f->tc[0] / tz + cam->cx;
  f->mean2d[1] = cam->fy * f->tc[1] / tz + cam->cy;
  /* Jacobian of the pinhole map, with x/z and y/z clamped to jac_clamp times
   * the half field of view */
  double limx = o->jac_clamp * (0.5 * cam->W / cam->fx);
  double limy = o->jac_clamp * (0.5 * cam->H / cam->fy);
  double ux = f->tc[0] / tz, uy = f->tc[1] / tz;
  f->grad_margin = fmin(f->grad_margin, rel_margin(fabs(ux), limx));
  f->grad_margin = fmin(f->grad_margin, rel_margin(fabs(uy), limy));
  f->clamp_u = fabs(ux) > limx;
  f->clamp_v = fabs(uy) > limy;
  f->u = f->clamp_u ? copysign(limx, ux) : ux;
  f->v = f->clamp_v ? copysign(limy, uy) : uy;
  f->J[0] = cam->fx / tz; f->J[1] = 0;              f->J[2] = -cam->fx * f->u / tz;
  f->J[3] = 0;            f->J[4] = cam->fy / tz;   f->J[5] = -cam->fy * f->v / tz;
  /* 2D covariance: J W Sigma W^T J^T + eps I */
  double T[6];
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 3; j++) {
      double acc = 0;
      for (int k = 0; k < 3; k++) acc += f->J[i * 3 + k] * f->Wc[k * 3 + j];
      T[i * 3 + j] = acc;
    }
  double S2[4];
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) {
      double acc = 0;
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) acc += T[i * 3 + k] * f->Sigma[k * 3 + l] * T[j * 3 + l];
      S2[i * 2 + j] = acc;
    }
  f->a = S2[0] + o->eps2d;
  f->b = S2[1];
  f->c = S2[3] + o->eps2d;
  f->det = f->a * f->c - f->b * f->b;
  f->margin = fmin(f->margin, fabs(f->det) / (fabs(f->a * f->c) + f->b * f->b));
  if (!(f->det > 0)) {
    f->culled_det = 1;
    return;
  }
  f->conic[0] = f->c / f->det;
  f->conic[1] = -f->b / f->det;
  f->conic[2] = f->a / f->det;
  /* footprint: ceil(sigma_extent * sqrt(largest eigenvalue)) */
  double mid = 0.5 * (f->a + f->c);
  double half = 0.5 * (f->a - f->c);
  f->lam = mid + sqrt(half * half + f->b * f->b);
  f->radius_f = o->sigma_extent * sqrt(f->lam);
  f->margin = fmin(f->margin, frac_margin(f->radius_f));
  f->radius = (int)ceil(f->radius_f);
  /* tile rectangle (inclusive), clamped to the view's tile grid */
  int tiles_x = (cam->W + o->tile_w - 1) / o->tile_w;
  int tiles_y = (cam->H + o->tile_h - 1) / o->tile_h;
  double ex0 = (f->mean2d[0] - f->radius) / o->tile_w, ex1 = (f->mean2d[0] + f->radius) / o->tile_w;
  double ey0 = (f->mean2d[1] - f->radius) / o->tile_h, ey1 = (f->mean2d[1] + f->radius) / o->tile_h;
  f->margin = fmin(f->margin, fmin(fmin(frac_margin(ex0), frac_margin(ex1)), fmin(frac_margin(ey0), frac_margin(ey1))));
  double fx0 = floor(ex0), fx1 = floor(ex1), fy0 = floor(ey0), fy1 = floor(ey1);
  int x0 = fx0 < 0 ? 0 : (fx0 > tiles_x - 1 ? tiles_x : (int)fx0);
  int x1 = fx1 > tiles_x - 1 ? tiles_x - 1 : (fx1 < 0 ? -1 : (int)fx1);
  int y0 = fy0 < 0 ? 0 : (fy0 > tiles_y - 1 ? tiles_y : (int)fy0);
  int y1 = fy1 > tiles_y - 1 ? tiles_y - 1 : (fy1 < 0 ? -1 : (int)fy1);
  f->rect[0] = x0; f->rect[1] = y0; f->rect[2] = x1; f->rect[3] = y1;
  f->visible = keep && x0 <= x1 && y0 <= y1;
  f->ntiles = f->visible ? (x1 - x0 + 1) * (y1 - y0 + 1) : 0;
  /* colour: SH evaluated in the direction from the camera centre to the mean */
  double cc[3];
  for (int i = 0; i < 3; i++) {
    cc[i] = 0;
    for (int k = 0; k < 3; k++) cc[i] -= cam->R[k * 3 + i] * cam->t[k];
  }
  double d[3] = {mu[0] - cc[0], mu[1] - cc[1], mu[2] - cc[2]};
  f->dnorm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int i = 0; i < 3; i++) f->dirn[i] = d[i] / f->dnorm;
  ora_sh_basis(sh_degree, f->dirn, f->Y, NULL);
  int K = (sh_degree + 1) * (sh_degree + 1);
  for (int ch = 0; ch < 3; ch++) {
    double acc = 0;
    for (int k = 0; k < K; k++) acc += shv[k * 3 + ch] * f->Y[k];
    f->color_raw[ch] = acc + 0.5;
    f->color[ch] = f->color_raw[ch] > 0 ? f->color_raw[ch] : 0.0;
    f->color_margin = fmin(f->color_margin, fabs(f->color_raw[ch]) / fmax(1.0, fabs(acc)));
  }
}

/* Forward projection of n Gaussians into one view.
 * Parameters are structure-of-arrays planes of length n (means [3][n],
 * log_scales [3][n], quats [4][n] in (w, x, y, z) order, logits [n],
 * sh [3K][n] with plane k*3 + channel); keep may be NULL.
 * Outputs are planes of length n as well. */
void ora_project(const ora_opts *o, const ora_cam *cam, int64_t n, int sh_degree,
                 const double *means, const double *log_scales, const double *quats,
                 const double *logits, const double *sh, const uint8_t *keep,
                 int32_t *visible, double *mean2d, double *conic, double *cov2d, double *depth,
                 double *opacity, double *color, double *color_raw, int32_t *radius, int32_t *rect,
                 int32_t *ntiles, double *margin, double *grad_margin, double *depth_margin,
                 double *color_margin) {
  int K = (sh_degree + 1) * (sh_degree + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double mu[3], ls[3], q[4], shv[3 * ORA_MAX_SH];
    for (int a = 0; a < 3; a++) { mu[a] = means[a * n + i]; ls[a] = log_scales[a * n + i]; }
    for (int a = 0; a < 4; a++) q[a] = quats[a * n + i];
    for (int k = 0; k < 3 * K; k++) shv[k] = sh[(int64_t)k * n + i];
    ora_fwd f;
    project_one(o, cam, sh_degree, mu, ls, q, logits[i], shv, keep ? keep[i] != 0 : 1, &f);
    visible[i] = f.visible;
    mean2d[i] = f.mean2d[0]; mean2d[n + i] = f.mean2d[1];
    for (int a = 0; a < 3; a++) conic[a * n + i] = f.conic[a];
    cov2d[i] = f.a; cov2d[n + i] = f.b; cov2d[2 * n + i] = f.c;
    depth[i] = f.tc[2];
    opacity[i] = f.opacity;
    for (int a = 0; a < 3; a++) { color[a * n + i] = f.color[a]; color_raw[a * n + i] = f.color_raw[a]; }
    radius[i] = f.radius;
    for (int a = 0; a < 4; a++) rect[a * n + i] = f.rect[a];
    ntiles[i] = f.ntiles;
    margin[i] = f.margin;
    grad_margin[i] = f.grad_margin;
    depth_margin[i] = f.depth_margin;
    color_margin[i] = f.color_margin;
  }
}

/* ------------------------------------------------------------------------
 * Tile binning and ordering.  Every visible record r contributes one entry
 * per tile of its rectangle; entries are ordered by the total order
 * (global tile id, fp32 depth bits, tiebreak) with qsort, then each tile's
 * [start, end) range is read off.  Global tile id = tile_base[r] +
 * ty * tiles_x[r] + tx.  Returns the number of entries, or -1 when it exceeds
 * capacity (call with capacity 0 to obtain the count).
 */
typedef struct { int64_t tile; uint32_t depth; int64_t tie; int64_t rec; } ora_entry;

static int cmp_entry(const void *pa, const void *pb) {
  const ora_entry *a = pa, *b = pb;
  if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
  if (a->depth != b->depth) return a->depth < b->depth ? -1 : 1;
  if (a->tie != b->tie) return a->tie < b->tie ? -1 : 1;
  return 0;
}

int64_t ora_bin(int64_t n_rec, const int32_t *rect /* [4][n_rec] */, const int32_t *visible,
                const uint32_t *depth_bits, const int64_t *tiebreak, const int64_t *tile_base,
                const int32_t *tiles_x, int64_t n_tiles_total, int64_t capacity, int64_t *out_tile,
                uint32_t *out_depth, int64_t *out_value, int64_t *ranges /* [n_tiles_total][2] */) {
  int64_t count = 0;
  for (int64_t r = 0; r < n_rec; r++)
    if (visible[r])
      count += (int64_t)(rect[2 * n_rec + r] - rect[r] + 1) * (rect[3 * n_rec + r] - rect[n_rec + r] + 1);
  if (count > capacity) return capacity == 0 ? count : -1;
  ora_entry *e = malloc(sizeof(ora_entry) * (count > 0 ? count : 1));
  int64_t m = 0;
  for (int64_t r = 0; r < n_rec; r++) {
    if (!visible[r]) continue;
    for (int ty = rect[n_rec + r]; ty <= rect[3 * n_rec + r]; ty++)
      for (int tx = rect[r]; tx <= rect[2 * n_rec + r]; tx++) {
        e[m].tile = tile_base[r] + (int64_t)ty * tiles_x[r] + tx;
        e[m].depth = depth_bits[r];
        e[m].tie = tiebreak[r];
        e[m].rec = r;
        m++;
      }
  }
  qsort(e, (size_t)count, sizeof(ora_entry), cmp_entry);
  for (int64_t t = 0; t < n_tiles_total; t++) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
  for (int64_t k = 0; k < count; k++) {
    out_tile[k] = e[k].tile;
    out_depth[k] = e[k].depth;
    out_value[k] = e[k].rec;
    if (k == 0 || e[k].tile != e[k - 1].tile) ranges[2 * e[k].tile] = k;
    ranges[2 * e[k].tile + 1] = k + 1;
  }
  free(e);
  return count;
}

/* ------------------------------------------------------------------------
 * Per-pixel front-to-back compositing (Sec. 3.2 blending equation, with the
 * 3DGS alpha rules):
 *   d = pixel centre - mean2d;  p = -(A dx^2 + C dy^2)/2 - B dx dy
 *   skip if p > 0;  alpha = min(alpha_max, o e^p);  skip if alpha < alpha_min
 *   stop before blending an entry whose T (1 - alpha) would fall below T_min
 *   C += alpha T colour;  D += alpha T depth;  T *= 1 - alpha
 * Output colour C + T bg, final T, and `last` = number of list entries
 * processed before the stop (or the list length).
 * Records are planes indexed by record id: mean2d [2][nr], conic [3][nr],
 * opacity [nr], color [3][nr], depth [nr].  A pixel is marked ambiguous when
 * an alpha decision has relative margin below delta, the stop decision one
 * below delta_T, a record flagged ambiguous (rec_amb bit 0) could blend into
 * it, or two entries that may blend into it (alpha within delta of
 * alpha_min or above) follow each other in an order another evaluation could
 * flip: depths closer than delta_depth relative, or float32 depths at most
 * one unit in the last place apart where one of the two records has a depth
 * whose float32 rounding is itself ambiguous (rec_amb bit 1).
 */
typedef struct {
  int64_t nr;
  const double *mean2d, *conic, *opacity, *color, *depth;
  const uint8_t *rec_amb; /* may be NULL */
} ora_records;

static int composite_pixel(const ora_opts *o, const ora_records *rc, const int64_t *vals,
                           int64_t len, double px, double py, double delta, double delta_T,
                           double delta_depth, double C[3], double *D, double *Tout, int *amb,
                           double *alpha_hist, double *T_hist, int64_t *sig, int *n_blended) {
  double T = 1.0;
  int nb = 0; /* entries blended (alpha >= alpha_min before the stop) */
  double prev_depth = NAN; /* depth of the last entry that may blend into this pixel */
  int64_t prev_r = -1;
  C[0] = C[1] = C[2] = 0;
  *D = 0;
  *amb = 0;
  uint64_t h = 0; /* signature of the set of blended entries (for finite differences) */
  int64_t j;
  for (j = 0; j < len; j++) {
    int64_t r = vals[j];
    double dx = px + 0.5 - rc->mean2d[r];
    double dy = py + 0.5 - rc->mean2d[rc->nr + r];
    double A = rc->conic[r], B = rc->conic[rc->nr + r], Cc = rc->conic[2 * rc->nr + r];
    double p = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
    if (alpha_hist) alpha_hist[j] = 0;
    if (p > 0) continue;
    double raw = rc->opacity[r] * exp(p);
    /* a record with an ambiguous decision of its own matters where it could blend */
    if (rc->rec_amb && (rc->rec_amb[r] & 1) && raw >= 0.5 * o->alpha_min) *amb = 1;
    if (rel_margin(raw, o->alpha_min) < delta || rel_margin(raw, o->alpha_max) < delta) *amb = 1;
    if (raw >= o->alpha_min * (1.0 - delta)) {
      double dep = rc->depth[r];
      if (fabs(dep - prev_depth) < delta_depth * fabs(dep)) *amb = 1; /* false while prev_depth is NaN */
      if (prev_r >= 0 && rc->rec_amb && ((rc->rec_amb[r] | rc->rec_amb[prev_r]) & 2)) {
        float a = (float)dep, b = (float)prev_depth;
        if (a == b || nextafterf(b, INFINITY) == a || nextafterf(b, -INFINITY) == a) *amb = 1;
      }
      prev_depth = dep;
      prev_r = r;
    }
    double alpha = raw < o->alpha_max ? raw : o->alpha_max;
    if (alpha < o->alpha_min) continue;
    double Tn = T * (1.0 - alpha);
    if (rel_margin(Tn, o->T_min) < delta_T) *amb = 1;
    if (Tn < o->T_min) break;
    for (int ch = 0; ch < 3; ch++) C[ch] += alpha * T * rc->color[ch * rc->nr + r];
    *D += alpha * T * rc->depth[r];
    if (alpha_hist) { alpha_hist[j] = alpha; T_hist[j] = T; }
    h = h * 1000003u + (uint64_t)(r + 1) * (uint64_t)(j + 1);
    T = Tn;
    nb++;
  }
  *Tout = T;
  if (n_blended) *n_blended = nb;
  if (sig) *sig = (int64_t)(h ^ (uint64_t)j);
  return (int)j;
}

/* Renders one view.  ranges_view points at this view's [tiles][2] ranges;
 * values are record ids in sorted order.  image [3][H][W]. */
void ora_render(const ora_opts *o, int32_t W, int32_t H, const int64_t *ranges_view,
                const int64_t *values, int64_t nr, const double *mean2d, const double *conic,
                const double *opacity, const double *color, const double *depth,
                const uint8_t *rec_amb, double delta, double delta_T, double delta_depth, double *image,
                double *T_final, int32_t *last, double *depth_out, uint8_t *ambiguous, int64_t *signature,
                int32_t *blended) {
  ora_records rc = {nr, mean2d, conic, opacity, color, depth, rec_amb};
  int tiles_x = (W + o->tile_w - 1) / o->tile_w;
  int64_t P = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t pix = 0; pix < P; pix++) {
    int px = (int)(pix % W), py = (int)(pix / W);
    int64_t t = (int64_t)(py / o->tile_h) * tiles_x + px / o->tile_w;
    int64_t s = ranges_view[2 * t], e = ranges_view[2 * t + 1];
    double C[3], D, T;
    int amb;
    int64_t sg;
    int nb;
    int n = composite_pixel(o, &rc, values + s, e - s, px, py, delta, delta_T, delta_depth, C, &D, &T, &amb, NULL,
                            NULL, &sg, &nb);
    if (blended) blended[pix] = nb;
    for (int ch = 0; ch < 3; ch++) image[ch * P + pix] = C[ch] + T * o->bg[ch];
    T_final[pix] = T;
    last[pix] = n;
    if (signature) signature[pix] = sg;
    if (depth_out) depth_out[pix] = D;
    if (ambiguous) ambiguous[pix] = (uint8_t)amb;
  }
}

/* Per-pixel brute force: every visible record of the view whose rectangle
 * covers the pixel's tile, ordered by (depth bits, tiebreak) with qsort.
 * Used only to check the binned path on tiny inputs. */
typedef struct { uint32_t depth; int64_t tie; int64_t rec; } ora_bentry;
static int cmp_bentry(const void *pa, const void *pb) {
  const ora_bentry *a = pa, *b = pb;
  if (a->depth != b->depth) return a->depth < b->depth ? -1 : 1;
  if (a->tie != b->tie) return a->tie < b->tie ? -1 : 1;
  return 0;
}

void ora_render_brute(const ora_opts *o, int32_t W, int32_t H, int64_t nr, const int32_t *visible,
                      const int32_t *rect, const uint32_t *depth_bits, const int64_t *tiebreak,
                      const double *mean2d, const double *conic, const double *opacity,
                      const double *color, const double *depth, double *image, double *T_final,
                      int32_t *last) {
  ora_records rc = {nr, mean2d, conic, opacity, color, depth, NULL};
  int64_t P = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t pix = 0; pix < P; pix++) {
    int px = (int)(pix % W), py = (int)(pix / W);
    int tx = px / o->tile_w, ty = py / o->tile_h;
    ora_bentry *list = malloc(sizeof(ora_bentry) * (nr > 0 ? nr : 1));
    int64_t m = 0;
    for (int64_t r = 0; r < nr; r++) {
      if (!visible[r]) continue;
      if (tx < rect[r] || tx > rect[2 * nr + r] || ty < rect[nr + r] || ty > rect[3 * nr + r]) continue;
      list[m].depth = depth_bits[r];
      list[m].tie = tiebreak[r];
      list[m].rec = r;
      m++;
    }
    qsort(list, (size_t)m, sizeof(ora_bentry), cmp_bentry);
    int64_t *vals = malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    for (int64_t k = 0; k < m; k++) vals[k] = list[k].rec;
    double C[3], D, T;
    int amb;
    int n = composite_pixel(o, &rc, vals, m, px, py, 0.0, 0.0, 0.0, C, &D, &T, &amb, NULL, NULL, NULL, NULL);
    for (int ch = 0; ch < 3; ch++) image[ch * P + pix] = C[ch] + T * o->bg[ch];
    T_final[pix] = T;
    last[pix] = n;
    free(vals);
    free(list);
  }
}

/* ------------------------------------------------------------------------
 * Reverse mode of the compositing for one view.  Given dL/dC_out per pixel
 * ([3][H][W]), accumulates into g2d ([9][nr] planes: dmean2d x, y;
 * dconic A, B, C; dopacity; dcolor r, g, b).  Per blended entry i with
 * transmittance T_i and B_i = sum_{j>i} alpha_j T_j c_j + T_final bg:
 *   dC/dc_i = alpha_i T_i,   dC/dalpha_i = T_i c_i - B_i / (1 - alpha_i)
 *   alpha = o G below the clamp: dalpha/do = G, dalpha/dp = alpha;
 *   above the clamp (alpha = alpha_max) both are zero.
 *   dp/dmean = (A dx + B dy, B dx + C dy);  dp/d(A, B, C) = (-dx^2/2, -dx dy, -dy^2/2)
 * The pixel's depth channel carries no gradient.
 */
void ora_render_bwd(const ora_opts *o, int32_t W, int32_t H, const int64_t *ranges_view,
                    const int64_t *values, int64_t nr, const double *mean2d, const double *conic,
                    const double *opacity, const double *color, const double *depth,
                    const double *dL_dimg, double *g2d) {
  ora_records rc = {nr, mean2d, conic, opacity, color, depth, NULL};
  int tiles_x = (W + o->tile_w - 1) / o->tile_w;
  int64_t P = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t pix = 0; pix < P; pix++) {
    int px = (int)(pix % W), py = (int)(pix / W);
    int64_t t = (int64_t)(py / o->tile_h) * tiles_x + px / o->tile_w;
    int64_t s = ranges_view[2 * t], e = ranges_view[2 * t + 1];
    int64_t len = e - s;
    if (len == 0) continue;
    double *ah = malloc(sizeof(double) * len), *th = malloc(sizeof(double) * len);
    double C[3], D, T;
    int amb;
    int n = composite_pixel(o, &rc, values + s, len, px, py, 0.0, 0.0, 0.0, C, &D, &T, &amb, ah, th, NULL, NULL);
    double g[3] = {dL_dimg[pix], dL_dimg[P + pix], dL_dimg[2 * P + pix]};
    double Bacc[3] = {T * o->bg[0], T * o->bg[1], T * o->bg[2]};
    for (int j = n - 1; j >= 0; j--) {
      double alpha = ah[j];
      if (alpha == 0) continue; /* skipped entry */
      int64_t r = values[s + j];
      double Ti = th[j];
      double col[3] = {color[r], color[nr + r], color[2 * nr + r]};
      double dL_dalpha = 0;
      for (int ch = 0; ch < 3; ch++) {
        dL_dalpha += g[ch] * (Ti * col[ch] - Bacc[ch] / (1.0 - alpha));
#pragma omp atomic
        g2d[(6 + ch) * nr + r] += g[ch] * alpha * Ti;
      }
      for (int ch = 0; ch < 3; ch++) Bacc[ch] += alpha * Ti * col[ch];
      double dx = px + 0.5 - mean2d[r], dy = py + 0.5 - mean2d[nr + r];
      double A = conic[r], B = conic[nr + r], Cc = conic[2 * nr + r];
      double p = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
      double G = exp(p);
      double raw = opacity[r] * G;
      if (raw >= o->alpha_max) continue; /* clamped: no gradient to o or the shape */
      double dL_dp = dL_dalpha * alpha;
#pragma omp atomic
      g2d[5 * nr + r] += dL_dalpha * G;
#pragma omp atomic
      g2d[0 * nr + r] += dL_dp * (A * dx + B * dy);
#pragma omp atomic
      g2d[1 * nr + r] += dL_dp * (B * dx + Cc * dy);
#pragma omp atomic
      g2d[2 * nr + r] += dL_dp * (-0.5 * dx * dx);
#pragma omp atomic
      g2d[3 * nr + r] += dL_dp * (-dx * dy);
#pragma omp atomic
      g2d[4 * nr + r] += dL_dp * (-0.5 * dy * dy);
    }
    free(ah);
    free(th);
  }
}

/* ------------------------------------------------------------------------
 * Reverse mode of the projection for one view.  g2d points at this view's
 * [9] planes with stride g2d_stride.  Adds the raw-parameter gradients into
 * grads ([3 means][3 log_scales][4 quats][1 logit][3K sh] planes of length n)
 * and, for every visible Gaussian, adds stat_scale * |dL/dmean2d|_2 to
 * stat_S and 1 to stat_n (the view-space positional statistic that
 * selective densification reads, Sec. 3.3).
 */
void ora_project_bwd(const ora_opts *o, const ora_cam *cam, int64_t n, int sh_degree,
                     const double *means, const double *log_scales, const double *quats,
                     const double *logits, const double *sh, const uint8_t *keep,
                     const double *g2d, int64_t g2d_stride, double stat_scale, double *grads,
                     double *stat_S, int32_t *stat_n) {
  int K = (sh_degree + 1) * (sh_degree + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double mu[3], ls[3], q[4], shv[3 * ORA_MAX_SH];
    for (int a = 0; a < 3; a++) { mu[a] = means[a * n + i]; ls[a] = log_scales[a * n + i]; }
    for (int a = 0; a < 4; a++) q[a] = quats[a * n + i];
    for (int k = 0; k < 3 * K; k++) shv[k] = sh[(int64_t)k * n + i];
    ora_fwd f;
    project_one(o, cam, sh_degree, mu, ls, q, logits[i], shv, keep ? keep[i] != 0 : 1, &f);
    if (!f.visible) continue;
    double gm2[2] = {g2d[0 * g2d_stride + i], g2d[1 * g2d_stride + i]};
    double gA = g2d[2 * g2d_stride + i], gB = g2d[3 * g2d_stride + i], gC = g2d[4 * g2d_stride + i];
    double go = g2d[5 * g2d_stride + i];
    double gcol[3] = {g2d[6 * g2d_stride + i], g2d[7 * g2d_stride + i], g2d[8 * g2d_stride + i]};
    double gmu[3] = {0, 0, 0};

    /* statistics */
    stat_S[i] += stat_scale * sqrt(gm2[0] * gm2[0] + gm2[1] * gm2[1]);
    stat_n[i] += 1;

    /* colour -> SH coefficients and view direction */
    double Y[ORA_MAX_SH], dY[ORA_MAX_SH * 3];
    ora_sh_basis(sh_degree, f.dirn, Y, dY);
    double gdir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ch++) {
      double graw = f.color_raw[ch] > 0 ? gcol[ch] : 0.0;
      for (int k = 0; k < K; k++) {
        grads[(int64_t)(11 + k * 3 + ch) * n + i] += graw * Y[k];
        for (int a = 0; a < 3; a++) gdir[a] += graw * shv[k * 3 + ch] * dY[k * 3 + a];
      }
    }
    double dd = gdir[0] * f.dirn[0] + gdir[1] * f.dirn[1] + gdir[2] * f.dirn[2];
    for (int a = 0; a < 3; a++) gmu[a] += (gdir[a] - dd * f.dirn[a]) / f.dnorm;

    /* opacity */
    grads[(int64_t)10 * n + i] += go * f.opacity * (1.0 - f.opacity);

    /* conic (A, B, C) = (c, -b, a) / det  ->  2D covariance (a, b, c) */
    double a = f.a, b = f.b, c = f.c, det2 = f.det * f.det;
    double ga = (-gA * c * c + gB * b * c - gC * b * b) / det2;
    double gb = (2 * gA * b * c - gB * (a * c + b * b) + 2 * gC * a * b) / det2;
    double gc = (-gA * b * b + gB * a * b - gC * a * a) / det2;
    double GS[4] = {ga, 0.5 * gb, 0.5 * gb, gc}; /* symmetric 2x2 gradient */

    /* S2 = T Sigma T^T with T = J W:  dL/dSigma = T^T GS T,  dL/dT = 2 GS T Sigma */
    double T[6];
    for (int r = 0; r < 2; r++)
      for (int j = 0; j < 3; j++) {
        double acc = 0;
        for (int k = 0; k < 3; k++) acc += f.J[r * 3 + k] * f.Wc[k * 3 + j];
        T[r * 3 + j] = acc;
      }
    double GSig[9];
    for (int k = 0; k < 3; k++)
      for (int l = 0; l < 3; l++) {
        double acc = 0;
        for (int r = 0; r < 2; r++)
          for (int s = 0; s < 2; s++) acc += T[r * 3 + k] * GS[r * 2 + s] * T[s * 3 + l];
        GSig[k * 3 + l] = acc;
      }
    double GT[6];
    for (int r = 0; r < 2; r++)
      for (int j = 0; j < 3; j++) {
        double acc = 0;
        for (int s = 0; s < 2; s++)
          for (int k = 0; k < 3; k++) acc += GS[r * 2 + s] * T[s * 3 + k] * f.Sigma[k * 3 + j];
        GT[r * 3 + j] = 2 * acc;
      }
    /* T = J W  ->  dL/dJ = dL/dT W^T */
    double GJ[6];
    for (int r = 0; r < 2; r++)
      for (int k = 0; k < 3; k++) {
        double acc = 0;
        for (int j = 0; j < 3; j++) acc += GT[r * 3 + j] * f.Wc[k * 3 + j];
        GJ[r * 3 + k] = acc;
      }
    /* J -> camera-space mean.  J02 = -fx u / tz with u = tx/tz unless clamped */
    double tx = f.tc[0], ty = f.tc[1], tz = f.tc[2];
    double fx = cam->fx, fy = cam->fy;
    double gt[3] = {0, 0, 0};
    gt[2] += GJ[0] * (-fx / (tz * tz)) + GJ[4] * (-fy / (tz * tz));
    double du_dtx = f.clamp_u ? 0.0 : 1.0 / tz, du_dtz = f.clamp_u ? 0.0 : -tx / (tz * tz);
    double dv_dty = f.clamp_v ? 0.0 : 1.0 / tz, dv_dtz = f.clamp_v ? 0.0 : -ty / (tz * tz);
    gt[0] += GJ[2] * (-fx / tz * du_dtx);
    gt[2] += GJ[2] * (fx * f.u / (tz * tz) - fx / tz * du_dtz);
    gt[1] += GJ[5] * (-fy / tz * dv_dty);
    gt[2] += GJ[5] * (fy * f.v / (tz * tz) - fy / tz * dv_dtz);
    /* mean2d -> camera-space mean */
    gt[0] += gm2[0] * fx / tz;
    gt[2] += gm2[0] * (-fx * tx / (tz * tz));
    gt[1] += gm2[1] * fy / tz;
    gt[2] += gm2[1] * (-fy * ty / (tz * tz));
    /* t = W mu + t_v */
    for (int a = 0; a < 3; a++)
      for (int k = 0; k < 3; k++) gmu[a] += cam->R[k * 3 + a] * gt[k];

    /* Sigma = M M^T, M = Rq diag(s) */
    double GM[9];
    for (int r = 0; r < 3; r++)
      for (int j = 0; j < 3; j++) {
        double acc = 0;
        for (int k = 0; k < 3; k++) acc += GSig[r * 3 + k] * f.M[k * 3 + j];
        GM[r * 3 + j] = 2 * acc;
      }
    double GR[9];
    for (int j = 0; j < 3; j++) {
      double gs = 0;
      for (int r = 0; r < 3; r++) {
        gs += GM[r * 3 + j] * f.Rq[r * 3 + j];
        GR[r * 3 + j] = GM[r * 3 + j] * f.s[j];
      }
      grads[(int64_t)(3 + j) * n + i] += gs * f.s[j];
    }
    /* rotation matrix -> unit quaternion (w, x, y, z) */
    double w = f.qh[0], x = f.qh[1], y = f.qh[2], z = f.qh[3];
    double gq[4];
    gq[0] = 2 * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
    gq[1] = 2 * (y * GR[1] + z * GR[2] + y * GR[3] - 2 * x * GR[4] - w * GR[5] + z * GR[6] + w * GR[7] - 2 * x * GR[8]);
    gq[2] = 2 * (-2 * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] + z * GR[7] - 2 * y * GR[8]);
    gq[3] = 2 * (-2 * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2 * z * GR[4] + y * GR[5] + x * GR[6] + y * GR[7]);
    /* normalisation q_hat = q / |q| */
    double gd = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;
    for (int a = 0; a < 4; a++) grads[(int64_t)(6 + a) * n + i] += (gq[a] - gd * f.qh[a]) / f.qn;
    for (int a = 0; a < 3; a++) grads[(int64_t)a * n + i] += gmu[a];
  }
}

/* Mean absolute error of one view and its gradient scaled by `scale`:
 * dL/dC = scale * sign(C - target) with sign(0) = 0.  Returns the sum of
 * |C - target| (the caller divides). */
double ora_l1(int64_t count, const double *img, const double *target, double scale, double *grad) {
  double acc = 0;
  for (int64_t k = 0; k < count; k++) {
    double d = img[k] - target[k];
    acc += fabs(d);
    grad[k] = d > 0 ? scale : (d < 0 ? -scale : 0.0);
  }
  return acc;
}
