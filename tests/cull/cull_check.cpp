// Host build of the kernels' sub-block cull (paper_2510_01767_amd/csrc/gsr_cull.h)
// checked against brute force: for random records made the way the
// projection makes them (conic of a 2D covariance with the 0.3 px dilation,
// base-2 exponent coefficients, the alpha_min level with its slack, the reach
// radius) and random 16 x 4 strips of four 4 x 4 sub-blocks, no sub-block
// that holds a pixel centre whose float32 exponent passes the per-pair
// test may be culled.  The device's 1-ulp reciprocal and square root are
// modelled by nudging each result by one ulp either way at random.
//
// usage: cull_check SEED COUNT  -> prints counts; exit status 1 on a dropped sub-block
#include <algorithm>
#include <cmath>
#include <math.h>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>

static std::mt19937_64 g_rng;

static float rcp_1ulp(float x) {
  const float r = 1.0f / x;
  const int s = (int)(g_rng() % 3) - 1;
  return s == 0 ? r : std::nextafter(r, s > 0 ? INFINITY : -INFINITY);
}
static float sqrt_1ulp(float x) {
  const float r = std::sqrt(x);
  const int s = (int)(g_rng() % 3) - 1;
  return s == 0 || !(r > 0.0f) || std::isinf(r) ? r : std::nextafter(r, s > 0 ? INFINITY : -INFINITY);
}
static float med3(float a, float b, float c) { return std::max(std::min(a, b), std::min(std::max(a, b), c)); }

struct float4 {
  float x, y, z, w;
};
#define __device__
#define __forceinline__ inline
#define __builtin_amdgcn_rcpf(x) rcp_1ulp(x)
#define __builtin_amdgcn_sqrtf(x) sqrt_1ulp(x)
#define __builtin_amdgcn_fmed3f(a, b, c) med3(a, b, c)
#define __fmaf_rn(a, b, c) std::fmaf(a, b, c)
#define __fma_rn(a, b, c) std::fma(a, b, c)
#include "gsr_cull.h"

using gsr::LdsRec;

static double U(double a, double b) { return std::uniform_real_distribution<double>(a, b)(g_rng); }

// a pixel (pxc, pyc) can blend the record only if pmin2 <= p2 <= 0: the
// kernels skip p2 > 0, and below the record's pmin2 their alpha test cannot
// pass (o 2^p2 < alpha_min there with margin), so this set holds every pixel
// the kernels can blend
static bool pixel_can_blend(const LdsRec &R, float pxc, float pyc) {
  const float dx = (pxc - R.r0.x) - R.r0.z, dy = (pyc - R.r0.y) - R.r0.w;
  const float t = std::fmaf(R.r1.x, dx, R.r1.y * dy);
  const float cdy = R.r1.z * dy;
  const float p2 = std::fmaf(t, dx, cdy * dy);
  return !(p2 > 0.0f || p2 < R.r2.w);
}

// The three tile shapes' strips: TW x kRows pixels split into four sub-blocks
// of SW x SH, SNX of them side by side (16 x 16 tiles: 16 x 4 strips of 4 x 4;
// 32 x 8: 32 x 2 of 8 x 2; 8 x 32: 8 x 8 of 4 x 4 in two bands).
struct StripShape {
  int tw, rows, sw, sh, snx;
};
static const StripShape kShapes[3] = {{16, 4, 4, 4, 4}, {32, 2, 8, 2, 4}, {8, 8, 4, 4, 2}};

// one strip: the cull's outcome for each of its four sub-blocks (as the
// kernels' sub-list pass takes it), brute force beside it
struct Outcome {
  bool kept[4], truth[4];
};

static Outcome classify(const LdsRec &R, const StripShape &sh, float wx0, float wy0) {
  Outcome v;
  const float wx1 = wx0 + (float)(sh.tw - 1), wy1 = wy0 + (float)(sh.rows - 1);
  const bool strip = gsr::reaches_strip(R, wx0, wx1, wy0, wy1);
  const gsr::ReachShape S = gsr::reach_shape(R);
  float xl = 3.0e38f, xr = -3.0e38f;
  for (int q = 0; q < 4; q++) {
    const float bx0 = wx0 + (float)((q % sh.snx) * sh.sw), by0 = wy0 + (float)((q / sh.snx) * sh.sh);
    if (q % sh.snx == 0) gsr::band_interval(R, S, by0, by0 + (float)(sh.sh - 1), xl, xr);
    const float x0 = (bx0 - R.r0.x) - R.r0.z, x1 = ((bx0 + (float)(sh.sw - 1)) - R.r0.x) - R.r0.z;
    v.kept[q] = strip && (S.thin || (x1 >= xl && x0 <= xr));
    bool t = false;
    for (int yy = 0; yy < sh.sh && !t; yy++)
      for (int xx = 0; xx < sh.sw && !t; xx++) t = pixel_can_blend(R, bx0 + (float)xx, by0 + (float)yy);
    v.truth[q] = t;
  }
  return v;
}

// a record from a 2D covariance (s1, s2, angle), opacity and mean, as the projection stores it
static LdsRec make_record(double s1, double s2, double th, double opac, double mx, double my, double alpha_min) {
  const double cs = std::cos(th), sn = std::sin(th);
  const double sxx = s1 * s1 * cs * cs + s2 * s2 * sn * sn + 0.3;
  const double syy = s1 * s1 * sn * sn + s2 * s2 * cs * cs + 0.3;
  const double sxy = (s1 * s1 - s2 * s2) * cs * sn;
  const double det = sxx * syy - sxy * sxy;
  const double A = syy / det, B = -sxy / det, C = sxx / det;
  const double lam = 0.5 * (sxx + syy) + std::sqrt(0.25 * (sxx - syy) * (sxx - syy) + sxy * sxy);
  const double c2 = 2.0 * std::log(opac / alpha_min) + 1e-5;
  const double l2e = 1.44269504088896340736;
  LdsRec R;
  const float hx = (float)mx, hy = (float)my;
  R.r0 = {hx, hy, (float)(mx - (double)hx), (float)(my - (double)hy)};
  R.r1 = {(float)(-0.5 * l2e * A), (float)(-l2e * B), (float)(-0.5 * l2e * C), (float)opac};
  R.r2 = {0.5f, 0.5f, 0.5f, c2 > 0.0 ? (float)(-0.5 * c2 * l2e) : 0.0f};
  R.reach = c2 > 0.0 ? (float)(std::sqrt(c2 * lam) * 1.001 + 0.01) : -1.0f;
  return R;
}

int main(int argc, char **argv) {
  const unsigned long long seed = argc > 1 ? strtoull(argv[1], nullptr, 10) : 1;
  const long n = argc > 2 ? atol(argv[2]) : 200000;
  g_rng.seed(seed);
  const double alpha_min = 1.0 / 255.0;
  long tests = 0, truth = 0, kept = 0, dropped = 0, thin = 0;
  for (long it = 0; it < n; it++) {
    // sizes from sub-pixel to a few thousand pixels, aspect up to 1e4 : 1 on a quarter of them
    const double s1 = std::exp(U(std::log(0.05), std::log(3000.0)));
    const double s2 = s1 / std::exp(U(0.0, std::log(it % 4 == 0 ? 1e4 : 30.0)));
    const double th = U(0.0, M_PI);
    const double opac = std::exp(U(std::log(alpha_min * 0.9), 0.0));
    // strips anywhere on a 3840 x 2160 view, means near them
    const double ox = std::floor(U(0.0, 3824.0)), oy = std::floor(U(0.0, 2156.0));
    const double mx = ox + U(-40.0, 72.0), my = oy + U(-40.0, 48.0);
    const LdsRec R = make_record(s1, s2, th, opac, mx, my, alpha_min);
    thin += gsr::reach_shape(R).thin;
    const Outcome v = classify(R, kShapes[it % 3], (float)ox + 0.5f, (float)oy + 0.5f);
    for (int q = 0; q < 4; q++) {
      tests++;
      truth += v.truth[q];
      kept += v.kept[q];
      if (v.truth[q] && !v.kept[q]) {
        if (dropped < 5)
          printf("dropped: it %ld q %d s1 %.9g s2 %.9g th %.9g opac %.9g mean (%.9g, %.9g) strip (%g, %g)\n", it, q,
                 s1, s2, th, opac, mx, my, ox, oy);
        dropped++;
      }
    }
  }
  // special cases: a record that reaches alpha_min nowhere is never kept; one
  // whose mean lies in a sub-block keeps it; a degenerate conic (det <= 0
  // after rounding) falls back to the circle
  long special = 0;
  {
    LdsRec R = make_record(3.0, 2.0, 0.3, alpha_min * 0.5, 100.0, 100.0, alpha_min);
    const Outcome v = classify(R, kShapes[0], 96.5f, 98.5f);
    for (int q = 0; q < 4; q++) special += v.kept[q];
    R = make_record(0.2, 0.2, 0.0, 0.9, 101.7, 100.2, alpha_min);
    const Outcome w = classify(R, kShapes[0], 96.5f, 98.5f);
    special += !w.kept[1] || !w.truth[1];
    R.r1.y = 2.0f * std::sqrt(R.r1.x * R.r1.z) * 1.0001f;  // 4ac - b^2 < 0
    special += !gsr::reach_shape(R).thin;
  }
  printf("tests %ld truth %ld kept %ld dropped %ld thin %ld special_failures %ld\n", tests, truth, kept, dropped,
         thin, special);
  if (special) return 1;
  return dropped != 0;
}
