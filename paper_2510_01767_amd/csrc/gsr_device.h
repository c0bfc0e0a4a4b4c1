// Device-side math of the rasterizer: per-Gaussian geometry, projection of
// one Gaussian into one view, the SH colour, the per-pair compositing step
// and wavefront reductions.  Everything per Gaussian-view runs in float64
// (MI355X issues a wave64 FP64 FMA at the rate of an unpacked FP32 one, and
// the projected mean must be exact to ~1e-6 px at city-scale coordinates);
// everything per (pixel, Gaussian) pair runs in float32.
#pragma once

#include <hip/hip_runtime.h>

#include "gsr_internal.h"

namespace gsr {

// ------------------------------------------------------------ camera, geometry

// One view's camera in float64, with the per-view constants of the
// projection computed once per workgroup (kept in LDS).
struct Cam64 {
  double R[9], t[3], fx, fy, cx, cy;
  double limx, limy;  // clamp of x/z and y/z inside the Jacobian
  double itw, ith;    // 1 / tile size (powers of two, so x * itw == x / tile_w)
  double cc[3];       // R^T t: mean + cc is the mean relative to the camera centre
  int W, H, tiles_x, tiles_y;
};

__device__ __forceinline__ Cam64 cam64(const gsr_camera &c, const ViewInfo &vi, const KOpts &o) {
  Cam64 k;
#pragma unroll
  for (int a = 0; a < 9; a++) k.R[a] = (double)c.R[a];
#pragma unroll
  for (int a = 0; a < 3; a++) k.t[a] = (double)c.t[a];
  k.fx = c.fx;
  k.fy = c.fy;
  k.cx = c.cx;
  k.cy = c.cy;
  k.W = vi.W;
  k.H = vi.H;
  k.tiles_x = vi.tiles_x;
  k.tiles_y = vi.tiles_y;
  k.limx = (double)o.jac_clamp * (0.5 * k.W / k.fx);
  k.limy = (double)o.jac_clamp * (0.5 * k.H / k.fy);
  k.itw = 1.0 / (double)o.tile_w;
  k.ith = 1.0 / (double)o.tile_h;
#pragma unroll
  for (int a = 0; a < 3; a++) k.cc[a] = k.R[a] * k.t[0] + k.R[3 + a] * k.t[1] + k.R[6 + a] * k.t[2];
  return k;
}

// The cameras of views [0, n_views) into LDS (one per thread, then a barrier).
__device__ __forceinline__ void load_cams(Cam64 *s_cam, const gsr_camera *cams, const ViewInfo *views, int n_views,
                                          const KOpts &o) {
  for (int v = threadIdx.x; v < n_views; v += blockDim.x) s_cam[v] = cam64(cams[v], views[v], o);
  __syncthreads();
}

// View-independent part of one Gaussian.
struct Geo {
  double mu[3];
  double s[3];   // exp(log_scale)
  double q[4];   // unit quaternion (w, x, y, z)
  double qn;     // |q_raw|
  double Rq[9];  // rotation of q, row major
  double Sig[6]; // covariance, symmetric: xx xy xz yy yz zz
  double opac;
};

__device__ __forceinline__ void rot_of_quat(const double q[4], double Rq[9]) {
  // R = (w^2 - |v|^2) I + 2 v v^T + 2 w [v]x   for the unit quaternion (w, v)
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  const double d = w * w - (x * x + y * y + z * z);
  Rq[0] = d + 2 * x * x;   Rq[1] = 2 * x * y - 2 * w * z; Rq[2] = 2 * x * z + 2 * w * y;
  Rq[3] = 2 * y * x + 2 * w * z; Rq[4] = d + 2 * y * y;   Rq[5] = 2 * y * z - 2 * w * x;
  Rq[6] = 2 * z * x - 2 * w * y; Rq[7] = 2 * z * y + 2 * w * x; Rq[8] = d + 2 * z * z;
}

// Activations and the 3D covariance of Gaussian i.  Both the forward (lean
// GeoF) and the reverse pass (full Geo) go through these helpers, so they
// see bit-identical covariances.
__device__ __forceinline__ void geo_core(const KParams &p, int64_t i, double mu[3], double s[3], double q[4],
                                         double &qn, double Rq[9], double Sig[6], double &opac) {
  const int64_t n = p.n;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    mu[a] = (double)p.means[a * n + i];
    s[a] = exp((double)p.log_scales[a * n + i]);
  }
  double qr[4];
#pragma unroll
  for (int a = 0; a < 4; a++) qr[a] = (double)p.quats[a * n + i];
  qn = sqrt(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
  const double inv = 1.0 / qn;
#pragma unroll
  for (int a = 0; a < 4; a++) q[a] = qr[a] * inv;
  rot_of_quat(q, Rq);
  // Sigma = Rq diag(s^2) Rq^T
  const double s2[3] = {s[0] * s[0], s[1] * s[1], s[2] * s[2]};
  const int idx[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
#pragma unroll
  for (int e = 0; e < 6; e++) {
    const int r = idx[e][0], c = idx[e][1];
    Sig[e] = Rq[r * 3 + 0] * s2[0] * Rq[c * 3 + 0] + Rq[r * 3 + 1] * s2[1] * Rq[c * 3 + 1] +
             Rq[r * 3 + 2] * s2[2] * Rq[c * 3 + 2];
  }
  opac = 1.0 / (1.0 + exp(-(double)p.logits[i]));
}

__device__ __forceinline__ void load_geo(const KParams &p, int64_t i, Geo &g) {
  geo_core(p, i, g.mu, g.s, g.q, g.qn, g.Rq, g.Sig, g.opac);
}

// What the forward keeps per Gaussian across views.
struct GeoF {
  double mu[3];
  double Sig[6];
  double opac;
  double smax2;  // largest eigenvalue of Sigma = max scale^2
};

__device__ __forceinline__ void load_geo_fwd(const KParams &p, int64_t i, GeoF &g) {
  double s[3], q[4], qn, Rq[9];
  geo_core(p, i, g.mu, s, q, qn, Rq, g.Sig, g.opac);
  g.smax2 = fmax(fmax(s[0] * s[0], s[1] * s[1]), s[2] * s[2]);
}

__device__ __forceinline__ double sig_at(const double S[6], int r, int c) {
  const int m = r < c ? r * 3 - (r * (r + 1)) / 2 + c : c * 3 - (c * (c + 1)) / 2 + r;
  return S[m];
}

// Projection of one Gaussian into one view.
struct Proj {
  double tc[3];
  double mx, my;
  double u, v;       // x/z, y/z as used inside J (clamped)
  bool cu, cv;       // clamp active
  double T0[3], T1[3];  // rows of J W
  double a, b, c, det;  // dilated 2D covariance
  double A, B, C;       // conic
  double lam;           // largest eigenvalue of the dilated 2D covariance
  int x0, y0, x1, y1;   // inclusive tile rectangle
};

// Returns true when the Gaussian is visible (depth inside (near, far),
// positive-definite 2D covariance, non-empty tile rectangle).
// Cheap conservative test: false only when the Gaussian is certainly not
// visible.  lambda_max(J W Sigma W^T J^T) <= |J|_F^2 max(s)^2, so the exact
// tile rectangle lies inside the one built from this bound.
__device__ __forceinline__ bool maybe_visible(const GeoF &g, const Cam64 &k, const KOpts &o) {
  double tc[3];
#pragma unroll
  for (int r = 0; r < 3; r++)
    tc[r] = k.R[r * 3 + 0] * g.mu[0] + k.R[r * 3 + 1] * g.mu[1] + k.R[r * 3 + 2] * g.mu[2] + k.t[r];
  const double tz = tc[2];
  if (!(tz > (double)o.near_plane && tz < (double)o.far_plane)) return false;
  const double iz = 1.0 / tz;
  const double ux = tc[0] * iz, uy = tc[1] * iz;
  const double mx = k.fx * ux + k.cx, my = k.fy * uy + k.cy;
  const double u = fmin(fabs(ux), k.limx), v = fmin(fabs(uy), k.limy);
  const double jn2 = (k.fx * iz) * (k.fx * iz) * (1.0 + u * u) + (k.fy * iz) * (k.fy * iz) * (1.0 + v * v);
  const double rb = ceil((double)o.sigma * sqrt(jn2 * g.smax2 + (double)o.eps2d)) + 1.0;
  return !(floor((mx + rb) * k.itw) < 0.0 || floor((my + rb) * k.ith) < 0.0 ||
           floor((mx - rb) * k.itw) > k.tiles_x - 1 || floor((my - rb) * k.ith) > k.tiles_y - 1);
}

// RECT = false (the reverse pass, on pairs known to be visible) stops after
// the conic: no eigenvalue, radius or tile rectangle.
template <bool RECT = true, class G>
__device__ __forceinline__ bool project_view(const G &g, const Cam64 &k, const KOpts &o, Proj &P) {
#pragma unroll
  for (int r = 0; r < 3; r++)
    P.tc[r] = k.R[r * 3 + 0] * g.mu[0] + k.R[r * 3 + 1] * g.mu[1] + k.R[r * 3 + 2] * g.mu[2] + k.t[r];
  const double tz = P.tc[2];
  if (!(tz > (double)o.near_plane && tz < (double)o.far_plane)) return false;
  const double iz = 1.0 / tz;
  const double ux = P.tc[0] * iz, uy = P.tc[1] * iz;
  P.mx = k.fx * ux + k.cx;
  P.my = k.fy * uy + k.cy;
  P.cu = fabs(ux) > k.limx;
  P.cv = fabs(uy) > k.limy;
  P.u = P.cu ? copysign(k.limx, ux) : ux;
  P.v = P.cv ? copysign(k.limy, uy) : uy;
  // J = [[fx/z, 0, -fx u / z], [0, fy/z, -fy v / z]];  T = J W
  const double j00 = k.fx * iz, j02 = -k.fx * P.u * iz, j11 = k.fy * iz, j12 = -k.fy * P.v * iz;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    P.T0[c] = j00 * k.R[c] + j02 * k.R[6 + c];
    P.T1[c] = j11 * k.R[3 + c] + j12 * k.R[6 + c];
  }
  double ST0[3], ST1[3];
#pragma unroll
  for (int r = 0; r < 3; r++) {
    ST0[r] = sig_at(g.Sig, r, 0) * P.T0[0] + sig_at(g.Sig, r, 1) * P.T0[1] + sig_at(g.Sig, r, 2) * P.T0[2];
    ST1[r] = sig_at(g.Sig, r, 0) * P.T1[0] + sig_at(g.Sig, r, 1) * P.T1[1] + sig_at(g.Sig, r, 2) * P.T1[2];
  }
  P.a = P.T0[0] * ST0[0] + P.T0[1] * ST0[1] + P.T0[2] * ST0[2] + (double)o.eps2d;
  P.b = P.T0[0] * ST1[0] + P.T0[1] * ST1[1] + P.T0[2] * ST1[2];
  P.c = P.T1[0] * ST1[0] + P.T1[1] * ST1[1] + P.T1[2] * ST1[2] + (double)o.eps2d;
  P.det = P.a * P.c - P.b * P.b;
  if (!(P.det > 0.0)) return false;
  const double idet = 1.0 / P.det;
  P.A = P.c * idet;
  P.B = -P.b * idet;
  P.C = P.a * idet;
  if (!RECT) return true;
  const double hd = 0.5 * (P.a - P.c);
  const double lam = 0.5 * (P.a + P.c) + sqrt(hd * hd + P.b * P.b);
  P.lam = lam;
  const double rad = ceil((double)o.sigma * sqrt(lam));
  const double lox = floor((P.mx - rad) * k.itw), hix = floor((P.mx + rad) * k.itw);
  const double loy = floor((P.my - rad) * k.ith), hiy = floor((P.my + rad) * k.ith);
  if (hix < 0.0 || hiy < 0.0 || lox > k.tiles_x - 1 || loy > k.tiles_y - 1) return false;
  P.x0 = lox < 0.0 ? 0 : (int)lox;
  P.y0 = loy < 0.0 ? 0 : (int)loy;
  P.x1 = hix > k.tiles_x - 1 ? k.tiles_x - 1 : (int)hix;
  P.y1 = hiy > k.tiles_y - 1 ? k.tiles_y - 1 : (int)hiy;
  return true;
}

// --------------------------------------------------------- spherical harmonics
// Real orthonormal SH with the Condon-Shortley phase, index l*l + l + m.
// The polynomials below agree with the textbook functions on the unit sphere;
// their gradients are only ever used projected onto the tangent plane.
constexpr double kY0 = 0.28209479177387814;   // 1/(2 sqrt(pi))
constexpr double kY1 = 0.48860251190291992;   // sqrt(3/(4 pi))
constexpr double kY2a = 1.0925484305920792;   // sqrt(15/pi)/2
constexpr double kY2b = 0.31539156525252005;  // sqrt(5/pi)/4
constexpr double kY2c = 0.54627421529603959;  // sqrt(15/pi)/4
constexpr double kY3a = 0.59004358992664352;  // sqrt(35/(2 pi))/4
constexpr double kY3b = 2.8906114426405538;   // sqrt(105/pi)/2
constexpr double kY3c = 0.45704579946446572;  // sqrt(21/(2 pi))/4
constexpr double kY3d = 0.37317633259011540;  // sqrt(7/pi)/4
constexpr double kY3e = 1.4453057213202769;   // sqrt(105/pi)/4

template <int D, class T>
__device__ __forceinline__ void sh_eval(T x, T y, T z, T *Y) {
  Y[0] = (T)kY0;
  if (D >= 1) {
    Y[1] = -(T)kY1 * y;
    Y[2] = (T)kY1 * z;
    Y[3] = -(T)kY1 * x;
  }
  if (D >= 2) {
    const T xx = x * x, yy = y * y, zz = z * z;
    Y[4] = (T)kY2a * x * y;
    Y[5] = -(T)kY2a * y * z;
    Y[6] = (T)kY2b * ((T)2 * zz - xx - yy);
    Y[7] = -(T)kY2a * x * z;
    Y[8] = (T)kY2c * (xx - yy);
    if (D >= 3) {
      Y[9] = -(T)kY3a * y * ((T)3 * xx - yy);
      Y[10] = (T)kY3b * x * y * z;
      Y[11] = -(T)kY3c * y * ((T)4 * zz - xx - yy);
      Y[12] = (T)kY3d * z * ((T)2 * zz - (T)3 * xx - (T)3 * yy);
      Y[13] = -(T)kY3c * x * ((T)4 * zz - xx - yy);
      Y[14] = (T)kY3e * z * (xx - yy);
      Y[15] = -(T)kY3a * x * (xx - (T)3 * yy);
    }
  }
}

// Gradient w.r.t. (x, y, z) of sum_k w_k Y_k (polynomial forms above).
template <int D, class T>
__device__ __forceinline__ void sh_grad(T x, T y, T z, const T *w, T g[3]) {
  g[0] = g[1] = g[2] = (T)0;
  if (D >= 1) {
    g[1] += -(T)kY1 * w[1];
    g[2] += (T)kY1 * w[2];
    g[0] += -(T)kY1 * w[3];
  }
  if (D >= 2) {
    g[0] += (T)kY2a * y * w[4];
    g[1] += (T)kY2a * x * w[4];
    g[1] += -(T)kY2a * z * w[5];
    g[2] += -(T)kY2a * y * w[5];
    g[0] += -(T)2 * (T)kY2b * x * w[6];
    g[1] += -(T)2 * (T)kY2b * y * w[6];
    g[2] += (T)4 * (T)kY2b * z * w[6];
    g[0] += -(T)kY2a * z * w[7];
    g[2] += -(T)kY2a * x * w[7];
    g[0] += (T)2 * (T)kY2c * x * w[8];
    g[1] += -(T)2 * (T)kY2c * y * w[8];
    if (D >= 3) {
      const T xx = x * x, yy = y * y, zz = z * z;
      g[0] += -(T)kY3a * (T)6 * x * y * w[9];
      g[1] += -(T)kY3a * ((T)3 * xx - (T)3 * yy) * w[9];
      g[0] += (T)kY3b * y * z * w[10];
      g[1] += (T)kY3b * x * z * w[10];
      g[2] += (T)kY3b * x * y * w[10];
      g[0] += (T)kY3c * (T)2 * x * y * w[11];
      g[1] += -(T)kY3c * ((T)4 * zz - xx - (T)3 * yy) * w[11];
      g[2] += -(T)kY3c * (T)8 * y * z * w[11];
      g[0] += -(T)kY3d * (T)6 * x * z * w[12];
      g[1] += -(T)kY3d * (T)6 * y * z * w[12];
      g[2] += (T)kY3d * ((T)6 * zz - (T)3 * xx - (T)3 * yy) * w[12];
      g[0] += -(T)kY3c * ((T)4 * zz - (T)3 * xx - yy) * w[13];
      g[1] += (T)kY3c * (T)2 * x * y * w[13];
      g[2] += -(T)kY3c * (T)8 * x * z * w[13];
      g[0] += (T)kY3e * (T)2 * x * z * w[14];
      g[1] += -(T)kY3e * (T)2 * y * z * w[14];
      g[2] += (T)kY3e * (xx - yy) * w[14];
      g[0] += -(T)kY3a * ((T)3 * xx - (T)3 * yy) * w[15];
      g[1] += (T)kY3a * (T)6 * x * y * w[15];
    }
  }
}

// ------------------------------------------------------------ per-pair step
// The alpha of one (pixel, record) pair.  Written with explicit fused
// multiply-adds so that the forward and the reverse kernels evaluate the
// identical float32 expression and replay the same skip / stop decisions.
struct PairAlpha {
  float dx, dy, G, raw, alpha;
  float t, cdy;  // a dx + b dy and c dy (parts of the exponent)
  bool in;       // p <= 0: a pair with a positive exponent (rounding) is skipped
};

// The record holds the exponent's coefficients in base 2, so the exponent
// p log2 e = a dx^2 + b dx dy + c dy^2 = (a dx + b dy) dx + (c dy) dy takes
// five operations and feeds the hardware 2^x directly (for
// ln(alpha_min / o) <= p <= 0, |p log2 e| < 12: the instruction's error stays
// below 6e-7 relative).  Callers take a pair only where `in` holds and
// alpha >= alpha_min.  Below the record's pmin (ln(alpha_min / o) minus a
// 5e-6 slack) o e^p stays under alpha_min by more than the rounding of the
// float32 steps, so the alpha test alone rejects those pairs.  With
// FINITE_G a positive exponent enters 2^x as 0, so that G (which the reverse
// pass multiplies by zero on skipped pairs) stays finite; without it G and
// raw may be infinite on skipped pairs, alpha is still at most alpha_max.
template <bool FINITE_G>
__device__ __forceinline__ PairAlpha pair_alpha(float pxc, float pyc, const float4 &r0, const float4 &r1,
                                                float alpha_max) {
  PairAlpha a;
  a.dx = (pxc - r0.x) - r0.z;
  a.dy = (pyc - r0.y) - r0.w;
  a.t = __fmaf_rn(r1.x, a.dx, r1.y * a.dy);
  a.cdy = r1.z * a.dy;
  const float p2 = __fmaf_rn(a.t, a.dx, a.cdy * a.dy);
  a.G = __builtin_amdgcn_exp2f(FINITE_G ? fminf(p2, 0.0f) : p2);
  a.in = !(p2 > 0.0f);
  a.raw = r1.w * a.G;
  // min(raw, alpha_max) as a signed integer minimum of the bit patterns:
  // alpha_max > 0, and raw is either >= 0 (where integer and float order
  // agree) or negative (sign bit set, so the integer minimum picks it, as the
  // float one does).  One operation, with no canonicalisation of alpha_max
  // inside the loop (a float minimum in IEEE mode re-quiets its operand).
  a.alpha = __int_as_float(min(__float_as_int(a.raw), __float_as_int(alpha_max)));
  return a;
}

// ------------------------------------------------------- wavefront reduction

template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ float dpp_or_zero(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK,
                                                               BANK_MASK, false));
}

// Sum over the 64 lanes of a wavefront; the total is valid in lane 63.
__device__ __forceinline__ float wave_sum_lane63(float x) {
  x += dpp_or_zero<0xB1>(x);       // quad_perm [1,0,3,2]
  x += dpp_or_zero<0x4E>(x);       // quad_perm [2,3,0,1]
  x += dpp_or_zero<0x141>(x);      // row_half_mirror
  x += dpp_or_zero<0x140>(x);      // row_mirror
  x += dpp_or_zero<0x142, 0xa>(x); // row_bcast:15 into rows 1 and 3
  x += dpp_or_zero<0x143, 0xc>(x); // row_bcast:31 into rows 2 and 3
  return x;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// ------------------------------------------------------------ shared helpers

constexpr int kBlock = 256;
constexpr double kLog2e = 1.44269504088896340736;  // log2(e)

__device__ __forceinline__ const float4 *rec_ptr(const KWs &ws, int64_t r) {
  return reinterpret_cast<const float4 *>(ws.records) + r * kRecordFloat4;
}

// Global tile id -> view (linear search over at most 32 views).
__device__ __forceinline__ int view_of_tile(const ViewInfo *views, int n_views, int64_t t) {
  int v = 0;
  while (v + 1 < n_views && views[v + 1].tile_base <= t) v++;
  return v;
}

// Workgroups of a grid are dispatched to the 8 XCDs round-robin (block b on
// XCD b % 8).  Give XCD x the contiguous chunk [x * per, (x + 1) * per) of
// tiles, so neighbouring tiles, which share Gaussians, hit the same L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t count) {
  const int64_t per = (count + 7) / 8;
  return (b % 8) * per + b / 8;
}

__host__ __device__ __forceinline__ int64_t xcd_grid(int64_t count) { return ((count + 7) / 8) * 8; }

static inline int grid_for(int64_t count, int block = kBlock) {
  int64_t g = (count + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 1048576) g = 1048576;
  return (int)g;
}

static inline int last_err() { return (int)hipGetLastError(); }

}  // namespace gsr
