// Sub-block culling of tile-list entries: the geometry the rasterization
// kernels use to decide, per batch, which entries each 16-pixel sub-block
// walks.  Kept apart from the kernels so that the host test suite can build
// these functions for the CPU and check them against brute force over pixel
// centres.  Includers provide float4, fmaf-style builtins and the device
// qualifiers (the HIP runtime header does).
#pragma once

namespace gsr {

struct LdsRec {
  float4 r0, r1, r2;  // mean (hi, lo), base-2 exponent coefficients + opacity, colour + base-2 pmin
  float reach;
};

// Which sub-blocks can an entry's alpha reach alpha_min in?  alpha >=
// alpha_min needs the base-2 exponent q(x, y) = a x^2 + b x y + c y^2 (x, y
// relative to the mean) to reach pmin2.  On a lowered level p_s the points of
// the ellipse {q >= p_s} at height y form the chord centred at sig y with
// half-width kap sqrt(ey^2 - y^2) (|y| <= ey), where, with
// det = 4 a c - b^2 > 0,
//   ey^2 = 4 a p_s / det,  sig = -b / (2a),  kap = sqrt(det) / (2 |a|),
// and the rightmost point of the ellipse lies at height yr = -b ex / (2c),
// ex^2 = 4 c p_s / det (the leftmost at -yr).  Over a band of heights
// [y0, y1] the chords reach furthest right at yr clamped into the band and
// furthest left at -yr clamped, so a box of pixel centres spanning the band
// meets the ellipse exactly when its x-range meets that interval [xl, xr]:
// one interval per band of sub-blocks, then two compares per sub-block,
// instead of an exact box test per sub-block.
//
// Conservative in float32:
//  * p_s = pmin2 (1.0001 + 1e-6 m) - 7.2e-5, m = (8 a c + 2 |b| (|a| + |c|))
//    / det >= 2, the ellipse's condition: a pixel's float32 exponent differs
//    from the exact q of the stored coefficients by at most ~4 ulp of its
//    terms' magnitudes, which on the ellipse stay below |p_s| m;
//  * det in double, where the float products are exact (thin ellipses);
//  * reciprocals and square roots by the hardware instructions (1 ulp),
//    far inside the pads below;
//  * the interval is padded by 1e-3 px, 1e-3 of the central half-chord
//    kap ey (the square root's error near a tangent) and 1e-5 of the shear
//    term;
//  * records with m > 1e6 (thinner than about 1000 : 1) or a rounded det
//    that is not positive are kept whenever the circle of radius `reach`
//    meets the strip.
// The box offsets are formed like the per-pixel offsets ((centre - hi) -
// lo).
struct ReachShape {
  float ey, ey2, sig, kap, yr;
  bool thin;
};

__device__ __forceinline__ ReachShape reach_shape(const LdsRec &R) {
  ReachShape S;
  const float a = R.r1.x, b = R.r1.y, c = R.r1.z;
  const double det = __fma_rn(-(double)b, (double)b, 4.0 * ((double)a * (double)c));
  const float detf = (float)det;
  const float inv_det = __builtin_amdgcn_rcpf(detf);
  const float m = __fmaf_rn(2.0f * fabsf(b), fabsf(a) + fabsf(c), 8.0f * (a * c)) * inv_det;
  S.thin = !(detf > 0.0f && m <= 1.0e6f);
  const float ps = __fmaf_rn(R.r2.w, __fmaf_rn(1.0e-6f, m, 1.0001f), -7.2135e-5f);
  const float ia = -0.5f * __builtin_amdgcn_rcpf(a);
  const float q4 = 4.0f * ps * inv_det;
  S.ey2 = q4 * a;
  S.ey = __builtin_amdgcn_sqrtf(S.ey2);
  S.sig = b * ia;
  S.kap = __builtin_amdgcn_sqrtf(detf) * ia;
  S.yr = (-0.5f * b * __builtin_amdgcn_rcpf(c)) * __builtin_amdgcn_sqrtf(q4 * c);
  return S;
}

// The entry's x-interval [xl, xr] (pad included) over the band of pixel-centre
// rows [by0, by1]; empty (xl > xr) when the ellipse misses the band.
__device__ __forceinline__ void band_interval(const LdsRec &R, const ReachShape &S, float by0, float by1, float &xl,
                                              float &xr) {
  const float y0 = (by0 - R.r0.y) - R.r0.w, y1 = (by1 - R.r0.y) - R.r0.w;
  const float ys = __builtin_amdgcn_fmed3f(S.yr, y0, y1), yl = __builtin_amdgcn_fmed3f(-S.yr, y0, y1);
  const float hr = S.kap * __builtin_amdgcn_sqrtf(fmaxf(0.0f, __fmaf_rn(-ys, ys, S.ey2)));
  const float hl = S.kap * __builtin_amdgcn_sqrtf(fmaxf(0.0f, __fmaf_rn(-yl, yl, S.ey2)));
  const float pad = __fmaf_rn(1.0e-5f * fabsf(S.sig), fmaxf(fabsf(y0), fabsf(y1)),
                              __fmaf_rn(1.0e-3f * S.kap, S.ey, 1.0e-3f));
  const bool miss = y0 > S.ey || y1 < -S.ey;
  xr = miss ? -3.0e38f : __fmaf_rn(S.sig, ys, hr) + pad;
  xl = miss ? 3.0e38f : __fmaf_rn(S.sig, yl, -hl) - pad;
}

// Can the entry reach the box of the strip's pixel centres at all: the
// circle of radius `reach` (negative: the entry reaches alpha_min nowhere).
__device__ __forceinline__ bool reaches_strip(const LdsRec &R, float bx0, float bx1, float by0, float by1) {
  const float reach = R.reach;
  const float mx = R.r0.x + R.r0.z, my = R.r0.y + R.r0.w;
  const float ddx = fmaxf(0.0f, fmaxf(bx0 - mx, mx - bx1));
  const float ddy = fmaxf(0.0f, fmaxf(by0 - my, my - by1));
  return reach >= 0.0f && __fmaf_rn(ddx, ddx, ddy * ddy) <= reach * reach;
}

}  // namespace gsr
