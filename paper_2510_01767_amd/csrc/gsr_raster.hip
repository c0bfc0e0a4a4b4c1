// Tile rasterization kernels (gfx950): front-to-back compositing (the
// blending sum of Sec. 3.2), the L1 image gradient and the back-to-front
// reverse pass, as plain per-tile kernels and as one persistent fused kernel.
//
// Work decomposition.  One workgroup (4 wavefronts, 256 lanes) owns one tile
// of 256 pixels, one lane per pixel.  The tile's ordered entry list is
// streamed through LDS in batches of B records.  Each wavefront owns a
// 64-pixel strip of the tile and each 16-lane row of it a 16-pixel
// sub-block; the batch is culled against the strip, then against each
// sub-block: an entry is kept for a sub-block only if the ellipse on which
// its alpha reaches alpha_min (its "reach", precomputed per record) can
// touch a pixel centre of the sub-block.  Each row then walks its own kept
// list in depth order.  Culled entries have alpha < alpha_min at every pixel
// they skip, so the result is identical to evaluating them; on city-scale
// scenes most entries of a tile list miss most sub-blocks, which is where
// the time would otherwise go.
//
// Reverse pass.  Each row reduces the nine per-pixel terms of its entry
// (the moments of dL/dp over the pixel offset, which the reverse projection
// maps through the record's conic, then dL/dopacity and dL/dcolour) by a
// reduce-scatter over its 16 lanes; lanes 0..8 then either add the sums to
// the record's gradient slot with device atomics, or (the other variants the
// autotuner weighs) into a per-batch LDS accumulator flushed with one device
// atomic per (entry, component).
#include <hip/hip_runtime.h>

#include "gsr_cull.h"
#include "gsr_device.h"

namespace gsr {

struct TileCtx {
  int64_t t;  // global tile id
  int v;      // view
  ViewInfo vi;
  int px, py;  // this lane's pixel
  bool inside;
  int64_t start, end;  // entry range [start, end) in keys
  int64_t pix;         // pixel index within the view
  float wx0, wx1, wy0, wy1;  // pixel-centre box of this lane's wavefront
  int sw, sh, snx;           // sub-block width and height, sub-blocks per strip row
};

template <int TW, int TH>
__device__ __forceinline__ void tile_ctx(const KWs &ws, const ViewInfo *views, int n_views, int64_t t,
                                         TileCtx &c) {
  static_assert(TW * TH == kBlock && 64 % TW == 0, "tile must be 256 pixels, whole rows per wavefront");
  constexpr int kRows = 64 / TW;
  c.t = t;
  c.v = view_of_tile(views, n_views, t);
  c.vi = views[c.v];
  const int64_t local = t - c.vi.tile_base;
  const int tx0 = (int)(local % c.vi.tiles_x) * TW, ty0 = (int)(local / c.vi.tiles_x) * TH;
  // Each wavefront owns a strip of 64 pixels (TW x kRows) and each 16-lane
  // row of it a sub-block of 16 pixels: 4 x 4 for 8- and 16-wide tiles, 8 x 2
  // for 32-wide ones (SNX sub-blocks side by side).
  constexpr int SW = TW == 32 ? 8 : 4, SH = 16 / SW, SNX = TW / SW;
  static_assert((kRows / SH) * SNX == 4, "four sub-blocks per strip");
  const int wave = threadIdx.x >> 6, lane = (int)threadIdx.x & 63, row = lane >> 4, sl = lane & 15;
  c.px = tx0 + (row % SNX) * SW + sl % SW;
  c.py = ty0 + wave * kRows + (row / SNX) * SH + sl / SW;
  c.sw = SW;
  c.sh = SH;
  c.snx = SNX;
  c.inside = c.px < c.vi.W && c.py < c.vi.H;
  c.pix = (int64_t)c.py * c.vi.W + c.px;
  c.start = ws.tile_start[t];
  c.end = min((int64_t)ws.tile_start[t + 1], ws.capacity);
  if (c.end < c.start) c.end = c.start;
  c.wx0 = (float)tx0 + 0.5f;
  c.wx1 = (float)(tx0 + TW) - 0.5f;
  c.wy0 = (float)(ty0 + wave * kRows) + 0.5f;
  c.wy1 = c.wy0 + (float)(kRows - 1);
}

// A batch of records in LDS as separate arrays: the four 16-lane rows of a
// wavefront read four different entries at once, which in a 64-byte record
// array would start on the same banks.
template <int B>
struct LdsBatch {
  float4 r0[B], r1[B], r2[B];
  float reach[B];
};

template <int B>
__device__ __forceinline__ LdsRec rec_at(const LdsBatch<B> &s, int j) {
  LdsRec R;
  R.r0 = s.r0[j];
  R.r1 = s.r1[j];
  R.r2 = s.r2[j];
  R.reach = s.reach[j];
  return R;
}

template <int B>
__device__ __forceinline__ void load_batch(const KWs &ws, int64_t lo, int nb, LdsBatch<B> &s_rec, uint32_t *s_idx,
                                           float *s_depth = nullptr) {
  if ((int)threadIdx.x < nb) {
    const uint32_t r = (uint32_t)ws.keys[lo + threadIdx.x];
    const float4 *rec = rec_ptr(ws, r);
    s_rec.r0[threadIdx.x] = rec[0];
    s_rec.r1[threadIdx.x] = rec[1];
    s_rec.r2[threadIdx.x] = rec[2];
    const uint4 r3 = reinterpret_cast<const uint4 *>(rec)[3];
    s_rec.reach[threadIdx.x] = __uint_as_float(r3.w);
    if (s_idx) s_idx[threadIdx.x] = r;
    if (s_depth) s_depth[threadIdx.x] = __uint_as_float(r3.z);
  }
}

// The kept entries of the batch for each of the wavefront's four
// sub-blocks, in list order: an entry is tested against the strip's circle,
// then each band of sub-blocks gets its interval and each sub-block two
// compares.  lists[q] of sub-block q gets cnt[q] entries; returns the count
// of this lane's own sub-block.
template <int B>
__device__ __forceinline__ int sub_lists(const LdsBatch<B> &s_rec, int nb, const TileCtx &c, uint8_t (*lists)[B],
                                         int cnt[4]) {
  static_assert(B <= 256, "byte indices");
  const int lane = lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0;
  for (int jb = 0; jb < nb; jb += 64) {
    const int j = jb + lane;
    const LdsRec R = rec_at(s_rec, j < nb ? j : 0);
    const bool strip = j < nb && reaches_strip(R, c.wx0, c.wx1, c.wy0, c.wy1);
    const ReachShape S = reach_shape(R);
    float xl = 3.0e38f, xr = -3.0e38f;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const float bx0 = c.wx0 + (float)((q % c.snx) * c.sw), by0 = c.wy0 + (float)((q / c.snx) * c.sh);
      if (q % c.snx == 0) band_interval(R, S, by0, by0 + (float)(c.sh - 1), xl, xr);
      const float x0 = (bx0 - R.r0.x) - R.r0.z, x1 = ((bx0 + (float)(c.sw - 1)) - R.r0.x) - R.r0.z;
      const bool keep = strip && (S.thin || (x1 >= xl && x0 <= xr));
      const uint64_t m = __ballot(keep);
      if (keep) lists[q][cnt[q] + __popcll(m & below)] = (uint8_t)j;
      cnt[q] += __popcll(m);
    }
  }
  return cnt[lane >> 4];
}

// The batch that a tile pass left in LDS: entries [lo, lo + nb) of the list
// in s_rec (and s_idx), and this wavefront's culled list of it (cnt entries
// in s_list).  nb == 0: nothing usable.
struct Resident {
  int64_t lo;
  int nb, cnt;  // cnt: this lane's sub-block list length
};

// Front-to-back compositing of one tile.  Returns the colour, the final
// transmittance and `last` (list entries processed before the stop, or the
// list length).  With HIST it stores, for every evaluated entry, the
// transmittance in front of it (0 when the entry was skipped).  Batches
// start at c.start + k B; the last one loaded stays resident (`res`).  The
// pair update is branch-free: a skipped pair adds 0 * colour and keeps T.
// With DEPTH it also composites the records' depths, D = sum d alpha T
// (the depth form of the blending sum, Sec. 3.2), from s_depth.  With COUNT
// (profiling) it counts the pairs this lane evaluates after the culling and
// the pairs it blends.
template <int B, bool HIST, bool DEPTH = false, bool COUNT = false>
__device__ __forceinline__ void tile_forward(const KWs &ws, const KOpts &o, const TileCtx &c, LdsBatch<B> &s_rec,
                                             uint32_t *s_idx, uint8_t (*s_list)[4][B], float C[3], float &T,
                                             int &last, float *hist, Resident &res, float *s_depth = nullptr,
                                             float *D = nullptr, uint32_t *n_eval = nullptr,
                                             uint32_t *n_blend = nullptr) {
  const float pxc = (float)c.px + 0.5f, pyc = (float)c.py + 0.5f;
  const float amax = o.alpha_max;
  const int wave = threadIdx.x >> 6, row = ((int)threadIdx.x & 63) >> 4;
  T = 1.0f;
  C[0] = C[1] = C[2] = 0.0f;
  bool done = !c.inside;
  bool stopped = false;
  last = 0;
  res.nb = 0;
  for (int64_t b = c.start; b < c.end; b += B) {
    if (__syncthreads_and(done)) break;
    const int nb = (int)min((int64_t)B, c.end - b);
    load_batch(ws, b, nb, s_rec, s_idx, DEPTH ? s_depth : nullptr);
    __syncthreads();
    int cq[4];
    const int cnt = sub_lists<B>(s_rec, nb, c, s_list[wave], cq);
    const int kmax = max(max(cq[0], cq[1]), max(cq[2], cq[3]));  // the same in every lane
    __syncthreads();
    res.lo = b;
    res.nb = nb;
    res.cnt = cnt;
    const uint8_t *mine = s_list[wave][row];
    const bool stopped_before = stopped;
    // each 16-lane row walks its own sub-block's list; a row whose list is
    // shorter idles (valid = false) while the others finish
    for (int k = 0; k < kmax && !done; k++) {
      const bool valid = k < cnt;
      // past the row's count the list byte is stale and may name an entry the
      // batch did not load: clamped into the loaded entries (no branch), the
      // pair marked invalid
      const int j = min((int)mine[k], nb - 1);
      const LdsRec R = rec_at(s_rec, j);
      const PairAlpha a = pair_alpha<false>(pxc, pyc, R.r0, R.r1, amax);
      const bool hit = valid && a.in && a.alpha >= o.alpha_min;
      const float Tn = T * (1.0f - a.alpha);
      const bool stop = hit && Tn < o.T_min;
      const bool take = hit && !stop;
      const float w = take ? a.alpha * T : 0.0f;
      C[0] = __fmaf_rn(w, R.r2.x, C[0]);
      C[1] = __fmaf_rn(w, R.r2.y, C[1]);
      C[2] = __fmaf_rn(w, R.r2.z, C[2]);
      if (DEPTH) *D = __fmaf_rn(w, s_depth[j], *D);
      if (COUNT) {
        *n_eval += valid ? 1u : 0u;
        *n_blend += take ? 1u : 0u;
      }
      if (HIST && valid && !stop) hist[(b + j) * 256 + threadIdx.x] = take ? T : 0.0f;
      T = take ? Tn : T;
      last = stop ? j : last;  // the batch's offset is added below
      stopped = stopped || stop;
      done = stop;
    }
    if (stopped && !stopped_before) last += (int)(b - c.start);
  }
  if (!stopped) last = c.inside ? (int)(c.end - c.start) : 0;
}

// Reduce-scatter of the nine terms over each 16-lane row: four butterfly
// steps between lanes i and i ^ 7, i ^ 1, i ^ 2, i ^ 8 (row_half_mirror, two
// quad permutations, row_ror:8), each step leaving a lane half of the
// components it carried, summed with its partner's.  Lanes 0..8 of a row end
// with the row sums of components 0, 2, 1, 3, 5, 7, 6, 8, 4 (comp_of_lane);
// 27 operations where four full row sums and a select take 44.
__device__ __forceinline__ float row_reduce_scatter(const float v[9], bool lb0, bool lb1, bool lb2, bool lb3) {
  float r[5], t0, t1, u;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const float keep = lb2 ? v[k + 5] : v[k], send = lb2 ? v[k] : v[k + 5];
    r[k] = keep + dpp_or_zero<0x141>(send);  // row_half_mirror: lane i ^ 7
  }
  r[4] = v[4] + dpp_or_zero<0x141>(v[4]);
  float s3[3];
#pragma unroll
  for (int k = 0; k < 2; k++) {
    const float keep = lb0 ? r[k + 2] : r[k], send = lb0 ? r[k] : r[k + 2];
    s3[k] = keep + dpp_or_zero<0xB1>(send);  // quad_perm [1,0,3,2]: lane i ^ 1
  }
  s3[2] = r[4] + dpp_or_zero<0xB1>(r[4]);
  {
    const float keep = lb1 ? s3[1] : s3[0], send = lb1 ? s3[0] : s3[1];
    t0 = keep + dpp_or_zero<0x4E>(send);  // quad_perm [2,3,0,1]: lane i ^ 2
    t1 = s3[2] + dpp_or_zero<0x4E>(s3[2]);
  }
  {
    const float keep = lb3 ? t1 : t0, send = lb3 ? t0 : t1;
    u = keep + dpp_or_zero<0x128>(send);  // row_ror:8: lane i ^ 8
  }
  return u;
}

// Back-to-front reverse pass of one tile.  g = dL/dC_out of this lane's
// pixel, T its final transmittance (recovered entry by entry unless the
// forward stored it).  Each contributing pair gives nine terms, summed per
// entry into its slot: the five moments of dL/dp over the pixel offset, then
// dL/dopacity and dL/dcolour.
//   RED = 0: per row entry, the reduce-scatter of the nine terms over the
//            row and one device atomic per component from lanes 0..8.
//   RED = 1: contributing lanes add their terms into an LDS accumulator
//            of the batch (ds_add_f32, combining the four wavefronts); one
//            device atomic per non-zero (entry, component) after the batch.
//   RED = 2, 3, 4: as 1 after DPP sums over lane quads (2), over 16-lane
//            rows (3), or a reduce-scatter over 16-lane rows (4).
// Batches are aligned like the forward's (c.start + k B), so when the
// forward's last batch `res` is the first one needed here it is used as it
// sits in LDS, culled lists included.
template <int B, int RED, bool HIST>
__device__ __forceinline__ void tile_backward(const KWs &ws, const KOpts &o, const TileCtx &c, LdsBatch<B> &s_rec,
                                              uint32_t *s_idx, uint8_t (*s_list)[4][B], float (*s_acc)[9],
                                              int *s_max, float T, int last, const float g[3],
                                              const float *hist, Resident res) {
  const float pxc = (float)c.px + 0.5f, pyc = (float)c.py + 0.5f;
  const float amax = o.alpha_max;  // as in the forward pass
  const int wave = threadIdx.x >> 6, lane = lane_id();
  // the reduce-scatter's lane roles (RED = 4): which component lane q of a
  // 16-lane row ends with, -1 for none
  const bool lb0 = lane & 1, lb1 = lane & 2, lb2 = lane & 4, lb3 = lane & 8;
  const int rq = lane & 15;
  const int comp_of_lane = rq < 8 ? (lb2 ? 5 : 0) + (lb1 ? (lb0 ? 3 : 1) : (lb0 ? 2 : 0)) : (rq == 8 ? 4 : -1);
  // gS = sum_ch g_ch S_ch with S the colour composited behind the current
  // entry (T_final bg to start); dL/dalpha_i = T_i (g . c_i) - gS / (1 - alpha_i)
  float gS = T * (g[0] * o.bg[0] + g[1] * o.bg[1] + g[2] * o.bg[2]);
  const bool active = c.inside && (g[0] != 0.0f || g[1] != 0.0f || g[2] != 0.0f);
  __syncthreads();
  if (threadIdx.x == 0) *s_max = 0;
  __syncthreads();
  if (active && last > 0) atomicMax(s_max, last);
  __syncthreads();
  const int top = *s_max;  // entries [0, top) of the list can contribute
  for (int64_t lo = c.start + (int64_t)((top - 1) / B) * B; top > 0 && lo >= c.start; lo -= B) {
    const int nb_top = (int)min((int64_t)B, c.start + top - lo);
    int nb, cnt;
    __syncthreads();
    if (res.nb > 0 && res.lo == lo) {
      // the forward's last batch, still in LDS with this wavefront's list
      nb = res.nb;
      cnt = res.cnt;
      res.nb = 0;
      if (RED >= 1)
        for (int e = threadIdx.x; e < nb * 9; e += blockDim.x) (&s_acc[0][0])[e] = 0.0f;
      __syncthreads();
    } else {
      nb = nb_top;
      load_batch(ws, lo, nb, s_rec, s_idx);
      if (RED >= 1)
        for (int e = threadIdx.x; e < nb * 9; e += blockDim.x) (&s_acc[0][0])[e] = 0.0f;
      __syncthreads();
      int cq[4];
      cnt = sub_lists<B>(s_rec, nb, c, s_list[wave], cq);
      __syncthreads();
    }
    // entries at or past `top` contribute to no pixel
    const uint8_t *mine = s_list[wave][(lane & 63) >> 4];
    while (cnt > 0 && (int)mine[cnt - 1] >= nb_top) cnt--;
    int kmax = max(cnt, __shfl_xor(cnt, 16));  // the longest of the wavefront's four row lists
    kmax = __builtin_amdgcn_readfirstlane(max(kmax, __shfl_xor(kmax, 32)));  // uniform: a scalar loop counter
    const int jj_last = active ? last - (int)(lo - c.start) : 0;  // this pixel's entries: jj < jj_last
    for (int k = kmax - 1; k >= 0; k--) {
      const bool valid = k < cnt;
      const int jj = min((int)mine[k], nb - 1);  // as in the forward pass
      const int64_t j = lo + jj;
      const LdsRec R = rec_at(s_rec, jj);
      const PairAlpha a = pair_alpha<true>(pxc, pyc, R.r0, R.r1, amax);
      const bool contrib = valid && a.in && jj < jj_last && a.alpha >= o.alpha_min;
      if (__ballot(contrib) == 0ull) continue;
      // Every lane evaluates the terms (all finite: alpha <= 0.99).  The
      // non-contributing lanes take alpha = 0 here: 1 / (1 - 0) is exactly 1,
      // so their T and suffix stay as they are and they add exact zeros.
      // 1 / (1 - alpha) by the hardware reciprocal (1 ulp): T and the
      // suffix only feed gradients, never a discrete decision.
      const float al = contrib ? a.alpha : 0.0f;
      const float inv_om = __builtin_amdgcn_rcpf(1.0f - al);
      const float Ti = HIST ? (contrib ? hist[j * 256 + threadIdx.x] : T) : T * inv_om;
      const float wgt = al * Ti;
      const float col[3] = {R.r2.x, R.r2.y, R.r2.z};
      float v[9];
      const float gc = __fmaf_rn(g[2], col[2], __fmaf_rn(g[1], col[1], g[0] * col[0]));
      const float dLda = __fmaf_rn(Ti, gc, -gS * inv_om);
      gS = __fmaf_rn(wgt, gc, gS);
#pragma unroll
      for (int ch = 0; ch < 3; ch++) v[6 + ch] = g[ch] * wgt;
      // the geometric terms vanish where alpha is clamped at alpha_max
      const float dLdam = (contrib && a.raw < o.alpha_max) ? dLda : 0.0f;
      const float gp = dLdam * a.alpha;  // dL/dp
      v[5] = dLdam * a.G;
      // the moments of dL/dp over the pixel offsets d = pixel - mean:
      // sum gp dx, gp dy, gp dx^2, gp dx dy, gp dy^2.  The geometric 2D
      // gradient is linear in them with the record's conic Q as coefficients
      // (dL/dmean = Q (m0, m1), dL/dQ = -(m2 / 2, m3, m4 / 2)), so the
      // reverse projection applies Q once per record instead of every pixel
      // applying it here.
      const float gpx = gp * a.dx, gpy = gp * a.dy;
      v[0] = gpx;
      v[1] = gpy;
      v[2] = gpx * a.dx;
      v[3] = gpx * a.dy;
      v[4] = gpy * a.dy;
      T = Ti;
      if (RED == 0) {
        // the row's reduce-scatter, then one device atomic per component from
        // lanes 0..8 of the row into its entry's gradient slot
        const float u = row_reduce_scatter(v, lb0, lb1, lb2, lb3);
        if (valid && comp_of_lane >= 0 && u != 0.0f)
          unsafeAtomicAdd(&ws.grad2d[(int64_t)s_idx[jj] * kGrad2dStride + comp_of_lane], u);
      } else if (RED == 1) {
        if (contrib) {
#pragma unroll
          for (int q = 0; q < 9; q++)
            if (v[q] != 0.0f) atomicAdd(&s_acc[jj][q], v[q]);
        }
      } else if (RED == 3) {
        // row sums (four DPP steps leave every lane of a 16-lane row with the
        // row's total), then lane 16 row + q adds component q: one LDS atomic
        // instruction per entry, four rows per address
        // (the nine chains interleaved step by step, so no DPP result is
        // read back-to-back)
#pragma unroll
        for (int q = 0; q < 9; q++) v[q] += dpp_or_zero<0xB1>(v[q]);   // quad_perm [1,0,3,2]
#pragma unroll
        for (int q = 0; q < 9; q++) v[q] += dpp_or_zero<0x4E>(v[q]);   // quad_perm [2,3,0,1]
#pragma unroll
        for (int q = 0; q < 9; q++) v[q] += dpp_or_zero<0x141>(v[q]);  // row_half_mirror
#pragma unroll
        for (int q = 0; q < 9; q++) v[q] += dpp_or_zero<0x140>(v[q]);  // row_mirror
        const int q = lane & 15;
        float mine = v[0];
#pragma unroll
        for (int k = 1; k < 9; k++) mine = q == k ? v[k] : mine;
        if (valid && q < 9 && mine != 0.0f) atomicAdd(&s_acc[jj][q], mine);
      } else if (RED == 4) {
        const float u = row_reduce_scatter(v, lb0, lb1, lb2, lb3);
        if (valid && comp_of_lane >= 0 && u != 0.0f) atomicAdd(&s_acc[jj][comp_of_lane], u);
      } else {
        // quad sums (two DPP steps), then one LDS atomic per quad and component
#pragma unroll
        for (int q = 0; q < 9; q++) v[q] += dpp_or_zero<0xB1>(v[q]);  // quad_perm [1,0,3,2]
#pragma unroll
        for (int q = 0; q < 9; q++) v[q] += dpp_or_zero<0x4E>(v[q]);  // quad_perm [2,3,0,1]
#pragma unroll
        for (int q = 0; q < 9; q++)
          if (valid && (lane & 3) == 0 && v[q] != 0.0f) atomicAdd(&s_acc[jj][q], v[q]);
      }
    }
    if (RED >= 1) {
      __syncthreads();
      for (int e = threadIdx.x; e < nb * 9; e += blockDim.x) {
        const int jj = e / 9, q = e - jj * 9;
        const float val = s_acc[jj][q];
        if (val != 0.0f) unsafeAtomicAdd(&ws.grad2d[(int64_t)s_idx[jj] * kGrad2dStride + q], val);
      }
    }
  }
}

__device__ __forceinline__ float block_sum_fixed(float x, float *s_w) {
  x = wave_sum_lane63(x);
  if (lane_id() == 63) s_w[threadIdx.x >> 6] = x;
  __syncthreads();
  const float r = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
  __syncthreads();
  return r;
}

// COUNT (profiling): pair_counts[p] = pairs blended into pixel p,
// pair_counts[pixels_total + p] = pairs its lane evaluated.
template <int TW, int TH, int B, bool HIST, bool DEPTH, bool COUNT>
__global__ __launch_bounds__(kBlock) void k_raster_fwd(KWs ws, KOpts o, int64_t tile_lo, int64_t tile_count,
                                                       float *images, int n_views, float *depth,
                                                       uint32_t *pair_counts) {
  __shared__ LdsBatch<B> s_rec;
  __shared__ float s_depth[DEPTH ? B : 1];
  __shared__ uint8_t s_list[4][4][B];  // [wavefront][sub-block][entry index in the batch]
  __shared__ ViewInfo s_views[GSR_MAX_VIEWS];
  for (int v = threadIdx.x; v < n_views; v += blockDim.x) s_views[v] = ws.views[v];
  __syncthreads();
  const int64_t b = xcd_remap(blockIdx.x, tile_count);
  if (b >= tile_count) return;
  TileCtx c;
  tile_ctx<TW, TH>(ws, s_views, n_views, tile_lo + b, c);
  float C[3], T;
  int last;
  Resident res;
  float D = 0.0f;
  uint32_t n_eval = 0u, n_blend = 0u;
  tile_forward<B, HIST, DEPTH, COUNT>(ws, o, c, s_rec, nullptr, s_list, C, T, last, ws.history, res, s_depth, &D,
                                      &n_eval, &n_blend);
  if (c.inside) {
    const int64_t P = (int64_t)c.vi.W * c.vi.H;
    float *img = images + c.vi.pix_base * 3;
#pragma unroll
    for (int ch = 0; ch < 3; ch++) img[ch * P + c.pix] = __fmaf_rn(T, o.bg[ch], C[ch]);
    ws.pix_T[c.vi.pix_base + c.pix] = T;
    ws.pix_last[c.vi.pix_base + c.pix] = (uint32_t)last;
    if (DEPTH) depth[c.vi.pix_base + c.pix] = D;
    if (COUNT) {
      pair_counts[c.vi.pix_base + c.pix] = n_blend;
      pair_counts[ws.pixels_total + c.vi.pix_base + c.pix] = n_eval;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_l1(KWs ws, KOpts o, int64_t tile_lo, int64_t tile_count,
                                               const float *images, const float *targets, int n_views, int tw,
                                               int th) {
  __shared__ float s_w[4];
  __shared__ ViewInfo s_views[GSR_MAX_VIEWS];
  for (int v = threadIdx.x; v < n_views; v += blockDim.x) s_views[v] = ws.views[v];
  __syncthreads();
  const int64_t t = tile_lo + blockIdx.x;
  const int v = view_of_tile(s_views, n_views, t);
  const ViewInfo vi = s_views[v];
  const int64_t local = t - vi.tile_base;
  const int px = (int)(local % vi.tiles_x) * tw + (int)(threadIdx.x % tw);
  const int py = (int)(local / vi.tiles_x) * th + (int)(threadIdx.x / tw);
  float acc = 0.0f;
  if (px < vi.W && py < vi.H) {
    const int64_t P = (int64_t)vi.W * vi.H;
    const int64_t base = vi.pix_base * 3 + (int64_t)py * vi.W + px;
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
      const float d = images[base + ch * P] - targets[base + ch * P];
      acc += fabsf(d);
      ws.pix_dLdC[base + ch * P] = d > 0.0f ? vi.loss_scale : (d < 0.0f ? -vi.loss_scale : 0.0f);
    }
  }
  const float s = block_sum_fixed(acc, s_w);
  if (threadIdx.x == 0) ws.tile_loss[t] = s;
}

template <int TW, int TH, int B, int RED, bool HIST>
__global__ __launch_bounds__(kBlock) void k_raster_bwd(KWs ws, KOpts o, int64_t tile_lo, int64_t tile_count,
                                                       const float *dLdC, int n_views) {
  __shared__ LdsBatch<B> s_rec;
  __shared__ uint32_t s_idx[B];
  __shared__ uint8_t s_list[4][4][B];  // [wavefront][sub-block][entry index in the batch]
  __shared__ float s_acc[RED >= 1 ? B : 1][9];
  __shared__ int s_max;
  __shared__ ViewInfo s_views[GSR_MAX_VIEWS];
  for (int v = threadIdx.x; v < n_views; v += blockDim.x) s_views[v] = ws.views[v];
  __syncthreads();
  const int64_t b = xcd_remap(blockIdx.x, tile_count);
  if (b >= tile_count) return;
  TileCtx c;
  tile_ctx<TW, TH>(ws, s_views, n_views, tile_lo + b, c);
  float g[3] = {0.f, 0.f, 0.f};
  float T = 1.0f;
  int last = 0;
  if (c.inside) {
    const int64_t P = (int64_t)c.vi.W * c.vi.H;
    const float *d = dLdC + c.vi.pix_base * 3 + c.pix;
    g[0] = d[0];
    g[1] = d[P];
    g[2] = d[2 * P];
    T = ws.pix_T[c.vi.pix_base + c.pix];
    last = (int)ws.pix_last[c.vi.pix_base + c.pix];
  }
  tile_backward<B, RED, HIST>(ws, o, c, s_rec, s_idx, s_list, s_acc, &s_max, T, last, g, ws.history,
                              Resident{0, 0, 0});
}

// Persistent fused forward + L1 + reverse pass.  Workgroups take tiles
// (in `order` when given) until their counter passes the last tile; no
// workgroup ever waits for another.  Workgroup class x = blockIdx mod 8 takes
// items x, x + 8, x + 16, ... from a counter of its own: the hardware hands
// consecutive workgroups to the 8 XCDs in turn, so each counter is shared by
// one XCD's workgroups instead of one counter by the whole chip.  The grid
// is a multiple of 8, so every class has workgroups and every tile is taken.
// The reduce-scatter form (RED 0) is held to 64 VGPRs, eight wavefronts per
// SIMD, which its LDS also allows (a few registers spill); the LDS
// accumulator forms are limited by their LDS anyway.
template <int TW, int TH, int B, int RED, bool HIST>
__global__ __launch_bounds__(kBlock, RED == 0 && !HIST ? 8 : 1) void k_fused(KWs ws, KOpts o, const float *targets, float *images,
                                                  int n_views, const uint32_t *order) {
  __shared__ LdsBatch<B> s_rec;
  __shared__ uint32_t s_idx[B];
  __shared__ uint8_t s_list[4][4][B];  // [wavefront][sub-block][entry index in the batch]
  __shared__ float s_acc[RED >= 1 ? B : 1][9];
  __shared__ int s_max;
  __shared__ float s_w[4];
  __shared__ int64_t s_item;
  __shared__ ViewInfo s_views[GSR_MAX_VIEWS];
  for (int v = threadIdx.x; v < n_views; v += blockDim.x) s_views[v] = ws.views[v];
  float *hist = ws.history;
  const int cls = (int)(blockIdx.x & 7u);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = cls + 8 * (int64_t)atomicAdd(&ws.hdr->queue[cls][0], 1u);
    __syncthreads();
    const int64_t item = s_item;
    if (item >= ws.tiles_total) break;
    const int64_t t = order ? (int64_t)order[item] : item;
    TileCtx c;
    tile_ctx<TW, TH>(ws, s_views, n_views, t, c);
    float C[3], T;
    int last;
    Resident res;
    tile_forward<B, HIST>(ws, o, c, s_rec, s_idx, s_list, C, T, last, hist, res);
    float g[3] = {0.f, 0.f, 0.f};
    float acc = 0.0f;
    if (c.inside) {
      const int64_t P = (int64_t)c.vi.W * c.vi.H;
      const int64_t base = c.vi.pix_base * 3 + c.pix;
#pragma unroll
      for (int ch = 0; ch < 3; ch++) {
        const float out = __fmaf_rn(T, o.bg[ch], C[ch]);
        images[base + ch * P] = out;
        const float d = out - targets[base + ch * P];
        acc += fabsf(d);
        g[ch] = d > 0.0f ? c.vi.loss_scale : (d < 0.0f ? -c.vi.loss_scale : 0.0f);
      }
      ws.pix_T[c.vi.pix_base + c.pix] = T;
      ws.pix_last[c.vi.pix_base + c.pix] = (uint32_t)last;
    }
    const float s = block_sum_fixed(acc, s_w);
    if (threadIdx.x == 0) ws.tile_loss[t] = s;
    tile_backward<B, RED, HIST>(ws, o, c, s_rec, s_idx, s_list, s_acc, &s_max, T, last, g, hist, res);
  }
}

// ------------------------------------------------------- longest list first
// The persistent kernel takes tiles in descending list length (bins of 4
// entries), so the longest tiles start first and the tail of the launch is
// made of short ones.  The order only schedules work: every tile's result is
// the same whichever workgroup computes it, whenever.

__device__ __forceinline__ int order_bin(const KWs &ws, int64_t t) {
  const uint32_t n = ws.tile_start[t + 1] - ws.tile_start[t];
  return kOrderBins - 1 - (int)min(n >> 2, (uint32_t)(kOrderBins - 1));
}

__global__ __launch_bounds__(kBlock) void k_order_hist(KWs ws) {
  __shared__ uint32_t s_h[kOrderBins];
  for (int k = threadIdx.x; k < kOrderBins; k += blockDim.x) s_h[k] = 0;
  __syncthreads();
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ws.tiles_total;
       t += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&s_h[order_bin(ws, t)], 1u);
  __syncthreads();
  for (int k = threadIdx.x; k < kOrderBins; k += blockDim.x)
    if (s_h[k]) atomicAdd(&ws.hdr->order_bins[k], s_h[k]);
}

__global__ __launch_bounds__(kOrderBins) void k_order_scan(KWs ws) {
  __shared__ uint32_t s[kOrderBins];
  const int k = threadIdx.x;
  const uint32_t x = ws.hdr->order_bins[k];
  s[k] = x;
  __syncthreads();
  for (int off = 1; off < kOrderBins; off <<= 1) {
    const uint32_t y = k >= off ? s[k - off] : 0u;
    __syncthreads();
    s[k] += y;
    __syncthreads();
  }
  ws.hdr->order_cursor[k] = s[k] - x;
}

// Each workgroup places its tiles with one device atomic per bin it holds
// (the ranks inside the workgroup from LDS atomics): the bins of the many
// short or empty tiles would otherwise take one atomic per tile on a single
// address.
__global__ __launch_bounds__(kBlock) void k_order_scatter(KWs ws) {
  __shared__ uint32_t s_cnt[kOrderBins], s_base[kOrderBins];
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < ws.tiles_total; t0 += (int64_t)gridDim.x * blockDim.x) {
    for (int k = threadIdx.x; k < kOrderBins; k += blockDim.x) s_cnt[k] = 0u;
    __syncthreads();
    const int64_t t = t0 + threadIdx.x;
    int bin = -1;
    uint32_t off = 0u;
    if (t < ws.tiles_total) {
      bin = order_bin(ws, t);
      off = atomicAdd(&s_cnt[bin], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kOrderBins; k += blockDim.x)
      if (s_cnt[k]) s_base[k] = atomicAdd(&ws.hdr->order_cursor[k], s_cnt[k]);
    __syncthreads();
    if (bin >= 0) ws.tile_order[s_base[bin] + off] = (uint32_t)t;
    __syncthreads();
  }
}

int launch_tile_order(const KWs &ws, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const int g = (int)min((int64_t)256, (ws.tiles_total + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_order_hist, dim3(g), dim3(kBlock), 0, s, ws);
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(kOrderBins), 0, s, ws);
  hipLaunchKernelGGL(k_order_scatter, dim3(grid_for(ws.tiles_total)), dim3(kBlock), 0, s, ws);
  return last_err();
}

// ---------------------------------------------------------------- launchers

#define GSR_TILE_DISPATCH(TW_, TH_, CALL)                                   \
  if (o.tile_w == TW_ && o.tile_h == TH_) {                                 \
    if (lds_batch == 64) {                                                  \
      constexpr int B = 64;                                                 \
      CALL(TW_, TH_, B);                                                    \
    } else if (lds_batch == 128) {                                          \
      constexpr int B = 128;                                                \
      CALL(TW_, TH_, B);                                                    \
    } else {                                                                \
      constexpr int B = 256;                                                \
      CALL(TW_, TH_, B);                                                    \
    }                                                                       \
    return last_err();                                                      \
  }

// reverse-pass kernels also select the reduction mode; the stored-history
// variant always takes the row reduce-scatter (4)
#define GSR_RED_CALL(KER, TW_, TH_, B_, ...)                                                           \
  do {                                                                                               \
    if (hist) hipLaunchKernelGGL((KER<TW_, TH_, B_, 4, true>), grid, block, 0, s, __VA_ARGS__);      \
    else if (red == 4) hipLaunchKernelGGL((KER<TW_, TH_, B_, 4, false>), grid, block, 0, s, __VA_ARGS__); \
    else if (red == 3) hipLaunchKernelGGL((KER<TW_, TH_, B_, 3, false>), grid, block, 0, s, __VA_ARGS__); \
    else if (red == 2) hipLaunchKernelGGL((KER<TW_, TH_, B_, 2, false>), grid, block, 0, s, __VA_ARGS__); \
    else if (red == 1) hipLaunchKernelGGL((KER<TW_, TH_, B_, 1, false>), grid, block, 0, s, __VA_ARGS__); \
    else hipLaunchKernelGGL((KER<TW_, TH_, B_, 0, false>), grid, block, 0, s, __VA_ARGS__);               \
  } while (0)

int launch_raster_fwd(const KWs &ws, const KOpts &o, int64_t tile_lo, int64_t tile_count, float *images,
                      int n_views, int store_history, int lds_batch, float *depth, uint32_t *pair_counts,
                      void *stream) {
  if (tile_count <= 0) return 0;
  const dim3 grid((unsigned)xcd_grid(tile_count)), block(kBlock);
  hipStream_t s = (hipStream_t)stream;
#define CALL_FWD(a, b_, B)                                                                                        \
  do {                                                                                                              \
    if (pair_counts)                                                                                                \
      hipLaunchKernelGGL((k_raster_fwd<a, b_, B, false, false, true>), grid, block, 0, s, ws, o, tile_lo,           \
                         tile_count, images, n_views, depth, pair_counts);                                          \
    else if (depth)                                                                                                 \
      hipLaunchKernelGGL((k_raster_fwd<a, b_, B, false, true, false>), grid, block, 0, s, ws, o, tile_lo,           \
                         tile_count, images, n_views, depth, pair_counts);                                          \
    else if (store_history)                                                                                         \
      hipLaunchKernelGGL((k_raster_fwd<a, b_, B, true, false, false>), grid, block, 0, s, ws, o, tile_lo,           \
                         tile_count, images, n_views, depth, pair_counts);                                          \
    else                                                                                                            \
      hipLaunchKernelGGL((k_raster_fwd<a, b_, B, false, false, false>), grid, block, 0, s, ws, o, tile_lo,          \
                         tile_count, images, n_views, depth, pair_counts);                                          \
  } while (0)
  GSR_TILE_DISPATCH(16, 16, CALL_FWD)
  GSR_TILE_DISPATCH(32, 8, CALL_FWD)
  GSR_TILE_DISPATCH(8, 32, CALL_FWD)
#undef CALL_FWD
  return (int)hipErrorInvalidValue;
}

int launch_l1(const KWs &ws, const KOpts &o, int64_t tile_lo, int64_t tile_count, const float *images,
              const float *targets, int n_views, void *stream) {
  if (tile_count <= 0) return 0;
  hipLaunchKernelGGL(k_l1, dim3((unsigned)tile_count), dim3(kBlock), 0, (hipStream_t)stream, ws, o, tile_lo,
                     tile_count, images, targets, n_views, o.tile_w, o.tile_h);
  return last_err();
}

int launch_raster_bwd(const KWs &ws, const KOpts &o, int64_t tile_lo, int64_t tile_count, const float *dLdC,
                      int n_views, int use_history, int lds_batch, int red, void *stream) {
  if (tile_count <= 0) return 0;
  const dim3 grid((unsigned)xcd_grid(tile_count)), block(kBlock);
  hipStream_t s = (hipStream_t)stream;
  const bool hist = use_history != 0;
#define CALL_BWD(a, b_, B) GSR_RED_CALL(k_raster_bwd, a, b_, B, ws, o, tile_lo, tile_count, dLdC, n_views)
  GSR_TILE_DISPATCH(16, 16, CALL_BWD)
  GSR_TILE_DISPATCH(32, 8, CALL_BWD)
  GSR_TILE_DISPATCH(8, 32, CALL_BWD)
#undef CALL_BWD
  return (int)hipErrorInvalidValue;
}

int launch_fused(const KWs &ws, const KOpts &o, const float *targets, float *images, int n_views, int use_history,
                 int lds_batch, int red, int grid_blocks, void *stream) {
  // a multiple of 8: every workgroup class of the per-XCD counters is present
  const dim3 grid((unsigned)xcd_grid(grid_blocks > 8 ? grid_blocks : 8)), block(kBlock);
  hipStream_t s = (hipStream_t)stream;
  const uint32_t *order = ws.tile_order;
  const bool hist = use_history != 0;
#define CALL_FUSED(a, b_, B) GSR_RED_CALL(k_fused, a, b_, B, ws, o, targets, images, n_views, order)
  GSR_TILE_DISPATCH(16, 16, CALL_FUSED)
  GSR_TILE_DISPATCH(32, 8, CALL_FUSED)
  GSR_TILE_DISPATCH(8, 32, CALL_FUSED)
#undef CALL_FUSED
  return (int)hipErrorInvalidValue;
}

}  // namespace gsr
