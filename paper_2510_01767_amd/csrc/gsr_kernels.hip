// HIP kernels of the differentiable Gaussian rasterizer for gfx950 (MI355X).
//
// Step structure (one training step of a block, Sec. 3 / App. A.1):
//   setup        view table + counters into the workspace (graph-safe: no memset nodes)
//   project      per Gaussian, all requested views: cull, EWA projection, SH colour,
//                64-byte record, per-tile intersection counts (device atomics)
//   scan         exclusive scan of the per-tile counts -> tile ranges, overflow flag
//   emit         per visible record, one 64-bit key (fp32 depth bits << 32 | record)
//                per covered tile, scattered into its tile's bucket
//   sort         per tile, order the bucket by key in LDS (bitonic; merge passes for
//                buckets larger than one LDS load)
//   raster, l1, raster_bwd, fused   (gsr_raster.hip)
//   project_bwd  per Gaussian, all views: chain rule to the raw parameters and the
//                densification statistics (Sec. 3.3)
//
// No kernel waits on another workgroup; persistent kernels take work from an
// atomic counter and exit when it runs past the last tile.
#include <hip/hip_runtime.h>

#include "gsr_device.h"

namespace gsr {


// ------------------------------------------------------------------ set-up

__global__ void k_setup(ViewTable table, KWs ws, int64_t zlo, int64_t zcount, int zero_bits, int64_t n) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (gid < table.n_views) ws.views[gid] = table.v[gid];
  if (gid == 0) {
    WsHeader *h = ws.hdr;
    h->overflow = 0;
    h->nonfinite = 0;
    h->union_count = 0;
    h->isect_total = 0;
  }
  if (gid < 8) ws.hdr->queue[gid][0] = 0;
  if (gid < GSR_MAX_VIEWS) {
    ws.hdr->isect[gid] = 0;
    ws.hdr->visible[gid] = 0;
  }
  for (int64_t k = gid; k < kOrderBins; k += stride) ws.hdr->order_bins[k] = 0;
  for (int64_t k = gid; k < zcount; k += stride) {
    ws.tile_count[zlo + k] = 0;
    ws.tile_fill[zlo + k] = 0;
  }
  if (zero_bits)
    for (int64_t k = gid; k < n; k += stride) ws.view_bits[k] = 0;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t count) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

__global__ void k_fill_f32(float *p, float v, int64_t count) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
    p[k] = v;
}

// ------------------------------------------------------------------ project

__device__ __forceinline__ bool finite_params(const KParams &p, int64_t i) {
  const int64_t n = p.n;
  float acc = 0.0f;
  for (int a = 0; a < 3; a++) acc += p.means[a * n + i] * 0.0f + p.log_scales[a * n + i] * 0.0f;
  for (int a = 0; a < 4; a++) acc += p.quats[a * n + i] * 0.0f;
  acc += p.logits[i] * 0.0f;
  return acc == 0.0f;  // any Inf or NaN makes the product NaN
}

// With TABLE, a workgroup's table of the tiles its records touch, in LDS:
// open addressing on the tile id, linear probing.  cnt counts the ranked
// entries (the LDS atomic's return value is the rank within the workgroup),
// fill the overflow ones; base receives the workgroup's start in the tile's
// bucket.
constexpr int kTileTable = 1024, kTileProbes = 16;
constexpr uint32_t kNoTile = 0xffffffffu;

template <int N>
struct TileTable {
  uint32_t key[N], cnt[N], fill[N], base[N];
};

// The table slot of tile t, inserting it if absent; -1 when the probe
// sequence is full.
__device__ __forceinline__ int tile_table_slot(TileTable<kTileTable> &tt, uint32_t t) {
  const uint32_t h = (t * 2654435761u) >> 22;  // 10 bits
  for (int k = 0; k < kTileProbes; k++) {
    const int e = (int)((h + (uint32_t)k) & (uint32_t)(kTileTable - 1));
    const uint32_t cur = *reinterpret_cast<volatile uint32_t *>(&tt.key[e]);
    if (cur == t) return e;
    if (cur == kNoTile) {
      const uint32_t prev = atomicCAS(&tt.key[e], kNoTile, t);
      if (prev == kNoTile || prev == t) return e;
    }
  }
  return -1;
}

template <int D, bool TABLE>
__global__ __launch_bounds__(kBlock) void k_project(KParams p, const gsr_camera *cams, KOpts o, KWs ws,
                                                    int view_lo, int view_hi, int or_bits) {
  constexpr int K = (D + 1) * (D + 1);
  __shared__ Cam64 s_cam[GSR_MAX_VIEWS];
  __shared__ ViewInfo s_view[GSR_MAX_VIEWS];
  __shared__ TileTable<TABLE ? kTileTable : 1> s_tt;
  for (int v = threadIdx.x; v < p.n_views; v += blockDim.x) s_view[v] = ws.views[v];
  if (TABLE)
    for (int e = threadIdx.x; e < kTileTable; e += blockDim.x) {
      s_tt.key[e] = kNoTile;
      s_tt.cnt[e] = 0u;
      s_tt.fill[e] = 0u;
    }
  load_cams(s_cam, cams, ws.views, p.n_views, o);
  const int64_t n = p.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  bool keep = valid && (p.keep == nullptr || p.keep[i] != 0);
  if (keep && o.check_finite && !finite_params(p, i)) {
    atomicOr(&ws.hdr->nonfinite, 1u);
    keep = false;
  }
  GeoF g;
  if (keep) load_geo_fwd(p, i, g);
  // reach of the alpha >= alpha_min ellipse {d : d^T Q d <= 2 ln(o / alpha_min)}
  // is sqrt(2 ln(o / alpha_min) lambda_max); the exponent gets 1e-5 of slack
  // (the float32 exponent and opacity are accurate to ~1e-6).  Below pmin the
  // float32 exponent cannot give alpha >= alpha_min (same slack).
  const double c2 = keep ? 2.0 * log(g.opac / (double)o.alpha_min) + 1e-5 : 0.0;
  const float pmin = c2 > 0.0 ? (float)(-0.5 * c2 * kLog2e) : 0.0f;  // in base 2, like the record's exponent
  uint32_t bits = (valid && or_bits) ? ws.view_bits[i] : 0u;
  uint32_t fresh = 0u;  // views found visible by this call
  const int lane = lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  for (int v = view_lo; v < view_hi; v++) {
    const ViewInfo &vi = s_view[v];
    const Cam64 &cam = s_cam[v];
    Proj P;
    // the exact projection only where the conservative bound leaves a chance
    const bool vis = keep && maybe_visible(g, cam, o) && project_view(g, cam, o, P);
    // (the whole wavefront, with TABLE the whole workgroup, stays in the loop)
    if (TABLE ? !__syncthreads_or(vis) : __ballot(vis) == 0ull) continue;
    const int64_t r = (int64_t)v * n + i;
    uint4 r3 = make_uint4(0u, 0u, 0u, 0u);
    int wx = 1, ntiles = 0;
    if (vis) {
      fresh |= 1u << v;
      float4 *rec = reinterpret_cast<float4 *>(ws.records) + r * kRecordFloat4;
      const float mxh = (float)P.mx, myh = (float)P.my;
      rec[0] = make_float4(mxh, myh, (float)(P.mx - (double)mxh), (float)(P.my - (double)myh));
      rec[1] = make_float4((float)(-0.5 * kLog2e * P.A), (float)(-kLog2e * P.B), (float)(-0.5 * kLog2e * P.C),
                           (float)g.opac);
      // the reach gets a relative and an absolute pad, so no pixel that the
      // float32 alpha test accepts lies outside it; -1 when even the centre
      // cannot reach alpha_min
      const float reach = c2 > 0.0 ? (float)(sqrt(c2 * P.lam) * 1.001 + 0.01) : -1.0f;
      r3 = make_uint4((uint32_t)P.x0 | ((uint32_t)P.y0 << 16), (uint32_t)P.x1 | ((uint32_t)P.y1 << 16),
                      __float_as_uint((float)P.tc[2]), __float_as_uint(reach));
      reinterpret_cast<uint4 *>(rec)[3] = r3;
      wx = P.x1 - P.x0 + 1;
      ntiles = wx * (P.y1 - P.y0 + 1);
    }
    // Count the record into each tile it touches.  For the first four tiles
    // (row-major) the record's rank in the tile's bucket comes out of the
    // count, kept so that the scatter needs no atomics; further tiles (large
    // footprints) are counted apart and placed after the ranked ones.
    const int x0 = P.x0, y0 = P.y0;
    auto tile_q = [&](int q) -> int32_t {
      const int dy = q / wx, dx = q - dy * wx;
      return (int32_t)(vi.tile_base + (int64_t)(y0 + dy) * vi.tiles_x + (x0 + dx));
    };
    uint32_t rk[4];
    if constexpr (TABLE) {
      // The workgroup counts into its table first (the rank within the
      // workgroup from the LDS atomic), then takes one device atomic per
      // distinct tile for all of it; a tile the table cannot hold takes
      // device atomics directly.  For wide footprints (many tiles per record,
      // many records per tile) the device atomics' throughput is what limits
      // this kernel, and the table divides their number.
      int slot[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        slot[q] = -1;
        rk[q] = 0u;
        if (q < ntiles) {
          const int32_t t = tile_q(q);
          slot[q] = tile_table_slot(s_tt, (uint32_t)t);
          if (slot[q] >= 0) rk[q] = atomicAdd(&s_tt.cnt[slot[q]], 1u);
          else rk[q] = atomicAdd(&ws.tile_count[t], 1u);
        }
      }
      for (int q = 4; q < ntiles; q++) {
        const int32_t t = tile_q(q);
        const int e = tile_table_slot(s_tt, (uint32_t)t);
        if (e >= 0) atomicAdd(&s_tt.fill[e], 1u);
        else atomicAdd(&ws.tile_fill[t], 1u);
      }
      __syncthreads();
      for (int e = threadIdx.x; e < kTileTable; e += blockDim.x) {
        const uint32_t t = s_tt.key[e];
        if (t != kNoTile) {
          const uint32_t c = s_tt.cnt[e], f = s_tt.fill[e];
          s_tt.base[e] = c ? atomicAdd(&ws.tile_count[t], c) : 0u;
          if (f) atomicAdd(&ws.tile_fill[t], f);
          s_tt.key[e] = kNoTile;
          s_tt.cnt[e] = 0u;
          s_tt.fill[e] = 0u;
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (slot[q] >= 0) rk[q] += s_tt.base[slot[q]];
    } else {
      // When the wavefront's records sit close together on the tile grid
      // (Gaussians stored in spatial order), lanes that share a tile take one
      // atomic for all of them, ranked by lane within it; otherwise, and for
      // what a few rounds leave, one atomic per (record, tile).
      const int32_t t0 = vis ? tile_q(0) : 0;
      int32_t tmin = vis ? t0 : INT32_MAX, tmax = vis ? t0 : -1;
  #pragma unroll
      for (int m = 1; m < 64; m <<= 1) {
        tmin = min(tmin, __shfl_xor(tmin, m));
        tmax = max(tmax, __shfl_xor(tmax, m));
      }
      const bool gather = tmax - tmin <= 2 * vi.tiles_x + 2;
      // Group the lanes that share a tile (per rank slot q) with ballots only:
      // which group no atomic result decides, so the groups are formed first,
      // each group's lowest lane then takes one atomic for the group, and all
      // of a lane's atomics are in flight together.  Lanes left after the
      // rounds, or all lanes when the wavefront is spread out, form groups of
      // one.
      int32_t tq[4];
      bool pending[4];
      int ldr[4];
      uint32_t off[4], cnt[4];
  #pragma unroll
      for (int q = 0; q < 4; q++) {
        tq[q] = q < ntiles ? tile_q(q) : -1;
        pending[q] = tq[q] >= 0;
        ldr[q] = lane;
        off[q] = 0u;
        cnt[q] = 0u;
      }
      for (int round = 0; gather && round < 8; round++) {
        bool any = false;
  #pragma unroll
        for (int q = 0; q < 4; q++) {
          const uint64_t act = __ballot(pending[q]);
          if (act == 0ull) continue;
          any = true;
          const int L = __ffsll((unsigned long long)act) - 1;
          const int32_t lt = __shfl(tq[q], L);
          const bool same = pending[q] && tq[q] == lt;
          const uint64_t m = __ballot(same);
          if (same) {
            ldr[q] = L;
            off[q] = (uint32_t)__popcll(m & below);
            pending[q] = false;
          }
          if (lane == L) cnt[q] = (uint32_t)__popcll(m);
        }
        if (!any) break;
      }
      uint32_t base[4];
  #pragma unroll
      for (int q = 0; q < 4; q++) {
        if (pending[q]) cnt[q] = 1u;  // a group of one (ldr = lane, off = 0)
        base[q] = cnt[q] ? atomicAdd(&ws.tile_count[tq[q]], cnt[q]) : 0u;
      }
  #pragma unroll
      for (int q = 0; q < 4; q++) rk[q] = __shfl(base[q], ldr[q]) + off[q];
      for (int q = 4; q < ntiles; q++) atomicAdd(&ws.tile_fill[tile_q(q)], 1u);
    }
    if (vis) {
      // the record's slot in one 64-byte write: cleared gradient, ranks, rectangle, depth
      uint4 *sl = reinterpret_cast<uint4 *>(ws.grad2d + r * kGrad2dStride);
      sl[0] = make_uint4(0u, 0u, 0u, 0u);
      sl[1] = make_uint4(0u, 0u, 0u, 0u);
      sl[2] = make_uint4(0u, rk[0], rk[1], rk[2]);
      sl[3] = make_uint4(rk[3], r3.x, r3.y, r3.z);
    }
  }
  if (valid) ws.view_bits[i] = bits | fresh;
  if (fresh == 0u) return;
  // Colour of every visible view: SH (float32) in the direction from the
  // camera centre c = -R^T t to the mean.  The coefficients are read once.
  float sh[3 * K];
#pragma unroll
  for (int k = 0; k < 3 * K; k++) sh[k] = p.sh[(int64_t)k * n + i];
  for (uint32_t b = fresh; b; b &= b - 1) {
    const int v = __ffs(b) - 1;
    const Cam64 &cam = s_cam[v];
    double d[3];
#pragma unroll
    for (int a = 0; a < 3; a++) d[a] = g.mu[a] + cam.cc[a];
    const double idn = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    float Y[K];
    sh_eval<D, float>((float)(d[0] * idn), (float)(d[1] * idn), (float)(d[2] * idn), Y);
    float col[3];
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
      float acc = 0.5f;
#pragma unroll
      for (int k = 0; k < K; k++) acc = __fmaf_rn(sh[k * 3 + ch], Y[k], acc);
      col[ch] = acc > 0.0f ? acc : 0.0f;
    }
    const int64_t r = (int64_t)v * n + i;
    reinterpret_cast<float4 *>(ws.records)[r * kRecordFloat4 + 2] = make_float4(col[0], col[1], col[2], pmin);
  }
}

// Per-view visible counts and the union, from view_bits (run on demand by the
// count query, never inside a step: per-view counters are single addresses
// that every workgroup would hit).  LDS counters per block, then one device
// atomic per block and view.
__global__ __launch_bounds__(kBlock) void k_count_visible(KWs ws, int64_t n, int n_views) {
  __shared__ uint32_t s_cnt[GSR_MAX_VIEWS + 1];
  if (threadIdx.x <= GSR_MAX_VIEWS) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t bits = i < n ? ws.view_bits[i] : 0u;
  for (int v = 0; v < n_views; v++) {
    const uint64_t m = __ballot((bits >> v) & 1u);
    if (lane_id() == 0 && m) atomicAdd(&s_cnt[v], (uint32_t)__popcll(m));
  }
  const uint64_t u = __ballot(bits != 0u);
  if (lane_id() == 0 && u) atomicAdd(&s_cnt[GSR_MAX_VIEWS], (uint32_t)__popcll(u));
  __syncthreads();
  if ((int)threadIdx.x < n_views && s_cnt[threadIdx.x]) atomicAdd(&ws.hdr->visible[threadIdx.x], s_cnt[threadIdx.x]);
  if (threadIdx.x == GSR_MAX_VIEWS && s_cnt[GSR_MAX_VIEWS]) atomicAdd(&ws.hdr->union_count, s_cnt[GSR_MAX_VIEWS]);
}

__global__ void k_zero_visible(KWs ws) {
  if (threadIdx.x < GSR_MAX_VIEWS) ws.hdr->visible[threadIdx.x] = 0;
  if (threadIdx.x == 0) ws.hdr->union_count = 0;
}

int launch_count_visible(const KWs &ws, int64_t n, int n_views, void *stream) {
  hipLaunchKernelGGL(k_zero_visible, dim3(1), dim3(64), 0, (hipStream_t)stream, ws);
  hipLaunchKernelGGL(k_count_visible, dim3(grid_for(n)), dim3(kBlock), 0, (hipStream_t)stream, ws, n, n_views);
  return last_err();
}

// --------------------------------------------------------------------- scan
// One workgroup of 1024 threads scans tile_count[lo, hi) into tile_start
// (absolute slots, starting at `base`), writes tile_start[hi], the per-view
// intersection counts and the overflow flag.

constexpr int kScanThreads = 1024;

// Inclusive sum over the 64 lanes of a wavefront (Hillis-Steele with shuffles).
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_up(x, (unsigned)off);
    if (lane >= off) x += y;
  }
  return x;
}

// Three passes over chunks of kScanChunk consecutive tiles (counts plus
// overflow counts): the sum of every chunk, then one workgroup scans the chunk
// sums and finds where each view starts, then every chunk scans itself from
// its prefix.  The chunk sums live in the tile-order array, which is written
// only after the sort.  No workgroup waits on another.
constexpr int kScanChunk = 4 * kScanThreads;

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) x += __shfl_xor(x, m);
  return x;
}

// Sum over the workgroup (kScanThreads threads); every thread gets it.
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t x, uint64_t *s_w) {
  constexpr int kWaves = kScanThreads / 64;
  x = wave_sum_u64(x);
  __syncthreads();
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = x;
  __syncthreads();
  uint64_t t = 0;
#pragma unroll
  for (int w = 0; w < kWaves; w++) t += s_w[w];
  return t;
}

__device__ __forceinline__ uint32_t tile_total(const KWs &ws, int64_t t, int64_t hi) {
  return t < hi ? ws.tile_count[t] + ws.tile_fill[t] : 0u;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(KWs ws, int64_t lo, int64_t hi) {
  __shared__ uint64_t s_w[kScanThreads / 64];
  const int64_t t0 = lo + (int64_t)blockIdx.x * kScanChunk + 4 * (int64_t)threadIdx.x;
  uint64_t x = 0;
#pragma unroll
  for (int q = 0; q < 4; q++) x += tile_total(ws, t0 + q, hi);
  const uint64_t sum = block_sum_u64(x, s_w);
  if (threadIdx.x == 0) reinterpret_cast<uint64_t *>(ws.tile_order)[blockIdx.x] = sum;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(KWs ws, int64_t lo, int64_t hi, int64_t base,
                                                               int view_lo, int view_hi, int nchunks) {
  constexpr int kWaves = kScanThreads / 64;
  __shared__ uint64_t s_wave[kWaves];
  __shared__ uint64_t s_vstart[GSR_MAX_VIEWS];
  uint64_t *sums = reinterpret_cast<uint64_t *>(ws.tile_order);
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  // exclusive scan of the chunk sums (at most kScanChunk chunks), plus base
  uint64_t x[4];
#pragma unroll
  for (int q = 0; q < 4; q++) x[q] = 4 * tid + q < nchunks ? sums[4 * tid + q] : 0ull;
  const uint64_t s = x[0] + x[1] + x[2] + x[3];
  const uint64_t incl = wave_incl_scan(s);
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  uint64_t before = 0;
  for (int w = 0; w < wave; w++) before += s_wave[w];
  uint64_t pre = (uint64_t)base + before + (incl - s);
  uint64_t total = (uint64_t)base;
  for (int w = 0; w < kWaves; w++) total += s_wave[w];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; q++) {
    if (4 * tid + q < nchunks) sums[4 * tid + q] = pre;
    pre += x[q];
  }
  __syncthreads();
  // where each view's first tile starts: its chunk's prefix plus the counts
  // in front of it within the chunk (one wavefront per view, all at once)
  const int nv = view_hi - view_lo;
  for (int v = wave; v < nv; v += kWaves) {
    const int64_t tb = ws.views[view_lo + v].tile_base;
    const int64_t c = (tb - lo) / kScanChunk;
    const int64_t c0 = lo + c * kScanChunk;
    uint64_t part = 0;
    for (int64_t t = c0 + lane; t < tb; t += 64) part += tile_total(ws, t, hi);
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) part += __shfl_xor(part, m);
    if (lane == 0) s_vstart[v] = sums[c] + part;
  }
  __syncthreads();
  const uint64_t cap = (uint64_t)ws.capacity;
  if (tid == 0) {
    ws.tile_start[hi] = (uint32_t)min(total, cap);
    if (total > cap) ws.hdr->overflow = 1u;
    ws.hdr->isect_total = (uint32_t)min(total, (uint64_t)0xffffffffu);
  }
  if (tid < nv) {
    const uint64_t a = s_vstart[tid], b = tid + 1 < nv ? s_vstart[tid + 1] : total;
    ws.hdr->isect[view_lo + tid] = (uint32_t)min(b - a, (uint64_t)0xffffffffu);
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(KWs ws, int64_t lo, int64_t hi) {
  constexpr int kWaves = kScanThreads / 64;
  __shared__ uint64_t s_wave[kWaves];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const int64_t t0 = lo + (int64_t)blockIdx.x * kScanChunk + 4 * (int64_t)tid;
  uint32_t x[4];
#pragma unroll
  for (int q = 0; q < 4; q++) x[q] = tile_total(ws, t0 + q, hi);
  const uint64_t s = (uint64_t)x[0] + x[1] + x[2] + x[3];
  const uint64_t incl = wave_incl_scan(s);
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  uint64_t before = 0;
  for (int w = 0; w < wave; w++) before += s_wave[w];
  uint64_t pre = reinterpret_cast<const uint64_t *>(ws.tile_order)[blockIdx.x] + before + (incl - s);
  const uint64_t cap = (uint64_t)ws.capacity;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    if (t0 + q < hi) ws.tile_start[t0 + q] = (uint32_t)min(pre, cap);
    pre += x[q];
  }
}

// --------------------------------------------------------------------- emit

// One thread per (view, Gaussian) pair: grid x over Gaussians, y over the
// views (or the one view of a plain-mode call), so the pairs of one Gaussian
// are placed in parallel rather than one after another.
__global__ __launch_bounds__(kBlock) void k_emit(KWs ws, int64_t n, int n_views, int view_only) {
  const int v = view_only >= 0 ? view_only : (int)blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !((ws.view_bits[i] >> v) & 1u)) return;
  const ViewInfo vi = ws.views[v];
  const int64_t r = (int64_t)v * n + i;
  const uint4 *sl = reinterpret_cast<const uint4 *>(ws.grad2d + r * kGrad2dStride);
  const uint4 s2 = sl[2], s3 = sl[3];
  const int x0 = s3.y & 0xffff, y0 = s3.y >> 16, x1 = s3.z & 0xffff;
  const int wx = x1 - x0 + 1, ntiles = wx * ((int)(s3.z >> 16) - y0 + 1);
  const uint64_t key = ((uint64_t)s3.w << 32) | (uint64_t)(uint32_t)r;
  const uint32_t rk[4] = {s2.y, s2.z, s2.w, s3.x};
  // the ranked first four tiles (row-major), their loads issued together
#pragma unroll
  for (int q = 0; q < 4; q++) {
    if (q < ntiles) {
      const int dy = q / wx, dx = q - dy * wx;
      const int64_t t = vi.tile_base + (int64_t)(y0 + dy) * vi.tiles_x + (x0 + dx);
      // rk[q] < the tile's count, so the slot lies in the tile's bucket; the
      // capacity bound is what an overflowing step can break
      const uint64_t slot = (uint64_t)ws.tile_start[t] + rk[q];
      if (slot < (uint64_t)ws.capacity) ws.keys[slot] = key;
    }
  }
  // the overflow entries of large footprints follow the ranked ones
  // (tile_fill counted them; counting it back down places them)
  for (int q = 4; q < ntiles; q++) {
    const int dy = q / wx, dx = q - dy * wx;
    const int64_t t = vi.tile_base + (int64_t)(y0 + dy) * vi.tiles_x + (x0 + dx);
    const uint32_t rank = ws.tile_count[t] + atomicSub(&ws.tile_fill[t], 1u) - 1u;
    const uint64_t slot = (uint64_t)ws.tile_start[t] + rank;
    if (slot < (uint64_t)ws.capacity && slot < (uint64_t)ws.tile_start[t + 1]) ws.keys[slot] = key;
  }
}

// --------------------------------------------------------------------- sort
// Keys of one tile are unique (the record slot is in the low word), so any
// correct sort gives the one ascending order.
//
// Tiles of at most kWaveSortMax entries: one wavefront per tile, the keys in
// registers, R per lane, lane-major (element e = lane * R + r in x[r]).  A
// bitonic network: partners closer than R sit in the same lane, the others
// in lane ^ (j / R), reached by DPP moves for lane distances 1, 2, 4, 8 and
// by shuffles for 16 and 32.  No LDS traffic besides those shuffles, no
// barrier.  Longer tiles are sorted as runs: tiles of up to 2048 or 4096
// entries as one run of that many keys, longer ones cut into runs of 8192; a
// workgroup sorts a run with two, four or eight wavefronts (1024 keys each,
// in registers as above) and one to three merge levels in LDS.  Tiles
// longer than one run are then merged run by run in global memory.

constexpr int kWaveSortMax = 1024;  // 64 lanes x 16 keys
constexpr int kSortBigThreads = 1024;
constexpr int kRunLong = 8192;      // the runs of tiles longer than 4096

template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, 0xf, 0xf, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// x from lane ^ m (m a power of two below 64), the whole wavefront active
template <int M>
__device__ __forceinline__ uint64_t lane_xor(uint64_t x) {
  if (M == 1) return dpp_u64<0xB1>(x);                     // quad_perm [1,0,3,2]
  if (M == 2) return dpp_u64<0x4E>(x);                     // quad_perm [2,3,0,1]
  if (M == 4) return dpp_u64<0x141>(dpp_u64<0x1B>(x));     // quad_perm [3,2,1,0] then row_half_mirror
  if (M == 8) return dpp_u64<0x128>(x);                    // row_ror:8
  return __shfl_xor(x, M);
}

template <int R, int JS, int KS>
__device__ __forceinline__ void bitonic_stage(uint64_t (&x)[R], int lane) {
  constexpr int k = 1 << KS, j = 1 << JS;
  if (j < R) {
    // partners in the same lane: e = lane R + r and lane R + (r ^ j)
#pragma unroll
    for (int r = 0; r < R; r++) {
      if ((r & j) == 0) {
        const int q = r | j;
        const bool up = (((lane * R) | r) & k) == 0;
        const uint64_t lo = x[r] < x[q] ? x[r] : x[q], hi = x[r] < x[q] ? x[q] : x[r];
        x[r] = up ? lo : hi;
        x[q] = up ? hi : lo;
      }
    }
  } else {
    constexpr int m = j / R;
    const bool lower = (lane & m) == 0;
#pragma unroll
    for (int r = 0; r < R; r++) {
      const uint64_t y = lane_xor<m>(x[r]);
      const bool up = (((lane * R) | r) & k) == 0;
      x[r] = (lower == up) == (x[r] < y) ? x[r] : y;
    }
  }
}

template <int R, int KS, int JS>
struct BitonicMerge {
  __device__ __forceinline__ static void run(uint64_t (&x)[R], int lane) {
    bitonic_stage<R, JS, KS>(x, lane);
    BitonicMerge<R, KS, JS - 1>::run(x, lane);
  }
};
template <int R, int KS>
struct BitonicMerge<R, KS, -1> {
  __device__ __forceinline__ static void run(uint64_t (&)[R], int) {}
};

template <int R, int KS, int LOGN>
struct BitonicSort {
  __device__ __forceinline__ static void run(uint64_t (&x)[R], int lane) {
    BitonicMerge<R, KS, KS - 1>::run(x, lane);
    BitonicSort<R, KS + 1, LOGN>::run(x, lane);
  }
};
template <int R, int LOGN>
struct BitonicSort<R, LOGN + 1, LOGN> {
  __device__ __forceinline__ static void run(uint64_t (&)[R], int) {}
};

template <int R>
__device__ __forceinline__ void wave_sort_tile(uint64_t *keys, int n) {
  constexpr int kLogN = 6 + (R >= 2) + (R >= 4) + (R >= 8) + (R >= 16) + (R >= 32) + (R >= 64);
  const int lane = lane_id();
  uint64_t x[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int e = lane * R + r;
    x[r] = e < n ? keys[e] : ~0ull;
  }
  BitonicSort<R, 1, kLogN>::run(x, lane);
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int e = lane * R + r;
    if (e < n) keys[e] = x[r];
  }
}

// Four tiles of at most kWaveSortMax entries per workgroup, one per
// wavefront (the whole wavefront stays active through the network), the
// register count sized to the tile.
__global__ __launch_bounds__(kBlock) void k_sort_wave(KWs ws, int64_t tile_lo, int64_t tile_count) {
  const int64_t groups = (tile_count + 3) / 4;
  const int64_t g = xcd_remap(blockIdx.x, groups);
  if (g >= groups) return;
  const int64_t b = g * 4 + (threadIdx.x >> 6);
  if (b >= tile_count) return;
  const int64_t t = tile_lo + b;
  const int64_t start = ws.tile_start[t];
  const int n = (int)((int64_t)ws.tile_start[t + 1] - start);
  if (n <= 1 || n > kWaveSortMax) return;
  uint64_t *keys = ws.keys + start;
  if (n <= 64) wave_sort_tile<1>(keys, n);
  else if (n <= 128) wave_sort_tile<2>(keys, n);
  else if (n <= 256) wave_sort_tile<4>(keys, n);
  else if (n <= 512) wave_sort_tile<8>(keys, n);
  else wave_sort_tile<16>(keys, n);
}

// Merge two sorted runs A[0, la), B[0, lb) into out.  Each thread takes a
// contiguous chunk of kMergeChunk outputs: one co-rank binary search finds
// where the chunk starts in A and in B (keys are unique), then the chunk is
// merged sequentially.
constexpr int kMergeChunk = 16;

__device__ void merge_runs(const uint64_t *A, int64_t la, const uint64_t *B, int64_t lb, uint64_t *out) {
  const int64_t total = la + lb;
  for (int64_t k0 = (int64_t)threadIdx.x * kMergeChunk; k0 < total; k0 += (int64_t)blockDim.x * kMergeChunk) {
    int64_t lo = k0 > lb ? k0 - lb : 0, hi = k0 < la ? k0 : la;
    while (lo < hi) {
      const int64_t ia = (lo + hi) >> 1;
      if (A[ia] < B[k0 - ia - 1]) lo = ia + 1;
      else hi = ia;
    }
    int64_t ia = lo, ib = k0 - lo;
    const int64_t k1 = min(k0 + (int64_t)kMergeChunk, total);
    for (int64_t k = k0; k < k1; k++) {
      const bool takeA = ib >= lb || (ia < la && A[ia] < B[ib]);
      out[k] = takeA ? A[ia++] : B[ib++];
    }
  }
}

// One workgroup merges the sorted runs of one tile of more than kRunLong entries.
__device__ void merge_tile_block(const KWs &ws, int64_t t) {
  const int64_t start = ws.tile_start[t];
  const int64_t n = (int64_t)ws.tile_start[t + 1] - start;
  uint64_t *keys = ws.keys + start;
  uint64_t *src = keys, *dst = ws.keys_alt + start;
  for (int64_t w = kRunLong; w < n; w <<= 1) {
    for (int64_t a = 0; a < n; a += 2 * w) {
      const int64_t la = min(w, n - a);
      const int64_t lb = min(w, max((int64_t)0, n - a - w));
      merge_runs(src + a, la, src + a + la, lb, dst + a);
    }
    __syncthreads();
    uint64_t *tmp = src;
    src = dst;
    dst = tmp;
  }
  if (src != keys) {
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) keys[k] = src[k];
  }
  __syncthreads();
}

// Runs of the tiles longer than one wavefront's register sort, listed per
// sort call in keys_alt (tile ids of the 2048-key runs from word 0, of the
// 4096-key runs from word capacity / 2, (tile, run index) pairs of the
// 8192-key runs from word `capacity`), which the merge passes use only after
// the runs are sorted; the tiles longer than one run in tile_order (free
// between the scan and the schedule).  Workgroups take the runs in a fixed
// stride (runs of one size cost alike), then the long tiles from a counter,
// so long tiles spread over the whole chip.
__global__ void k_big_reset(KWs ws) {
  ws.hdr->big_count = 0u;
  ws.hdr->big_next = 0u;
  ws.hdr->run2_count = 0u;
  ws.hdr->run_count = 0u;
  ws.hdr->run8_count = 0u;
}

__device__ __forceinline__ uint32_t *run_list(const KWs &ws, int run) {
  return reinterpret_cast<uint32_t *>(ws.keys_alt) + (run == 2048 ? 0 : run == 4096 ? ws.capacity / 2 : ws.capacity);
}

// One atomic per wavefront and list, the lanes' places following from a
// prefix sum over the wavefront: a single counter hit by every long tile of
// a 2160p view would serialise on its address.
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool take, uint32_t count) {
  const int lane = lane_id();
  uint32_t before = 0u, total = 0u;
  // lanes append `count` entries each; the prefix over lower lanes by shuffles
  uint32_t c = take ? count : 0u, incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, (unsigned)off);
    if (lane >= off) incl += y;
  }
  total = __shfl(incl, 63);
  before = incl - c;
  uint32_t base = 0u;
  if (total != 0u && lane == 0) base = atomicAdd(counter, total);
  return __shfl(base, 0) + before;
}

__global__ __launch_bounds__(kBlock) void k_big_collect(KWs ws, int64_t tile_lo, int64_t tile_count) {
  // (every lane of a wavefront goes through the same iterations: the appends are wavefront-wide)
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < tile_count; b0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = b0 + threadIdx.x;
    const int64_t t = tile_lo + b;
    const int64_t n = b < tile_count ? (int64_t)ws.tile_start[t + 1] - ws.tile_start[t] : 0;
    const bool r2 = n > kWaveSortMax && n <= 2048, r4 = n > 2048 && n <= 4096, r8 = n > 4096;
    const uint32_t runs = r8 ? (uint32_t)((n + kRunLong - 1) / kRunLong) : 0u;
    const uint32_t a2 = wave_append(&ws.hdr->run2_count, r2, 1u);
    const uint32_t a4 = wave_append(&ws.hdr->run_count, r4, 1u);
    const uint32_t a8 = wave_append(&ws.hdr->run8_count, r8, runs);
    const uint32_t ab = wave_append(&ws.hdr->big_count, n > kRunLong, 1u);
    if (r2) run_list(ws, 2048)[a2] = (uint32_t)t;
    if (r4) run_list(ws, 4096)[a4] = (uint32_t)t;
    if (r8) {
      uint32_t *list = run_list(ws, kRunLong);
      for (uint32_t c = 0; c < runs; c++) {
        list[2 * (a8 + c)] = (uint32_t)t;
        list[2 * (a8 + c) + 1] = c;
      }
    }
    if (n > kRunLong) ws.tile_order[ab] = (uint32_t)t;
  }
}

// One level of merges inside a run of RUN keys in LDS: the sorted blocks of
// w keys are merged in pairs into blocks of 2w.  Each of the THREADS threads
// produces RUN / THREADS consecutive outputs after one co-rank search (keys
// are unique), holds them in registers over a barrier and stores them in
// place.
template <int RUN, int THREADS>
__device__ __forceinline__ void merge_level_lds(uint64_t *s, int w) {
  constexpr int kPer = RUN / THREADS;
  const int o0 = (int)threadIdx.x * kPer;
  const int pair = o0 / (2 * w), k0 = o0 - pair * 2 * w;
  const uint64_t *A = s + pair * 2 * w, *B = A + w;
  int lo = k0 > w ? k0 - w : 0, hi = k0 < w ? k0 : w;
  while (lo < hi) {
    const int ia = (lo + hi) >> 1;
    if (A[ia] < B[k0 - ia - 1]) lo = ia + 1;
    else hi = ia;
  }
  int ia = lo, ib = k0 - lo;
  uint64_t out[kPer];
#pragma unroll
  for (int k = 0; k < kPer; k++) {
    const uint64_t a = A[min(ia, w - 1)], b = B[min(ib, w - 1)];  // (reads stay inside the pair)
    const bool takeA = ib >= w || (ia < w && a < b);
    out[k] = takeA ? a : b;
    ia += takeA ? 1 : 0;
    ib += takeA ? 0 : 1;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; k++) s[o0 + k] = out[k];
  __syncthreads();
}

// Sorts the listed runs of RUN keys: each wavefront sorts its 1024 keys of
// the run in registers, then merge levels in LDS give the sorted run.
// Missing keys of a short run are padded with distinct values above every
// key, ascending with the position (depth bits of a finite float stay below
// 0x7f800000 in the high word), so a wavefront's share of padding only is
// sorted.
template <int RUN>
__global__ __launch_bounds__(RUN / 16) void k_sort_runs(KWs ws) {
  constexpr int kWaves = RUN / 1024, kThreads = 64 * kWaves, R = 16;
  __shared__ uint64_t s[RUN];
  const uint32_t count = RUN == 2048 ? ws.hdr->run2_count : RUN == 4096 ? ws.hdr->run_count : ws.hdr->run8_count;
  const uint32_t *list = run_list(ws, RUN);
  const int wave = threadIdx.x >> 6, lane = lane_id();
  // runs of one size cost alike: workgroups take them in a fixed stride
  for (uint32_t k = blockIdx.x; k < count; k += gridDim.x) {
    const int64_t t = RUN <= 4096 ? list[k] : list[2 * k];
    const int64_t c0 = RUN <= 4096 ? 0 : (int64_t)list[2 * k + 1] * RUN;
    const int64_t start = ws.tile_start[t];
    const int m = (int)min((int64_t)RUN, (int64_t)ws.tile_start[t + 1] - start - c0);
    uint64_t *keys = ws.keys + start + c0;
    const int q0 = wave * 1024;
    uint64_t x[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int e = q0 + lane * R + r;
      x[r] = e < m ? keys[e] : ~0ull - (uint64_t)(RUN - 1 - e);
    }
    if (q0 < m) BitonicSort<R, 1, 10>::run(x, lane);  // (uniform per wavefront)
#pragma unroll
    for (int r = 0; r < R; r++) s[q0 + lane * R + r] = x[r];
    __syncthreads();
#pragma unroll
    for (int w = 1024; w < RUN; w <<= 1) merge_level_lds<RUN, kThreads>(s, w);
    for (int e = threadIdx.x; e < m; e += kThreads) keys[e] = s[e];
    __syncthreads();
  }
}

// Merges the runs of the tiles longer than one run, one tile per workgroup.
__global__ __launch_bounds__(kSortBigThreads) void k_sort_big(KWs ws) {
  __shared__ uint32_t s_k;
  const uint32_t count = ws.hdr->big_count;
  for (;;) {
    if (threadIdx.x == 0) s_k = atomicAdd(&ws.hdr->big_next, 1u);
    __syncthreads();
    const uint32_t k = s_k;
    if (k >= count) break;
    merge_tile_block(ws, ws.tile_order[k]);  // ends with a barrier, before s_k is written again
  }
}

// --------------------------------------------------------------- loss total

// Deterministic: fixed thread mapping and reduction tree, double
// accumulation.  One workgroup per view sums its tiles' losses; one thread
// then adds the views in order.
__global__ __launch_bounds__(kScanThreads) void k_loss_views(KWs ws) {
  constexpr int kWaves = kScanThreads / 64;
  __shared__ double s_w[kWaves];
  const int v = blockIdx.x;
  const ViewInfo vi = ws.views[v];
  const int64_t nt = (int64_t)vi.tiles_x * vi.tiles_y;
  double a = 0.0;
  for (int64_t k = threadIdx.x; k < nt; k += kScanThreads) a += (double)ws.tile_loss[vi.tile_base + k];
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) a += __shfl_xor(a, m);
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) t += s_w[w];
    ws.hdr->view_loss[v] = t * (double)vi.loss_scale;
  }
}

__global__ void k_loss_total(KWs ws, int n_views, float *loss) {
  if (threadIdx.x == 0) {
    double total = 0.0;
    for (int v = 0; v < n_views; v++) total += ws.hdr->view_loss[v];
    *loss = (float)total;
  }
}

// -------------------------------------------------------------- project_bwd
// Reverse mode of the projection for every view in which the Gaussian is
// visible (view_only >= 0 restricts to one view and adds into the gradients).

template <int D>
__global__ __launch_bounds__(kBlock) void k_project_bwd(KParams p, const gsr_camera *cams, KOpts o, KWs ws,
                                                        KGrads gr, float *stat_S, uint32_t *stat_n,
                                                        int view_only) {
  constexpr int K = (D + 1) * (D + 1);
  __shared__ Cam64 s_cam[GSR_MAX_VIEWS];
  load_cams(s_cam, cams, ws.views, p.n_views, o);
  const int64_t n = p.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t bits = ws.view_bits[i];
  if (view_only >= 0) bits &= 1u << view_only;
  const bool add = view_only >= 0 || o.accumulate;
  if (bits == 0) {
    if (!add) {
      for (int a = 0; a < 3; a++) gr.means[a * n + i] = 0.f, gr.log_scales[a * n + i] = 0.f;
      for (int a = 0; a < 4; a++) gr.quats[a * n + i] = 0.f;
      gr.logits[i] = 0.f;
      for (int k = 0; k < 3 * K; k++) gr.sh[(int64_t)k * n + i] = 0.f;
    }
    return;
  }
  // the view loop needs the mean and the covariance only; the rest of the
  // geometry is rebuilt after it (bit-identical, from the same helper)
  GeoF gf;
  load_geo_fwd(p, i, gf);
  double gmu[3] = {0, 0, 0}, gSig[6] = {0, 0, 0, 0, 0, 0}, gopac = 0.0;
  float Sacc = 0.f;
  uint32_t cnt = 0;
  const double stat_scale = o.stat_scale;
  for (uint32_t b = bits; b; b &= b - 1) {
    // the chain rule below only feeds gradients: multiply-adds may fuse (the
    // projection it starts from, and the colour replay after the loop, whose
    // clamp must take the forward's decision, are not fused)
#pragma clang fp contract(fast)
    const int v = __ffs(b) - 1;
    const Cam64 &cam = s_cam[v];
    Proj P;
    project_view<false>(gf, cam, o, P);  // visible by construction of view_bits
    const float4 *g2 = reinterpret_cast<const float4 *>(ws.grad2d + ((int64_t)v * n + i) * kGrad2dStride);
    const float4 q0 = g2[0], q1 = g2[1];
    // the reverse raster's moments of dL/dp over the pixel offsets d (sums of
    // gp dx, gp dy, gp dx^2, gp dx dy, gp dy^2; p = -d^T Q d / 2) give the 2D
    // gradient: dL/dmean = Q (m0, m1), dL/d(A, B, C) = -(m2 / 2, m3, m4 / 2)
    const double QA = P.A, QB = P.B, QC = P.C;
    const double m0 = q0.x, m1 = q0.y;
    const double gmx = QA * m0 + QB * m1, gmy = QB * m0 + QC * m1;
    const double gA = -0.5 * (double)q0.z, gB = -(double)q0.w, gC = -0.5 * (double)q1.x, go = q1.y;
    Sacc += (float)(stat_scale * sqrt(gmx * gmx + gmy * gmy));
    cnt += 1;
    gopac += go;
    // conic -> 2D covariance:  dL/dS = -Q G_Q Q with G_Q = [[gA, gB/2], [gB/2, gC]]
    const double h = 0.5 * gB;
    const double m00 = gA * QA + h * QB, m01 = gA * QB + h * QC;  // G_Q Q
    const double m10 = h * QA + gC * QB, m11 = h * QB + gC * QC;
    const double gs00 = -(QA * m00 + QB * m10);
    const double gs01 = -(QA * m01 + QB * m11);
    const double gs11 = -(QB * m01 + QC * m11);
    // S = T Sigma T^T (T = J W, rows T0, T1):  dL/dSigma = T^T G_S T
    const double *T0 = P.T0, *T1 = P.T1;
    {
      int e = 0;
#pragma unroll
      for (int r = 0; r < 3; r++)
#pragma unroll
        for (int cidx = r; cidx < 3; cidx++, e++) {
          double val = T0[r] * gs00 * T0[cidx] + T0[r] * gs01 * T1[cidx] + T1[r] * gs01 * T0[cidx] +
                       T1[r] * gs11 * T1[cidx];
          gSig[e] += (r == cidx) ? val : 2.0 * val;  // off-diagonals stored once, used twice
        }
    }
    // dL/dT = 2 G_S T Sigma
    double ST0[3], ST1[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
      ST0[r] = sig_at(gf.Sig, r, 0) * T0[0] + sig_at(gf.Sig, r, 1) * T0[1] + sig_at(gf.Sig, r, 2) * T0[2];
      ST1[r] = sig_at(gf.Sig, r, 0) * T1[0] + sig_at(gf.Sig, r, 1) * T1[1] + sig_at(gf.Sig, r, 2) * T1[2];
    }
    double GT0[3], GT1[3];
#pragma unroll
    for (int cidx = 0; cidx < 3; cidx++) {
      GT0[cidx] = 2.0 * (gs00 * ST0[cidx] + gs01 * ST1[cidx]);
      GT1[cidx] = 2.0 * (gs01 * ST0[cidx] + gs11 * ST1[cidx]);
    }
    // T = J W:  dL/dJ = dL/dT W^T
    double gj00 = 0, gj02 = 0, gj11 = 0, gj12 = 0;
#pragma unroll
    for (int cidx = 0; cidx < 3; cidx++) {
      gj00 += GT0[cidx] * cam.R[cidx];
      gj02 += GT0[cidx] * cam.R[6 + cidx];
      gj11 += GT1[cidx] * cam.R[3 + cidx];
      gj12 += GT1[cidx] * cam.R[6 + cidx];
    }
    const double tx = P.tc[0], ty = P.tc[1], tz = P.tc[2];
    const double iz = 1.0 / tz, iz2 = iz * iz;
    double gt[3] = {0, 0, 0};
    gt[2] += -gj00 * cam.fx * iz2 - gj11 * cam.fy * iz2;
    if (P.cu) {
      gt[2] += gj02 * cam.fx * P.u * iz2;
    } else {
      gt[0] += -gj02 * cam.fx * iz2;
      gt[2] += gj02 * 2.0 * cam.fx * tx * iz2 * iz;
    }
    if (P.cv) {
      gt[2] += gj12 * cam.fy * P.v * iz2;
    } else {
      gt[1] += -gj12 * cam.fy * iz2;
      gt[2] += gj12 * 2.0 * cam.fy * ty * iz2 * iz;
    }
    // projected mean
    gt[0] += gmx * cam.fx * iz;
    gt[1] += gmy * cam.fy * iz;
    gt[2] += -(gmx * cam.fx * tx + gmy * cam.fy * ty) * iz2;
    // t = W mu + t_v
#pragma unroll
    for (int a = 0; a < 3; a++) gmu[a] += cam.R[a] * gt[0] + cam.R[3 + a] * gt[1] + cam.R[6 + a] * gt[2];
  }
  // colour -> SH coefficients and viewing direction, per visible view.  The
  // forward's float32 colour is replayed operation for operation, so the
  // clamp at zero takes the same decision here.
  float sh[3 * K], gsh[3 * K];
#pragma unroll
  for (int k = 0; k < 3 * K; k++) {
    sh[k] = p.sh[(int64_t)k * n + i];
    gsh[k] = 0.f;
  }
  for (uint32_t b = bits; b; b &= b - 1) {
    const int v = __ffs(b) - 1;
    const Cam64 &cam = s_cam[v];
    const float *g2 = ws.grad2d + ((int64_t)v * n + i) * kGrad2dStride;
    const float gcol[3] = {g2[6], g2[7], g2[8]};
    double d[3];
#pragma unroll
    for (int a = 0; a < 3; a++) d[a] = gf.mu[a] + cam.cc[a];
    const double idn = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const float x = (float)(d[0] * idn), y = (float)(d[1] * idn), z = (float)(d[2] * idn);
    float Y[K];
    sh_eval<D, float>(x, y, z, Y);
    float wk[K];
#pragma unroll
    for (int k = 0; k < K; k++) wk[k] = 0.0f;
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
      float raw = 0.5f;
#pragma unroll
      for (int k = 0; k < K; k++) raw = __fmaf_rn(sh[k * 3 + ch], Y[k], raw);
      const float gr_ch = raw > 0.0f ? gcol[ch] : 0.0f;
#pragma unroll
      for (int k = 0; k < K; k++) {
        gsh[k * 3 + ch] += gr_ch * Y[k];
        wk[k] += gr_ch * sh[k * 3 + ch];
      }
    }
    if (D > 0) {
      float gd[3];
      sh_grad<D, float>(x, y, z, wk, gd);
      const float dot = gd[0] * x + gd[1] * y + gd[2] * z;
      gmu[0] += (double)(gd[0] - dot * x) * idn;
      gmu[1] += (double)(gd[1] - dot * y) * idn;
      gmu[2] += (double)(gd[2] - dot * z) * idn;
    }
  }
  {
#pragma clang fp contract(fast)
  Geo g;
  load_geo(p, i, g);
  // Sigma = Rq diag(s^2) Rq^T  (gSig holds dL/dSigma_ij for i <= j, off-diagonals doubled)
  double G[9];
  {
    const int idx[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
#pragma unroll
    for (int e = 0; e < 6; e++) {
      const int r = idx[e][0], cidx = idx[e][1];
      const double val = r == cidx ? gSig[e] : 0.5 * gSig[e];
      G[r * 3 + cidx] = val;
      G[cidx * 3 + r] = val;
    }
  }
  // dL/dM = 2 G M with M = Rq diag(s);  s_j = exp(l_j)
  double gl[3], GR[9];
#pragma unroll
  for (int j = 0; j < 3; j++) {
    double gs = 0.0;
#pragma unroll
    for (int r = 0; r < 3; r++) {
      const double gm = 2.0 * (G[r * 3 + 0] * g.Rq[0 * 3 + j] + G[r * 3 + 1] * g.Rq[1 * 3 + j] + G[r * 3 + 2] * g.Rq[2 * 3 + j]) * g.s[j];
      gs += gm * g.Rq[r * 3 + j];
      GR[r * 3 + j] = gm * g.s[j];
    }
    gl[j] = gs * g.s[j];
  }
  // R = (w^2 - |v|^2) I + 2 v v^T + 2 w [v]x  ->  unit quaternion
  const double w = g.q[0], qx = g.q[1], qy = g.q[2], qz = g.q[3];
  const double tr = GR[0] + GR[4] + GR[8];
  const double cw = -qz * GR[1] + qy * GR[2] + qz * GR[3] - qx * GR[5] - qy * GR[6] + qx * GR[7];
  double gq[4];
  gq[0] = 2.0 * w * tr + 2.0 * cw;
  const double vv[3] = {qx, qy, qz};
  const double cross_k[3] = {-GR[5] + GR[7], GR[2] - GR[6], -GR[1] + GR[3]};
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const double sym = (GR[k * 3 + 0] + GR[0 * 3 + k]) * vv[0] + (GR[k * 3 + 1] + GR[1 * 3 + k]) * vv[1] +
                       (GR[k * 3 + 2] + GR[2 * 3 + k]) * vv[2];
    gq[1 + k] = -2.0 * vv[k] * tr + 2.0 * sym + 2.0 * w * cross_k[k];
  }
  const double gd = gq[0] * g.q[0] + gq[1] * g.q[1] + gq[2] * g.q[2] + gq[3] * g.q[3];
  const double inv_qn = 1.0 / g.qn;
  float outq[4];
#pragma unroll
  for (int a = 0; a < 4; a++) outq[a] = (float)((gq[a] - gd * g.q[a]) * inv_qn);
  const float glogit = (float)(gopac * g.opac * (1.0 - g.opac));
  if (add) {
    for (int a = 0; a < 3; a++) {
      gr.means[a * n + i] += (float)gmu[a];
      gr.log_scales[a * n + i] += (float)gl[a];
    }
    for (int a = 0; a < 4; a++) gr.quats[a * n + i] += outq[a];
    gr.logits[i] += glogit;
#pragma unroll
    for (int k = 0; k < 3 * K; k++) gr.sh[(int64_t)k * n + i] += gsh[k];
  } else {
    for (int a = 0; a < 3; a++) {
      gr.means[a * n + i] = (float)gmu[a];
      gr.log_scales[a * n + i] = (float)gl[a];
    }
    for (int a = 0; a < 4; a++) gr.quats[a * n + i] = outq[a];
    gr.logits[i] = glogit;
#pragma unroll
    for (int k = 0; k < 3 * K; k++) gr.sh[(int64_t)k * n + i] = gsh[k];
  }
  if (stat_S) stat_S[i] += Sacc;
  if (stat_n) stat_n[i] += cnt;
  }
}

// -------------------------------------------------------------- visibility

__global__ __launch_bounds__(kBlock) void k_visibility(KParams p, const gsr_camera *cams, KOpts o, KWs ws,
                                                       float bx0, float by0, float bz0, float bx1, float by1,
                                                       float bz1, uint32_t *bits_out, uint8_t *keep_out,
                                                       uint8_t *in_block) {
  __shared__ Cam64 s_cam[GSR_MAX_VIEWS];
  load_cams(s_cam, cams, ws.views, p.n_views, o);
  const int64_t n = p.n;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool keep = p.keep == nullptr || p.keep[i] != 0;
  uint32_t bits = 0;
  if (keep) {
    GeoF g;
    load_geo_fwd(p, i, g);
    for (int v = 0; v < p.n_views; v++) {
      Proj P;
      if (maybe_visible(g, s_cam[v], o) && project_view(g, s_cam[v], o, P)) bits |= 1u << v;
    }
  }
  if (bits_out) bits_out[i] = bits;
  if (keep_out) keep_out[i] = bits != 0 ? 1 : 0;
  if (in_block) {
    const float x = p.means[i], y = p.means[n + i], z = p.means[2 * n + i];
    in_block[i] = (x >= bx0 && x < bx1 && y >= by0 && y < by1 && z >= bz0 && z < bz1) ? 1 : 0;
  }
}

__global__ void k_copy_pixels(KWs ws, float *T_out, uint32_t *last_out) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ws.pixels_total;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (T_out) T_out[k] = ws.pix_T[k];
    if (last_out) last_out[k] = ws.pix_last[k];
  }
}

// ---------------------------------------------------------------- launchers


int launch_setup(const ViewTable &table, const KWs &ws, int64_t zlo, int64_t zcount, int zero_bits, int64_t n,
                 void *stream) {
  int64_t work = zcount;
  if (zero_bits && n > work) work = n;
  if (work < GSR_MAX_VIEWS) work = GSR_MAX_VIEWS;
  hipLaunchKernelGGL(k_setup, dim3(grid_for(work)), dim3(kBlock), 0, (hipStream_t)stream, table, ws, zlo, zcount,
                     zero_bits, n);
  return last_err();
}

int launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, void *stream) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count)), dim3(kBlock), 0, (hipStream_t)stream, p, value, count);
  return last_err();
}

int launch_fill_f32(float *p, float value, int64_t count, void *stream) {
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(count)), dim3(kBlock), 0, (hipStream_t)stream, p, value, count);
  return last_err();
}

int launch_project(const KParams &p, const gsr_camera *cams, const KOpts &o, const KWs &ws, int view_lo,
                   int view_hi, int or_bits, int table, void *stream) {
  const dim3 grid(grid_for(p.n)), block(kBlock);
  hipStream_t s = (hipStream_t)stream;
#define GSR_PROJECT(D_)                                                                                        \
  do {                                                                                                        \
    if (table) hipLaunchKernelGGL((k_project<D_, true>), grid, block, 0, s, p, cams, o, ws, view_lo, view_hi, or_bits); \
    else hipLaunchKernelGGL((k_project<D_, false>), grid, block, 0, s, p, cams, o, ws, view_lo, view_hi, or_bits);      \
  } while (0)
  switch (p.sh_degree) {
    case 0: GSR_PROJECT(0); break;
    case 1: GSR_PROJECT(1); break;
    case 2: GSR_PROJECT(2); break;
    default: GSR_PROJECT(3); break;
  }
#undef GSR_PROJECT
  return last_err();
}

int launch_scan(const KWs &ws, int64_t lo, int64_t hi, int64_t base, int view_lo, int view_hi, void *stream) {
  if (hi <= lo) return (int)hipErrorInvalidValue;
  const int64_t nchunks = (hi - lo + kScanChunk - 1) / kScanChunk;
  // chunk sums in the tile-order array (sized for 8 bytes per chunk of the
  // largest tile grid); one workgroup scans at most kScanChunk of them
  if (nchunks > kScanChunk) return (int)hipErrorInvalidValue;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nchunks), dim3(kScanThreads), 0, s, ws, lo, hi);
  hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(kScanThreads), 0, s, ws, lo, hi, base, view_lo, view_hi,
                     (int)nchunks);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nchunks), dim3(kScanThreads), 0, s, ws, lo, hi);
  return last_err();
}

int launch_emit(const KWs &ws, int64_t n, int n_views, int view_only, void *stream) {
  const unsigned gy = view_only >= 0 ? 1u : (unsigned)n_views;
  hipLaunchKernelGGL(k_emit, dim3(grid_for(n), gy), dim3(kBlock), 0, (hipStream_t)stream, ws, n, n_views, view_only);
  return last_err();
}

int launch_sort(const KWs &ws, int64_t tile_lo, int64_t tile_count, void *stream) {
  if (tile_count <= 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  const dim3 wgrid((unsigned)xcd_grid((tile_count + 3) / 4));
  hipLaunchKernelGGL(k_sort_wave, wgrid, dim3(kBlock), 0, s, ws, tile_lo, tile_count);
  hipLaunchKernelGGL(k_big_reset, dim3(1), dim3(1), 0, s, ws);
  hipLaunchKernelGGL(k_big_collect, dim3((unsigned)min((tile_count + kBlock - 1) / kBlock, (int64_t)4096)),
                     dim3(kBlock), 0, s, ws, tile_lo, tile_count);
  hipLaunchKernelGGL(k_sort_runs<2048>, dim3(4096), dim3(128), 0, s, ws);
  hipLaunchKernelGGL(k_sort_runs<4096>, dim3(2048), dim3(256), 0, s, ws);
  hipLaunchKernelGGL(k_sort_runs<kRunLong>, dim3(1024), dim3(kRunLong / 16), 0, s, ws);
  hipLaunchKernelGGL(k_sort_big, dim3(512), dim3(kSortBigThreads), 0, s, ws);
  return last_err();
}

int launch_project_bwd(const KParams &p, const gsr_camera *cams, const KOpts &o, const KWs &ws, const KGrads &g,
                       float *stat_S, uint32_t *stat_n, int view_only, void *stream) {
  const dim3 grid(grid_for(p.n)), block(kBlock);
  hipStream_t s = (hipStream_t)stream;
  switch (p.sh_degree) {
    case 0: hipLaunchKernelGGL(k_project_bwd<0>, grid, block, 0, s, p, cams, o, ws, g, stat_S, stat_n, view_only); break;
    case 1: hipLaunchKernelGGL(k_project_bwd<1>, grid, block, 0, s, p, cams, o, ws, g, stat_S, stat_n, view_only); break;
    case 2: hipLaunchKernelGGL(k_project_bwd<2>, grid, block, 0, s, p, cams, o, ws, g, stat_S, stat_n, view_only); break;
    default: hipLaunchKernelGGL(k_project_bwd<3>, grid, block, 0, s, p, cams, o, ws, g, stat_S, stat_n, view_only); break;
  }
  return last_err();
}

int launch_loss(const KWs &ws, int n_views, float *loss, void *stream) {
  hipLaunchKernelGGL(k_loss_views, dim3((unsigned)n_views), dim3(kScanThreads), 0, (hipStream_t)stream, ws);
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, (hipStream_t)stream, ws, n_views, loss);
  return last_err();
}

int launch_visibility(const KParams &p, const gsr_camera *cams, const KOpts &o, const KWs &ws, const float *aabb6,
                      uint32_t *bits, uint8_t *keep_out, uint8_t *in_block, void *stream) {
  hipLaunchKernelGGL(k_visibility, dim3(grid_for(p.n)), dim3(kBlock), 0, (hipStream_t)stream, p, cams, o, ws,
                     aabb6[0], aabb6[1], aabb6[2], aabb6[3], aabb6[4], aabb6[5], bits, keep_out, in_block);
  return last_err();
}

int launch_copy_pixels(const KWs &ws, float *T_out, uint32_t *last_out, void *stream) {
  hipLaunchKernelGGL(k_copy_pixels, dim3(grid_for(ws.pixels_total)), dim3(kBlock), 0, (hipStream_t)stream, ws, T_out,
                     last_out);
  return last_err();
}

}  // namespace gsr
