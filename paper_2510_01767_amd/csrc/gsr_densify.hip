// Selective densification and pruning (Sec. 3.3; the clone / split / prune
// rules of vanilla 3DGS that the fine stage follows, App. A.1).
//
// Every Gaussian i yields c_i in {0, 1, 2} outputs, written at the exclusive
// prefix sum of c, so the outputs keep the input's storage order (a clone or
// the two children of a split sit next to their parent, and a Morton-ordered
// set stays nearly Morton-ordered).  Two launches count (per-block sums, one
// block scanning the block sums; the host reads the total), one launch
// recomputes each block's local offsets and writes every plane.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gsr_device.h"
#include "gsr_stages.h"

namespace gsr {

namespace {

constexpr int kItems = 4;                       // consecutive Gaussians per thread
constexpr int kChunk = kBlock * kItems;         // Gaussians per workgroup
constexpr int kPlaneSplit = 4;                  // workgroups sharing a chunk's planes

struct Decision {
  int kind;  // 0 keep, 1 clone, 2 split
  int c;     // outputs written
};

__device__ __forceinline__ Decision decide(const KDensify &k, int64_t i) {
  if (k.keep && !k.keep[i]) return {0, 0};
  const int64_t n = k.n;
  const float lmax = fmaxf(fmaxf(k.ls[i], k.ls[n + i]), k.ls[2 * n + i]);
  const bool opa_ok = !k.opa_on || (double)k.opa[i] >= k.logit_min;
  const uint32_t cnt = k.cnt[i];
  // S / n >= threshold, exactly: the product of a float and a count below
  // 2^29 is exact in double
  const bool cand = cnt > 0 && (double)k.S[i] >= k.grad_thr * (double)cnt && (!k.selective || k.in_block[i]);
  if (!cand) {
    const bool ok = opa_ok && (!k.world_on || (double)lmax <= k.log_world_max);
    return {0, ok ? 1 : 0};
  }
  if ((double)lmax <= k.log_clone_max) {
    const bool ok = opa_ok && (!k.world_on || (double)lmax <= k.log_world_max);
    return {1, ok ? 2 : 0};
  }
  // a child's log scales are l - d rounded to float; rounding is monotone,
  // so the child's largest is the rounded lmax - d
  const float lc = lmax - k.child_dlog;
  const bool ok = opa_ok && (!k.world_on || (double)lc <= k.log_world_max);
  return {2, ok ? 2 : 0};
}

__device__ __forceinline__ uint64_t block_exclusive_sum(uint64_t x, uint64_t *s_tmp, uint64_t *total) {
  // wave inclusive scan with shuffles, then the wave totals in LDS
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  uint64_t incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) s_tmp[wave] = incl;
  __syncthreads();
  uint64_t before = 0, all = 0;
  for (int w = 0; w < kBlock / 64; w++) {
    if (w < wave) before += s_tmp[w];
    all += s_tmp[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

__global__ __launch_bounds__(kBlock) void k_densify_count(KDensify k) {
  __shared__ uint64_t s_tmp[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kItems;
  uint64_t sum = 0;
#pragma unroll
  for (int j = 0; j < kItems; j++)
    if (base + j < k.n) sum += (uint64_t)decide(k, base + j).c;
  uint64_t total;
  block_exclusive_sum(sum, s_tmp, &total);
  if (threadIdx.x == 0) k.block_sums[blockIdx.x] = total;
}

// exclusive scan of the block sums in place, the grand total after them
__global__ __launch_bounds__(1024) void k_densify_scan(uint64_t *sums, int64_t nb) {
  __shared__ uint64_t s_w[16];
  uint64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    const int64_t b = b0 + threadIdx.x;
    const uint64_t x = b < nb ? sums[b] : 0;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    uint64_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint64_t before = 0, all = 0;
    for (int w = 0; w < 16; w++) {
      if (w < wave) before += s_w[w];
      all += s_w[w];
    }
    if (b < nb) sums[b] = carry + before + incl - x;
    carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

// The two children's means of split Gaussian i at pos, pos + 1:
// mean + R(q / |q|) (exp(log_scale) * eps_j), in double, rounded once.
__device__ void child_means(const KDensify &k, int64_t i, int64_t pos) {
  const int64_t n = k.n, no = k.n_out;
  const double qw = k.quat[i], qx = k.quat[n + i], qy = k.quat[2 * n + i], qz = k.quat[3 * n + i];
  const double inv = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const double w = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
  const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
                       2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                       2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
  const double s[3] = {exp((double)k.ls[i]), exp((double)k.ls[n + i]), exp((double)k.ls[2 * n + i])};
  for (int j = 0; j < 2; j++) {
    double d[3];
#pragma unroll
    for (int a = 0; a < 3; a++) d[a] = s[a] * (double)k.samples[(int64_t)(j * 3 + a) * n + i];
#pragma unroll
    for (int a = 0; a < 3; a++)
      k.o_mean[a * no + pos + j] =
          (float)((double)k.mean[a * n + i] + R[3 * a] * d[0] + R[3 * a + 1] * d[1] + R[3 * a + 2] * d[2]);
  }
}

enum PlaneMode { kMeans, kLogScales, kCopied, kMoments };

// One plane of the block's Gaussians: consecutive lanes read consecutive
// Gaussians and write their outputs, which are consecutive too; the
// kItems loads of a thread are issued before its stores.  dec / pos: the
// thread's Gaussians (threadIdx.x + r kBlock), c = 0 for none.
template <int MODE>
__device__ __forceinline__ void copy_plane(const KDensify &k, const int *dec, const int64_t *pos, const float *src,
                                           float *dst) {
  float v[kItems];
#pragma unroll
  for (int r = 0; r < kItems; r++) {
    const bool load = (dec[r] & 3) != 0 && !(MODE == kMoments && (dec[r] >> 2) == 2);
    v[r] = load ? src[threadIdx.x + r * kBlock] : 0.0f;
  }
#pragma unroll
  for (int r = 0; r < kItems; r++) {
    const int c = dec[r] & 3, kind = dec[r] >> 2;
    // the children's means are written apart; a moment of a clone or a
    // child starts from zero
    const bool skip = MODE == kMeans && kind == 2;
    const float x = (MODE == kLogScales && kind == 2) ? v[r] - k.child_dlog : v[r];
    const float x1 = MODE == kMoments ? 0.0f : x;
    if (c != 0 && !skip) dst[pos[r]] = x;
    if (c == 2 && !skip) dst[pos[r] + 1] = x1;
  }
}

// Decisions and block-local offsets first (kItems consecutive Gaussians per
// thread, as in the count), kept in LDS; then plane by plane, each plane of
// the block's Gaussians read and written in contiguous runs.
__global__ __launch_bounds__(kBlock) void k_densify_apply(KDensify k) {
  __shared__ uint64_t s_tmp[kBlock / 64];
  __shared__ uint16_t s_off[kChunk];  // block-local output offset (< 2 kChunk)
  __shared__ uint8_t s_dec[kChunk];   // kind * 4 + c
  const int64_t first = (int64_t)blockIdx.x * kChunk;
  const int64_t base = first + (int64_t)threadIdx.x * kItems;
  uint8_t dec[kItems];
  uint64_t sum = 0;
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    const Decision d = base + j < k.n ? decide(k, base + j) : Decision{0, 0};
    dec[j] = (uint8_t)(d.kind * 4 + d.c);
    sum += (uint64_t)d.c;
  }
  uint64_t total;
  uint64_t off = block_exclusive_sum(sum, s_tmp, &total);
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    s_off[threadIdx.x * kItems + j] = (uint16_t)off;
    s_dec[threadIdx.x * kItems + j] = dec[j];
    off += dec[j] & 3;
  }
  __syncthreads();
  const int64_t bp = (int64_t)k.block_sums[blockIdx.x];
  const int count = (int)min((int64_t)kChunk, k.n - first);
  const int64_t n = k.n, no = k.n_out;
  // this thread's Gaussians for every plane, from LDS once
  int mdec[kItems];
  int64_t mpos[kItems];
#pragma unroll
  for (int r = 0; r < kItems; r++) {
    const int t = threadIdx.x + r * kBlock;
    mdec[r] = t < count ? s_dec[t] : 0;
    mpos[r] = t < count ? bp + s_off[t] : 0;
    if (mpos[r] + (mdec[r] & 3) > no) mdec[r] = 0;  // fewer outputs than counted: the caller's n_out is short
  }
  if (blockIdx.y == 0) {
#pragma unroll
    for (int r = 0; r < kItems; r++) {
      const int c = mdec[r] & 3;
      const int64_t i = first + threadIdx.x + r * kBlock;
      if (c == 0) continue;
      if ((mdec[r] >> 2) == 2) child_means(k, i, mpos[r]);  // split Gaussians (a minority)
      if (k.parent) {
        k.parent[mpos[r]] = i;
        if (c == 2) k.parent[mpos[r] + 1] = i;
      }
    }
  }
  // the planes, spread over the chunk's kPlaneSplit workgroups (plane number
  // u of the parameters, then of each moment when present, goes to the
  // workgroup u mod kPlaneSplit)
  int u = 0;
  const int y = blockIdx.y;
  constexpr int G = kPlaneSplit;  // gridDim.y
  for (int p = 0; p < 3; p++, u++)
    if (u % G == y) copy_plane<kMeans>(k, mdec, mpos, k.mean + p * n + first, k.o_mean + p * no);
  for (int p = 0; p < 3; p++, u++)
    if (u % G == y) copy_plane<kLogScales>(k, mdec, mpos, k.ls + p * n + first, k.o_ls + p * no);
  for (int p = 0; p < 4; p++, u++)
    if (u % G == y) copy_plane<kCopied>(k, mdec, mpos, k.quat + p * n + first, k.o_quat + p * no);
  if (u++ % G == y) copy_plane<kCopied>(k, mdec, mpos, k.opa + first, k.o_opa);
  for (int p = 0; p < k.sh_planes; p++, u++)
    if (u % G == y) copy_plane<kCopied>(k, mdec, mpos, k.sh + p * n + first, k.o_sh + p * no);
  if (!k.om[0]) return;
  const int rows[5] = {3, 3, 4, 1, k.sh_planes};
  for (int g = 0; g < 5; g++)
    for (int p = 0; p < rows[g]; p++) {
      if (u++ % G == y) copy_plane<kMoments>(k, mdec, mpos, k.m[g] + p * n + first, k.om[g] + p * no);
      if (u++ % G == y) copy_plane<kMoments>(k, mdec, mpos, k.v[g] + p * n + first, k.ov[g] + p * no);
    }
}

}  // namespace

int64_t densify_blocks(int64_t n) { return (n + kChunk - 1) / kChunk; }

int launch_densify_count(const KDensify &k, void *stream) {
  const int64_t nb = densify_blocks(k.n);
  hipStream_t s = (hipStream_t)stream;
  if (nb > 0) hipLaunchKernelGGL(k_densify_count, dim3((unsigned)nb), dim3(kBlock), 0, s, k);
  hipLaunchKernelGGL(k_densify_scan, dim3(1), dim3(1024), 0, s, k.block_sums, nb);
  return last_err();
}

int launch_densify_apply(const KDensify &k, void *stream) {
  const int64_t nb = densify_blocks(k.n);
  // each chunk's planes over kPlaneSplit workgroups: more loads in flight, at
  // the price of deciding each Gaussian kPlaneSplit times
  if (nb > 0)
    hipLaunchKernelGGL(k_densify_apply, dim3((unsigned)nb, kPlaneSplit), dim3(kBlock), 0, (hipStream_t)stream, k);
  return last_err();
}

}  // namespace gsr

// ---------------------------------------------------------------- C ABI

namespace {

gsr_status fill_densify(gsr::KDensify &k, int64_t n, int32_t sh_degree, const gsr_densify_opts *o,
                        const gsr_gaussians *g, const gsr_stats *stats, const uint8_t *in_block, void *ws,
                        size_t ws_bytes) {
  if (n < 0 || sh_degree < 0 || sh_degree > 3 || !o || !g || !stats || !ws) return GSR_ERR_INVALID_ARG;
  // the per-Gaussian arrays may be null when there are no Gaussians
  if (n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh ||
                !stats->grad2d_norm_sum || !stats->visible_count))
    return GSR_ERR_INVALID_ARG;
  if (n > 0 && o->selective && !in_block) return GSR_ERR_INVALID_ARG;
  if (std::isnan(o->grad_threshold) || !(o->clone_max_scale > 0.0f) || !(o->min_opacity >= 0.0f) ||
      !(o->min_opacity < 1.0f) || std::isnan(o->max_world_scale) || std::isinf(o->clone_max_scale))
    return GSR_ERR_INVALID_ARG;
  size_t need = 0;
  gsr_densify_workspace_size(n, &need);
  if (ws_bytes < need) return GSR_ERR_WORKSPACE_TOO_SMALL;
  k = gsr::KDensify{};
  k.mean = g->means;
  k.ls = g->log_scales;
  k.quat = g->quats;
  k.opa = g->opacity_logits;
  k.sh = g->sh;
  k.keep = g->keep;
  k.S = stats->grad2d_norm_sum;
  k.cnt = stats->visible_count;
  k.in_block = in_block;
  k.n = n;
  k.sh_planes = 3 * (sh_degree + 1) * (sh_degree + 1);
  k.selective = o->selective ? 1 : 0;
  k.grad_thr = (double)o->grad_threshold;
  k.log_clone_max = std::log((double)o->clone_max_scale);
  k.opa_on = o->min_opacity > 0.0f;
  k.logit_min = k.opa_on ? std::log((double)o->min_opacity / (1.0 - (double)o->min_opacity)) : 0.0;
  k.world_on = o->max_world_scale > 0.0f;
  k.log_world_max = k.world_on ? std::log((double)o->max_world_scale) : 0.0;
  k.child_dlog = (float)std::log(1.6);
  k.block_sums = (uint64_t *)(((uintptr_t)ws + 15) & ~(uintptr_t)15);
  return GSR_OK;
}

bool full(const gsr_grads *p) { return p && p->means && p->log_scales && p->quats && p->opacity_logits && p->sh; }

}  // namespace

extern "C" gsr_status gsr_densify_workspace_size(int64_t n, size_t *bytes) {
  if (n < 0 || !bytes) return GSR_ERR_INVALID_ARG;
  *bytes = 16 + 8 * (size_t)(gsr::densify_blocks(n) + 1);
  return GSR_OK;
}

extern "C" gsr_status gsr_densify_count(int64_t n, int32_t sh_degree, const gsr_densify_opts *opts,
                                        const gsr_gaussians *g, const gsr_stats *stats, const uint8_t *in_block,
                                        void *ws, size_t ws_bytes, void *stream, int64_t *n_out) {
  if (!n_out) return GSR_ERR_INVALID_ARG;
  gsr::KDensify k;
  const gsr_status st = fill_densify(k, n, sh_degree, opts, g, stats, in_block, ws, ws_bytes);
  if (st != GSR_OK) return st;
  if (gsr::launch_densify_count(k, stream)) return GSR_ERR_HIP;
  uint64_t total = 0;
  if (hipMemcpyAsync(&total, k.block_sums + gsr::densify_blocks(n), sizeof total, hipMemcpyDeviceToHost,
                     (hipStream_t)stream) != hipSuccess ||
      hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return GSR_ERR_HIP;
  *n_out = (int64_t)total;
  return GSR_OK;
}

extern "C" gsr_status gsr_densify_apply(int64_t n, int32_t sh_degree, const gsr_densify_opts *opts,
                                        const gsr_gaussians *g, const gsr_grads *m_in, const gsr_grads *v_in,
                                        const gsr_stats *stats, const uint8_t *in_block, const float *samples,
                                        int64_t n_out, const gsr_grads *out, const gsr_grads *m_out,
                                        const gsr_grads *v_out, int64_t *parent_out, void *ws, size_t ws_bytes,
                                        void *stream) {
  gsr::KDensify k;
  const gsr_status st = fill_densify(k, n, sh_degree, opts, g, stats, in_block, ws, ws_bytes);
  if (st != GSR_OK) return st;
  if (n_out < 0) return GSR_ERR_INVALID_ARG;
  if (n_out == 0 || n == 0) return GSR_OK;  // nothing to write
  if (!samples || !full(out)) return GSR_ERR_INVALID_ARG;
  const bool moments = m_out || v_out || m_in || v_in;
  if (moments && !(full(m_in) && full(v_in) && full(m_out) && full(v_out))) return GSR_ERR_INVALID_ARG;
  k.samples = samples;
  k.n_out = n_out;
  k.o_mean = out->means;
  k.o_ls = out->log_scales;
  k.o_quat = out->quats;
  k.o_opa = out->opacity_logits;
  k.o_sh = out->sh;
  k.parent = parent_out;
  if (moments) {
    const gsr_grads *io[4] = {m_in, v_in, m_out, v_out};
    for (int t = 0; t < 4; t++) {
      float *ptr[5] = {io[t]->means, io[t]->log_scales, io[t]->quats, io[t]->opacity_logits, io[t]->sh};
      for (int q = 0; q < 5; q++) {
        if (t == 0) k.m[q] = ptr[q];
        if (t == 1) k.v[q] = ptr[q];
        if (t == 2) k.om[q] = ptr[q];
        if (t == 3) k.ov[q] = ptr[q];
      }
    }
  }
  return gsr::launch_densify_apply(k, stream) ? GSR_ERR_HIP : GSR_OK;
}
