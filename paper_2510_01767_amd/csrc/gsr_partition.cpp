// Load-balanced KD-tree scene partition with cutline refinement (Sec. 3.1,
// App. A.5).  The tree is grown on the host, best-first: the leaf with the
// most cameras is split along the longer of its x / y extents, at a
// percentile of the Gaussian centres it holds; a bisection on the percentile
// within [q_min, q_max] moves the cut toward the heavier child.  Each child's
// cameras are those of the parent whose back-projected pixels fall into it
// with a ratio of at least tau (fast camera selection, Sec. 3.2).
//
// Counting pixels into candidate boxes is the only part that touches the
// pixels.  gsr_partition_blocks counts on the host, one evaluated split at a
// time; gsr_partition_blocks_device counts on the GPU, from points resident
// in device memory, and evaluates every percentile the bisection can reach
// (2^steps - 1 of them) for both children in one pass per split, then walks
// the bisection over that table.  Both count the same float32 points with
// the same comparisons, so their results are identical.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <queue>
#include <vector>

#include "gsr.h"
#include "gsr_internal.h"
#include "gsr_stages.h"

namespace {

struct Node {
  float box[6];              // xmin ymin zmin xmax ymax zmax, half-open
  std::vector<int> cams;     // ascending camera ids
  std::vector<int64_t> pts;  // Gaussian centres inside the box
  int64_t id;                // creation order
};

bool inside(const float *b, float x, float y, float z) {
  return x >= b[0] && x < b[3] && y >= b[1] && y < b[4] && z >= b[2] && z < b[5];
}

// count / n_pix >= tau, exactly: tau * n_pix is exact in double (24-bit
// mantissa times an integer below 2^29).
bool selected(int64_t count, int64_t n_pix, float tau) {
  return n_pix > 0 && (double)count >= (double)tau * (double)n_pix;
}

struct Input {
  const float *centers;
  int64_t n;
  const int64_t *offsets;
  int n_views;
  float tau;
};

// The bisection's reachable percentiles as a complete binary tree: node k
// holds q; child 2k + 1 follows "left heavier" (q_high = q, q = (q_low + q)/2),
// child 2k + 2 "right heavier" (q_low = q, q = (q_high + q)/2).
std::vector<double> percentile_tree(int steps, double q_min, double q_max) {
  const int64_t count = ((int64_t)1 << steps) - 1;
  std::vector<double> q(count), lo(count), hi(count);
  q[0] = 0.5;
  lo[0] = q_min;
  hi[0] = q_max;
  for (int64_t k = 0; 2 * k + 2 < count; k++) {
    q[2 * k + 1] = 0.5 * (lo[k] + q[k]);
    lo[2 * k + 1] = lo[k];
    hi[2 * k + 1] = q[k];
    q[2 * k + 2] = 0.5 * (hi[k] + q[k]);
    lo[2 * k + 2] = q[k];
    hi[2 * k + 2] = hi[k];
  }
  return q;
}

// Order statistics of a at the sorted, distinct indices idx[lo, hi), the
// range [first, last) of a holding them, by recursive selection.
void order_stats(std::vector<float> &a, int64_t first, int64_t last, const std::vector<int64_t> &idx, size_t lo,
                 size_t hi, std::vector<float> &out) {
  if (lo >= hi) return;
  const size_t mid = (lo + hi) / 2;
  const int64_t k = idx[mid];
  std::nth_element(a.begin() + first, a.begin() + k, a.begin() + last);
  out[mid] = a[k];
  order_stats(a, first, k, idx, lo, mid, out);
  order_stats(a, k + 1, last, idx, mid + 1, hi, out);
}

// Counts, per camera of `cams` and per box, of that camera's pixels inside
// the box: counts[j * nb + b].
struct HostCounter {
  const float *xyz;  // [3][total]
  int64_t total;
  const int64_t *offsets;
  gsr_status operator()(const std::vector<int> &cams, const float *boxes, int nb, std::vector<int64_t> &counts) {
    counts.assign(cams.size() * (size_t)nb, 0);
    for (size_t j = 0; j < cams.size(); j++)
      for (int64_t k = offsets[cams[j]]; k < offsets[cams[j] + 1]; k++) {
        const float x = xyz[k], y = xyz[total + k], z = xyz[2 * total + k];
        for (int b = 0; b < nb; b++) counts[j * nb + b] += inside(boxes + 6 * b, x, y, z) ? 1 : 0;
      }
    return GSR_OK;
  }
};

struct DeviceCounter {
  const float *xyz;  // device [3][total]
  int64_t total;
  const int64_t *offsets;  // host
  int n_views;
  char *ws;  // device
  hipStream_t stream;
  std::vector<uint32_t> h_counts;
  std::vector<gsr::PartitionView> h_list;

  gsr_status operator()(const std::vector<int> &cams, const float *boxes, int nb, std::vector<int64_t> &counts) {
    counts.assign(cams.size() * (size_t)nb, 0);
    if (cams.empty()) return GSR_OK;
    const gsr::PartitionWs w = gsr::partition_ws(ws, n_views);
    h_list.resize(cams.size());
    int64_t pmax = 1;
    for (size_t j = 0; j < cams.size(); j++) {
      h_list[j].first = offsets[cams[j]];
      h_list[j].count = offsets[cams[j] + 1] - offsets[cams[j]];
      pmax = std::max(pmax, h_list[j].count);
    }
    h_counts.resize(cams.size() * (size_t)nb);
    if (hipMemcpyAsync(w.views, h_list.data(), cams.size() * sizeof(gsr::PartitionView), hipMemcpyHostToDevice,
                       stream) != hipSuccess ||
        hipMemcpyAsync(w.boxes, boxes, (size_t)nb * 6 * sizeof(float), hipMemcpyHostToDevice, stream) != hipSuccess)
      return GSR_ERR_HIP;
    if (gsr::launch_count_points(xyz, total, w.views, (int)cams.size(), pmax, w.boxes, nb, w.counts, stream))
      return GSR_ERR_HIP;
    if (hipMemcpyAsync(h_counts.data(), w.counts, h_counts.size() * sizeof(uint32_t), hipMemcpyDeviceToHost,
                       stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return GSR_ERR_HIP;
    for (size_t k = 0; k < h_counts.size(); k++) counts[k] = h_counts[k];
    return GSR_OK;
  }
};

gsr_status check_args(const float *scene_aabb, const float *centers, int64_t n, const float *points,
                      const int64_t *view_offsets, int32_t n_views, int32_t n_blocks, float tau, int32_t refine_steps,
                      float q_min, float q_max, const float *blocks_out) {
  if (!scene_aabb || (!centers && n > 0) || !points || !view_offsets || !blocks_out || n < 0 || n_views < 1 ||
      n_blocks < 1 || refine_steps < 1 || refine_steps > GSR_MAX_REFINE_STEPS ||
      !(q_min > 0.0f && q_min < q_max && q_max < 1.0f) || !std::isfinite(tau))
    return GSR_ERR_INVALID_ARG;
  if (view_offsets[0] != 0) return GSR_ERR_INVALID_ARG;
  for (int v = 0; v < n_views; v++)
    if (view_offsets[v + 1] < view_offsets[v]) return GSR_ERR_INVALID_ARG;
  return GSR_OK;
}

// Alg. 1 with the camera selection of each candidate child by `count`.
// Eager: all reachable percentiles of a split in one call; else one call
// per evaluated split.
template <class Counter>
gsr_status partition(const Input &in, const float *scene_aabb, int n_blocks, int steps, float q_min, float q_max,
                     bool eager, Counter &count, float *blocks_out, uint8_t *assign_out, int32_t *workload_out) {
  const std::vector<double> qtree = percentile_tree(steps, q_min, q_max);
  auto lighter = [](const Node *a, const Node *b) {  // max-heap; equal workloads: earliest node first
    if (a->cams.size() != b->cams.size()) return a->cams.size() < b->cams.size();
    return a->id > b->id;
  };
  std::vector<std::unique_ptr<Node>> all;
  std::priority_queue<Node *, std::vector<Node *>, decltype(lighter)> pq(lighter);
  all.emplace_back(new Node());
  Node *root = all.back().get();
  std::memcpy(root->box, scene_aabb, sizeof root->box);
  for (int c = 0; c < in.n_views; c++) root->cams.push_back(c);
  const float *C = in.centers;
  for (int64_t i = 0; i < in.n; i++)
    if (inside(root->box, C[i], C[in.n + i], C[2 * in.n + i])) root->pts.push_back(i);
  root->id = 0;
  pq.push(root);
  int64_t next_id = 1;
  std::vector<float> coord, boxes, cuts;
  std::vector<int64_t> counts, idx;
  std::vector<int> cams_l, cams_r;

  while ((int32_t)pq.size() < n_blocks) {
    Node *p = pq.top();
    pq.pop();
    const int a = (p->box[3] - p->box[0]) >= (p->box[4] - p->box[1]) ? 0 : 1;
    const int64_t m = (int64_t)p->pts.size();
    // the cut at percentile q: the order statistic of index floor(q (m - 1))
    // of the node's centres along a, or the extent's middle for m = 0
    const size_t nq = eager ? qtree.size() : 0;
    std::vector<float> cut_of(qtree.size());
    if (m == 0) {
      std::fill(cut_of.begin(), cut_of.end(), 0.5f * (p->box[a] + p->box[3 + a]));
    } else {
      coord.resize(m);
      for (int64_t j = 0; j < m; j++) coord[j] = C[(int64_t)a * in.n + p->pts[j]];
      idx.clear();
      for (double q : qtree) idx.push_back((int64_t)std::floor(q * (double)(m - 1)));
      std::vector<int64_t> uniq(idx);
      std::sort(uniq.begin(), uniq.end());
      uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
      cuts.assign(uniq.size(), 0.0f);
      order_stats(coord, 0, m, uniq, 0, uniq.size(), cuts);
      for (size_t k = 0; k < qtree.size(); k++)
        cut_of[k] = cuts[std::lower_bound(uniq.begin(), uniq.end(), idx[k]) - uniq.begin()];
    }
    auto child_boxes = [&](float cut, float *l, float *r) {
      std::memcpy(l, p->box, 6 * sizeof(float));
      std::memcpy(r, p->box, 6 * sizeof(float));
      l[3 + a] = cut;
      r[a] = cut;
    };
    auto select = [&](const int64_t *cnt_l, const int64_t *cnt_r, int stride) {
      cams_l.clear();
      cams_r.clear();
      for (size_t j = 0; j < p->cams.size(); j++) {
        const int c = p->cams[j];
        const int64_t np = in.offsets[c + 1] - in.offsets[c];
        if (selected(cnt_l[j * stride], np, in.tau)) cams_l.push_back(c);
        if (selected(cnt_r[j * stride], np, in.tau)) cams_r.push_back(c);
      }
    };
    if (eager) {
      boxes.resize(12 * nq);
      for (size_t k = 0; k < nq; k++) child_boxes(cut_of[k], &boxes[12 * k], &boxes[12 * k + 6]);
      const gsr_status st = count(p->cams, boxes.data(), (int)(2 * nq), counts);
      if (st != GSR_OK) return st;
    }
    float box_l[6], box_r[6];
    int64_t k = 0;  // node of the percentile tree being evaluated
    for (int it = 0; it < steps; it++) {
      child_boxes(cut_of[k], box_l, box_r);
      if (eager) {
        select(&counts[2 * k], &counts[2 * k + 1], (int)(2 * nq));
      } else {
        float pair[12];
        std::memcpy(pair, box_l, sizeof box_l);
        std::memcpy(pair + 6, box_r, sizeof box_r);
        const gsr_status st = count(p->cams, pair, 2, counts);
        if (st != GSR_OK) return st;
        select(&counts[0], &counts[1], 2);
      }
      if (cams_l.size() > cams_r.size())
        k = 2 * k + 1;
      else if (cams_r.size() > cams_l.size())
        k = 2 * k + 2;
      else
        break;
    }
    // the children of the last evaluated split
    all.emplace_back(new Node());
    Node *L = all.back().get();
    all.emplace_back(new Node());
    Node *R = all.back().get();
    std::memcpy(L->box, box_l, sizeof box_l);
    std::memcpy(R->box, box_r, sizeof box_r);
    L->cams = cams_l;
    R->cams = cams_r;
    for (int64_t i : p->pts) (C[(int64_t)a * in.n + i] < box_l[3 + a] ? L->pts : R->pts).push_back(i);
    p->pts = std::vector<int64_t>();
    L->id = next_id++;
    R->id = next_id++;
    pq.push(L);
    pq.push(R);
  }
  std::vector<Node *> leaves;
  while (!pq.empty()) {
    leaves.push_back(pq.top());
    pq.pop();
  }
  std::sort(leaves.begin(), leaves.end(), [](const Node *x, const Node *y) { return x->id < y->id; });
  for (int b = 0; b < n_blocks; b++) {
    std::memcpy(blocks_out + 6 * b, leaves[b]->box, 6 * sizeof(float));
    if (workload_out) workload_out[b] = (int32_t)leaves[b]->cams.size();
    if (assign_out) {
      std::memset(assign_out + (int64_t)b * in.n_views, 0, (size_t)in.n_views);
      for (int c : leaves[b]->cams) assign_out[(int64_t)b * in.n_views + c] = 1;
    }
  }
  return GSR_OK;
}

}  // namespace

extern "C" gsr_status gsr_partition_blocks(const float *scene_aabb, const float *centers, int64_t n,
                                           const float *points, const int64_t *view_offsets, int32_t n_views,
                                           int32_t n_blocks, float tau, int32_t refine_steps, float q_min,
                                           float q_max, float *blocks_out, uint8_t *assign_out,
                                           int32_t *workload_out) {
  const gsr_status st = check_args(scene_aabb, centers, n, points, view_offsets, n_views, n_blocks, tau,
                                   refine_steps, q_min, q_max, blocks_out);
  if (st != GSR_OK) return st;
  const Input in{centers, n, view_offsets, n_views, tau};
  HostCounter count{points, view_offsets[n_views], view_offsets};
  return partition(in, scene_aabb, n_blocks, refine_steps, q_min, q_max, false, count, blocks_out, assign_out,
                   workload_out);
}

extern "C" gsr_status gsr_partition_workspace_size(int32_t n_views, size_t *bytes) {
  if (n_views < 1 || !bytes) return GSR_ERR_INVALID_ARG;
  *bytes = gsr::partition_ws_bytes(n_views);
  return GSR_OK;
}

extern "C" gsr_status gsr_partition_blocks_device(const float *scene_aabb, const float *centers, int64_t n,
                                                  const float *points, const int64_t *view_offsets, int32_t n_views,
                                                  int32_t n_blocks, float tau, int32_t refine_steps, float q_min,
                                                  float q_max, void *ws, size_t ws_bytes, void *stream,
                                                  float *blocks_out, uint8_t *assign_out, int32_t *workload_out) {
  const gsr_status st = check_args(scene_aabb, centers, n, points, view_offsets, n_views, n_blocks, tau,
                                   refine_steps, q_min, q_max, blocks_out);
  if (st != GSR_OK) return st;
  if (!ws || ws_bytes < gsr::partition_ws_bytes(n_views)) return GSR_ERR_WORKSPACE_TOO_SMALL;
  const Input in{centers, n, view_offsets, n_views, tau};
  DeviceCounter count{points, view_offsets[n_views], view_offsets, n_views, (char *)ws, (hipStream_t)stream, {}, {}};
  // every reachable percentile's two children in one pass when the boxes fit
  const bool eager = 2 * (((int64_t)1 << refine_steps) - 1) <= GSR_MAX_COVERAGE_BLOCKS;
  return partition(in, scene_aabb, n_blocks, refine_steps, q_min, q_max, eager, count, blocks_out, assign_out,
                   workload_out);
}
