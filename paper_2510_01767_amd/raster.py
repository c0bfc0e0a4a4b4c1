"""Torch face of the rasterizer: device buffers, the C calls, autograd.

PyTorch supplies device memory and streams only; every step runs in
libgsr.so.  Layouts follow include/gsr.h: parameters are SoA float32 planes,
images/targets are per-view [3][H][W] blocks packed back to back, cameras a
[n_views][16] float32 device tensor (R row-major, t, fx, fy, cx, cy).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import gsr as C

PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


def camera_tensor(cameras, device="cuda") -> torch.Tensor:
    rows = []
    for c in cameras:
        rows.append(np.concatenate([np.asarray(c["R"], np.float32).ravel(), np.asarray(c["t"], np.float32),
                                    np.array([c["fx"], c["fy"], c["cx"], c["cy"]], np.float32)]))
    return torch.from_numpy(np.stack(rows).astype(np.float32)).to(device)


def pack_images(images) -> np.ndarray:
    return np.concatenate([np.ascontiguousarray(im, np.float32).ravel() for im in images])


def unpack_images(flat, sizes):
    out, o = [], 0
    for (W, H) in sizes:
        out.append(flat[o:o + 3 * W * H].reshape(3, H, W))
        o += 3 * W * H
    return out


def scene_tensors(scene, device="cuda") -> dict:
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
    return dict(means=t(scene.means), log_scales=t(scene.log_scales), quats=t(scene.quats),
                opacity_logits=t(scene.opacity_logits), sh=t(scene.sh))


def partition_blocks_device(scene_aabb, centers, points, view_offsets, n_blocks, tau=0.1, refine_steps=3,
                            q_min=0.1, q_max=0.9, stream=None):
    """gsr_partition_blocks_device: the KD-tree partition with the pixel counting on the GPU.
    points: float32 CUDA tensor [3][total]; the other inputs are host arrays.  Returns host
    (blocks [M][6], assign [M][V] uint8, workload [M])."""
    assert points.is_cuda and points.dtype == torch.float32 and points.is_contiguous() and points.shape[0] == 3
    n_views = len(view_offsets) - 1
    ws_bytes = C.gsr_partition_workspace_size(n_views)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=points.device)
    s = torch.cuda.current_stream(points.device) if stream is None else stream
    return C.gsr_partition_blocks_device(scene_aabb, centers, points.data_ptr(), view_offsets, n_blocks,
                                         ws.data_ptr(), ws_bytes, s.cuda_stream, tau, refine_steps, q_min, q_max)


def densify(params, S, count, samples, grad_threshold, clone_max_scale, min_opacity=0.0, max_world_scale=0.0,
            in_block=None, keep=None, m=None, v=None, stream=None):
    """gsr_densify_count + gsr_densify_apply on dicts of CUDA planes (PARAM_NAMES keys).
    Selective densification when in_block (uint8 [n]) is given.  Returns (params, m, v, parent)
    with m / v None unless given."""
    n = params["opacity_logits"].shape[-1]
    sh_degree = int(round((params["sh"].shape[0] // 3) ** 0.5)) - 1
    dev = params["means"].device
    opts = C.gsr_densify_opts(grad_threshold, clone_max_scale, min_opacity, max_world_scale,
                              1 if in_block is not None else 0, 0)
    g = Rasterizer.gaussians(params, keep)
    stats = C.gsr_stats(S.data_ptr(), count.data_ptr())
    ws_bytes = C.gsr_densify_workspace_size(n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    s = (torch.cuda.current_stream(dev) if stream is None else stream).cuda_stream
    blk = in_block.data_ptr() if in_block is not None else None
    n_out = C.gsr_densify_count(n, sh_degree, opts, g, stats, blk, ws.data_ptr(), ws_bytes, s)
    new = lambda: {k: torch.empty((params[k].shape[0], n_out) if params[k].dim() == 2 else (n_out,),
                                  dtype=torch.float32, device=dev) for k in PARAM_NAMES}
    out = new()
    mo, vo = (new(), new()) if m is not None else (None, None)
    parent = torch.empty(n_out, dtype=torch.int64, device=dev)
    gs = lambda d: C.gsr_grads(*[d[k].data_ptr() for k in PARAM_NAMES]) if d is not None else None
    C.gsr_densify_apply(n, sh_degree, opts, g, gs(m), gs(v), stats, blk, samples.data_ptr(), n_out, gs(out),
                        gs(mo), gs(vo), parent.data_ptr(), ws.data_ptr(), ws_bytes, s)
    return out, mo, vo, parent


class Rasterizer:
    """One plan + workspace for a fixed problem shape."""

    def __init__(self, n, sh_degree, sizes, mode="plain", tile=(16, 16), bwd="recompute", lds_batch=128,
                 grid_per_cu=4, capacity=0, history_budget=None, device="cuda", **conventions):
        self.n, self.sh_degree, self.sizes = int(n), int(sh_degree), [tuple(map(int, s)) for s in sizes]
        self.V = len(self.sizes)
        self.device = torch.device(device)
        if history_budget is None:
            # the stored blend history is used only where it fits in a quarter
            # of the device memory free now (otherwise the reverse pass
            # recomputes the transmittance)
            history_budget = torch.cuda.mem_get_info(self.device)[0] // 4 if torch.cuda.is_available() else 0
        # bumped by every call that rewrites the workspace; the autograd
        # functions compare it to catch a reverse pass whose forward state
        # was overwritten
        self.generation = 0
        o = C.gsr_default_options()
        o.mode = C.GSR_MODE_BATCHED if mode == "batched" else C.GSR_MODE_PLAIN
        o.tile_w, o.tile_h = tile
        o.bwd_variant = {"auto": C.GSR_BWD_AUTO, "recompute": C.GSR_BWD_RECOMPUTE,
                         "stored": C.GSR_BWD_STORED}[bwd]
        o.lds_batch, o.grid_per_cu = lds_batch, grid_per_cu
        o.capacity_intersections = int(capacity)
        o.history_budget_bytes = int(history_budget)
        for k, v in conventions.items():
            if k == "bg":
                o.bg = (ctypes.c_float * 3)(*v)
            else:
                setattr(o, k, v)
        self._W = (ctypes.c_int32 * self.V)(*[s[0] for s in self.sizes])
        self._H = (ctypes.c_int32 * self.V)(*[s[1] for s in self.sizes])
        self.problem = C.gsr_problem(self.n, self.sh_degree, self.V, self._W, self._H)
        self.plan = C.gsr_plan_create(self.problem, o)
        self.ws_bytes = C.gsr_workspace_size(self.plan)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        assert self.ws.data_ptr() % 256 == 0
        self.pixels = sum(W * H for W, H in self.sizes)
        self.images = torch.empty(3 * self.pixels, dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        K3 = 3 * (self.sh_degree + 1) ** 2
        z = lambda *s: torch.zeros(*s, dtype=torch.float32, device=self.device)
        self.grads = dict(means=z(3, self.n), log_scales=z(3, self.n), quats=z(4, self.n),
                          opacity_logits=z(self.n), sh=z(K3, self.n))
        self.S = z(self.n)
        self.count = torch.zeros(self.n, dtype=torch.int32, device=self.device)

    def __del__(self):
        try:
            if getattr(self, "plan", None):
                C.gsr_plan_destroy(self.plan)
                self.plan = None
        except Exception:
            pass

    # ------------------------------------------------------------ marshalling
    @staticmethod
    def gaussians(params, keep=None) -> C.gsr_gaussians:
        for k in PARAM_NAMES:
            assert params[k].is_contiguous() and params[k].dtype == torch.float32
        return C.gsr_gaussians(*[params[k].data_ptr() for k in PARAM_NAMES],
                               keep.data_ptr() if keep is not None else None)

    def grads_struct(self, grads=None) -> C.gsr_grads:
        g = self.grads if grads is None else grads
        return C.gsr_grads(*[g[k].data_ptr() for k in PARAM_NAMES])

    def stats_struct(self, stats=True):
        if not stats:
            return None
        return C.gsr_stats(self.S.data_ptr(), self.count.data_ptr())

    @staticmethod
    def stream_handle(stream=None):
        s = stream if stream is not None else torch.cuda.current_stream()
        return s.cuda_stream

    @property
    def options(self) -> C.gsr_options:
        return C.gsr_plan_options(self.plan)

    @property
    def layout(self) -> C.gsr_layout:
        return C.gsr_workspace_layout(self.plan)

    # ------------------------------------------------------------ the calls
    def step_l1(self, params, cams, targets, keep=None, stats=True, stream=None):
        """gsr_forward_backward_l1: returns (loss [1], images [3P]); gradients land in self.grads."""
        self.generation += 1
        C.gsr_forward_backward_l1(self.plan, self.gaussians(params, keep), cams.data_ptr(), targets.data_ptr(),
                                  self.images.data_ptr(), self.loss.data_ptr(), self.grads_struct(),
                                  self.stats_struct(stats), self.ws.data_ptr(), self.ws_bytes,
                                  self.stream_handle(stream))
        return self.loss, self.images

    def forward(self, params, cams, keep=None, T_final=None, last=None, images=None, stream=None):
        self.generation += 1
        img = self.images if images is None else images
        C.gsr_forward(self.plan, self.gaussians(params, keep), cams.data_ptr(), img.data_ptr(),
                      T_final.data_ptr() if T_final is not None else None,
                      last.data_ptr() if last is not None else None, self.ws.data_ptr(), self.ws_bytes,
                      self.stream_handle(stream))
        return img

    def backward(self, params, cams, dL_dimages, keep=None, grads=None, stats=True, stream=None):
        self.generation += 1
        C.gsr_backward(self.plan, self.gaussians(params, keep), cams.data_ptr(), dL_dimages.data_ptr(),
                       self.grads_struct(grads), self.stats_struct(stats), self.ws.data_ptr(), self.ws_bytes,
                       self.stream_handle(stream))
        return self.grads if grads is None else grads

    def visibility_mask(self, params, cams, aabb=None, keep=None, stream=None):
        self.generation += 1
        bits = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        keep_out = torch.zeros(self.n, dtype=torch.uint8, device=self.device)
        inb = torch.zeros(self.n, dtype=torch.uint8, device=self.device)
        C.gsr_visibility_mask(self.plan, self.gaussians(params, keep), cams.data_ptr(),
                              None if aabb is None else [float(x) for x in aabb], bits.data_ptr(),
                              keep_out.data_ptr(), inb.data_ptr() if aabb is not None else None,
                              self.ws.data_ptr(), self.ws_bytes, self.stream_handle(stream))
        return bits, keep_out, (inb if aabb is not None else None)

    def capture(self, params, cams, targets, keep=None, stats=True, stream=None):
        self.generation += 1
        C.gsr_graph_capture(self.plan, self.gaussians(params, keep), cams.data_ptr(), targets.data_ptr(),
                            self.images.data_ptr(), self.loss.data_ptr(), self.grads_struct(),
                            self.stats_struct(stats), self.ws.data_ptr(), self.ws_bytes,
                            self.stream_handle(stream))

    def launch(self, stream=None):
        self.generation += 1
        C.gsr_graph_launch(self.plan, self.stream_handle(stream))

    def counts(self, stream=None, check=True) -> C.gsr_counts:
        return C.gsr_query_counts(self.plan, self.ws.data_ptr(), self.stream_handle(stream), check)

    def autotune(self, params, cams, targets, reps=3, stream=None):
        self.generation += 1
        best, ms = C.gsr_autotune(self.plan, self.gaussians(params), cams.data_ptr(), targets.data_ptr(),
                                  self.images.data_ptr(), self.loss.data_ptr(), self.grads_struct(),
                                  self.ws.data_ptr(), self.ws_bytes, reps, self.stream_handle(stream))
        return best, ms

    def set_tuning(self, tile=None, bwd=None, lds_batch=None, grid_per_cu=None):
        o = self.options
        if tile is not None:
            o.tile_w, o.tile_h = tile
        if bwd is not None:
            o.bwd_variant = {"auto": C.GSR_BWD_AUTO, "recompute": C.GSR_BWD_RECOMPUTE,
                             "stored": C.GSR_BWD_STORED}[bwd]
        if lds_batch is not None:
            o.lds_batch = lds_batch
        if grid_per_cu is not None:
            o.grid_per_cu = grid_per_cu
        C.gsr_plan_set_tuning(self.plan, o)

    def render_depth(self, params, cams, keep=None, images=None, stream=None):
        """gsr_render_depth: (images [3P], depth [P]) with D = sum_i d_i alpha_i T_i per pixel."""
        self.generation += 1
        img = self.images if images is None else images
        depth = torch.empty(self.pixels, dtype=torch.float32, device=self.device)
        C.gsr_render_depth(self.plan, self.gaussians(params, keep), cams.data_ptr(), img.data_ptr(),
                           depth.data_ptr(), self.ws.data_ptr(), self.ws_bytes, self.stream_handle(stream))
        return img, depth

    def pair_counts(self, params, cams, keep=None, images=None, stream=None):
        """gsr_pair_counts (profiling): per pixel, the pairs blended and the pairs evaluated
        after the culling; returns (blended [P], evaluated [P]) as int32 views of u32."""
        self.generation += 1
        img = self.images if images is None else images
        counts = torch.empty(2 * self.pixels, dtype=torch.int32, device=self.device)
        C.gsr_pair_counts(self.plan, self.gaussians(params, keep), cams.data_ptr(), img.data_ptr(),
                          counts.data_ptr(), self.ws.data_ptr(), self.ws_bytes, self.stream_handle(stream))
        return counts[:self.pixels], counts[self.pixels:]

    def camera_coverage(self, cams, depth, blocks, tau=0.1, stream=None):
        """gsr_camera_coverage: counts [V][M] (int32 view of u32), ratio V_{c,b} [V][M], selected [V][M]."""
        assert blocks.dtype == torch.float32 and blocks.is_contiguous() and blocks.shape[-1] == 6
        M = blocks.shape[0]
        counts = torch.empty((self.V, M), dtype=torch.int32, device=self.device)
        ratio = torch.empty((self.V, M), dtype=torch.float32, device=self.device)
        selected = torch.empty((self.V, M), dtype=torch.uint8, device=self.device)
        C.gsr_camera_coverage(self.plan, cams.data_ptr(), depth.data_ptr(), blocks.data_ptr(), M, float(tau),
                              counts.data_ptr(), ratio.data_ptr(), selected.data_ptr(), self.stream_handle(stream))
        return counts, ratio, selected

    def back_project(self, cams, depth, stream=None):
        """gsr_back_project: the world points [3][P] of every pixel's composited depth."""
        points = torch.empty((3, self.pixels), dtype=torch.float32, device=self.device)
        C.gsr_back_project(self.plan, cams.data_ptr(), depth.data_ptr(), points.data_ptr(), self.stream_handle(stream))
        return points

    def adam_step(self, params, grads, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-15, visible_only=False,
                  stream=None):
        """gsr_adam_step on parameter / gradient / moment dicts (PARAM_NAMES keys).  lr: six learning
        rates (means, log_scales, quats, opacity_logits, SH band 0, SH bands >= 1).  visible_only:
        update only the Gaussians visible in this plan's last step (its workspace view masks)."""
        hp = C.gsr_adam((ctypes.c_float * 6)(*lr), beta1, beta2, eps, int(step))
        bits = self.ws.data_ptr() + self.layout.view_bits if visible_only else None
        C.gsr_adam_step(self.plan, hp, self.grads_struct(params), self.grads_struct(grads), self.grads_struct(m),
                        self.grads_struct(v), bits, self.stream_handle(stream))

    # ------------------------------------------------------------ workspace views
    def ws_tensor(self, field, dtype, count):
        off = getattr(self.layout, field)
        nbytes = count * torch.tensor([], dtype=dtype).element_size()
        return self.ws[off:off + nbytes].view(dtype)

    def image_list(self, flat=None):
        return unpack_images(self.images if flat is None else flat, self.sizes)


class RasterizeL1Fn(torch.autograd.Function):
    """L1 training step as an autograd op: forward runs the fused
    gsr_forward_backward_l1 and keeps its gradients (copies, so later calls
    on the same Rasterizer do not change them); backward scales them by the
    incoming gradient of the loss.  The images are a non-differentiable side
    output.  The step's capacity and finiteness flags are checked before
    returning (one synchronisation): an overflowing step raises GsrError."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, rast: Rasterizer, cams, targets):
        params = dict(means=means.contiguous(), log_scales=log_scales.contiguous(), quats=quats.contiguous(),
                      opacity_logits=opacity_logits.contiguous(), sh=sh.contiguous())
        loss, images = rast.step_l1(params, cams, targets)
        rast.counts()
        g = [rast.grads[k].clone() for k in PARAM_NAMES]
        ctx.save_for_backward(*g)
        ctx.mark_non_differentiable(images)
        return loss.clone()[0], images.clone()

    @staticmethod
    def backward(ctx, grad_loss, grad_images):
        g = ctx.saved_tensors
        return tuple(x * grad_loss for x in g) + (None, None, None)


class StaleForwardError(RuntimeError):
    """The reverse pass of a render whose forward state (kept in the
    Rasterizer's workspace) was overwritten by a later call."""


class RasterizeFn(torch.autograd.Function):
    """Images as a differentiable function of the parameters (gsr_forward /
    gsr_backward with an arbitrary image gradient).

    The reverse pass reads the forward's state from the Rasterizer's
    workspace (records, tile lists, per-pixel T_final and `last`).  Each
    render stamps the Rasterizer's generation; backward raises
    StaleForwardError if any call rewrote the workspace since, rather than
    returning gradients of another render.  One Rasterizer per render that
    must stay differentiable (or backward before the next render) avoids it.
    The capacity and finiteness flags are checked before returning."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, rast: Rasterizer, cams):
        params = dict(means=means.contiguous(), log_scales=log_scales.contiguous(), quats=quats.contiguous(),
                      opacity_logits=opacity_logits.contiguous(), sh=sh.contiguous())
        img = rast.forward(params, cams).clone()
        rast.counts()
        ctx.rast, ctx.params, ctx.cams = rast, params, cams
        ctx.generation = rast.generation
        return img

    @staticmethod
    def backward(ctx, grad_images):
        rast = ctx.rast
        if rast.generation != ctx.generation:
            raise StaleForwardError("the Rasterizer's workspace was rewritten after this render's forward "
                                    f"(generation {ctx.generation} -> {rast.generation}); its reverse pass "
                                    "cannot run")
        grads = rast.backward(ctx.params, ctx.cams, grad_images.contiguous())
        return tuple(grads[k].clone() for k in PARAM_NAMES) + (None, None)


def render_l1(params, rast: Rasterizer, cams, targets):
    """(loss, images) with loss differentiable w.r.t. the five parameter tensors."""
    return RasterizeL1Fn.apply(params["means"], params["log_scales"], params["quats"], params["opacity_logits"],
                               params["sh"], rast, cams, targets)


def render(params, rast: Rasterizer, cams):
    return RasterizeFn.apply(params["means"], params["log_scales"], params["quats"], params["opacity_logits"],
                             params["sh"], rast, cams)
