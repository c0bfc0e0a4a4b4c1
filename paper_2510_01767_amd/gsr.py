"""ctypes binding of libgsr.so (the C ABI declared in include/gsr.h).

Argument marshalling only: every step of the rasterizer runs in the HIP
kernels of the library.  The functions below carry the C names; device
buffers are passed as integer addresses (``tensor.data_ptr()``) and streams
as ``hipStream_t`` handles (``torch.cuda.current_stream().cuda_stream``).
If the library is missing it is built once with hipcc; if that is impossible
the import fails loudly - there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# GSR_LIBRARY selects another build of the same library (e.g. one whose host
# code carries sanitizers); the default is the in-tree libgsr.so.
LIB_PATH = os.environ.get("GSR_LIBRARY") or os.path.join(HERE, "libgsr.so")

GSR_OK = 0
GSR_ERR_INVALID_ARG = 1
GSR_ERR_WORKSPACE_TOO_SMALL = 2
GSR_ERR_CAPACITY = 3
GSR_ERR_NONFINITE = 4
GSR_ERR_HIP = 5
GSR_ERR_STATE = 6
GSR_MAX_VIEWS = 32
GSR_SLOT_FLOATS = 16
GSR_MAX_COVERAGE_BLOCKS = 1024
GSR_MAX_REFINE_STEPS = 16
GSR_MODE_PLAIN = 0
GSR_MODE_BATCHED = 1
GSR_BWD_AUTO = 0
GSR_BWD_RECOMPUTE = 1
GSR_BWD_STORED = 2

_i32, _i64, _f32, _vp, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t


class gsr_camera(ctypes.Structure):
    _fields_ = [("R", _f32 * 9), ("t", _f32 * 3), ("fx", _f32), ("fy", _f32), ("cx", _f32), ("cy", _f32)]


class gsr_options(ctypes.Structure):
    _fields_ = [
        ("mode", _i32), ("tile_w", _i32), ("tile_h", _i32), ("bwd_variant", _i32),
        ("lds_batch", _i32), ("grid_per_cu", _i32), ("accumulate_grads", _i32), ("check_finite", _i32),
        ("profile_stages", _i32), ("bwd_reduce", _i32), ("project_table", _i32), ("near_plane", _f32), ("far_plane", _f32), ("eps2d", _f32), ("sigma_extent", _f32),
        ("jac_clamp", _f32), ("alpha_min", _f32), ("alpha_max", _f32), ("T_min", _f32),
        ("bg", _f32 * 3), ("stat_scale", _f32),
        ("capacity_intersections", _i64), ("history_budget_bytes", _i64),
    ]


class gsr_problem(ctypes.Structure):
    _fields_ = [("n", _i64), ("sh_degree", _i32), ("n_views", _i32),
                ("widths", ctypes.POINTER(_i32)), ("heights", ctypes.POINTER(_i32))]


class gsr_gaussians(ctypes.Structure):
    _fields_ = [("means", _vp), ("log_scales", _vp), ("quats", _vp), ("opacity_logits", _vp),
                ("sh", _vp), ("keep", _vp)]


class gsr_grads(ctypes.Structure):
    _fields_ = [("means", _vp), ("log_scales", _vp), ("quats", _vp), ("opacity_logits", _vp), ("sh", _vp)]


class gsr_stats(ctypes.Structure):
    _fields_ = [("grad2d_norm_sum", _vp), ("visible_count", _vp)]


class gsr_densify_opts(ctypes.Structure):
    _fields_ = [("grad_threshold", _f32), ("clone_max_scale", _f32), ("min_opacity", _f32),
                ("max_world_scale", _f32), ("selective", _i32), ("reserved", _i32)]


class gsr_counts(ctypes.Structure):
    _fields_ = [("visible", _i64 * GSR_MAX_VIEWS), ("intersections", _i64 * GSR_MAX_VIEWS),
                ("visible_total", _i64), ("intersections_total", _i64), ("visible_union", _i64),
                ("overflow", _i32), ("nonfinite", _i32), ("tile_w", _i32), ("tile_h", _i32),
                ("bwd_variant", _i32), ("lds_batch", _i32), ("grid_per_cu", _i32), ("mode", _i32)]


class gsr_layout(ctypes.Structure):
    _fields_ = [(k, _sz) for k in ("header", "view_table", "view_bits", "records", "grad2d", "tile_count",
                                   "tile_start", "tile_fill", "tile_loss", "tile_order", "keys", "keys_alt",
                                   "pix_T", "pix_last", "pix_dLdC", "history", "total")] + \
               [(k, _i64) for k in ("vn", "tiles_total", "pixels_total", "capacity", "history_entries")]


GSR_MAX_STAGES = 16


class gsr_stage_times(ctypes.Structure):
    _fields_ = [("count", _i32), ("launches", _i32 * GSR_MAX_STAGES), ("ms", _f32 * GSR_MAX_STAGES),
                ("name", (ctypes.c_char * 32) * GSR_MAX_STAGES)]

    def as_dict(self) -> dict:
        return {self.name[k].value.decode(): (float(self.ms[k]), int(self.launches[k])) for k in range(self.count)}


class gsr_adam(ctypes.Structure):
    _fields_ = [("lr", _f32 * 6), ("beta1", _f32), ("beta2", _f32), ("eps", _f32), ("step", _i32)]


EXPORTS = (
    "gsr_last_stage_times", "gsr_adam_step", "gsr_render_depth", "gsr_pair_counts", "gsr_camera_coverage",
    "gsr_back_project", "gsr_forward_backward_l1_static",
    "gsr_partition_blocks", "gsr_partition_workspace_size", "gsr_partition_blocks_device",
    "gsr_densify_workspace_size", "gsr_densify_count", "gsr_densify_apply",
    "gsr_default_options", "gsr_plan_create", "gsr_plan_destroy", "gsr_workspace_size",
    "gsr_workspace_layout", "gsr_image_offset", "gsr_forward", "gsr_backward",
    "gsr_forward_backward_l1", "gsr_visibility_mask", "gsr_graph_capture", "gsr_graph_launch",
    "gsr_query_counts", "gsr_autotune", "gsr_plan_options", "gsr_plan_set_tuning",
    "gsr_status_string", "gsr_last_error",
)

_lib = None


def load(build_if_missing: bool = True):
    """Loads libgsr.so (building it first if it does not exist)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise RuntimeError(f"{LIB_PATH} is not built")
        from . import build as _build
        _build.build()
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.gsr_default_options.argtypes = [P(gsr_options)]
    L.gsr_default_options.restype = None
    L.gsr_plan_create.argtypes = [P(_vp), P(gsr_problem), P(gsr_options)]
    L.gsr_plan_destroy.argtypes = [_vp]
    L.gsr_workspace_size.argtypes = [_vp, P(_sz)]
    L.gsr_workspace_layout.argtypes = [_vp, P(gsr_layout)]
    L.gsr_image_offset.argtypes = [_vp, _i32, P(_i64)]
    L.gsr_forward.argtypes = [_vp, P(gsr_gaussians), _vp, _vp, _vp, _vp, _vp, _sz, _vp]
    L.gsr_backward.argtypes = [_vp, P(gsr_gaussians), _vp, _vp, P(gsr_grads), P(gsr_stats), _vp, _sz, _vp]
    L.gsr_forward_backward_l1.argtypes = [_vp, P(gsr_gaussians), _vp, _vp, _vp, _vp, P(gsr_grads),
                                          P(gsr_stats), _vp, _sz, _vp]
    L.gsr_visibility_mask.argtypes = [_vp, P(gsr_gaussians), _vp, P(_f32), _vp, _vp, _vp, _vp, _sz, _vp]
    L.gsr_graph_capture.argtypes = [_vp, P(gsr_gaussians), _vp, _vp, _vp, _vp, P(gsr_grads), P(gsr_stats),
                                    _vp, _sz, _vp]
    L.gsr_graph_launch.argtypes = [_vp, _vp]
    L.gsr_query_counts.argtypes = [_vp, _vp, P(gsr_counts), _vp]
    L.gsr_autotune.argtypes = [_vp, P(gsr_gaussians), _vp, _vp, _vp, _vp, P(gsr_grads), _vp, _sz, _i32,
                               P(gsr_options), P(_f32), _vp]
    L.gsr_last_stage_times.argtypes = [_vp, P(gsr_stage_times)]
    L.gsr_back_project.argtypes = [_vp, _vp, _vp, _vp, _vp]
    L.gsr_partition_blocks.argtypes = [P(_f32), P(_f32), _i64, P(_f32), P(_i64), _i32, _i32, _f32, _i32, _f32,
                                       _f32, P(_f32), P(ctypes.c_uint8), P(_i32)]
    L.gsr_partition_workspace_size.argtypes = [_i32, P(_sz)]
    L.gsr_partition_blocks_device.argtypes = [P(_f32), P(_f32), _i64, _vp, P(_i64), _i32, _i32, _f32, _i32, _f32,
                                              _f32, _vp, _sz, _vp, P(_f32), P(ctypes.c_uint8), P(_i32)]
    L.gsr_densify_workspace_size.argtypes = [_i64, P(_sz)]
    L.gsr_densify_count.argtypes = [_i64, _i32, P(gsr_densify_opts), P(gsr_gaussians), P(gsr_stats), _vp, _vp, _sz,
                                    _vp, P(_i64)]
    L.gsr_densify_apply.argtypes = [_i64, _i32, P(gsr_densify_opts), P(gsr_gaussians), P(gsr_grads), P(gsr_grads),
                                    P(gsr_stats), _vp, _vp, _i64, P(gsr_grads), P(gsr_grads), P(gsr_grads), _vp,
                                    _vp, _sz, _vp]
    L.gsr_render_depth.argtypes = [_vp, P(gsr_gaussians), _vp, _vp, _vp, _vp, _sz, _vp]
    L.gsr_pair_counts.argtypes = [_vp, P(gsr_gaussians), _vp, _vp, _vp, _vp, _sz, _vp]
    L.gsr_forward_backward_l1_static.argtypes = [_vp, P(gsr_gaussians), _vp, _vp, _vp, _vp, P(gsr_grads),
                                                 P(gsr_stats), _vp]
    L.gsr_camera_coverage.argtypes = [_vp, _vp, _vp, _vp, _i32, _f32, _vp, _vp, _vp, _vp]
    L.gsr_adam_step.argtypes = [_vp, P(gsr_adam), P(gsr_grads), P(gsr_grads), P(gsr_grads), P(gsr_grads), _vp,
                                _vp]
    L.gsr_plan_options.argtypes = [_vp, P(gsr_options)]
    L.gsr_plan_set_tuning.argtypes = [_vp, P(gsr_options)]
    L.gsr_status_string.argtypes = [_i32]
    L.gsr_status_string.restype = ctypes.c_char_p
    L.gsr_last_error.argtypes = [_vp]
    L.gsr_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        f = getattr(L, name)
        if f.restype is ctypes.c_int:  # ctypes default
            f.restype = _i32
    _lib = L
    return L


class GsrError(RuntimeError):
    def __init__(self, status, message=""):
        self.status = status
        super().__init__(f"{gsr_status_string(status)} ({status}): {message}")


def _check(status, plan=None):
    if status != GSR_OK:
        msg = gsr_last_error(plan) if plan else ""
        raise GsrError(status, msg)


# ---------------------------------------------------------------- C names


def gsr_default_options() -> gsr_options:
    o = gsr_options()
    load().gsr_default_options(ctypes.byref(o))
    return o


def gsr_plan_create(problem: gsr_problem, options: gsr_options):
    plan = _vp()
    _check(load().gsr_plan_create(ctypes.byref(plan), ctypes.byref(problem), ctypes.byref(options)))
    return plan


def gsr_plan_destroy(plan):
    _check(load().gsr_plan_destroy(plan))


def gsr_workspace_size(plan) -> int:
    b = _sz()
    _check(load().gsr_workspace_size(plan, ctypes.byref(b)), plan)
    return b.value


def gsr_workspace_layout(plan) -> gsr_layout:
    L = gsr_layout()
    _check(load().gsr_workspace_layout(plan, ctypes.byref(L)), plan)
    return L


def gsr_image_offset(plan, view: int) -> int:
    o = _i64()
    _check(load().gsr_image_offset(plan, view, ctypes.byref(o)), plan)
    return o.value


def gsr_forward(plan, g: gsr_gaussians, cams, images, T_final, last, ws, ws_bytes, stream):
    _check(load().gsr_forward(plan, ctypes.byref(g), cams, images, T_final, last, ws, ws_bytes, stream), plan)


def gsr_backward(plan, g: gsr_gaussians, cams, dL_dimages, grads: gsr_grads, stats, ws, ws_bytes, stream):
    _check(load().gsr_backward(plan, ctypes.byref(g), cams, dL_dimages, ctypes.byref(grads),
                               ctypes.byref(stats) if stats is not None else None, ws, ws_bytes, stream), plan)


def gsr_forward_backward_l1(plan, g, cams, targets, images, loss, grads, stats, ws, ws_bytes, stream):
    _check(load().gsr_forward_backward_l1(plan, ctypes.byref(g), cams, targets, images, loss, ctypes.byref(grads),
                                          ctypes.byref(stats) if stats is not None else None, ws, ws_bytes,
                                          stream), plan)


def gsr_visibility_mask(plan, g, cams, aabb, view_bits, keep_out, in_block, ws, ws_bytes, stream):
    box = (_f32 * 6)(*aabb) if aabb is not None else None
    _check(load().gsr_visibility_mask(plan, ctypes.byref(g), cams, box, view_bits, keep_out, in_block, ws,
                                      ws_bytes, stream), plan)


def gsr_render_depth(plan, g, cams, images, depth, ws, ws_bytes, stream):
    _check(load().gsr_render_depth(plan, ctypes.byref(g), cams, images, depth, ws, ws_bytes, stream), plan)


GSR_STATIC_SCRATCH_BYTES = 64 << 20


def gsr_forward_backward_l1_static(plan, g, cams, targets, images, loss, grads, stats, stream):
    _check(load().gsr_forward_backward_l1_static(plan, ctypes.byref(g), cams, targets, images, loss,
                                                 ctypes.byref(grads), ctypes.byref(stats) if stats else None,
                                                 stream), plan)


def gsr_pair_counts(plan, g, cams, images, counts, ws, ws_bytes, stream):
    _check(load().gsr_pair_counts(plan, ctypes.byref(g), cams, images, counts, ws, ws_bytes, stream), plan)


def gsr_camera_coverage(plan, cams, depth, blocks, n_blocks, tau, counts, ratio, selected, stream):
    _check(load().gsr_camera_coverage(plan, cams, depth, blocks, n_blocks, tau, counts, ratio, selected, stream),
           plan)


def gsr_back_project(plan, cams, depth, points, stream):
    _check(load().gsr_back_project(plan, cams, depth, points, stream), plan)


def _partition_host_args(scene_aabb, centers, view_offsets, n_blocks):
    import numpy as np
    aabb = np.ascontiguousarray(scene_aabb, np.float32)
    c = np.ascontiguousarray(centers, np.float32)
    off = np.ascontiguousarray(view_offsets, np.int64)
    V = off.size - 1
    out = (np.zeros((n_blocks, 6), np.float32), np.zeros((n_blocks, V), np.uint8), np.zeros(n_blocks, np.int32))
    return aabb, c, off, V, out


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def gsr_partition_blocks(scene_aabb, centers, points, view_offsets, n_blocks, tau=0.1, refine_steps=3, q_min=0.1,
                         q_max=0.9):
    """Host KD-tree partition on NumPy arrays: centers [3][n], points [3][total] (float32),
    view_offsets [V + 1] (int64).  Returns (blocks [M][6], assign [M][V] uint8, workload [M])."""
    import numpy as np
    aabb, c, off, V, (blocks, assign, work) = _partition_host_args(scene_aabb, centers, view_offsets, n_blocks)
    pts = np.ascontiguousarray(points, np.float32)
    P = ctypes.POINTER
    _check(load().gsr_partition_blocks(_ptr(aabb, _f32), _ptr(c, _f32), c.shape[1], _ptr(pts, _f32), _ptr(off, _i64),
                                       V, n_blocks, tau, refine_steps, q_min, q_max, _ptr(blocks, _f32),
                                       _ptr(assign, ctypes.c_uint8), _ptr(work, _i32)), None)
    return blocks, assign, work


def gsr_partition_workspace_size(n_views):
    out = _sz(0)
    _check(load().gsr_partition_workspace_size(n_views, ctypes.byref(out)), None)
    return out.value


def gsr_partition_blocks_device(scene_aabb, centers, points_ptr, view_offsets, n_blocks, ws_ptr, ws_bytes, stream,
                                tau=0.1, refine_steps=3, q_min=0.1, q_max=0.9):
    """The same partition with the pixel counting on the GPU: points_ptr is the device address
    of float32 [3][total] points; the rest are host NumPy arrays."""
    aabb, c, off, V, (blocks, assign, work) = _partition_host_args(scene_aabb, centers, view_offsets, n_blocks)
    _check(load().gsr_partition_blocks_device(_ptr(aabb, _f32), _ptr(c, _f32), c.shape[1], points_ptr,
                                              _ptr(off, _i64), V, n_blocks, tau, refine_steps, q_min, q_max, ws_ptr,
                                              ws_bytes, stream, _ptr(blocks, _f32), _ptr(assign, ctypes.c_uint8),
                                              _ptr(work, _i32)), None)
    return blocks, assign, work


def gsr_densify_workspace_size(n):
    out = _sz(0)
    _check(load().gsr_densify_workspace_size(n, ctypes.byref(out)), None)
    return out.value


def gsr_densify_count(n, sh_degree, opts, g, stats, in_block, ws, ws_bytes, stream):
    """Returns the output count (synchronizes the stream)."""
    out = _i64(0)
    _check(load().gsr_densify_count(n, sh_degree, ctypes.byref(opts), ctypes.byref(g), ctypes.byref(stats), in_block,
                                    ws, ws_bytes, stream, ctypes.byref(out)), None)
    return out.value


def gsr_densify_apply(n, sh_degree, opts, g, m_in, v_in, stats, in_block, samples, n_out, out, m_out, v_out,
                      parent_out, ws, ws_bytes, stream):
    ref = lambda x: ctypes.byref(x) if x is not None else None
    _check(load().gsr_densify_apply(n, sh_degree, ctypes.byref(opts), ctypes.byref(g), ref(m_in), ref(v_in),
                                    ctypes.byref(stats), in_block, samples, n_out, ref(out), ref(m_out), ref(v_out),
                                    parent_out, ws, ws_bytes, stream), None)


def gsr_adam_step(plan, hp, params, grads, m, v, visible_bits, stream):
    _check(load().gsr_adam_step(plan, ctypes.byref(hp), ctypes.byref(params), ctypes.byref(grads),
                                ctypes.byref(m), ctypes.byref(v), visible_bits, stream), plan)


def gsr_graph_capture(plan, g, cams, targets, images, loss, grads, stats, ws, ws_bytes, stream):
    _check(load().gsr_graph_capture(plan, ctypes.byref(g), cams, targets, images, loss, ctypes.byref(grads),
                                    ctypes.byref(stats) if stats is not None else None, ws, ws_bytes, stream),
           plan)


def gsr_graph_launch(plan, stream):
    _check(load().gsr_graph_launch(plan, stream), plan)


def gsr_query_counts(plan, ws, stream, check=True) -> gsr_counts:
    c = gsr_counts()
    s = load().gsr_query_counts(plan, ws, ctypes.byref(c), stream)
    if check:
        _check(s, plan)
    return c


def gsr_autotune(plan, g, cams, targets, images, loss, grads, ws, ws_bytes, reps, stream):
    best = gsr_options()
    ms = _f32()
    _check(load().gsr_autotune(plan, ctypes.byref(g), cams, targets, images, loss, ctypes.byref(grads), ws,
                               ws_bytes, reps, ctypes.byref(best), ctypes.byref(ms), stream), plan)
    return best, ms.value


def gsr_last_stage_times(plan) -> dict:
    t = gsr_stage_times()
    _check(load().gsr_last_stage_times(plan, ctypes.byref(t)), plan)
    return t.as_dict()


def gsr_plan_options(plan) -> gsr_options:
    o = gsr_options()
    _check(load().gsr_plan_options(plan, ctypes.byref(o)), plan)
    return o


def gsr_plan_set_tuning(plan, o: gsr_options):
    _check(load().gsr_plan_set_tuning(plan, ctypes.byref(o)), plan)


def gsr_status_string(s: int) -> str:
    return load().gsr_status_string(s).decode()


def gsr_last_error(plan) -> str:
    r = load().gsr_last_error(plan)
    return r.decode() if r else ""
