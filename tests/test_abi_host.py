"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/gsr.h declares, validates arguments before
enqueuing anything, and lays out the workspace consistently."""
import ctypes
import os
import re

import pytest

from paper_2510_01767_amd import gsr as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gsr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    lib = C.load()
    names = declared_functions()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(C.EXPORTS)


def test_struct_sizes_match_the_header():
    assert ctypes.sizeof(C.gsr_camera) == 64
    assert ctypes.sizeof(C.gsr_options) == 4 * 11 + 4 * 12 + 4 + 8 * 2  # 4 bytes of padding before the int64s
    assert ctypes.sizeof(C.gsr_stage_times) == 4 + 16 * 4 + 16 * 4 + 16 * 32


def problem(n=1000, sh=3, sizes=((64, 48), (33, 17))):
    W = (ctypes.c_int32 * len(sizes))(*[s[0] for s in sizes])
    H = (ctypes.c_int32 * len(sizes))(*[s[1] for s in sizes])
    p = C.gsr_problem(n, sh, len(sizes), W, H)
    p._keep = (W, H)
    return p


def create(p, o=None):
    plan = ctypes.c_void_p()
    o = o or C.gsr_default_options()
    s = C.load().gsr_plan_create(ctypes.byref(plan), ctypes.byref(p), ctypes.byref(o))
    return s, plan


def test_defaults():
    o = C.gsr_default_options()
    assert (o.tile_w, o.tile_h, o.mode, o.lds_batch) == (16, 16, C.GSR_MODE_PLAIN, 128)
    assert abs(o.alpha_min - 1 / 255) < 1e-9 and abs(o.alpha_max - 0.99) < 1e-7
    assert abs(o.T_min - 1e-4) < 1e-10 and abs(o.eps2d - 0.3) < 1e-7 and o.sigma_extent == 3.0
    assert abs(o.jac_clamp - 1.3) < 1e-7 and list(o.bg) == [0, 0, 0]


@pytest.mark.parametrize("mutate", [
    lambda p, o: setattr(p, "n", 0),
    lambda p, o: setattr(p, "sh_degree", 4),
    lambda p, o: setattr(p, "sh_degree", -1),
    lambda p, o: setattr(p, "n_views", 0),
    lambda p, o: setattr(p, "n_views", 33),
    lambda p, o: setattr(p, "n", 1 << 31),  # n * n_views >= 2^32
    lambda p, o: setattr(p, "n", (1 << 28) + 1),  # above GSR_MAX_GAUSSIANS (per-Gaussian grids)
    lambda p, o: p.widths.__setitem__(0, 0),
    lambda p, o: p.heights.__setitem__(1, 16385),
    lambda p, o: setattr(o, "tile_h", 8),
    lambda p, o: setattr(o, "lds_batch", 100),
    lambda p, o: setattr(o, "grid_per_cu", 0),
    lambda p, o: setattr(o, "mode", 7),
    lambda p, o: setattr(o, "bwd_reduce", 5),
    lambda p, o: setattr(o, "project_table", 2),
    lambda p, o: setattr(o, "alpha_max", 1.0),
    lambda p, o: setattr(o, "T_min", 0.0),
    lambda p, o: setattr(o, "near_plane", -1.0),
    lambda p, o: setattr(o, "capacity_intersections", -5),
])
def test_invalid_arguments_are_rejected(mutate):
    p = problem()
    o = C.gsr_default_options()
    mutate(p, o)
    s, plan = create(p, o)
    assert s == C.GSR_ERR_INVALID_ARG and not plan.value


def test_largest_gaussian_count_is_accepted():
    p = problem()
    p.n = 1 << 28
    s, plan = create(p, C.gsr_default_options())
    assert s == C.GSR_OK and plan.value
    C.load().gsr_plan_destroy(plan)


def test_null_problem():
    plan = ctypes.c_void_p()
    assert C.load().gsr_plan_create(ctypes.byref(plan), None, None) == C.GSR_ERR_INVALID_ARG


def test_layout_and_workspace_size():
    p = problem()
    o = C.gsr_default_options()
    o.capacity_intersections = 100000
    s, plan = create(p, o)
    assert s == C.GSR_OK
    L = C.gsr_workspace_layout(plan)
    size = C.gsr_workspace_size(plan)
    assert size == L.total
    fields = ["header", "view_table", "view_bits", "records", "grad2d", "tile_count", "tile_start",
              "tile_fill", "tile_loss", "tile_order", "keys", "keys_alt", "pix_T", "pix_last", "pix_dLdC",
              "history"]
    offs = [getattr(L, f) for f in fields]
    assert all(x % 256 == 0 for x in offs)
    assert offs == sorted(offs)
    assert L.vn == 2000 and L.capacity == 100000 and L.history_entries == 0
    assert L.pixels_total == 64 * 48 + 33 * 17
    assert L.tiles_total == 4 * 3 + 3 * 2
    assert L.keys_alt - L.keys >= 8 * 100000
    assert L.records + 64 * L.vn <= L.grad2d
    assert C.GSR_SLOT_FLOATS == 16 and L.grad2d + 4 * C.GSR_SLOT_FLOATS * L.vn <= L.tile_count
    assert C.gsr_image_offset(plan, 1) == 3 * 64 * 48
    C.gsr_plan_destroy(plan)
    # the stored-history variant reserves capacity * 256 floats within its budget
    o.bwd_variant = C.GSR_BWD_STORED
    o.history_budget_bytes = 200000 * 256 * 4
    s, plan2 = create(p, o)
    L2 = C.gsr_workspace_layout(plan2)
    assert L2.history_entries == 100000 * 256 and C.gsr_workspace_size(plan2) > size
    C.gsr_plan_destroy(plan2)
    o.history_budget_bytes = 1000
    s, plan3 = create(p, o)
    assert C.gsr_workspace_layout(plan3).history_entries == 0
    C.gsr_plan_destroy(plan3)


def test_calls_validate_before_touching_the_device():
    p = problem()
    s, plan = create(p)
    lib = C.load()
    fake = 0x100000  # never dereferenced: every check below fails on the host first
    g = C.gsr_gaussians(fake, fake, fake, fake, fake, None)
    gr = C.gsr_grads(fake, fake, fake, fake, fake)
    size = C.gsr_workspace_size(plan)
    # NULL workspace, too small, misaligned
    assert lib.gsr_forward(plan, ctypes.byref(g), fake, fake, None, None, None, size, None) == C.GSR_ERR_INVALID_ARG
    assert lib.gsr_forward(plan, ctypes.byref(g), fake, fake, None, None, fake, size - 1, None) == C.GSR_ERR_WORKSPACE_TOO_SMALL
    assert lib.gsr_forward(plan, ctypes.byref(g), fake, fake, None, None, fake + 8, size, None) == C.GSR_ERR_INVALID_ARG
    # null parameter plane
    g0 = C.gsr_gaussians(fake, None, fake, fake, fake, None)
    assert lib.gsr_forward(plan, ctypes.byref(g0), fake, fake, None, None, fake, size, None) == C.GSR_ERR_INVALID_ARG
    assert lib.gsr_forward_backward_l1(plan, ctypes.byref(g), fake, None, fake, fake, ctypes.byref(gr), None,
                                       fake, size, None) == C.GSR_ERR_INVALID_ARG
    # backward without a forward, launch without a capture, capture in plain mode
    assert lib.gsr_backward(plan, ctypes.byref(g), fake, fake, ctypes.byref(gr), None, fake, size, None) == C.GSR_ERR_STATE
    assert lib.gsr_graph_launch(plan, None) == C.GSR_ERR_STATE
    assert lib.gsr_graph_capture(plan, ctypes.byref(g), fake, fake, fake, fake, ctypes.byref(gr), None, fake, size,
                                 fake) == C.GSR_ERR_STATE
    assert "gsr_forward" in C.gsr_last_error(plan) or C.gsr_last_error(plan)
    # autotuning needs the batched form
    assert lib.gsr_autotune(plan, ctypes.byref(g), fake, fake, fake, fake, ctypes.byref(gr), fake, size, 1, None,
                            None, None) == C.GSR_ERR_STATE
    # tuning changes may not grow the workspace
    o = C.gsr_plan_options(plan)
    o.tile_w, o.tile_h = 32, 8
    C.gsr_plan_set_tuning(plan, o)
    assert C.gsr_workspace_size(plan) == size
    o.bwd_variant = C.GSR_BWD_STORED
    with pytest.raises(C.GsrError):
        C.gsr_plan_set_tuning(plan, o)
    C.gsr_plan_destroy(plan)


def test_status_strings():
    for s in range(7):
        assert C.gsr_status_string(s)
    assert C.gsr_status_string(3) == "intersection capacity exceeded"


def test_adam_step_rejects_bad_arguments_before_touching_the_device():
    s, plan = create(problem(), C.gsr_default_options())
    assert s == C.GSR_OK
    L = C.load()
    g = C.gsr_grads(1, 1, 1, 1, 1)
    hp = C.gsr_adam((ctypes.c_float * 6)(*([1e-3] * 6)), 0.9, 0.999, 1e-15, 0)
    assert L.gsr_adam_step(plan, ctypes.byref(hp), ctypes.byref(g), ctypes.byref(g), ctypes.byref(g),
                           ctypes.byref(g), None, None) == C.GSR_ERR_INVALID_ARG  # step 0
    hp.step, hp.beta1 = 1, 1.0
    assert L.gsr_adam_step(plan, ctypes.byref(hp), ctypes.byref(g), ctypes.byref(g), ctypes.byref(g),
                           ctypes.byref(g), None, None) == C.GSR_ERR_INVALID_ARG  # beta1 = 1
    hp.beta1 = 0.9
    null = C.gsr_grads(None, 1, 1, 1, 1)
    assert L.gsr_adam_step(plan, ctypes.byref(hp), ctypes.byref(null), ctypes.byref(g), ctypes.byref(g),
                           ctypes.byref(g), None, None) == C.GSR_ERR_INVALID_ARG
    C.gsr_plan_destroy(plan)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: asking for more exits non-zero with a message, before any device use."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_byte_model_matches_the_per_unit_budget():
    """The algorithmic byte model of bench.py: per visible (view, Gaussian)
    the plain form moves 1100 B at SH degree 3 and 380 B at degree 0; the
    batched form reads the geometry once (40 B per Gaussian) and writes each
    visible Gaussian's gradients once; the fused raster moves 80 B per
    intersection, 52 B per pixel and 36 B per visible record."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    for K, F, cv in ((48, 59, 1100), (3, 14, 380)):
        assert b.b_alg_plain(0, K, F, 1, 1, 0, 0) == cv
        assert b.b_alg_plain(1, K, F, 1, 0, 0, 0) == 12
    assert b.b_alg_plain(0, 48, 59, 1, 0, 1, 0) == 140 and b.b_alg_plain(0, 48, 59, 1, 0, 0, 1) == 52
    assert b.b_alg_batched(1, 0, 48, 59, 0, 0, 0) == 40
    assert b.b_alg_batched(0, 1, 48, 59, 0, 0, 0) == 4 + 4 * 48 + 8 * 59 + 16
    assert b.b_alg_batched(0, 0, 48, 59, 1, 0, 0) == 152
    assert b.b_alg_fused(1, 0, 0) == 36 and b.b_alg_fused(0, 1, 0) == 80 and b.b_alg_fused(0, 0, 1) == 52
