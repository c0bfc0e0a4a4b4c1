"""The allocation-free fused step (gsr_forward_backward_l1_static) against the
workspace form (gsr_forward_backward_l1) through the C ABI: two calls in a
row, the second on a smaller problem, each compared with the workspace form
on the same inputs (images and loss bit-identical, the same kernels; parameter
gradients and densification statistics equal up to the order of float
atomics; visible counts exact)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2510_01767_amd import gsr as C
from paper_2510_01767_amd import scenes
from paper_2510_01767_amd.raster import PARAM_NAMES, Rasterizer, camera_tensor, pack_images, scene_tensors

pytestmark = pytest.mark.gpu


def static_step(scene, mode):
    """Plan + output buffers only (no workspace), then the allocation-free call."""
    sizes = [(c["W"], c["H"]) for c in scene.cameras]
    V = len(sizes)
    o = C.gsr_default_options()
    o.mode = C.GSR_MODE_BATCHED if mode == "batched" else C.GSR_MODE_PLAIN
    Wa = (ctypes.c_int32 * V)(*[s[0] for s in sizes])
    Ha = (ctypes.c_int32 * V)(*[s[1] for s in sizes])
    prob = C.gsr_problem(scene.n, scene.sh_degree, V, Wa, Ha)
    plan = C.gsr_plan_create(prob, o)
    assert C.gsr_workspace_size(plan) <= C.GSR_STATIC_SCRATCH_BYTES
    params = scene_tensors(scene)
    cams = camera_tensor(scene.cameras)
    targets = torch.from_numpy(pack_images(scene.targets)).cuda()
    pixels = sum(w * h for w, h in sizes)
    images = torch.empty(3 * pixels, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    grads = {k: torch.empty_like(params[k]) for k in PARAM_NAMES}
    S = torch.zeros(scene.n, dtype=torch.float32, device="cuda")
    cnt = torch.zeros(scene.n, dtype=torch.int32, device="cuda")
    g = Rasterizer.gaussians(params)
    gr = C.gsr_grads(*[grads[k].data_ptr() for k in PARAM_NAMES])
    st = C.gsr_stats(S.data_ptr(), cnt.data_ptr())
    torch.cuda.synchronize()
    C.gsr_forward_backward_l1_static(plan, g, cams.data_ptr(), targets.data_ptr(), images.data_ptr(),
                                     loss.data_ptr(), gr, st, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out = dict(images=images.cpu().numpy(), loss=float(loss.item()), S=S.cpu().numpy(), count=cnt.cpu().numpy(),
               grads={k: v.cpu().numpy() for k, v in grads.items()})
    C.gsr_plan_destroy(plan)
    return out


def workspace_step(scene, mode):
    sizes = [(c["W"], c["H"]) for c in scene.cameras]
    r = Rasterizer(scene.n, scene.sh_degree, sizes, mode=mode, lds_batch=128, grid_per_cu=4)
    params = scene_tensors(scene)
    cams = camera_tensor(scene.cameras)
    targets = torch.from_numpy(pack_images(scene.targets)).cuda()
    r.S.zero_()
    r.count.zero_()
    loss, images = r.step_l1(params, cams, targets)
    torch.cuda.synchronize()
    return dict(images=images.cpu().numpy(), loss=float(loss.item()), S=r.S.cpu().numpy(),
                count=r.count.cpu().numpy(), grads={k: v.cpu().numpy() for k, v in r.grads.items()})


def check_same(a, b):
    assert np.array_equal(a["images"], b["images"])
    assert a["loss"] == b["loss"]
    assert np.array_equal(a["count"], b["count"])
    # the same kernels; the float32 atomic sums of the 2D gradients (and the
    # statistics built on them) may add up in another order between two runs,
    # ~1e-6 relative L2 on the small, cancelling quaternion gradient
    rel = lambda x, y: np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-30)
    assert rel(a["S"], b["S"]) <= 1e-5
    for k in a["grads"]:
        assert rel(a["grads"][k], b["grads"][k]) <= 1e-5, k


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_static_scratch_step_matches_the_workspace_step_twice(mode):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    C.load(build_if_missing=False)
    big, small = scenes.small_ragged(), scenes.config0()
    assert small.n < big.n and small.pixels < big.pixels
    for sc in (big, small):  # the second call on a smaller problem reuses the same array
        print("[gpu-case] static scratch", mode, sc.name, flush=True)
        check_same(static_step(sc, mode), workspace_step(sc, mode))


def test_static_scratch_rejects_a_plan_beyond_its_size():
    C.load(build_if_missing=False)
    o = C.gsr_default_options()
    o.mode = C.GSR_MODE_BATCHED
    Wa = (ctypes.c_int32 * 1)(1920)
    Ha = (ctypes.c_int32 * 1)(1080)
    plan = C.gsr_plan_create(C.gsr_problem(1_000_000, 3, 1, Wa, Ha), o)
    assert C.gsr_workspace_size(plan) > C.GSR_STATIC_SCRATCH_BYTES
    g = C.gsr_gaussians(1, 1, 1, 1, 1, None)
    gr = C.gsr_grads(1, 1, 1, 1, 1)
    with pytest.raises(C.GsrError) as e:
        C.gsr_forward_backward_l1_static(plan, g, 1, 1, 1, 1, gr, None, None)
    assert e.value.status == C.GSR_ERR_WORKSPACE_TOO_SMALL
    C.gsr_plan_destroy(plan)
