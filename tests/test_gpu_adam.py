"""GPU parity of the Adam step (gsr_adam_step) with the FP64 oracle.

Tolerance, from the float32 arithmetic (about ten roundings of 6e-8 each):
|p_gpu - p_ora| <= 2e-7 |p| + 2e-6 lr/(1 - b1^t) (|b1 m| + |(1 - b1) g|) /
(sqrt(v^) + eps), moments within 3e-7 of the magnitude of their two terms.  Each step feeds the GPU's float32 state to
the oracle, so errors do not compound across steps."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_01767_amd import scenes
from paper_2510_01767_amd.raster import PARAM_NAMES, Rasterizer, camera_tensor, pack_images, scene_tensors

pytestmark = pytest.mark.gpu
# the ABI carries float32 hyperparameters: the oracle gets the same values
f32 = lambda x: float(np.float32(x))
LR = tuple(f32(x) for x in (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 2.5e-3 / 20))
B1, B2, EPS = f32(0.9), f32(0.999), f32(1e-15)
ROWS = dict(means=3, log_scales=3, quats=4, opacity_logits=1, sh=48)


def announce(*a):
    print("[gpu-case]", *a, flush=True)


def rand_planes(gen, n, scale=1.0, positive=False):
    out = {}
    for k, r in ROWS.items():
        shape = (n,) if k == "opacity_logits" else (r, n)
        t = torch.randn(shape, generator=gen, dtype=torch.float32) * scale
        out[k] = (t.abs() if positive else t).cuda()
    return out


def np64(d):
    return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in d.items()}


def check(gpu_p, gpu_m, gpu_v, p, g, m, v, step, visible=None, beta1=B1, beta2=B2, eps=EPS):
    """The bounds scale with the magnitudes of the summed terms, so a first
    moment that nearly cancels (b1 m against (1 - b1) g) is judged by the
    size of its terms, not of its tiny result."""
    P, M, V = oracle.adam_step(p, g, m, v, LR, beta1, beta2, eps, step, visible)
    bc1, bc2 = 1 - beta1 ** step, 1 - beta2 ** step
    for k in ROWS:
        shape = P[k].shape
        gp = np64(gpu_p)[k].reshape(shape)
        gm = np64(gpu_m)[k].reshape(shape)
        gv = np64(gpu_v)[k].reshape(shape)
        p0 = np.asarray(p[k]).reshape(shape)
        g0 = np.asarray(g[k]).reshape(shape)
        mterm = np.abs(beta1 * np.asarray(m[k]).reshape(shape)) + np.abs((1 - beta1) * g0)
        vterm = np.abs(beta2 * np.asarray(v[k]).reshape(shape)) + (1 - beta2) * g0 ** 2
        if k == "sh":
            rate = np.full((shape[0], 1), LR[5])
            rate[:3] = LR[4]
        else:
            rate = LR[oracle.ADAM_GROUPS.index(k)]
        dscale = rate / bc1 * mterm / (np.sqrt(V[k] / bc2) + eps)
        assert np.all(np.abs(gp - P[k]) <= 2e-7 * np.abs(p0) + 2e-6 * dscale + 1e-30), k
        assert np.all(np.abs(gm - M[k]) <= 3e-7 * mterm + 1e-38), k
        assert np.all(np.abs(gv - V[k]) <= 3e-7 * vterm + 1e-38), k


def plan_for(n):
    return Rasterizer(n, 3, [(64, 48)], mode="batched")


def test_dense_steps_match_oracle():
    n = 100003
    announce("adam dense", n)
    gen = torch.Generator().manual_seed(7)
    r = plan_for(n)
    p, m, v = rand_planes(gen, n), rand_planes(gen, n, 1e-3), rand_planes(gen, n, 1e-6, positive=True)
    for t in range(1, 4):
        g = rand_planes(gen, n, 10.0 ** (-2 * t))
        before = (np64(p), np64(g), np64(m), np64(v))
        r.adam_step(p, g, m, v, LR, t, beta1=B1, beta2=B2, eps=EPS)
        torch.cuda.synchronize()
        check(p, m, v, *before, step=t)


def test_visible_only_step_uses_the_last_step_view_masks():
    s = scenes.small_ragged()
    announce("adam visible-only", s.n)
    sizes = [(c["W"], c["H"]) for c in s.cameras]
    r = Rasterizer(s.n, s.sh_degree, sizes, mode="batched")
    params = scene_tensors(s)
    # a keep mask crops 30 % of the Gaussians, so the step's view masks leave them out
    keep = torch.from_numpy((np.random.default_rng(11).random(s.n) < 0.7).astype(np.uint8)).cuda()
    r.step_l1(params, camera_tensor(s.cameras), torch.from_numpy(pack_images(s.targets)).cuda(), keep=keep,
              stats=False)
    torch.cuda.synchronize()
    bits = r.ws_tensor("view_bits", torch.int32, s.n).cpu().numpy().view(np.uint32)
    assert 0 < (bits != 0).sum() < s.n
    gen = torch.Generator().manual_seed(8)
    m, v = rand_planes(gen, s.n, 1e-3), rand_planes(gen, s.n, 1e-6, positive=True)
    p = {k: params[k].clone() for k in PARAM_NAMES}
    before = (np64(p), np64(r.grads), np64(m), np64(v))
    r.adam_step(p, r.grads, m, v, LR, 5, beta1=B1, beta2=B2, eps=EPS, visible_only=True)
    torch.cuda.synchronize()
    check(p, m, v, *before, step=5, visible=bits)
    off = bits == 0
    for k in PARAM_NAMES:
        assert np.array_equal(np64(p)[k][..., off], before[0][k][..., off])


def test_bench_size_step_matches_oracle_on_a_subset():
    n = 3_000_000
    announce("adam 3M", n)
    gen = torch.Generator().manual_seed(9)
    r = plan_for(n)
    p, g = rand_planes(gen, n), rand_planes(gen, n, 1e-3)
    m, v = rand_planes(gen, n, 1e-4), rand_planes(gen, n, 1e-8, positive=True)
    sub = torch.from_numpy(np.sort(np.random.default_rng(10).choice(n, n // 100, replace=False))).cuda()
    pick = lambda d: {k: x[..., sub].clone() for k, x in d.items()}
    before = tuple(np64(pick(d)) for d in (p, g, m, v))
    r.adam_step(p, g, m, v, LR, 12, beta1=B1, beta2=B2, eps=EPS)
    torch.cuda.synchronize()
    check(pick(p), pick(m), pick(v), *before, step=12)
