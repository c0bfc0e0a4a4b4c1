"""GPU parity at the benchmark's full sizes.

Config 1 (1M Gaussians, one 1080p view) is checked whole.  Config 2 (3M
Gaussians, 16 uneven views, the workload bench.py times, in its autotuned
batched launch) is checked stage by stage on outputs the oracle can compute
one by one: images and 2D gradients of sampled views, and the reverse
projection of a seeded 1 % subset of Gaussians fed with the GPU's own 2D
gradients of every view."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_01767_amd import scenes
from paper_2510_01767_amd.raster import Rasterizer, camera_tensor, pack_images, scene_tensors
from tests import parity

pytestmark = pytest.mark.gpu


def announce(*a):
    print("[gpu-case]", *a, flush=True)


def setup(scene, **kw):
    sizes = [(c["W"], c["H"]) for c in scene.cameras]
    r = Rasterizer(scene.n, scene.sh_degree, sizes, **kw)
    return r, scene_tensors(scene), camera_tensor(scene.cameras), torch.from_numpy(pack_images(scene.targets)).cuda()


def test_config1_full_step_matches_oracle():
    s = scenes.config1()
    announce("config1 full", s.n)
    r, params, cams, targets = setup(s, mode="batched", tile=(8, 32), lds_batch=256, grid_per_cu=8)
    r.S.zero_()
    r.count.zero_()
    loss, _ = r.step_l1(params, cams, targets)
    torch.cuda.synchronize()
    ora = oracle.step_l1(oracle.Params.from_scene(s), s.cameras, s.targets, parity.opts_for((8, 32)))
    rep = {}
    parity.compare_images(parity.gpu_images(r), ora, rep)
    assert abs(float(loss.item()) - ora["loss"]) <= 1e-5 * ora["loss"]
    ex = parity.excluded_gaussians(ora, s.n, parity.opts_for((8, 32)), s.targets)
    parity.compare_grads(parity.gpu_grad_groups(r.grads), ora["grads"], ex, report=rep)
    keep = ~ex
    S = r.S.cpu().numpy().astype(np.float64)
    rms = np.sqrt(np.mean(ora["S"] ** 2))
    assert np.all(np.abs(S[keep] - ora["S"][keep]) <= 1e-3 * (np.abs(ora["S"][keep]) + 1e-2 * rms))
    assert np.array_equal(r.count.cpu().numpy()[keep], ora["count"][keep])
    print("report", rep)


@pytest.fixture(scope="module")
def c2():
    s = scenes.config2()
    announce("config2 scene", s.n, s.n_views)
    r, params, cams, targets = setup(s, mode="batched")
    best, ms = r.autotune(params, cams, targets, reps=1)
    announce("autotuned", best.tile_w, best.tile_h, best.lds_batch, best.grid_per_cu, ms)
    r.S.zero_()
    r.count.zero_()
    r.step_l1(params, cams, targets)
    torch.cuda.synchronize()
    return s, r, params, cams, targets


def test_config2_sampled_views_match_oracle(c2):
    s, r, params, cams, targets = c2
    o = r.options
    opts = parity.opts_for((o.tile_w, o.tile_h))
    P = oracle.Params.from_scene(s)
    n, V = s.n, s.n_views
    gimgs = parity.gpu_images(r)
    L = r.layout
    g2d_all = r.ws_tensor("grad2d", torch.float32, 12 * L.vn).view(-1, 12)
    tile_loss = r.ws_tensor("tile_loss", torch.float32, L.tiles_total).cpu().numpy().astype(np.float64)
    views = [int(np.argmin([c["W"] * c["H"] for c in s.cameras])), 0]
    tile_base = 0
    bases = []
    for c in s.cameras:
        bases.append(tile_base)
        tile_base += ((c["W"] + o.tile_w - 1) // o.tile_w) * ((c["H"] + o.tile_h - 1) // o.tile_h)
    for v in views:
        c = s.cameras[v]
        W, H = c["W"], c["H"]
        announce("config2 view", v, W, H)
        fo = oracle.forward(P, [c], opts)
        rep = {}
        parity.compare_images([gimgs[v]], fo, rep)
        # per-view L1 sum from the GPU's tile partials
        nt = ((W + o.tile_w - 1) // o.tile_w) * ((H + o.tile_h - 1) // o.tile_h)
        l_gpu = tile_loss[bases[v]:bases[v] + nt].sum()
        l_ora = np.abs(fo["images"][0] - s.targets[v]).sum()
        assert abs(l_gpu - l_ora) <= 1e-5 * l_ora
        # 2D gradients of this view's records under the same dL/dC, away from L1 kinks
        d = np.sign(fo["images"][0] - s.targets[v]) / (3.0 * W * H * V)
        kink = np.abs(fo["images"][0] - s.targets[v]) < 1e-5
        d_g = np.sign(gimgs[v].astype(np.float64) - s.targets[v]) / (3.0 * W * H * V)
        assert np.array_equal((d == d_g)[~kink], np.ones((~kink).sum(), bool))
        bo = oracle.backward(P, [c], opts, fo, [d])
        vis = fo["records"][0]["visible"].astype(bool)
        ex = parity.excluded_gaussians(fo, n, opts)
        kinked = np.zeros(n, bool)
        if kink.any():
            ys, xs = np.nonzero(kink.any(axis=0))
            gx = (W + o.tile_w - 1) // o.tile_w
            for t in np.unique((ys // o.tile_h) * gx + xs // o.tile_w):
                a, b = fo["bins"]["ranges"][t]
                kinked[fo["bins"]["values"][a:b] % n] = True
        sel = vis & ~ex & ~kinked
        gg = g2d_all[v * n:(v + 1) * n, :9].cpu().numpy().astype(np.float64)[sel]
        go = bo["g2d"].T[sel]
        for k in range(9):
            a_, b_ = gg[:, k], go[:, k]
            rel = np.linalg.norm(a_ - b_) / max(np.linalg.norm(b_), 1e-300)
            rms = np.sqrt(np.mean(b_ ** 2))
            assert rel <= 1e-3, (v, k, rel)
            assert np.all(np.abs(a_ - b_) <= 1e-3 * (np.abs(b_) + 1e-2 * rms)), (v, k)
        print("view", v, rep, "grad2d records checked", int(sel.sum()), "kink-excluded", int(kinked.sum()))


def test_config2_reverse_projection_on_a_subset(c2):
    """Parameter gradients and statistics of a seeded 1 % of the Gaussians:
    the oracle's reverse projection fed with the GPU's 2D gradients."""
    s, r, params, cams, targets = c2
    n, V = s.n, s.n_views
    rng = np.random.default_rng(20251002)
    sub = np.sort(rng.choice(n, n // 100, replace=False))
    P = oracle.Params.from_scene(s)
    Ps = oracle.Params(P.means[:, sub].copy(), P.log_scales[:, sub].copy(), P.quats[:, sub].copy(),
                       P.logits[sub].copy(), P.sh[:, sub].copy(), P.sh_degree)
    L = r.layout
    g2d = r.ws_tensor("grad2d", torch.float32, 12 * L.vn).view(V, n, 12)[:, torch.from_numpy(sub).cuda(), :9]
    g2d = g2d.cpu().numpy().astype(np.float64)  # [V][m][9]
    bits = r.ws_tensor("view_bits", torch.int32, n).cpu().numpy().view(np.uint32)[sub]
    opts = parity.opts_for((r.options.tile_w, r.options.tile_h))
    m = sub.size
    grads = np.zeros((11 + P.sh.shape[0], m))
    S = np.zeros(m)
    cnt = np.zeros(m, np.int32)
    lib = oracle.lib()
    for v, c in enumerate(s.cameras):
        proj = oracle.project(Ps, c, opts)
        gv = np.ascontiguousarray(g2d[v].T)  # [9][m]
        # the GPU only writes 2D gradients of records visible in its own view mask
        vis_gpu = ((bits >> v) & 1).astype(bool)
        amb = proj["margin"] < parity.DELTA
        assert np.array_equal(vis_gpu[~amb], proj["visible"][~amb].astype(bool))
        gv[:, ~vis_gpu] = 0.0
        lib.ora_project_bwd(oracle.ctypes.byref(opts), oracle.ctypes.byref(oracle.make_cam(c)), m, Ps.sh_degree,
                            oracle._p(Ps.means, oracle._d), oracle._p(Ps.log_scales, oracle._d),
                            oracle._p(Ps.quats, oracle._d), oracle._p(Ps.logits, oracle._d),
                            oracle._p(Ps.sh, oracle._d), None, oracle._p(gv, oracle._d), m, float(V),
                            oracle._p(grads, oracle._d), oracle._p(S, oracle._d), oracle._p(cnt, oracle._i32))
    gpu = parity.gpu_grad_groups({k: v_[..., torch.from_numpy(sub).cuda()] for k, v_ in r.grads.items()})
    excl = np.zeros(m, bool)
    for c in s.cameras:
        excl |= oracle.project(Ps, c, opts)["margin"] < parity.DELTA
    rep = {}
    parity.compare_grads(gpu, grads, excl, report=rep)
    Sg = r.S.cpu().numpy().astype(np.float64)[sub]
    rms = np.sqrt(np.mean(S ** 2))
    assert np.all(np.abs(Sg - S)[~excl] <= 1e-3 * (np.abs(S[~excl]) + 1e-2 * rms))
    assert np.array_equal(r.count.cpu().numpy()[sub][~excl], cnt[~excl])
    print("subset", m, rep)
