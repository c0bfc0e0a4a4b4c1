"""GPU parity at the benchmark's full sizes.

Config 1 (1M Gaussians, one 1080p view) is checked whole.  Configs 2 (3M
Gaussians, 16 uneven views: the workload bench.py times, in its autotuned
batched launch) and 3 (8M Gaussians, 32 aerial 1080p views) are checked
stage by stage on outputs the oracle can compute one by one: images, tile
losses and 2D gradients of sampled views, and the parameter gradients and
densification statistics of a seeded 1 % subset of Gaussians against the
oracle's whole step (every view, forward and reverse).  Config 4 (20M Gaussians, 200+ per
pixel, 3840x2160) is checked on a window of one view: the oracle renders the
window through a camera cropped to it (same projection, same tile grid
phase, the Jacobian clamp scaled to the full frame), pixels, transmittance
and `last` are compared there, and 2D gradients of the records whose
footprint lies inside the window."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_01767_amd import gsr as C
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
    parity.assert_excluded_fraction(ex, ora["count"] > 0, rep)
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


def check_sampled_views(s, r, views):
    o = r.options
    opts = parity.opts_for((o.tile_w, o.tile_h))
    P = oracle.Params.from_scene(s)
    n, V = s.n, s.n_views
    gimgs = parity.gpu_images(r)
    L = r.layout
    g2d_all = r.ws_tensor("grad2d", torch.float32, C.GSR_SLOT_FLOATS * L.vn).view(-1, C.GSR_SLOT_FLOATS)
    tile_loss = r.ws_tensor("tile_loss", torch.float32, L.tiles_total).cpu().numpy().astype(np.float64)
    tile_base = 0
    bases = []
    for c in s.cameras:
        bases.append(tile_base)
        tile_base += ((c["W"] + o.tile_w - 1) // o.tile_w) * ((c["H"] + o.tile_h - 1) // o.tile_h)
    for v in views:
        c = s.cameras[v]
        W, H = c["W"], c["H"]
        announce(s.name, "view", v, W, H)
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
        amb = fo["ambiguous"][0].astype(bool)[None]
        assert np.all((d == d_g)[~kink & ~amb])
        bo = oracle.backward(P, [c], opts, fo, [d])
        vis = fo["records"][0]["visible"].astype(bool)
        # Gaussians touching an ambiguous pixel or one on the L1 kink
        ex = parity.excluded_gaussians(fo, n, opts, [s.targets[v]])
        parity.assert_excluded_fraction(ex, vis, rep)
        sel = vis & ~ex
        gg = parity.slot_grad2d(g2d_all[v * n:(v + 1) * n, :9].cpu().numpy()[sel], fo["records"][0]["conic"][:, sel])
        go = bo["g2d"].T[sel]
        for k in range(9):
            a_, b_ = gg[:, k], go[:, k]
            rel = np.linalg.norm(a_ - b_) / max(np.linalg.norm(b_), 1e-300)
            rms = np.sqrt(np.mean(b_ ** 2))
            assert rel <= 1e-3, (v, k, rel)
            assert np.all(np.abs(a_ - b_) <= 1e-3 * (np.abs(b_) + 1e-2 * rms)), (v, k)
        print("view", v, rep, "grad2d records checked", int(sel.sum()), "excluded", int((vis & ex).sum()))


def test_config2_sampled_views_match_oracle(c2):
    s, r, params, cams, targets = c2
    check_sampled_views(s, r, [int(np.argmin([c["W"] * c["H"] for c in s.cameras])), 0])


def check_subset(s, r):
    """Parameter gradients and statistics of a seeded 1 % of the Gaussians
    against the FP64 oracle's whole step, taken view by view (the view's
    forward, the L1 gradient of the oracle's own image, its reverse pass) and
    summed over the views."""
    n, V = s.n, s.n_views
    rng = np.random.default_rng(20251002)
    sub = np.sort(rng.choice(n, n // 100, replace=False))
    m = sub.size
    o = r.options
    opts = parity.opts_for((o.tile_w, o.tile_h))
    P = oracle.Params.from_scene(s)
    grads = np.zeros((11 + P.sh.shape[0], m))
    S = np.zeros(m)
    cnt = np.zeros(m, np.int64)
    excl = np.zeros(m, bool)
    for v, c in enumerate(s.cameras):
        fo = oracle.forward(P, [c], opts)
        d = np.sign(fo["images"][0] - s.targets[v]) / (3.0 * c["W"] * c["H"] * V)
        bo = oracle.backward(P, [c], opts, fo, [d], stat_scale=V)
        grads += bo["grads"][:, sub]
        S += bo["S"][sub]
        cnt += bo["count"][sub]
        excl |= parity.excluded_gaussians(fo, n, opts, [s.targets[v]])[sub]
        del fo, bo
    gpu = parity.gpu_grad_groups({k: v_[..., torch.from_numpy(sub).cuda()] for k, v_ in r.grads.items()})
    rep = {}
    parity.assert_excluded_fraction(excl, cnt > 0, rep)
    parity.compare_grads(gpu, grads, excl, report=rep)
    Sg = r.S.cpu().numpy().astype(np.float64)[sub]
    rms = np.sqrt(np.mean(S ** 2))
    assert np.all(np.abs(Sg - S)[~excl] <= 1e-3 * (np.abs(S[~excl]) + 1e-2 * rms))
    assert np.array_equal(r.count.cpu().numpy()[sub][~excl], cnt[~excl])
    print("subset", m, rep)


@pytest.mark.timeout(900)
def test_config2_gradients_on_a_subset(c2):
    s, r, params, cams, targets = c2
    check_subset(s, r)


@pytest.fixture(scope="module")
def c3():
    s = scenes.config3()
    announce("config3 scene", s.n, s.n_views)
    r, params, cams, targets = setup(s, mode="batched")
    best, ms = r.autotune(params, cams, targets, reps=1)
    announce("autotuned", best.tile_w, best.tile_h, best.lds_batch, best.grid_per_cu, ms)
    r.S.zero_()
    r.count.zero_()
    r.step_l1(params, cams, targets)
    torch.cuda.synchronize()
    return s, r


@pytest.mark.timeout(900)
def test_config3_sampled_views_match_oracle(c3):
    s, r = c3
    check_sampled_views(s, r, [0, s.n_views - 1])


@pytest.mark.timeout(900)
def test_config3_gradients_on_a_subset(c3):
    s, r = c3
    check_subset(s, r)


def window_camera(c, ox, oy, w, h, opts):
    """Camera cropped to the window [ox, ox + w) x [oy, oy + h) of c, and
    options with the Jacobian clamp scaled so that its limits (a fraction of
    the half frame over the focal length) stay those of the full frame."""
    assert c["W"] * h == c["H"] * w and c["W"] % w == 0
    wc = dict(c)
    wc["cx"] = c["cx"] - ox
    wc["cy"] = c["cy"] - oy
    wc["W"], wc["H"] = w, h
    o = oracle.default_opts(tile_w=opts.tile_w, tile_h=opts.tile_h)
    o.jac_clamp = opts.jac_clamp * (c["W"] // w)
    return wc, o


@pytest.mark.timeout(900)
def test_config4_window_matches_oracle():
    s = scenes.config4()
    announce("config4 scene", s.n, s.n_views)
    tile = (16, 16)
    r, params, cams, targets = setup(s, mode="batched", tile=tile, lds_batch=256, grid_per_cu=8)
    r.step_l1(params, cams, targets, stats=False)
    torch.cuda.synchronize()
    counts = r.counts()
    announce("config4 step", "intersections", counts.intersections_total, "pairs",
             int(r.ws_tensor("pix_last", torch.int32, r.pixels).sum().item()))
    v, (ox, oy, w, h) = 0, (1680, 960, 480, 270)
    c = s.cameras[v]
    W, H, V, n = c["W"], c["H"], s.n_views, s.n
    wc, wo = window_camera(c, ox, oy, w, h, parity.opts_for(tile))
    assert ox % tile[0] == 0 and oy % tile[1] == 0
    P = oracle.Params.from_scene(s)
    fo = oracle.forward(P, [wc], wo)
    img = parity.gpu_images(r)[v][:, oy:oy + h, ox:ox + w]
    rep = {}
    parity.compare_images([img], fo, rep)
    T = r.ws_tensor("pix_T", torch.float32, W * H).cpu().numpy().reshape(H, W)[oy:oy + h, ox:ox + w]
    last = r.ws_tensor("pix_last", torch.int32, W * H).cpu().numpy().reshape(H, W)[oy:oy + h, ox:ox + w]
    parity.compare_pixels([T], [last], fo)
    # 2D gradients of the records whose tiles lie strictly inside the window
    # (their whole footprint is window pixels), under the full frame's dL/dC
    t_img = s.targets[v][:, oy:oy + h, ox:ox + w]
    d = np.sign(fo["images"][0] - t_img) / (3.0 * W * H * V)
    bo = oracle.backward(P, [wc], wo, fo, [d])
    rec = fo["records"][0]
    gx, gy = fo["grids"][0]
    x0, y0, x1, y1 = rec["rect"]
    inner = rec["visible"].astype(bool) & (x0 >= 1) & (y0 >= 1) & (x1 <= gx - 2) & (y1 <= gy - 2)
    ex = parity.excluded_gaussians(fo, n, wo, [t_img])
    parity.assert_excluded_fraction(ex, inner, rep, limit=parity.MAX_EXCLUDED_DEEP)
    sel = np.nonzero(inner & ~ex)[0]
    L = r.layout
    g2d = r.ws_tensor("grad2d", torch.float32, C.GSR_SLOT_FLOATS * L.vn).view(-1, C.GSR_SLOT_FLOATS)
    gg = parity.slot_grad2d(g2d[v * n + torch.from_numpy(sel).cuda(), :9].cpu().numpy(), rec["conic"][:, sel])
    go = bo["g2d"].T[sel]
    assert sel.size > 1000, sel.size
    for k in range(9):
        a_, b_ = gg[:, k], go[:, k]
        rel = np.linalg.norm(a_ - b_) / max(np.linalg.norm(b_), 1e-300)
        rms = np.sqrt(np.mean(b_ ** 2))
        excess = np.abs(a_ - b_) - 1e-3 * (np.abs(b_) + parity.ELEM_FLOOR_DEEP * rms)
        if excess.max() > 0:
            w = np.argsort(-excess)[:5]
            print("component", k, "elements over", int((excess > 0).sum()), "of", excess.size, "rms", rms,
                  [(int(sel[j]), float(a_[j]), float(b_[j])) for j in w], flush=True)
        assert rel <= 1e-3, (k, rel)
        assert np.all(excess <= 0), k
    print("config4 window", rep, "records checked", sel.size, "depth complexity",
          float(fo["last"][0].mean()))
