"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_01767_amd import scenes
from paper_2510_01767_amd import gsr as C
from paper_2510_01767_amd.raster import Rasterizer, camera_tensor, pack_images, scene_tensors, unpack_images
from tests import parity

pytestmark = pytest.mark.gpu

# Two GPU runs of the same arithmetic whose float32 atomic sums (the 2D
# gradients, up to a few hundred terms per entry) add up in different orders
# differ by ~1e-6 relative L2 on the small, cancelling quaternion gradient.
ATOMIC_ORDER_RTOL = 1e-5


def announce(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    C.load(build_if_missing=False)
    yield
    torch.cuda.synchronize()


def setup(scene, mode="plain", tile=(16, 16), **kw):
    sizes = [(c["W"], c["H"]) for c in scene.cameras]
    r = Rasterizer(scene.n, scene.sh_degree, sizes, mode=mode, tile=tile, **kw)
    params = scene_tensors(scene)
    cams = camera_tensor(scene.cameras)
    targets = torch.from_numpy(pack_images(scene.targets)).cuda()
    return r, params, cams, targets


_ORA = {}


def ora_step(scene, tile=(16, 16)):
    key = (scene.name, tile)
    if key not in _ORA:
        P = oracle.Params.from_scene(scene)
        _ORA[key] = oracle.step_l1(P, scene.cameras, scene.targets, parity.opts_for(tile))
    return _ORA[key]


@pytest.fixture(scope="module")
def c0():
    return scenes.config0()


@pytest.fixture(scope="module")
def ragged():
    return scenes.small_ragged()


def run_step(scene, **kw):
    r, params, cams, targets = setup(scene, **kw)
    r.S.zero_()
    r.count.zero_()
    loss, _ = r.step_l1(params, cams, targets)
    torch.cuda.synchronize()
    return r, params, cams, targets, float(loss.item())


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_config0_step_matches_oracle(c0, mode):
    announce("config0 step", mode)
    r, params, cams, targets, loss = run_step(c0, mode=mode)
    ora = ora_step(c0)
    rep = {}
    parity.compare_images(parity.gpu_images(r), ora, rep)
    assert abs(loss - ora["loss"]) <= 1e-5 * abs(ora["loss"])
    T = r.ws_tensor("pix_T", torch.float32, r.pixels).cpu().numpy()
    last = r.ws_tensor("pix_last", torch.int32, r.pixels).cpu().numpy()
    parity.compare_pixels([T.reshape(128, 128)], [last.reshape(128, 128)], ora)
    ex = parity.excluded_gaussians(ora, c0.n, parity.opts_for(), c0.targets)
    parity.assert_excluded_fraction(ex, ora["count"] > 0, rep)
    parity.compare_grads(parity.gpu_grad_groups(r.grads), ora["grads"], ex, report=rep)
    S = r.S.cpu().numpy().astype(np.float64)
    keep = ~ex
    np.testing.assert_allclose(S[keep], ora["S"][keep], rtol=1e-3, atol=1e-3 * np.sqrt(np.mean(ora["S"] ** 2)))
    assert np.array_equal(r.count.cpu().numpy()[keep], ora["count"][keep])
    print("report", rep)


@pytest.mark.parametrize("project_table", [0, 1])
@pytest.mark.parametrize("scene_name", ["config0", "ragged"])
def test_records_and_binning_bit_exact(scene_name, project_table, c0, ragged):
    scene = c0 if scene_name == "config0" else ragged
    announce("records/binning", scene_name, "project table", project_table)
    r, params, cams, targets, _ = run_step(scene, mode="batched", project_table=project_table)
    ora = ora_step(scene)
    n, V = scene.n, scene.n_views
    L = r.layout
    rec = parity.gpu_records(r)
    bits = parity.ws_np(r, "view_bits", torch.int32, n).view(np.uint32)
    for v in range(V):
        o = ora["records"][v]
        vis_g = ((bits >> v) & 1).astype(bool)
        amb = o["margin"] < parity.DELTA
        assert np.array_equal(vis_g[~amb], o["visible"][~amb].astype(bool))
        sel = vis_g & o["visible"].astype(bool)
        rv = rec[v * n:(v + 1) * n][sel]
        m2 = rv[:, 0:2].astype(np.float64) + rv[:, 2:4].astype(np.float64)
        np.testing.assert_allclose(m2, o["mean2d"][:, sel].T, rtol=0, atol=1e-9 * max(1.0, np.abs(o["mean2d"]).max()))
        # the exponent's base-2 coefficients log2(e) (-A/2, -B, -C/2), rounded once
        L2E = 1.0 / np.log(2.0)
        coef = np.stack([-0.5 * L2E * o["conic"][0], -L2E * o["conic"][1], -0.5 * L2E * o["conic"][2]])
        np.testing.assert_allclose(rv[:, 4:7], coef[:, sel].T, rtol=3e-7)
        np.testing.assert_allclose(rv[:, 7], o["opacity"][sel], rtol=3e-7)
        # colours are evaluated in float32 (48 SH terms): ~1e-7 absolute error
        np.testing.assert_allclose(rv[:, 8:11], o["color"][:, sel].T, rtol=0, atol=2e-6)
        np.testing.assert_allclose(rv[:, 14], o["depth"][sel], rtol=3e-7)
        # the per-record reach bounds every pixel centre where the oracle's
        # alpha clears alpha_min (used to cull entries per wavefront)
        reach = rv[:, 15].astype(np.float64)
        # pmin lower-bounds the exponent of every pair the alpha test accepts
        pmin = rv[:, 11].astype(np.float64) * np.log(2.0)  # stored in base 2
        np.testing.assert_array_less(pmin, np.log(parity.opts_for().alpha_min / o["opacity"][sel]) + 1e-12)
        idx = np.nonzero(sel)[0]
        W, H = scene.cameras[v]["W"], scene.cameras[v]["H"]
        ys, xs = np.mgrid[0:H, 0:W]
        amin = parity.opts_for().alpha_min
        for k in range(0, idx.size, max(1, idx.size // 200)):
            i = idx[k]
            A, B, Cc = o["conic"][:, i]
            dx = xs + 0.5 - o["mean2d"][0, i]
            dy = ys + 0.5 - o["mean2d"][1, i]
            al = o["opacity"][i] * np.exp(-0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy)
            hit = al >= amin * (1 - 1e-5)
            if hit.any():
                assert np.sqrt(dx[hit] ** 2 + dy[hit] ** 2).max() <= reach[k], (v, i)
    # binning and order against the oracle's own binning of its own records:
    # bit-identical bucket sizes, starts, record order and depth keys in every
    # tile that lists no Gaussian with an ambiguous decision
    ob = ora["bins"]
    starts = parity.ws_np(r, "tile_start", torch.int32, L.tiles_total + 1).view(np.uint32).astype(np.int64)
    keys = parity.ws_np(r, "keys", torch.int64, int(starts[-1])).view(np.uint64)
    ok_tiles = parity.unambiguous_tiles(ora)
    clean = 0
    for t in range(L.tiles_total):
        a0, a1 = ob["ranges"][t]
        vals = ob["values"][a0:a1]
        if not ok_tiles[t]:
            continue
        g = keys[starts[t]:starts[t + 1]]
        assert np.array_equal((g & 0xffffffff).astype(np.int64), vals), t
        assert np.array_equal((g >> 32).astype(np.uint32), ob["depth"][a0:a1]), t
        clean += 1
    assert clean == L.tiles_total  # these scenes have no ambiguous Gaussian
    assert starts[-1] == ob["count"]
    assert np.array_equal(np.diff(starts), ob["ranges"][:, 1] - ob["ranges"][:, 0])
    nonempty = np.diff(starts) > 0
    assert np.array_equal(starts[:-1][nonempty], ob["ranges"][nonempty, 0])


@pytest.mark.parametrize("red", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("mode", ["plain", "batched"])
@pytest.mark.parametrize("tile", [(16, 16), (32, 8), (8, 32)])
def test_ragged_multiview_matches_oracle(ragged, mode, tile, red):
    announce("ragged", mode, tile, "reduce", red)
    r, params, cams, targets, loss = run_step(ragged, mode=mode, tile=tile, bwd_reduce=red)
    ora = ora_step(ragged, tile)
    rep = {}
    parity.compare_images(parity.gpu_images(r), ora, rep)
    assert abs(loss - ora["loss"]) <= 1e-5 * abs(ora["loss"])
    ex = parity.excluded_gaussians(ora, ragged.n, parity.opts_for(tile), ragged.targets)
    # a dense scene: about a hundred Gaussians reach alpha_min / 2 at each pixel,
    # so each flagged pixel removes that many
    parity.assert_excluded_fraction(ex, ora["count"] > 0, rep, limit=parity.MAX_EXCLUDED_DENSE)
    parity.compare_grads(parity.gpu_grad_groups(r.grads), ora["grads"], ex, report=rep)
    print("report", rep)


def test_batched_equals_plain_and_is_deterministic(ragged):
    announce("batched vs plain")
    rp, *_ = run_step(ragged, mode="plain")
    rb, params, cams, targets, _ = run_step(ragged, mode="batched")
    ip, ib = rp.images.cpu().numpy(), rb.images.cpu().numpy()
    assert np.array_equal(ip, ib)
    # the same arithmetic; the tiles run in another order, so the float32
    # atomic sums of the 2D gradients add up in another order
    for k in rp.grads:
        a, b = rp.grads[k].cpu().numpy(), rb.grads[k].cpu().numpy()
        assert np.linalg.norm(a - b) <= ATOMIC_ORDER_RTOL * max(np.linalg.norm(b), 1e-30), k
    rb.step_l1(params, cams, targets, stats=False)
    torch.cuda.synchronize()
    assert np.array_equal(rb.images.cpu().numpy(), ib)


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_storage_order_does_not_change_results(ragged, mode):
    """Gaussians stored in Morton order (lanes of a wavefront then share
    tiles and take one count atomic per distinct tile): the oracle's results,
    images bit-identical to the random order, gradients the same up to the
    order of float atomics."""
    announce("storage order", mode)
    perm = scenes.morton_order(ragged.means)
    sm = ragged.reordered(perm)
    rr, *_ = run_step(ragged, mode=mode)
    rm, *_ = run_step(sm, mode=mode)
    assert np.array_equal(rr.images.cpu().numpy(), rm.images.cpu().numpy())
    for k in rr.grads:
        a = rm.grads[k].cpu().numpy()
        b = rr.grads[k].cpu().numpy()[..., perm]
        assert np.linalg.norm(a - b) <= ATOMIC_ORDER_RTOL * max(np.linalg.norm(b), 1e-30), k
    assert np.array_equal(rm.count.cpu().numpy(), rr.count.cpu().numpy()[perm])
    ora = ora_step(sm)
    ex = parity.excluded_gaussians(ora, sm.n, parity.opts_for((16, 16)), sm.targets)
    parity.compare_images(parity.gpu_images(rm), ora)
    parity.compare_grads(parity.gpu_grad_groups(rm.grads), ora["grads"], ex)


def test_stored_history_equals_recompute(ragged):
    announce("stored vs recompute")
    rr, *_ = run_step(ragged, mode="batched", bwd="recompute")
    rs, *_ = run_step(ragged, mode="batched", bwd="stored", capacity=200000, history_budget=1 << 30)
    assert rs.layout.history_entries > 0 and rs.counts().bwd_variant == C.GSR_BWD_STORED
    assert np.array_equal(rr.images.cpu().numpy(), rs.images.cpu().numpy())
    for k in rr.grads:
        a, b = rr.grads[k].cpu().numpy(), rs.grads[k].cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-5 * max(np.linalg.norm(b), 1e-30), k
    rsp, *_ = run_step(ragged, mode="plain", bwd="stored", capacity=200000, history_budget=1 << 30)
    for k in rr.grads:
        a, b = rr.grads[k].cpu().numpy(), rsp.grads[k].cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-5 * max(np.linalg.norm(b), 1e-30), k


def test_forward_backward_split_equals_fused_l1(ragged):
    announce("forward/backward split")
    rf, params, cams, targets, _ = run_step(ragged, mode="batched")
    r2, *_ = setup(ragged, mode="batched")
    img = r2.forward(params, cams)
    torch.cuda.synchronize()
    assert np.array_equal(img.cpu().numpy(), rf.images.cpu().numpy())
    # dL/dimage of the L1 loss, computed from the images
    d = torch.sign(img - targets)
    scales = []
    for (W, H) in r2.sizes:
        scales.append(torch.full((3 * W * H,), 1.0 / (3 * W * H * len(r2.sizes)), device="cuda"))
    d = d * torch.cat(scales)
    r2.backward(params, cams, d.contiguous())
    torch.cuda.synchronize()
    # the same arithmetic; only the order of the float32 atomic sums differs
    for k in rf.grads:
        a, b = r2.grads[k].cpu().numpy(), rf.grads[k].cpu().numpy()
        assert np.linalg.norm(a - b) <= ATOMIC_ORDER_RTOL * max(np.linalg.norm(b), 1e-30), k


def test_visibility_mask_matches_oracle(ragged):
    announce("visibility mask")
    r, params, cams, targets = setup(ragged, mode="batched")
    bits, keep, inb = r.visibility_mask(params, cams, aabb=ragged.block_aabb)
    P = oracle.Params.from_scene(ragged)
    ob, ok, oi = oracle.visibility_mask(P, ragged.cameras, parity.opts_for(), ragged.block_aabb)
    amb = np.zeros(ragged.n, bool)
    for c in ragged.cameras:
        amb |= oracle.project(P, c, parity.opts_for())["margin"] < parity.DELTA
    gb = bits.cpu().numpy().view(np.uint32)
    assert np.array_equal(gb[~amb], ob[~amb])
    assert np.array_equal(keep.cpu().numpy()[~amb], ok[~amb])
    assert np.array_equal(inb.cpu().numpy(), oi)
    # keep mask culls everywhere
    km = torch.ones(ragged.n, dtype=torch.uint8, device="cuda")
    km[::3] = 0
    bits2, _, _ = r.visibility_mask(params, cams, keep=km)
    g2 = bits2.cpu().numpy().view(np.uint32)
    assert np.all(g2[::3] == 0)


def test_graph_capture_replays_match_eager(ragged):
    announce("graph capture")
    r, params, cams, targets, loss0 = run_step(ragged, mode="batched")
    img0 = r.images.cpu().numpy().copy()
    g0 = {k: v.cpu().numpy().copy() for k, v in r.grads.items()}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        r.capture(params, cams, targets, stats=False)
    s.synchronize()
    for rep in range(3):
        r.images.zero_()
        for v in r.grads.values():
            v.fill_(7.0)
        torch.cuda.synchronize()
        r.launch(stream=s)
        s.synchronize()
        assert np.array_equal(r.images.cpu().numpy(), img0), rep
        assert abs(float(r.loss.item()) - loss0) <= 1e-7 * abs(loss0)
        for k in g0:
            a = r.grads[k].cpu().numpy()
            assert np.linalg.norm(a - g0[k]) <= ATOMIC_ORDER_RTOL * max(np.linalg.norm(g0[k]), 1e-30), (rep, k)
        # eager work between replays
        r.forward(params, cams)
        torch.cuda.synchronize()


def test_capacity_overflow_is_reported(ragged):
    announce("capacity overflow")
    r, params, cams, targets = setup(ragged, mode="batched", capacity=1000)
    r.step_l1(params, cams, targets, stats=False)
    c = r.counts(check=False)
    assert c.overflow == 1 and c.intersections_total > 1000
    with pytest.raises(C.GsrError) as e:
        r.counts()
    assert e.value.status == C.GSR_ERR_CAPACITY
    rp, params, cams, targets = setup(ragged, mode="plain", capacity=1000)
    with pytest.raises(C.GsrError) as e:
        rp.step_l1(params, cams, targets, stats=False)
    assert e.value.status == C.GSR_ERR_CAPACITY
    r2, *_ = setup(ragged, mode="batched", capacity=int(c.intersections_total))
    r2.step_l1(params, cams, targets, stats=False)
    c2 = r2.counts()
    assert c2.overflow == 0 and c2.intersections_total == c.intersections_total


def test_nonfinite_parameters_are_flagged(ragged):
    announce("nonfinite")
    r, params, cams, targets = setup(ragged, mode="batched", check_finite=1)
    params["log_scales"][1, 5] = float("nan")
    r.step_l1(params, cams, targets, stats=False)
    with pytest.raises(C.GsrError) as e:
        r.counts()
    assert e.value.status == C.GSR_ERR_NONFINITE


def test_counts_match_oracle(ragged):
    announce("counts")
    r, params, cams, targets, _ = run_step(ragged, mode="batched")
    c = r.counts()
    ora = ora_step(ragged)
    for v in range(ragged.n_views):
        assert abs(c.visible[v] - int(ora["records"][v]["visible"].sum())) <= int((ora["records"][v]["margin"] < parity.DELTA).sum())
    assert c.intersections_total == r.ws_tensor("tile_start", torch.int32, r.layout.tiles_total + 1)[-1].item()
    assert c.visible_union == int(sum((r_["visible"] > 0) for r_ in ora["records"]).astype(bool).sum())


def test_persistent_schedule_is_a_longest_first_permutation(ragged):
    announce("tile order")
    r, params, cams, targets, _ = run_step(ragged, mode="batched", tile=(8, 32))
    L = r.layout
    order = r.ws_tensor("tile_order", torch.int32, L.tiles_total).cpu().numpy()
    assert np.array_equal(np.sort(order), np.arange(L.tiles_total))
    starts = r.ws_tensor("tile_start", torch.int32, L.tiles_total + 1).cpu().numpy().astype(np.int64)
    lengths = np.diff(starts)[order]
    assert np.all(np.diff(np.minimum(lengths // 4, 1023)) <= 0)


def test_autograd_function_returns_library_gradients(ragged):
    announce("autograd")
    from paper_2510_01767_amd.raster import render_l1
    r, params, cams, targets = setup(ragged, mode="batched")
    leaves = {k: v.clone().requires_grad_(True) for k, v in params.items()}
    loss, images = render_l1(leaves, r, cams, targets)
    (2.0 * loss).backward()
    r2, *_ = run_step(ragged, mode="batched")
    for k in leaves:
        a = leaves[k].grad.cpu().numpy()
        b = 2.0 * r2.grads[k].cpu().numpy()
        assert np.linalg.norm(a - b) <= ATOMIC_ORDER_RTOL * max(np.linalg.norm(b), 1e-30), k


def test_render_backward_after_a_second_render_raises_or_matches_oracle(ragged):
    """Two renders on one Rasterizer, then the first one's backward: it must
    raise (its forward state was overwritten), never return another render's
    gradients; the second one's backward gives the oracle's gradients."""
    announce("autograd: stale forward")
    from paper_2510_01767_amd.raster import StaleForwardError, render
    r, params, cams, targets = setup(ragged, mode="batched")
    leaves1 = {k: v.clone().requires_grad_(True) for k, v in params.items()}
    leaves2 = {k: v.clone().requires_grad_(True) for k, v in params.items()}
    img1 = render(leaves1, r, cams)
    img2 = render(leaves2, r, cams)
    assert torch.equal(img1, img2)
    # dL/dimage of the L1 loss of the oracle's definition (mean over views of the per-view mean)
    sizes = r.sizes
    w = torch.cat([torch.full((3 * W * H,), 1.0 / (3 * W * H * len(sizes)), device="cuda") for W, H in sizes])
    loss1 = ((img1 - targets).abs() * w).sum()
    loss2 = ((img2 - targets).abs() * w).sum()
    with pytest.raises(StaleForwardError):
        loss1.backward()
    loss2.backward()
    ora = ora_step(ragged)
    ex = parity.excluded_gaussians(ora, ragged.n, parity.opts_for(), ragged.targets)
    g = {k: v.grad for k, v in leaves2.items()}
    parity.compare_grads(parity.gpu_grad_groups(g), ora["grads"], ex)
    # a render followed by its own backward before the next render is fine
    leaves3 = {k: v.clone().requires_grad_(True) for k, v in params.items()}
    ((render(leaves3, r, cams) - targets).abs() * w).sum().backward()
    for k in leaves3:  # equal up to the order of float atomics
        a, b = leaves3[k].grad, leaves2[k].grad
        assert float(torch.linalg.norm(a - b)) <= ATOMIC_ORDER_RTOL * float(torch.linalg.norm(b)), k


def test_autograd_functions_raise_on_capacity_overflow(ragged):
    announce("autograd: overflow")
    from paper_2510_01767_amd.raster import render, render_l1
    r, params, cams, targets = setup(ragged, mode="batched", capacity=1000)
    leaves = {k: v.clone().requires_grad_(True) for k, v in params.items()}
    with pytest.raises(C.GsrError) as e:
        render_l1(leaves, r, cams, targets)
    assert e.value.status == C.GSR_ERR_CAPACITY
    with pytest.raises(C.GsrError) as e:
        render(leaves, r, cams)
    assert e.value.status == C.GSR_ERR_CAPACITY


@pytest.mark.parametrize("tile", [(16, 16), (32, 8)])
def test_pair_counts_match_oracle(ragged, tile):
    """Per pixel, the pairs the profiling forward counts as blended equal the
    oracle's blended entries (the compositing weights alpha T > 0 before the
    stop), on pixels without ambiguous decisions; evaluated pairs lie between
    the blended ones and the walked list length `last`."""
    announce("pair counts", tile)
    r, params, cams, targets = setup(ragged, mode="batched", tile=tile)
    blended, evaluated = r.pair_counts(params, cams)
    torch.cuda.synchronize()
    P = oracle.Params.from_scene(ragged)
    fo = oracle.forward(P, ragged.cameras, parity.opts_for(tile))
    o = 0
    bl, ev = blended.cpu().numpy(), evaluated.cpu().numpy()
    last = r.ws_tensor("pix_last", torch.int32, r.pixels).cpu().numpy()
    for v, (W, H) in enumerate(r.sizes):
        amb = fo["ambiguous"][v].astype(bool).ravel()
        # the oracle's blended count: entries with alpha >= alpha_min before the stop
        n_bl = fo["blended"][v].ravel()
        b_ = bl[o:o + W * H]
        assert np.array_equal(b_[~amb], n_bl[~amb]), v
        e_ = ev[o:o + W * H]
        assert np.all(e_ >= b_) and np.all(e_ <= last[o:o + W * H])
        o += W * H
    assert int(bl.sum()) > 0
    # the reverse pass cannot follow a profiling render
    with pytest.raises(C.GsrError) as e:
        r.backward(params, cams, torch.zeros_like(r.images))
    assert e.value.status == C.GSR_ERR_STATE


def test_gpu_gradient_agrees_with_oracle_finite_differences():
    """GPU analytic gradient vs central differences of the FP64 oracle loss."""
    announce("gpu vs oracle FD")
    from tests.oracle_helpers import tiny_scene
    P, cams, targets = tiny_scene(seed=11, n=30)
    # float32-representable copies so that both sides see the same inputs
    P32 = oracle.Params(*[np.asarray(a, np.float32).astype(np.float64) for a in
                          (P.means, P.log_scales, P.quats, P.logits, P.sh)], P.sh_degree)
    T32 = [np.asarray(t, np.float32) for t in targets]
    sc = scenes.Scene("tiny", P32.means.astype(np.float32), P32.log_scales.astype(np.float32),
                      P32.quats.astype(np.float32), P32.logits.astype(np.float32), P32.sh.astype(np.float32),
                      P32.sh_degree, cams, T32, np.zeros(6, np.float32), {})
    r, params, cams_t, targets_t, _ = run_step(sc, mode="batched")
    gpu = parity.gpu_grad_groups(r.grads)
    flat = P32.flat()
    opts = parity.opts_for()
    rng = np.random.default_rng(0)
    n = P32.n
    sel = rng.choice(flat.size, 120, replace=False)
    T64 = [t.astype(np.float64) for t in T32]
    gflat = np.concatenate([gpu["means"].ravel(), gpu["log_scales"].ravel(), gpu["quats"].ravel(),
                            gpu["opacity_logits"].ravel(), gpu["sh_dc"].ravel(), gpu["sh_rest"].ravel()])
    # sh_dc and sh_rest are consecutive planes of the same sh array
    fd, ga = [], []
    for k in sel:
        h = 1e-6 * max(1.0, abs(flat[k]))
        vp, vm = flat.copy(), flat.copy()
        vp[k] += h
        vm[k] -= h
        fp = oracle.forward(P32.with_flat(vp), cams, opts)
        fm = oracle.forward(P32.with_flat(vm), cams, opts)
        f0 = ora_step(sc)
        same = all(np.array_equal(a, b) and np.array_equal(a, c) for a, b, c in
                   zip(fp["signature"], fm["signature"], f0["signature"]))
        same &= all(np.array_equal(np.sign(a - t), np.sign(b - t)) for a, b, t in zip(fp["images"], fm["images"], T64))
        if not same:
            continue
        lp = oracle.l1_loss(fp["images"], T64)[0]
        lm = oracle.l1_loss(fm["images"], T64)[0]
        fd.append((lp - lm) / (2 * h))
        ga.append(gflat[k])
    fd, ga = np.array(fd), np.array(ga)
    assert fd.size > 80
    rms = np.sqrt(np.mean(fd ** 2))
    assert np.linalg.norm(ga - fd) <= 1e-3 * np.linalg.norm(fd)
    assert np.all(np.abs(ga - fd) <= 1e-3 * (np.abs(fd) + 1e-2 * rms))
