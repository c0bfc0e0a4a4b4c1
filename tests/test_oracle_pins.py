"""Pins of the FP64 oracle against facts that do not come from the oracle:
hand-derived worked examples (tests/golden/closed_forms.json), library
routines (scipy rotations, scipy spherical harmonics, numpy eigenvalues),
invariants of the compositing sum, brute force, and finite differences."""
import ctypes
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle
from tests.oracle_helpers import Y00, cam, params, tiny_scene

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
O = oracle.default_opts()


def render_one(P, c, opts=O):
    return oracle.forward(P, [c], opts)


def centre_pixel(f):
    return f["images"][0][:, 64, 64], f["T_final"][0][64, 64], f["last"][0][64, 64]


# ---------------------------------------------------------------- projection


def test_projection_worked_example():
    g = GOLD["projection"]
    c = cam(g["W"], g["H"], g["fx"], t=g["t"])
    P = params([g["mean"]])
    r = oracle.project(P, c, O)
    assert r["visible"][0] == 1
    np.testing.assert_allclose(r["mean2d"][:, 0], g["mean2d"], rtol=0, atol=1e-12)


def test_radius_and_rect_worked_example():
    g = GOLD["radius"]
    c = cam(128, 128, g["f"], t=(0, 0, g["z"]))
    rng = np.random.default_rng(0)
    for q in rng.standard_normal((5, 4)):  # isotropic: independent of the rotation
        P = params([[0.015625, 0.0, 0.0]], log_scales=[[math.log(g["scale"])] * 3], quats=[q])
        r = oracle.project(P, c, O)
        assert r["radius"][0] == g["radius"]
        assert list(r["rect"][:, 0]) == g["rect"]
        assert r["ntiles"][0] == g["ntiles"]
        # on the optical axis J = diag(f/z, f/z): Sigma_2D = (f s / z)^2 I + eps I
        Pa = params([[0.0, 0.0, 0.0]], log_scales=[[math.log(g["scale"])] * 3], quats=[q])
        ra = oracle.project(Pa, c, O)
        np.testing.assert_allclose(ra["cov2d"][:, 0], [g["lambda_max"], 0, g["lambda_max"]], atol=1e-12)
        assert ra["radius"][0] == g["radius"]


def pinhole(X, c):
    Xc = np.asarray(c["R"]) @ X + np.asarray(c["t"])
    return np.array([c["fx"] * Xc[0] / Xc[2] + c["cx"], c["fy"] * Xc[1] / Xc[2] + c["cy"]])


def fd_jacobian(X, c, h=1e-6):
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (pinhole(X + e, c) - pinhole(X - e, c)) / (2 * h)
    return J


def oblique_cam():
    R = Rotation.from_euler("xyz", [0.3, -0.2, 0.1]).as_matrix()
    return cam(96, 80, 90.0, R=R, t=(0.1, -0.2, 3.5), cx=47.0, cy=41.5)


@pytest.mark.parametrize("seed", range(6))
def test_cov2d_matches_library_rotation_and_fd_jacobian(seed):
    """Sigma_2D = J Sigma J^T + eps I with Sigma from scipy's rotation of the
    (w, x, y, z) quaternion and J the finite-difference Jacobian of the pinhole
    map (unclamped region)."""
    rng = np.random.default_rng(seed)
    c = oblique_cam()
    mu = rng.uniform(-0.5, 0.5, 3)
    ls = rng.normal(-2.0, 0.5, 3)
    q = rng.standard_normal(4) * rng.uniform(0.3, 3.0)
    P = params([mu], log_scales=[ls], quats=[q])
    r = oracle.project(P, c, O)
    Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    Sigma = Rq @ np.diag(np.exp(2 * ls)) @ Rq.T
    J = fd_jacobian(mu, c)
    S2 = J @ Sigma @ J.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(r["cov2d"][:, 0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-7)
    np.testing.assert_allclose(r["mean2d"][:, 0], pinhole(mu, c), rtol=1e-13)
    Q = np.linalg.inv(S2)
    np.testing.assert_allclose(r["conic"][:, 0], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-6)
    lam = np.linalg.eigvalsh(S2).max()
    assert r["radius"][0] == math.ceil(3 * math.sqrt(lam))
    np.testing.assert_allclose(r["depth"][0], (np.asarray(c["R"]) @ mu + c["t"])[2], rtol=1e-14)


def test_jacobian_clamp_evaluates_at_the_limit_point():
    """Beyond 1.3 half-fields of view the Jacobian is the one of the in-limit
    point at the same depth and height."""
    c = cam(64, 64, 64.0, t=(0, 0, 4.0))
    z = 4.0
    lim = 1.3 * 0.5 * 64 / 64.0
    for xr in (1.0, 1.5, -2.0):  # x/z beyond the limit of 0.65
        mu = np.array([xr * z, 0.1, 0.0])
        P = params([mu], log_scales=[[-1.5, -2.0, -2.5]], quats=[[0.9, 0.1, -0.3, 0.2]])
        r = oracle.project(P, c, O)
        q = P.quats[:, 0]
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Sigma = Rq @ np.diag(np.exp(2 * P.log_scales[:, 0])) @ Rq.T
        J = fd_jacobian(np.array([math.copysign(lim, xr) * z, 0.1, 0.0]), c)
        S2 = J @ Sigma @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(r["cov2d"][:, 0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-7)


def test_near_plane_culls():
    c = cam(t=(0, 0, 0.0))
    P = params([[0, 0, 0.005], [0, 0, 0.5]])
    r = oracle.project(P, c, O)
    assert list(r["visible"]) == [0, 1]


# ------------------------------------------------------------ spherical harmonics


def real_sh_scipy(l, m, d):
    theta = math.acos(max(-1.0, min(1.0, d[2])))
    phi = math.atan2(d[1], d[0])
    if m == 0:
        return float(np.real(sph_harm_y(l, 0, theta, phi)))
    Y = sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2) * float(np.real(Y) if m > 0 else np.imag(Y))


def test_sh_basis_matches_scipy_condon_shortley():
    rng = np.random.default_rng(1)
    for d in rng.standard_normal((25, 3)):
        d /= np.linalg.norm(d)
        Y, _ = oracle.sh_basis(3, d)
        ref = [real_sh_scipy(l, m, d) for l in range(4) for m in range(-l, l + 1)]
        np.testing.assert_allclose(Y, ref, atol=1e-13)


def test_sh_orthonormal_by_quadrature():
    x, w = np.polynomial.legendre.leggauss(24)
    nphi = 48
    Ys, ws = [], []
    for ct, wt in zip(x, w):
        st = math.sqrt(1 - ct * ct)
        for k in range(nphi):
            ph = 2 * math.pi * k / nphi
            Ys.append(oracle.sh_basis(3, np.array([st * math.cos(ph), st * math.sin(ph), ct]))[0])
            ws.append(wt * 2 * math.pi / nphi)
    Ys = np.array(Ys)
    G = (Ys * np.array(ws)[:, None]).T @ Ys
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_gradient_is_tangential_derivative():
    rng = np.random.default_rng(2)
    for d in rng.standard_normal((10, 3)):
        d /= np.linalg.norm(d)
        u = np.cross(d, rng.standard_normal(3))
        u /= np.linalg.norm(u)
        _, dY = oracle.sh_basis(3, d)
        h = 1e-6
        yp = oracle.sh_basis(3, (d + h * u) / np.linalg.norm(d + h * u))[0]
        ym = oracle.sh_basis(3, (d - h * u) / np.linalg.norm(d - h * u))[0]
        np.testing.assert_allclose(dY @ u, (yp - ym) / (2 * h), atol=1e-8)


def test_sh_degree0_is_constant_colour():
    rng = np.random.default_rng(4)
    cols = rng.uniform(0, 1, (50, 3))
    P = params(rng.uniform(-0.5, 0.5, (50, 3)), colors=cols)
    r = oracle.project(P, cam(), O)
    np.testing.assert_allclose(r["color"].T, cols, atol=1e-13)


# ------------------------------------------------------------- compositing


def test_single_gaussian_peak():
    g = GOLD["single_peak"]
    P = params([[0.015625, 0.015625, 0.0]], opacities=[g["opacity"]], colors=[g["color"]])
    C, T, last = centre_pixel(render_one(P, cam()))
    np.testing.assert_allclose(C, g["C"], atol=1e-12)
    assert abs(T - g["T_final"]) < 1e-12 and last == 1


def test_single_gaussian_footprint_is_the_alpha_ellipse():
    """T_final < 1 exactly on the lattice points with d^T Q d <= 2 ln(o / alpha_min)
    inside the tile rectangle, Q the inverse of the library-built covariance."""
    c = oblique_cam()
    o = 0.8
    mu = np.array([0.05, -0.02, 0.1])
    ls = np.array([-1.6, -2.4, -2.0])
    q = np.array([0.7, 0.2, -0.5, 0.3])
    P = params([mu], log_scales=[ls], quats=[q], opacities=[o])
    f = render_one(P, c)
    Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    S2 = fd_jacobian(mu, c) @ (Rq @ np.diag(np.exp(2 * ls)) @ Rq.T) @ fd_jacobian(mu, c).T + 0.3 * np.eye(2)
    Q = np.linalg.inv(S2)
    m2 = pinhole(mu, c)
    rect = f["records"][0]["rect"][:, 0]
    ys, xs = np.mgrid[0:c["H"], 0:c["W"]]
    d = np.stack([xs + 0.5 - m2[0], ys + 0.5 - m2[1]])
    e = np.einsum("i...,ij,j...->...", d, Q, d)
    inside = e <= 2 * math.log(o / O.alpha_min)
    tx, ty = xs // 16, ys // 16
    inside &= (tx >= rect[0]) & (tx <= rect[2]) & (ty >= rect[1]) & (ty <= rect[3])
    margin = np.abs(e - 2 * math.log(o / O.alpha_min))
    ok = margin > 1e-9
    assert inside.sum() > 20
    assert np.array_equal((f["T_final"][0] < 1.0)[ok], inside[ok])


def test_two_gaussian_stack_and_swap():
    g = GOLD["two_stack"]
    fr, bk = g["front"], g["back"]
    zb = 0.5  # the back mean is scaled so that it projects onto the same pixel centre
    P = params([[0.015625, 0.015625, 0.0], [0.015625 * (4 + zb) / 4, 0.015625 * (4 + zb) / 4, zb]],
               opacities=[fr["opacity"], bk["opacity"]], colors=[fr["color"], bk["color"]])
    C, T, _ = centre_pixel(render_one(P, cam()))
    np.testing.assert_allclose(C, g["C"], atol=1e-12)
    assert abs(T - g["T_final"]) < 1e-12
    # swap the depths: the back one is now in front (means scaled to keep the pixel)
    z2 = 0.5
    P2 = params([[0.015625 * (4 + z2) / 4, 0.015625 * (4 + z2) / 4, z2], [0.015625, 0.015625, 0.0]],
                opacities=[fr["opacity"], bk["opacity"]], colors=[fr["color"], bk["color"]])
    C2, T2, _ = centre_pixel(render_one(P2, cam()))
    exp = bk["opacity"] * np.array(bk["color"]) + (1 - bk["opacity"]) * fr["opacity"] * np.array(fr["color"])
    np.testing.assert_allclose(C2, exp, atol=1e-12)
    assert abs(T2 - g["T_final"]) < 1e-12


def test_early_stop_stack():
    g = GOLD["early_stop"]
    k = g["stack"]
    means = [[0.015625 * (4 + 0.1 * j) / 4, 0.015625 * (4 + 0.1 * j) / 4, 0.1 * j] for j in range(k)]
    P = params(means, opacities=[g["alpha"]] * k, colors=[[1.0, 0.5, 0.25]] * k)
    C, T, last = centre_pixel(render_one(P, cam()))
    assert last == g["blended"]
    assert abs(T - g["T_final"]) < 1e-15
    np.testing.assert_allclose(C, np.array([1.0, 0.5, 0.25]) * g["color_scale"], atol=1e-12)


@pytest.fixture(scope="module")
def ragged():
    from paper_2510_01767_amd import scenes
    s = scenes.small_ragged()
    return s, oracle.Params.from_scene(s)


def test_blend_weights_plus_transmittance_is_one(ragged):
    """With every colour 1 and bg 0 the image is sum alpha_i T_i = 1 - T_final;
    with bg 1 it is exactly 1."""
    s, P = ragged
    Pw = P.copy()
    Pw.sh[:] = 0
    Pw.sh[0:3] = 0.5 / Y00
    f = oracle.forward(Pw, s.cameras, O)
    for img, T in zip(f["images"], f["T_final"]):
        np.testing.assert_allclose(img, np.broadcast_to(1 - T, img.shape), atol=1e-12)
        assert T.min() >= 0 and T.max() <= 1
    fb = oracle.forward(Pw, s.cameras, oracle.default_opts(bg=(1.0, 1.0, 1.0)))
    for img in fb["images"]:
        np.testing.assert_allclose(img, 1.0, atol=1e-12)


def test_colour_in_convex_hull_and_transmittance_monotone(ragged):
    s, P = ragged
    f = oracle.forward(P, s.cameras, O)
    cmax = f["R"]["color"].max()
    for img, T in zip(f["images"], f["T_final"]):
        assert img.min() >= 0
        assert np.all(img <= (1 - T)[None] * cmax + 1e-12)
    # T never increases along a list: adding a Gaussian in front multiplies the
    # final transmittance by (1 - alpha) <= 1 wherever neither render stopped
    # early (an early stop may end a list sooner, at a larger T)
    Pf = P.copy()
    extra = params([[0.0, 0.0, -0.9]], log_scales=[[-1.0] * 3])
    for a in ("means", "log_scales", "quats", "sh"):
        setattr(Pf, a, np.concatenate([getattr(Pf, a), np.pad(getattr(extra, a), ((0, getattr(Pf, a).shape[0] - getattr(extra, a).shape[0]), (0, 0)))], 1))
    Pf.logits = np.concatenate([Pf.logits, extra.logits])
    f2 = oracle.forward(Pf, s.cameras, O)
    n = P.n
    for v, c in enumerate(s.cameras):
        W, H = c["W"], c["H"]
        gx = f["grids"][v][0]
        ys, xs = np.mgrid[0:H, 0:W]
        t = f["tile_base"][v] + (ys // 16) * gx + xs // 16
        len1 = f["bins"]["ranges"][t, 1] - f["bins"]["ranges"][t, 0]
        len2 = f2["bins"]["ranges"][t, 1] - f2["bins"]["ranges"][t, 0]
        full = (f["last"][v] == len1) & (f2["last"][v] == len2)
        assert full.mean() > 0.5
        assert np.all(f2["T_final"][v][full] <= f["T_final"][v][full] * (1 + 1e-14))
        assert np.any(f2["T_final"][v][full] < f["T_final"][v][full])


def test_binning_matches_python_brute_force(ragged):
    s, P = ragged
    f = oracle.forward(P, s.cameras, O)
    n = P.n
    entries = []
    for v in range(s.n_views):
        r = f["records"][v]
        gx = f["grids"][v][0]
        for i in range(n):
            if not r["visible"][i]:
                continue
            x0, y0, x1, y1 = r["rect"][:, i]
            db = int(np.float32(r["depth"][i]).view(np.uint32))
            for ty in range(y0, y1 + 1):
                for tx in range(x0, x1 + 1):
                    entries.append((int(f["tile_base"][v]) + ty * gx + tx, db, i, v * n + i))
    entries.sort()
    b = f["bins"]
    assert b["count"] == len(entries)
    assert np.array_equal(b["tiles"], [e[0] for e in entries])
    assert np.array_equal(b["depth"], [e[1] for e in entries])
    assert np.array_equal(b["values"], [e[3] for e in entries])


def test_binned_render_equals_per_pixel_brute_force(ragged):
    s, P = ragged
    f = oracle.forward(P, s.cameras, O)
    n = P.n
    L = oracle.lib()
    _p = oracle._p
    for v, c in enumerate(s.cameras):
        r = f["records"][v]
        W, H = c["W"], c["H"]
        img = np.zeros((3, H, W))
        T = np.zeros((H, W))
        last = np.zeros((H, W), np.int32)
        db = np.ascontiguousarray(np.float32(r["depth"]).view(np.uint32))
        tie = np.arange(n, dtype=np.int64)
        L.ora_render_brute(ctypes.byref(O), W, H, n, _p(r["visible"], oracle._i32), _p(np.ascontiguousarray(r["rect"]), oracle._i32),
                           _p(db, oracle._u32), _p(tie, oracle._i64), _p(r["mean2d"], oracle._d), _p(r["conic"], oracle._d),
                           _p(r["opacity"], oracle._d), _p(r["color"], oracle._d), _p(r["depth"], oracle._d),
                           _p(img, oracle._d), _p(T, oracle._d), _p(last, oracle._i32))
        assert np.array_equal(img, f["images"][v])
        assert np.array_equal(T, f["T_final"][v])
        assert np.array_equal(last, f["last"][v])


def test_l1_matches_numpy():
    rng = np.random.default_rng(5)
    imgs = [rng.uniform(0, 1, (3, 7, 9)), rng.uniform(0, 1, (3, 4, 5))]
    tg = [rng.uniform(0, 1, (3, 7, 9)), imgs[1].copy()]
    tg[1][0, 0, 0] += 0.5
    loss, grads = oracle.l1_loss(imgs, tg)
    exp = np.mean([np.abs(a - b).mean() for a, b in zip(imgs, tg)])
    assert abs(loss - exp) < 1e-15
    np.testing.assert_array_equal(grads[0], np.sign(imgs[0] - tg[0]) / (imgs[0].size * 2))
    assert np.count_nonzero(grads[1]) == 1  # sign(0) = 0


def test_visibility_mask_and_block_membership(ragged):
    s, P = ragged
    bits, keep, inb = oracle.visibility_mask(P, s.cameras, O, s.block_aabb)
    f = oracle.forward(P, s.cameras, O)
    n = P.n
    vals = f["bins"]["values"]
    for v in range(s.n_views):
        listed = np.zeros(n, bool)
        sel = vals[(vals >= v * n) & (vals < (v + 1) * n)] - v * n
        listed[sel] = True
        assert np.array_equal(((bits >> v) & 1).astype(bool), listed)
    assert np.array_equal(keep.astype(bool), bits != 0)
    lo, hi = s.block_aabb[:3].astype(np.float64), s.block_aabb[3:].astype(np.float64)
    for i in range(0, n, 7):
        m = P.means[:, i]
        assert inb[i] == int(all(lo[a] <= m[a] < hi[a] for a in range(3)))
    # a keep mask removes Gaussians from every view
    k2 = np.ones(n, np.uint8)
    k2[::2] = 0
    bits2, _, _ = oracle.visibility_mask(P, s.cameras, O, s.block_aabb, keep=k2)
    assert np.all(bits2[::2] == 0) and np.array_equal(bits2[1::2], bits[1::2])


# ----------------------------------------------------------------- gradients


def _signature(P, cams, targets):
    f = oracle.forward(P, cams, O)
    sig = [np.concatenate([x.ravel() for x in f["signature"]]),
           np.concatenate([x.ravel() for x in f["last"]]),
           np.concatenate([np.sign(a - b).ravel() for a, b in zip(f["images"], targets)]),
           np.concatenate([r["rect"].ravel() for r in f["records"]]),
           np.concatenate([r["color_raw"].ravel() > 0 for r in f["records"]])]
    return oracle.l1_loss(f["images"], targets)[0], sig


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.fixture(scope="module")
def tiny():
    P, cams, targets = tiny_scene()
    res = oracle.step_l1(P, cams, targets, O)
    return P, cams, targets, res


def test_tiny_scene_is_nontrivial(tiny):
    P, cams, targets, res = tiny
    assert res["bins"]["count"] > 60
    assert min(int(r["visible"].sum()) for r in res["records"]) > 20
    assert sum(int((l > 0).sum()) for l in res["last"]) > 500


def test_gradients_match_central_finite_differences(tiny):
    P, cams, targets, res = tiny
    flat = P.flat()
    ana = np.concatenate([res["grads"][0:3].ravel(), res["grads"][3:6].ravel(), res["grads"][6:10].ravel(),
                          res["grads"][10].ravel(), res["grads"][11:].ravel()])
    n = P.n
    K3 = P.sh.shape[0]
    group_rows = [("means", 3), ("log_scales", 3), ("quats", 4), ("logits", 1), ("sh", K3)]
    gids = np.concatenate([np.full(r * n, k) for k, (_, r) in enumerate(group_rows)])
    # every parameter of the first 12 Gaussians
    sel = np.nonzero(np.tile(np.arange(n) < 12, 3 + 3 + 4 + 1 + K3))[0]
    _, sig0 = _signature(P, cams, targets)
    fd = np.full(flat.size, np.nan)
    for k in sel:
        h = 1e-6 * max(1.0, abs(flat[k]))
        vp, vm = flat.copy(), flat.copy()
        vp[k] += h
        vm[k] -= h
        lp, sp = _signature(P.with_flat(vp), cams, targets)
        lm, sm = _signature(P.with_flat(vm), cams, targets)
        if _same(sp, sig0) and _same(sm, sig0):
            fd[k] = (lp - lm) / (2 * h)
    ok = ~np.isnan(fd)
    assert ok.sum() > 0.9 * sel.size
    for g, (name, _) in enumerate(group_rows):
        m = ok & (gids == g)
        a, b = ana[m], fd[m]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        assert rel < 1e-5, (name, rel)
        assert np.linalg.norm(b) > 0, name


def test_quaternion_gradient_invariants(tiny):
    P, cams, targets, res = tiny
    gq = res["grads"][6:10]
    # the loss does not depend on |q|: <dL/dq, q> = 0
    dots = np.sum(gq * P.quats, axis=0)
    assert np.max(np.abs(dots)) < 1e-12 * max(1.0, np.abs(gq).max()) + 1e-16
    # isotropic scales: the loss does not depend on q at all
    Pi = P.copy()
    Pi.log_scales[:] = Pi.log_scales.mean(axis=0, keepdims=True)
    ri = oracle.step_l1(Pi, cams, targets, O)
    assert np.abs(ri["grads"][6:10]).max() < 1e-12 * np.abs(ri["grads"][0:6]).max()


def test_logit_and_sh_chain_invariants(tiny):
    P, cams, targets, _ = tiny
    c = cams[:1]
    r = oracle.step_l1(P, c, targets[:1], O)
    o = 1 / (1 + np.exp(-P.logits))
    vis = r["records"][0]["visible"].astype(bool)
    np.testing.assert_allclose(r["grads"][10][vis], (o * (1 - o) * r["g2d"][5])[vis], rtol=1e-12, atol=1e-300)
    # dL/dc_{k,ch} / dL/dc_{0,ch} = Y_k(dir) / Y_0 where the colour is not clamped
    Rm, t = np.asarray(c[0]["R"]), np.asarray(c[0]["t"])
    centre = -Rm.T @ t
    for i in np.nonzero(vis)[0][:10]:
        d = P.means[:, i] - centre
        Y, _ = oracle.sh_basis(3, d / np.linalg.norm(d))
        for ch in range(3):
            if r["records"][0]["color_raw"][ch, i] <= 0:
                continue
            g0 = r["grads"][11 + ch, i]
            if abs(g0) < 1e-14:
                continue
            gk = r["grads"][11 + np.arange(16) * 3 + ch, i]
            np.testing.assert_allclose(gk / g0, Y / Y[0], rtol=1e-10)


def test_densification_statistic_matches_fd_in_screen_space(tiny):
    """S_i = V * |dL/dmean2d| per visible view; dL/dmean2d checked by central
    differences of the rasterize-only stage (records fixed, mean2d moved)."""
    P, cams, targets, res = tiny
    n = P.n
    V = len(cams)
    R = res["R"]
    L = oracle.lib()
    _p = oracle._p

    def loss_with(mean2d):
        total = 0.0
        for v, c in enumerate(cams):
            W, H = c["W"], c["H"]
            img = np.zeros((3, H, W)); T = np.zeros((H, W)); la = np.zeros((H, W), np.int32)
            rv = np.ascontiguousarray(res["bins"]["ranges"][res["tile_base"][v]:res["tile_base"][v] + res["tiles_per_view"][v]])
            L.ora_render(ctypes.byref(O), W, H, _p(rv, oracle._i64), _p(res["bins"]["values"], oracle._i64), n * V,
                         _p(mean2d, oracle._d), _p(R["conic"], oracle._d), _p(R["opacity"], oracle._d),
                         _p(R["color"], oracle._d), _p(R["depth"], oracle._d), None, 0.0, 0.0, 0.0,
                         _p(img, oracle._d), _p(T, oracle._d), _p(la, oracle._i32), None, None, None, None)
            total += np.abs(img - targets[v]).mean()
        return total / V

    checked = 0
    for r in np.nonzero(R["visible"])[0][:25]:
        g = np.zeros(2)
        for a in range(2):
            mp, mm = R["mean2d"].copy(), R["mean2d"].copy()
            mp[a, r] += 1e-6
            mm[a, r] -= 1e-6
            g[a] = (loss_with(mp) - loss_with(mm)) / 2e-6
        np.testing.assert_allclose(res["g2d"][0:2, r], g, rtol=1e-4, atol=1e-11)
        checked += 1
    assert checked >= 10
    S = np.zeros(n)
    for v in range(V):
        vis = res["records"][v]["visible"].astype(bool)
        S[vis] += V * np.hypot(res["g2d"][0, v * n:(v + 1) * n], res["g2d"][1, v * n:(v + 1) * n])[vis]
    np.testing.assert_allclose(res["S"], S, rtol=1e-12)
    assert np.array_equal(res["count"], sum(r["visible"] for r in res["records"]))
