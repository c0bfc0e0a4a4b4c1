"""Pins of the oracle's guard band (the parity protocol's ambiguity rules).

Each discrete decision of the method is built by hand so that its margin is
just inside the band (the oracle must flag it) and just outside (it must
not): the ceiling of the footprint radius, a floor of the tile rectangle,
alpha against alpha_min and alpha_max, the transmittance stop, the order of
two entries whose depths nearly coincide, the float32 rounding of a depth
next to an entry of an adjacent float32 depth, the colour clamp and the
Jacobian clamp.  A last pin checks which Gaussians a flagged pixel removes
from the gradient comparison: those whose alpha reaches alpha_min / 2 there,
and no others.  The cases follow from the compositing conventions alone
(Sec. 3.2 blending sum, prior-art alpha rules); the expected flags are the
band widths stated in the oracle."""
import math

import numpy as np
import pytest

import oracle
from tests import parity
from tests.oracle_helpers import cam, params

O = oracle.default_opts()
F = 128.0
Z = 4.0
CAM = cam(128, 128, F, t=(0.0, 0.0, Z))


def fwd(P):
    return oracle.forward(P, [CAM], O)


def px_to_x(u, z_cam=Z):
    """World x (= camera x, R = I) whose projection is the image column u."""
    return (u - 64.0) * z_cam / F


# --------------------------------------------------------- per-Gaussian decisions


@pytest.mark.parametrize("m, flagged", [(1e-11, True), (-1e-11, True), (1e-7, False), (-1e-7, False)])
def test_radius_ceil_band(m, flagged):
    """On the optical axis an isotropic Gaussian has lambda = (f s / z)^2 + eps,
    so 3 sqrt(lambda) = 6 (1 - m) fixes s."""
    lam = (6.0 * (1.0 - m)) ** 2 / 9.0
    s = Z / F * math.sqrt(lam - O.eps2d)
    P = params([[0.0, 0.0, 0.0]], log_scales=[[math.log(s)] * 3])
    r = oracle.project(P, CAM, O)
    assert r["visible"][0] == 1
    assert r["radius"][0] == (6 if m > 0 else 7)
    assert (r["margin"][0] < oracle.DELTA_GAUSS) == flagged
    f = fwd(P)
    # a record with an ambiguous decision marks the pixels it can reach
    assert bool(f["ambiguous"][0].any()) == flagged


@pytest.mark.parametrize("m, flagged", [(3e-11, True), (-3e-11, True), (3e-7, False), (-3e-7, False)])
def test_rect_floor_band(m, flagged):
    """(mean_x - r) / 16 = 3 (1 + m) with r = 6 (s = 0.05 at z = 4, f = 128)."""
    u = 16.0 * 3.0 * (1.0 + m) + 6.0
    P = params([[px_to_x(u), 0.0, 0.0]], log_scales=[[math.log(0.05)] * 3])
    r = oracle.project(P, CAM, O)
    assert r["radius"][0] == 6
    assert r["rect"][0, 0] == (3 if m > 0 else 2)
    assert (r["margin"][0] < oracle.DELTA_GAUSS) == flagged


@pytest.mark.parametrize("m, flagged", [(1e-10, True), (1e-6, False)])
def test_jacobian_clamp_band(m, flagged):
    """x/z at 1.3 half fields of view times (1 + m): a kink of the gradient."""
    lim = O.jac_clamp * 0.5 * CAM["W"] / CAM["fx"]
    P = params([[lim * (1.0 + m) * 3.0, 0.0, -1.0]])
    r = oracle.project(P, CAM, O)
    assert (r["grad_margin"][0] < oracle.DELTA_GAUSS) == flagged


@pytest.mark.parametrize("raw, flagged", [(1e-8, True), (-1e-8, True), (1e-4, False), (-1e-4, False)])
def test_colour_clamp_band(raw, flagged):
    """Degree-0 colour c0 Y0 + 1/2 = raw on every channel."""
    P = params([[0.0, 0.0, 0.0]], colors=[[raw, raw, raw]])
    r = oracle.project(P, CAM, O)
    np.testing.assert_allclose(r["color_raw"][:, 0], raw, atol=1e-15)
    assert (r["color_margin"][0] < oracle.DELTA_COLOR) == flagged


# ------------------------------------------------------------ per-pair decisions


def gaussian_at_offset(d, opacity, z=0.0):
    """A Gaussian whose projected mean sits d pixels right of the centre of
    pixel (64, 64), found by a few fixed-point steps (the conic depends
    slightly on the position through J)."""
    u = 64.5 + d
    for _ in range(4):
        P = params([[px_to_x(u, Z + z), px_to_x(64.5, Z + z), z]], opacities=[opacity])
        r = oracle.project(P, CAM, O)
        u += (64.5 + d) - r["mean2d"][0, 0]
    return P, r


def alpha_at_offset(r, target, o):
    """Offset d of the mean right of the pixel centre (64.5, 64.5) at which
    o exp(p) = target, for the conic and vertical offset of projection r:
    the root dx < 0 of (A/2) dx^2 + B dy dx + (C/2) dy^2 = ln(o / target)."""
    A, B, C = r["conic"][:, 0]
    dy = 64.5 - r["mean2d"][1, 0]
    a, b, c = 0.5 * A, B * dy, 0.5 * C * dy * dy - math.log(o / target)
    dx = (-b - math.sqrt(b * b - 4 * a * c)) / (2 * a)
    return -dx


@pytest.mark.parametrize("m, flagged", [(1e-6, True), (-1e-6, True), (1e-4, False), (-1e-4, False)])
def test_alpha_min_band(m, flagged):
    o = 0.6
    target = O.alpha_min * (1.0 + m)
    P, r = gaussian_at_offset(1.0, o)
    for _ in range(8):
        P, r = gaussian_at_offset(alpha_at_offset(r, target, o), o)
    dx = 64.5 - r["mean2d"][0, 0]
    dy = 64.5 - r["mean2d"][1, 0]
    A, B, C = r["conic"][:, 0]
    raw = o * math.exp(-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy)
    assert abs(raw / target - 1.0) < 1e-9
    f = fwd(P)
    assert bool(f["ambiguous"][0][64, 64]) == flagged
    # a pixel well inside the footprint is never ambiguous
    nx = int(math.floor(r["mean2d"][0, 0]))
    assert not f["ambiguous"][0][64, nx]


@pytest.mark.parametrize("m, flagged", [(1e-6, True), (-1e-6, True), (1e-3, False), (-1e-3, False)])
def test_alpha_max_band(m, flagged):
    """At the pixel centre on the mean, o e^0 = o = 0.99 (1 + m)."""
    o = O.alpha_max * (1.0 + m)
    P = params([[px_to_x(64.5), px_to_x(64.5), 0.0]], opacities=[o])
    f = fwd(P)
    assert bool(f["ambiguous"][0][64, 64]) == flagged


@pytest.mark.parametrize("m, flagged", [(1e-6, True), (-1e-6, True), (1e-3, False), (-1e-3, False)])
def test_transmittance_stop_band(m, flagged):
    """Three Gaussians on the centre of pixel (64, 64) at increasing depth,
    opacities 0.95, 0.95, o3 with (0.05)^2 (1 - o3) = T_min (1 + m): the third
    is blended when m > 0 and stops the pixel when m < 0."""
    o3 = 1.0 - O.T_min * (1.0 + m) / 0.05 ** 2
    zs = [0.0, 0.2, 0.4]
    means = [[px_to_x(64.5, Z + z), px_to_x(64.5, Z + z), z] for z in zs]
    P = params(means, opacities=[0.95, 0.95, o3])
    f = fwd(P)
    assert f["last"][0][64, 64] == (3 if m > 0 else 2)
    assert bool(f["ambiguous"][0][64, 64]) == flagged


# ---------------------------------------------------------------- list order


@pytest.mark.parametrize("m, flagged", [(1e-10, True), (1e-6, False)])
def test_depth_gap_band(m, flagged):
    """Two Gaussians blending into pixel (64, 64) with camera depths z and
    z (1 + m): an order that another float64 evaluation could flip when m is
    inside the band.  Both depths are far from a float32 rounding boundary."""
    z1 = 0.3
    z2 = (Z + z1) * (1.0 + m) - Z
    means = [[px_to_x(64.5, Z + z), px_to_x(64.5, Z + z), z] for z in (z1, z2)]
    P = params(means, opacities=[0.4, 0.4])
    r = oracle.project(P, CAM, O)
    assert np.all(r["depth_margin"] > oracle.DELTA_DEPTH_ROUND)
    f = fwd(P)
    assert f["last"][0][64, 64] == 2
    assert bool(f["ambiguous"][0][64, 64]) == flagged


@pytest.mark.parametrize("ulps, flagged", [(1, True), (0, True), (3, False)])
def test_depth_rounding_next_to_adjacent_depth(ulps, flagged):
    """Record 1's camera depth lies exactly on the midpoint between the
    float32 value f and its successor (it could round either way); record 2's
    depth is the float32 value `ulps` steps above f.  The order of the two may
    flip only when their float32 depths can coincide or swap."""
    f = np.float32(4.3)
    up = np.nextafter(f, np.float32(np.inf))
    mid = 0.5 * (float(f) + float(up))
    d2 = float(f)
    for _ in range(ulps):
        d2 = float(np.nextafter(np.float32(d2), np.float32(np.inf)))
    means = [[px_to_x(64.5, d), px_to_x(64.5, d), d - Z] for d in (mid, d2)]
    P = params(means, opacities=[0.4, 0.4])
    r = oracle.project(P, CAM, O)
    assert r["depth"][0] == mid
    assert r["depth_margin"][0] < oracle.DELTA_DEPTH_ROUND
    fo = fwd(P)
    assert fo["last"][0][64, 64] == 2
    assert bool(fo["ambiguous"][0][64, 64]) == flagged
    # the tile lists the two in the same order either way only when not flagged
    assert parity.unambiguous_tiles(fo)[fo["tile_base"][0] + 4 * 8 + 4] == (not flagged)


# ------------------------------------------------------ what a flagged pixel removes


def test_flagged_pixel_removes_only_gaussians_reaching_it():
    """Gaussian 0 sits on pixel (64, 64); Gaussian 1 is in the same tile 7 px
    away, where its alpha at (64, 64) is far below alpha_min / 2; Gaussian 2
    is 2 px away (alpha above alpha_min / 2 there).  Flagging (64, 64)
    removes 0 and 2 only."""
    us = [64.5, 71.5, 66.5]
    P = params([[px_to_x(u), px_to_x(64.5), 0.0] for u in us], opacities=[0.5, 0.5, 0.5])
    fo = fwd(P)
    r = fo["records"][0]
    A = r["conic"][0]
    al = 0.5 * np.exp(-0.5 * A * (np.array(us) - 64.5) ** 2)
    assert al[1] < 0.5 * O.alpha_min <= al[2]
    mask = np.zeros((128, 128), bool)
    mask[64, 64] = True
    hit = oracle.touching(fo, [mask], O)
    assert list(hit) == [True, False, True]
    # no flagged pixel: nothing removed
    assert not oracle.touching(fo, [np.zeros((128, 128), bool)], O).any()


def test_blended_count_of_the_early_stop_stack():
    """Five identical Gaussians with alpha 0.95 on one pixel centre: three are
    blended (T = 0.05^3 = 1.25e-4 >= 1e-4), the fourth would take T below
    1e-4 and stops the pixel; `last` counts the three processed entries and
    the blended count is 3 (the closed form of the early-stop golden)."""
    zs = [0.0, 0.1, 0.2, 0.3, 0.4]
    means = [[px_to_x(64.5, Z + z), px_to_x(64.5, Z + z), z] for z in zs]
    f = fwd(params(means, opacities=[0.95] * 5))
    assert f["blended"][0][64, 64] == 3
    assert f["last"][0][64, 64] == 3
    np.testing.assert_allclose(f["T_final"][0][64, 64], 0.05 ** 3, rtol=1e-12)
