"""Pins of the oracle's fast camera selection (Sec. 3.2): the composited
depth D = sum_i d_i alpha_i T_i shares its weights with the colour, so with
pure red / green Gaussians D = d_red C_r + d_green C_g at every pixel; the
back-projected points re-project to their pixel centres at depth D; blocks
that tile the points' box have ratios summing to 1; a hand-worked example."""
import math

import numpy as np

import oracle
from tests.oracle_helpers import cam, params


def test_depth_shares_the_colour_weights():
    # red Gaussian in front (camera z 3.8), green behind (4.3), both near the axis
    P = params([(0.02, -0.01, -0.2), (-0.03, 0.02, 0.3)], log_scales=[(math.log(0.2),) * 3] * 2,
               opacities=[0.6, 0.7], colors=[(1.0, 0.0, 0.0), (0.0, 1.0, 0.0)])
    c = cam(64, 48, 64.0)
    o = oracle.default_opts(tile_w=16, tile_h=16)
    fo = oracle.forward(P, [c], o)
    D, C = fo["depth"][0], fo["images"][0]
    d = fo["records"][0]["depth"]
    assert abs(d[0] - 3.8) < 1e-12 and abs(d[1] - 4.3) < 1e-12
    assert np.allclose(D, d[0] * C[0] + d[1] * C[1], rtol=1e-12, atol=1e-15)
    assert D.max() > 1.0  # the footprint covers pixels


def test_back_projection_reprojects_to_pixel_centres():
    rng = np.random.default_rng(1)
    # an exactly orthonormal rotation (so R^T is R's inverse to the last bit)
    R = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    c = cam(40, 30, 55.0, R=R, t=(0.3, -1.2, 9.0), cx=21.0, cy=13.5)
    D = rng.uniform(2.0, 30.0, (30, 40))
    p = oracle.back_project(D, c)
    Rm = np.asarray(c["R"]).reshape(3, 3)
    q = np.einsum("ab,bhw->ahw", Rm, p) + np.asarray(c["t"])[:, None, None]
    vs, us = np.mgrid[0:30, 0:40]
    assert np.allclose(q[2], D, rtol=1e-13)
    assert np.allclose(c["fx"] * q[0] / q[2] + c["cx"], us + 0.5, atol=1e-10)
    assert np.allclose(c["fy"] * q[1] / q[2] + c["cy"], vs + 0.5, atol=1e-10)


def test_blocks_tiling_the_points_give_ratios_summing_to_one():
    rng = np.random.default_rng(2)
    c = cam(32, 24, 30.0, t=(0.0, 0.0, 5.0))
    D = rng.uniform(1.0, 9.0, (24, 32))
    p = oracle.back_project(D, c).reshape(3, -1)
    lo, hi = p.min(axis=1) - 1e-3, p.max(axis=1) + 1e-3
    mid = 0.5 * (lo + hi)
    blocks = [(x0, y0, lo[2], x1, y1, hi[2]) for (x0, x1) in ((lo[0], mid[0]), (mid[0], hi[0]))
              for (y0, y1) in ((lo[1], mid[1]), (mid[1], hi[1]))]
    r = oracle.camera_coverage([D], [c], blocks, tau=0.1)
    assert r["counts"].sum() == 32 * 24
    assert abs(r["ratio"].sum() - 1.0) < 1e-12
    assert np.array_equal(r["selected"][0], r["ratio"][0] >= 0.1)


def test_hand_worked_two_by_two_view():
    # identity pose, camera at the origin, fx = fy = 2, cx = cy = 1: pixel
    # centres at offsets +-0.5 -> rays (+-0.25, +-0.25, 1)
    c = dict(R=np.eye(3), t=np.zeros(3), fx=2.0, fy=2.0, cx=1.0, cy=1.0, W=2, H=2)
    D = np.array([[4.0, 8.0], [2.0, 0.0]])
    p = oracle.back_project(D, c)
    assert np.allclose(p[:, 0, 0], (-1.0, -1.0, 4.0)) and np.allclose(p[:, 0, 1], (2.0, -2.0, 8.0))
    assert np.allclose(p[:, 1, 0], (-0.5, 0.5, 2.0)) and np.allclose(p[:, 1, 1], (0.0, 0.0, 0.0))
    r = oracle.camera_coverage([D], [c], [(-2, -2, 1, 0, 1, 5), (0, -3, 0, 3, 3, 10)], tau=0.3)
    # block 0 holds (-1,-1,4) and (-0.5,0.5,2); block 1 holds (2,-2,8) and the origin (z = 0 >= 0)
    assert r["counts"].tolist() == [[2, 2]]
    assert np.allclose(r["ratio"], [[0.5, 0.5]]) and r["selected"].tolist() == [[True, True]]
