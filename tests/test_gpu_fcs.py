"""GPU parity of fast camera selection (Sec. 3.2): the composited depth of
gsr_render_depth against the oracle's and the block counts of
gsr_camera_coverage against the oracle's counts on its own depth maps.

Depth tolerance, derived like the image guard bands: D = sum_i w_i d_i with
the weights w_i = alpha_i T_i summing to at most 1; the float32 weights carry
the transmittance's relative error (at most 2e-5 after ~1000 factors) plus
alpha's (4e-6), so |D_gpu - D_ora| <= 3e-5 max(1, |D_ora|) on pixels whose
decisions are not ambiguous.  A count may differ by the points that could
flip under that depth error (within 3e-5 D |ray| of a block face) or that
sit on an ambiguous pixel."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_01767_amd import scenes
from paper_2510_01767_amd.raster import Rasterizer, camera_tensor, scene_tensors, unpack_images
from tests import parity

pytestmark = pytest.mark.gpu


def announce(*a):
    print("[gpu-case]", *a, flush=True)


def unpack_depth(depth, sizes):
    out, o = [], 0
    d = depth.cpu().numpy()
    for W, H in sizes:
        out.append(d[o:o + W * H].reshape(H, W).astype(np.float64))
        o += W * H
    return out


def compare_depth(gpu, fo):
    for v, (g, o) in enumerate(zip(gpu, fo["depth"])):
        amb = fo["ambiguous"][v].astype(bool)
        err = np.abs(g - o) / np.maximum(1.0, np.abs(o))
        assert float(err[~amb].max()) <= 3e-5, (v, float(err[~amb].max()))


def grid_blocks(means, nx, ny, pad=1.0):
    lo, hi = means.min(axis=1) - pad, means.max(axis=1) + pad
    xs, ys = np.linspace(lo[0], hi[0], nx + 1), np.linspace(lo[1], hi[1], ny + 1)
    return np.array([(xs[i], ys[j], lo[2], xs[i + 1], ys[j + 1], hi[2]) for i in range(nx) for j in range(ny)],
                    np.float32)


def check_coverage(r, cams, depth, blocks, fo, cameras):
    counts, ratio, sel = r.camera_coverage(cams, depth, torch.from_numpy(blocks).cuda(), tau=0.1)
    torch.cuda.synchronize()
    ora = oracle.camera_coverage(fo["depth"], cameras, blocks.astype(np.float64), tau=0.1, margin_rel=3e-5,
                                 ambiguous=fo["ambiguous"])
    c = counts.cpu().numpy().astype(np.int64)
    assert np.all(np.abs(c - ora["counts"]) <= ora["unsure"]), (c, ora["counts"], ora["unsure"])
    npix = np.array([cc["W"] * cc["H"] for cc in cameras], np.float64)[:, None]
    assert np.allclose(ratio.cpu().numpy(), c / npix, rtol=1e-6)
    # V >= tau exactly: count >= tau N_p, tau the float32 value
    assert np.array_equal(sel.cpu().numpy().astype(bool), c >= float(np.float32(0.1)) * npix)
    return c, ora


@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_depth_and_coverage_on_a_ragged_scene(mode):
    s = scenes.small_ragged()
    announce("fcs ragged", mode)
    sizes = [(c["W"], c["H"]) for c in s.cameras]
    r = Rasterizer(s.n, s.sh_degree, sizes, mode=mode)
    params, cams = scene_tensors(s), camera_tensor(s.cameras)
    img_f = r.forward(params, cams).clone()
    img, depth = r.render_depth(params, cams)
    torch.cuda.synchronize()
    assert torch.equal(img, img_f)  # the same forward, plus the depth channel
    fo = oracle.forward(oracle.Params.from_scene(s), s.cameras, parity.opts_for((16, 16)))
    compare_depth(unpack_depth(depth, sizes), fo)
    blocks = grid_blocks(s.means.astype(np.float64), 2, 2, pad=0.05)
    c, ora = check_coverage(r, cams, depth, blocks, fo, s.cameras)
    assert c.sum() > 0 and ora["unsure"].sum() < 0.01 * c.sum() + 10


@pytest.mark.timeout(900)
def test_coverage_at_the_bench_workload():
    s = scenes.config2()
    announce("fcs config2", s.n, s.n_views)
    sizes = [(c["W"], c["H"]) for c in s.cameras]
    r = Rasterizer(s.n, s.sh_degree, sizes, mode="batched", tile=(8, 32), lds_batch=256, grid_per_cu=8)
    params, cams = scene_tensors(s), camera_tensor(s.cameras)
    img, depth = r.render_depth(params, cams)
    torch.cuda.synchronize()
    P = oracle.Params.from_scene(s)
    opts = parity.opts_for((8, 32))
    gd = unpack_depth(depth, sizes)
    depths, ambs = [], []
    for v, c in enumerate(s.cameras):
        fo = oracle.forward(P, [c], opts)
        compare_depth([gd[v]], fo)
        depths.append(fo["depth"][0])
        ambs.append(fo["ambiguous"][0])
        del fo
    blocks = grid_blocks(s.means.astype(np.float64), 4, 4)
    c, ora = check_coverage(r, cams, depth, blocks, dict(depth=depths, ambiguous=ambs), s.cameras)
    print("coverage counts", c.sum(), "unsure", int(ora["unsure"].sum()), "selected", int(ora["selected"].sum()))
