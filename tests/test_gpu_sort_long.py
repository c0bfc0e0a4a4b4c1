"""Bit-exact tile binning and order on long tile lists.

The GPU's own records of a dense scene (tile rectangle and float32 depth bits
of every (view, Gaussian) record, and its visibility bits) are binned and
ordered by the FP64 oracle's integer binning; the GPU's keys must equal the
oracle's entry for entry and its tile ranges must be identical.  The scene
is built so that every length class of the per-tile sort occurs: one
wavefront in registers up to 1024 entries, a workgroup's run sort (two,
four or eight wavefronts in registers, then merges in LDS) up to 2048, 4096
and 8192, and runs of 8192 plus merge passes in global memory beyond."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_01767_amd import gsr as C
from paper_2510_01767_amd import scenes
from paper_2510_01767_amd.raster import Rasterizer, camera_tensor, scene_tensors
from tests import parity

pytestmark = pytest.mark.gpu

# length classes of the per-tile sort: (lowest, highest, path)
CLASSES = ((2, 1024, "k_sort_wave"), (1025, 2048, "k_sort_runs<2048>"), (2049, 4096, "k_sort_runs<4096>"),
           (4097, 8192, "k_sort_runs<8192>"), (8193, 1 << 31, "k_sort_runs<8192> + k_sort_big"))


@pytest.mark.parametrize("tile,project_table", [((16, 16), 0), ((8, 32), 0), ((16, 16), 1)])
def test_long_tile_binning_and_order_bit_exact(tile, project_table):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    C.load(build_if_missing=False)
    s = scenes.dense_cloud()
    n, V = s.n, s.n_views
    print("[gpu-case] long-tile sort", s.name, tile, "project table", project_table, flush=True)
    sizes = [(c["W"], c["H"]) for c in s.cameras]
    r = Rasterizer(n, s.sh_degree, sizes, mode="batched", tile=tile, capacity=8_000_000,
                   project_table=project_table)
    r.forward(scene_tensors(s), camera_tensor(s.cameras))
    torch.cuda.synchronize()
    counts = r.counts()
    assert counts.overflow == 0
    L = r.layout
    rec = parity.gpu_records(r).view(np.uint32)
    bits = parity.ws_np(r, "view_bits", torch.int32, n).view(np.uint32)
    visible = np.concatenate([((bits >> v) & 1).astype(np.int32) for v in range(V)])
    lo, hi = rec[:, 12], rec[:, 13]
    rect = np.stack([lo & 0xffff, lo >> 16, hi & 0xffff, hi >> 16]).astype(np.int32)
    depth_bits = rec[:, 14].copy()
    opts = parity.opts_for(tile)
    grids = [oracle.tile_grid(c, opts) for c in s.cameras]
    tpv = [a * b for a, b in grids]
    tile_base = np.concatenate([[0], np.cumsum(tpv)[:-1]]).astype(np.int64)
    assert sum(tpv) == L.tiles_total
    ob = oracle.bin_records(rect, visible, depth_bits, np.tile(np.arange(n, dtype=np.int64), V),
                            np.repeat(tile_base, n), np.repeat(np.array([g[0] for g in grids], np.int32), n),
                            L.tiles_total)
    starts = parity.ws_np(r, "tile_start", torch.int32, L.tiles_total + 1).view(np.uint32).astype(np.int64)
    assert starts[-1] == ob["count"] == counts.intersections_total
    lens = np.diff(starts)
    assert np.array_equal(lens, ob["ranges"][:, 1] - ob["ranges"][:, 0])
    nonempty = lens > 0
    assert np.array_equal(starts[:-1][nonempty], ob["ranges"][nonempty, 0])
    keys = parity.ws_np(r, "keys", torch.int64, int(starts[-1])).view(np.uint64)
    # the record slot v * n + i in the low word, the float32 depth bits in the high word
    assert np.array_equal((keys & 0xffffffff).astype(np.int64), ob["values"])
    assert np.array_equal((keys >> 32).astype(np.uint32), ob["depth"])
    seen = {}
    for a, b, path in CLASSES:
        k = int(((lens >= a) & (lens <= b)).sum())
        seen[path] = k
        assert k > 0, (path, a, b)
    print("tiles checked per sort path", seen, "longest", int(lens.max()), "entries", int(starts[-1]), flush=True)
