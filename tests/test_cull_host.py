"""The rasterization kernels' sub-block cull, built for the CPU.

The kernels skip an entry for a 16-pixel sub-block when the entry's alpha
cannot reach alpha_min at any pixel centre of it (the skipped pairs would add
nothing to the blending sum of Sec. 3.2, so the result is the same as
evaluating them).  tests/cull/cull_check.cpp compiles the kernels' own cull
functions (csrc/gsr_cull.h) on the host and compares them with brute force
over the pixel centres of random strips, for records made the way the
projection makes them: no sub-block holding a pixel whose float32 exponent
passes the per-pair test may be culled, and the cull must stay tight (it keeps
at most a few percent more sub-blocks than brute force finds)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_01767_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "cull", "cull_check.cpp")


@pytest.fixture(scope="module")
def cull_check(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("needs g++")
    exe = str(tmp_path_factory.mktemp("cull") / "cull_check")
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-Wall", "-Werror", "-I", CSRC, SRC,
                           "-o", exe])
    return exe


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cull_drops_no_sub_block_a_pixel_accepts(cull_check, seed):
    r = subprocess.run([cull_check, str(seed), "1000000"], capture_output=True, text=True, timeout=120)
    out = r.stdout + r.stderr
    m = re.search(r"tests (\d+) truth (\d+) kept (\d+) dropped (\d+) thin (\d+) special_failures (\d+)", out)
    assert m, out
    tests, truth, kept, dropped, thin, special = map(int, m.groups())
    assert dropped == 0, out
    assert special == 0, out
    assert r.returncode == 0, out
    assert truth > 0.2 * tests, out          # the strips do meet the records
    assert kept <= 1.03 * truth, out         # and the cull keeps little beyond what brute force finds
    assert 0 < thin < 0.01 * (tests // 4), out
