"""Pins of the densification oracle (Sec. 3.3 with the vanilla 3DGS rules
of App. A.1): a hand-worked set of Gaussians covering keep / clone / split /
prune / out-of-block, the rotation against SciPy's quaternion conversion,
the children's spread against the parent's covariance, and the identities
that hold when densification and pruning are switched off."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import densify as od

f32 = np.float32


def gaussians(means, log_scales, quats, logits, sh_degree=0, seed=0):
    n = len(logits)
    K = (sh_degree + 1) ** 2
    rng = np.random.default_rng(seed)
    return dict(means=np.asarray(means, f32).T.copy(), log_scales=np.asarray(log_scales, f32).T.copy(),
                quats=np.asarray(quats, f32).T.copy(), opacity_logits=np.asarray(logits, f32),
                sh=rng.normal(size=(3 * K, n)).astype(f32))


def hand_set():
    I = (1, 0, 0, 0)
    small, big = [np.log(0.01)] * 3, [np.log(0.5)] * 3
    P = gaussians([(0, 0, 0), (1, 0, 0), (2, 0, 0), (3, 0, 0), (4, 0, 0), (5, 0, 0)],
                  [small, small, big, big, small, small], [I] * 6, [0.0, 0.0, 0.0, 0.0, -6.0, 0.0])
    S = np.array([1.0, 0.1, 3.0, 9.0, 9.0, 0.0], f32)
    n_seen = np.array([4, 1, 10, 3, 3, 0], np.uint32)
    in_block = np.array([1, 1, 1, 0, 1, 1], np.uint8)
    samples = np.zeros((2, 3, 6), f32)
    samples[0, 0, 2], samples[1, 1, 2] = 1.0, -2.0
    return P, S, n_seen, in_block, samples


def test_hand_worked_densification():
    # threshold 0.2: G0 0.25 (small: clone), G1 0.1 (keep), G2 0.3 (large:
    # split), G3 3.0 but outside the block (keep under SD), G4 3.0 but
    # opacity sigmoid(-6) = 0.0025 < 0.005 (pruned with its clone), G5 never
    # seen (keep)
    P, S, n_seen, in_block, samples = hand_set()
    m = {g: np.full_like(P[g], 7.0) for g in od.GROUPS}
    r = od.densify_prune(P, S, n_seen, in_block, samples, 0.2, 0.05, min_opacity=0.005, m=m, v=m)
    assert r["kind"].tolist() == [1, 0, 2, 0, 1, 0]
    assert r["parent"].tolist() == [0, 0, 1, 2, 2, 3, 5]
    out = r["params"]
    s = float(np.exp(np.float64(f32(np.log(0.5)))))
    assert np.allclose(out["means"][:, 3], (2 + s, 0, 0), atol=1e-12)
    assert np.allclose(out["means"][:, 4], (2, -2 * s, 0), atol=1e-12)
    assert np.allclose(np.exp(out["log_scales"][:, 3].astype(np.float64)), 0.5 / 1.6, rtol=1e-6)
    assert out["log_scales"][0, 3] == f32(f32(np.log(0.5)) - f32(np.log(1.6)))
    assert np.array_equal(out["means"][:, [0, 1, 2, 5, 6]], P["means"][:, [0, 0, 1, 3, 5]])
    assert np.array_equal(out["sh"], P["sh"][:, r["parent"]])
    # moments: the originals keep theirs, the clone and the children start at zero
    assert r["m"]["means"][0].tolist() == [7, 0, 7, 0, 0, 7, 7]
    # without SD the out-of-block G3 splits too
    r = od.densify_prune(P, S, n_seen, in_block, samples, 0.2, 0.05, min_opacity=0.005, selective=False)
    assert r["parent"].tolist() == [0, 0, 1, 2, 2, 3, 3, 5]
    # a size cap above the children's 0.3125 but below 0.5 prunes the large
    # Gaussian G3 and keeps G2's children
    r = od.densify_prune(P, S, n_seen, in_block, samples, 0.2, 0.05, max_world_scale=0.4)
    assert r["parent"].tolist() == [0, 0, 1, 2, 2, 4, 4, 5]


def test_clone_boundary_is_inclusive():
    P = gaussians([(0, 0, 0)], [[0.0, -1.0, -2.0]], [(1, 0, 0, 0)], [0.0])
    r = od.densify_prune(P, np.array([1.0], f32), np.array([1], np.uint32), np.array([1], np.uint8),
                         np.zeros((2, 3, 1), f32), 1.0, 1.0)
    assert r["kind"].tolist() == [1]  # largest scale exp(0) = 1 <= 1, and S / n = 1 >= 1
    r = od.densify_prune(P, np.array([1.0], f32), np.array([2], np.uint32), np.array([1], np.uint8),
                         np.zeros((2, 3, 1), f32), 0.5, 0.999)
    assert r["kind"].tolist() == [2]


def test_rotation_matches_scipy():
    rng = np.random.default_rng(3)
    q = rng.normal(size=(4, 200)) * rng.uniform(0.1, 5.0, 200)
    R = od.rotation(q)
    ref = Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], 1)).as_matrix()  # SciPy takes (x, y, z, w)
    assert np.allclose(R, ref, atol=1e-12)


def test_children_follow_the_parent_covariance():
    # many copies of one rotated anisotropic Gaussian, standard normal draws:
    # the children's positions have mean mu and covariance R diag(s^2) R^T
    n = 100_000
    q = np.array([0.9, 0.3, -0.2, 0.4])
    ls = np.log([2.0, 0.5, 0.1])
    P = gaussians(np.tile([1.0, 2.0, 3.0], (n, 1)), np.tile(ls, (n, 1)), np.tile(q, (n, 1)), np.zeros(n))
    rng = np.random.default_rng(4)
    samples = rng.standard_normal((2, 3, n)).astype(f32)
    r = od.densify_prune(P, np.ones(n, f32), np.ones(n, np.uint32), np.ones(n, np.uint8), samples, 0.5, 0.01)
    x = r["params"]["means"]
    Rs = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    s = np.exp(P["log_scales"][:, 0].astype(np.float64))
    cov = Rs @ np.diag(s ** 2) @ Rs.T
    assert np.allclose(x.mean(axis=1), (1, 2, 3), atol=0.03)
    assert np.allclose(np.cov(x), cov, atol=0.04 * np.abs(cov).max())


def test_switched_off_is_the_identity_and_keep_prunes():
    rng = np.random.default_rng(5)
    n = 500
    P = gaussians(rng.normal(size=(n, 3)), rng.normal(-3, 1, (n, 3)), rng.normal(size=(n, 4)),
                  rng.normal(size=n), sh_degree=2)
    S, cnt = rng.uniform(0, 1, n).astype(f32), rng.integers(0, 5, n).astype(np.uint32)
    blk = rng.integers(0, 2, n).astype(np.uint8)
    samples = rng.standard_normal((2, 3, n)).astype(f32)
    r = od.densify_prune(P, S, cnt, blk, samples, np.inf, 0.01)
    assert r["parent"].tolist() == list(range(n))
    for g in od.GROUPS:
        assert np.array_equal(r["params"][g], P[g])
    keep = rng.integers(0, 2, n).astype(np.uint8)
    r = od.densify_prune(P, S, cnt, blk, samples, np.inf, 0.01, keep=keep)
    assert r["parent"].tolist() == np.nonzero(keep)[0].tolist()
    # counts: every candidate yields two outputs
    r = od.densify_prune(P, S, cnt, blk, samples, 0.1, 0.05)
    kind = r["kind"]
    assert len(r["parent"]) == n + int((kind > 0).sum())
    assert not np.any(kind[blk == 0])
