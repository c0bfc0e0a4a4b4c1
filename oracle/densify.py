"""Selective densification and pruning (Sec. 3.3), with the clone / split /
prune rules of vanilla 3DGS that the fine stage keeps (App. A.1), written
from their definitions.

TEST INFRASTRUCTURE ONLY, like the rest of this package.  NumPy, float64
for the geometry.  Readings that the library documents and this follows:
  * a Gaussian is a densification candidate when it was seen (n_i > 0), its
    mean view-space gradient norm S_i / n_i reaches the threshold and, under
    selective densification, its centre lies in the block (in_block);
  * candidates no larger than clone_max_scale (largest exp(log_scale)) are
    cloned, larger ones split into two children drawn from the Gaussian
    itself: mean + R (s * eps) with the caller's normal draws eps, scales
    s / (0.8 * 2), i.e. log scales log_scale - ln(1.6) rounded to float32;
  * every output is then pruned when its opacity sigmoid(logit) is below
    min_opacity or its largest scale exceeds max_world_scale (each test
    off when its threshold is 0), and Gaussians with keep = 0 yield nothing;
  * a kept or cloned original keeps its Adam moments, a clone or a child
    starts from zero moments;
  * outputs follow the input order, a Gaussian's outputs next to each other
    (original before its clone, child 0 before child 1).
"""
from __future__ import annotations

import numpy as np

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")
LN_1_6_F32 = np.float32(np.log(1.6))


def rotation(q):
    """Rotation matrices [n][3][3] of quaternions q [4][n] (w, x, y, z), after
    normalisation (the usual unit-quaternion formula)."""
    q = np.asarray(q, np.float64)
    w, x, y, z = q / np.linalg.norm(q, axis=0)
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def decide(params, S, n_seen, in_block, grad_threshold, clone_max_scale, selective=True):
    """Per Gaussian: 0 keep as is, 1 clone, 2 split."""
    S = np.asarray(S, np.float32).astype(np.float64)
    n_seen = np.asarray(n_seen, np.int64)
    seen = n_seen > 0
    with np.errstate(invalid="ignore"):  # an infinite threshold times n = 0
        mean_grad_reaches = seen & (S >= float(np.float32(grad_threshold)) * n_seen)  # S / n >= t, exactly
    cand = mean_grad_reaches & (np.asarray(in_block, bool) if selective else True)
    largest = np.exp(np.asarray(params["log_scales"], np.float32).astype(np.float64)).max(axis=0)
    small = largest <= float(np.float32(clone_max_scale))
    return np.where(cand, np.where(small, 1, 2), 0)


def survives(opacity_logit, log_scales, min_opacity, max_world_scale):
    ok = np.ones(np.asarray(opacity_logit).shape, bool)
    if min_opacity > 0:
        o = 1.0 / (1.0 + np.exp(-np.asarray(opacity_logit, np.float64)))
        ok &= o >= float(np.float32(min_opacity))
    if max_world_scale > 0:
        ok &= np.exp(np.asarray(log_scales, np.float64)).max(axis=0) <= float(np.float32(max_world_scale))
    return ok


def densify_prune(params, S, n_seen, in_block, samples, grad_threshold, clone_max_scale, min_opacity=0.0,
                  max_world_scale=0.0, selective=True, keep=None, m=None, v=None):
    """Returns dict(params, m, v (None without moments), parent [n_out],
    kind [n] of decide()).  params / m / v: dicts of float32 planes; samples
    [2][3][n] float32 normal draws."""
    n = np.asarray(params["opacity_logits"]).shape[-1]
    kind = decide(params, S, n_seen, in_block, grad_threshold, clone_max_scale, selective)
    ls = np.asarray(params["log_scales"], np.float32)
    child_ls = (ls - LN_1_6_F32).astype(np.float32)
    # the two children's means, float64: mean + R (exp(log_scale) * eps_j)
    R = rotation(params["quats"])
    s = np.exp(ls.astype(np.float64))
    child_mean = [np.asarray(params["means"], np.float64) +
                  np.einsum("nab,bn->an", R, s * np.asarray(samples[j], np.float64)) for j in range(2)]
    ok_self = survives(params["opacity_logits"], ls, min_opacity, max_world_scale)
    ok_child = survives(params["opacity_logits"], child_ls, min_opacity, max_world_scale)
    if keep is not None:
        ok_self &= np.asarray(keep, bool)
        ok_child &= np.asarray(keep, bool)
    # outputs per Gaussian: (parent, child index or -1, moments kept)
    outs = []
    for i in range(n):
        if kind[i] == 0 and ok_self[i]:
            outs.append((i, -1, True))
        elif kind[i] == 1 and ok_self[i]:
            outs += [(i, -1, True), (i, -1, False)]
        elif kind[i] == 2 and ok_child[i]:
            outs += [(i, 0, False), (i, 1, False)]
    parent = np.array([o[0] for o in outs], np.int64)
    child = np.array([o[1] for o in outs], np.int64)
    kept = np.array([o[2] for o in outs], bool)
    out = {g: np.asarray(params[g], np.float32)[..., parent].copy() for g in GROUPS}
    # children's means stay float64 here; the library rounds them once to float32
    out["means"] = out["means"].astype(np.float64)
    for j in range(2):
        sel = child == j
        out["means"][:, sel] = child_mean[j][:, parent[sel]]
        out["log_scales"][:, sel] = child_ls[:, parent[sel]]
    res = dict(params=out, parent=parent, kind=kind, m=None, v=None)
    if m is not None:
        for name, st in (("m", m), ("v", v)):
            res[name] = {g: np.where(kept, np.asarray(st[g], np.float32)[..., parent], np.float32(0)) for g in GROUPS}
    return res
