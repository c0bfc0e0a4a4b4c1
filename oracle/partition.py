"""Load-balanced KD-tree scene partition with cutline refinement (Sec. 3.1,
App. A.5, Alg. 1), written from the algorithm's description.

TEST INFRASTRUCTURE ONLY, like the rest of this package.  Plain Python over
NumPy arrays; every comparison is made on the float32 values the library
receives.  Where the paper leaves a choice open, this follows the library's
documented reading:
  * the percentile q of a node's Gaussian centres along the split axis is the
    order statistic of index floor(q (m - 1)) of its m centres (q = 0.5 is
    the median of the initial cut); a node without centres is cut at the
    middle of its extent;
  * the split axis is x when the x extent is at least the y extent, else y;
  * boxes are half-open, [min, cut) on the left and [cut, max) on the right;
  * among leaves of equal workload the earliest created is split first;
  * after the refinement the children of the last evaluated split are kept;
  * a camera is selected when count / N_p >= tau, tau being the float32
    value, N_p the camera's pixel count.
"""
from __future__ import annotations

import math

import numpy as np

f32 = np.float32


def camera_in_box(points, offsets, cam, box, tau) -> bool:
    """Fast camera selection for one camera and one box (Sec. 3.2): the
    fraction of the camera's back-projected pixels inside the box is at least
    tau.  count >= tau * N_p is that comparison, exact in float64."""
    p = points[:, offsets[cam]:offsets[cam + 1]]
    if p.shape[1] == 0:
        return False
    lo, hi = np.asarray(box[:3], f32)[:, None], np.asarray(box[3:], f32)[:, None]
    count = int(np.all((p >= lo) & (p < hi), axis=0).sum())
    return count >= float(f32(tau)) * p.shape[1]


def split_axis(box) -> int:
    """0 (x) when the x extent is at least the y extent, else 1 (y)."""
    return 0 if (box[3] - box[0]) >= (box[4] - box[1]) else 1


def cut_at(box, axis, coords, q):
    """The cut of percentile q along `axis`: coords are the node's centres
    along that axis."""
    if len(coords) == 0:
        return f32(0.5) * (f32(box[axis]) + f32(box[3 + axis]))
    return np.sort(np.asarray(coords, f32))[int(math.floor(q * (len(coords) - 1)))]


def split(points, offsets, cams, box, axis, cut, tau):
    """Children boxes of a cut and the parent's cameras each one keeps."""
    bl, br = np.array(box, f32), np.array(box, f32)
    bl[3 + axis] = cut
    br[axis] = cut
    cl = [c for c in cams if camera_in_box(points, offsets, c, bl, tau)]
    cr = [c for c in cams if camera_in_box(points, offsets, c, br, tau)]
    return bl, br, cl, cr


def kd_partition(scene_aabb, centers, points, offsets, n_blocks, tau=0.1, steps=3, q_min=0.1, q_max=0.9,
                 trace=None):
    """Leaves [(box, cams)] in creation order.  trace, if a list, receives per
    split (node id, axis, [(q, cut, |C_L|, |C_R|) per evaluated split])."""
    centers = np.asarray(centers, f32)
    points = np.asarray(points, f32)
    root = np.asarray(scene_aabb, f32)
    in_root = np.all((centers >= root[:3, None]) & (centers < root[3:, None]), axis=0)
    leaves = [dict(box=root.copy(), cams=list(range(len(offsets) - 1)), pts=np.nonzero(in_root)[0], id=0)]
    next_id = 1
    while len(leaves) < n_blocks:
        # the leaf with the largest workload L = |C|
        k = max(range(len(leaves)), key=lambda j: (len(leaves[j]["cams"]), -leaves[j]["id"]))
        p = leaves.pop(k)
        a = split_axis(p["box"])
        coords = centers[a, p["pts"]]
        q_low, q_high, q = float(f32(q_min)), float(f32(q_max)), 0.5
        evals = []
        for _ in range(steps):
            cut = cut_at(p["box"], a, coords, q)
            bl, br, cl, cr = split(points, offsets, p["cams"], p["box"], a, cut, tau)
            evals.append((q, float(cut), len(cl), len(cr)))
            if len(cl) > len(cr):  # the left child is heavier: move the cut left
                q_high, q = q, 0.5 * (q_low + q)
            elif len(cr) > len(cl):
                q_low, q = q, 0.5 * (q_high + q)
            else:
                break
        if trace is not None:
            trace.append((p["id"], a, evals))
        left = coords < bl[3 + a]
        leaves.append(dict(box=bl, cams=cl, pts=p["pts"][left], id=next_id))
        leaves.append(dict(box=br, cams=cr, pts=p["pts"][~left], id=next_id + 1))
        next_id += 2
    leaves.sort(key=lambda d: d["id"])
    return [(d["box"], d["cams"]) for d in leaves]
