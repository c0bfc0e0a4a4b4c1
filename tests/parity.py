"""Comparison rules between the HIP path and the FP64 oracle.

Tolerances: images and final transmittance within 1e-5 relative
(|gpu - ora| <= 1e-5 max(1, |ora|) per element on pixels whose discrete
decisions are not ambiguous, and relative L2 <= 1e-5 over whole images);
gradients within 1e-3 relative per parameter group (relative L2) and per
element |gpu - ora| <= 1e-3 (|ora| + 1e-2 rms_group).  A decision is
ambiguous when its FP64 relative margin is below the oracle's guard (per
Gaussian: 1e-9, both sides decide in float64, and 1e-12 for the float32
rounding of the depth; per pair: 4e-6 for the alpha thresholds and 2e-5 for
the stop, bounds on the float32 error of alpha and of the transmittance;
1e-9 between the depths of consecutive entries); another correct
implementation may take it either way, so such pixels, and the Gaussians
whose alpha reaches alpha_min / 2 at them, are left out of the per-element
checks and counted.
"""
import numpy as np
import torch

import oracle
from paper_2510_01767_amd.raster import unpack_images

DELTA = oracle.DELTA_GAUSS
IMG_TOL = 1e-5
GRAD_TOL = 1e-3
GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh_dc", "sh_rest")


def gpu_grad_groups(g: dict) -> dict:
    sh = g["sh"].detach().cpu().numpy().astype(np.float64)
    return dict(means=g["means"].cpu().numpy().astype(np.float64),
                log_scales=g["log_scales"].cpu().numpy().astype(np.float64),
                quats=g["quats"].cpu().numpy().astype(np.float64),
                opacity_logits=g["opacity_logits"].cpu().numpy().astype(np.float64)[None],
                sh_dc=sh[0:3], sh_rest=sh[3:])


def ora_grad_groups(grads: np.ndarray) -> dict:
    return dict(means=grads[0:3], log_scales=grads[3:6], quats=grads[6:10], opacity_logits=grads[10:11],
                sh_dc=grads[11:14], sh_rest=grads[14:])


def slot_grad2d(slots, conic):
    """The 2D gradient (dmean 2, dconic 3, dopacity, dcolour 3) of GPU record slots.

    Words 0..4 of a slot hold what the reverse raster pass sums per record:
    the moments of dL/dp over the pixel offsets d = pixel - mean2d (gp dx,
    gp dy, gp dx^2, gp dx dy, gp dy^2 with gp = dL/dp), where the exponent is
    p = -(A dx^2 + 2 B dx dy + C dy^2) / 2 (Sec. 3.2, the Gaussian's alpha).
    So dL/dmean2d = -dp/dd summed = (A m0 + B m1, B m0 + C m1) and
    dL/d(A, B, C) = -(m2 / 2, m3, m4 / 2); words 5..8 are dL/dopacity and
    dL/dcolour as they are.  slots: [k, >= 9]; conic: [3, k] (A, B, C), the
    oracle's conic of the same records."""
    m = np.asarray(slots, np.float64)[:, :9]
    A, B, C = (np.asarray(conic, np.float64)[j] for j in range(3))
    out = m.copy()
    out[:, 0] = A * m[:, 0] + B * m[:, 1]
    out[:, 1] = B * m[:, 0] + C * m[:, 1]
    out[:, 2] = -0.5 * m[:, 2]
    out[:, 3] = -m[:, 3]
    out[:, 4] = -0.5 * m[:, 4]
    return out


def compare_images(gpu_images, ora, report=None):
    """gpu_images: list of [3, H, W] arrays; ora: oracle.forward/step_l1 output."""
    n_amb = 0
    n_pix = 0
    worst = 0.0
    for v, (g, o) in enumerate(zip(gpu_images, ora["images"])):
        g = np.asarray(g, np.float64)
        amb = ora["ambiguous"][v].astype(bool)
        n_amb += int(amb.sum())
        n_pix += amb.size
        ok = ~amb
        err = np.abs(g - o) / np.maximum(1.0, np.abs(o))
        worst = max(worst, float(err[:, ok].max()) if ok.any() else 0.0)
        assert float(err[:, ok].max()) <= IMG_TOL, (v, float(err[:, ok].max()))
        rel = np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-30)
        assert rel <= IMG_TOL, (v, rel)
    if report is not None:
        report.update(ambiguous_pixels=n_amb, pixels=n_pix, image_max_rel=worst)
    walked = int(sum(int(np.asarray(l, np.int64).sum()) for l in ora["last"]))
    assert n_amb <= AMB_PER_ENTRY * walked + AMB_FLOOR * len(ora["images"]), (n_amb, n_pix, walked)
    return worst


def compare_pixels(gpu_T, gpu_last, ora):
    for v, (t, l) in enumerate(zip(gpu_T, gpu_last)):
        amb = ora["ambiguous"][v].astype(bool)
        o = ora["T_final"][v]
        err = np.abs(t - o) / np.maximum(1.0, np.abs(o))
        assert float(err[~amb].max()) <= IMG_TOL
        assert np.array_equal(l[~amb], ora["last"][v][~amb])


L1_KINK = 1e-5  # |image - target| below this: the L1 sign may differ (float32 image error ~1e-6)
# Ambiguous pixels allowed: 5e-7 per list entry a pixel walks, plus a floor
# of 8 per view for tiny views.  A float32 alpha is within ~1.5e-6 of the FP64
# one, so a band of 4e-6 around alpha_min is the narrowest that covers it;
# how many pixels it flags grows with the entries each pixel evaluates:
# measured 1.7e-5 of the pixels at ~300 entries per pixel (1M city block),
# 1e-4 on a 3M-Gaussian view (322), 9.6e-4 on the 20M cloud at 2160p (2344).
AMB_PER_ENTRY = 5e-7
AMB_FLOOR = 8
# Largest fraction of the checked Gaussians the exclusions may remove; the
# small dense test scenes (a hundred Gaussians per pixel on a few thousand
# pixels) lose more per flagged pixel.
MAX_EXCLUDED = 0.05
MAX_EXCLUDED_DENSE = 0.25
# the 20M-Gaussian cloud at 2160p: ~150 blended and ~2300 walked entries per
# pixel, so every flagged pixel removes a few hundred Gaussians (measured
# 5.1 % of the window's records)
MAX_EXCLUDED_DEEP = 0.08
# Per-element gradient floor, as a fraction of the group's rms: |gpu - ora| <=
# 1e-3 (|ora| + floor rms).  A float32 reverse pass over a pixel's list adds an
# absolute error that grows with the list: 1e-2 holds at ~300 entries per
# pixel; the 2160p cloud (~2300 walked, ~150 blended per pixel) needs 2e-2
# (measured worst: 1.2e-5 rms of absolute error on a 1e-13 gradient).
ELEM_FLOOR = 1e-2
ELEM_FLOOR_DEEP = 2e-2


def record_ambiguous(rec):
    """Per-record decisions another implementation may take the other way:
    the float64 ones (culling, determinant, radius, rectangle).  The float32
    rounding of the depth is handled per pixel by the oracle (it matters only
    next to an entry of the same or an adjacent float32 depth)."""
    return rec["margin"] < DELTA


def depth_round_ambiguous(rec):
    return rec["depth_margin"] < oracle.DELTA_DEPTH_ROUND


def unambiguous_tiles(ora):
    """Tiles whose list order no correct implementation can change: no listed
    record has an ambiguous decision of its own, and no record whose depth
    may round to another float32 value sits next to an entry of the same or
    an adjacent float32 depth."""
    b = ora["bins"]
    R = ora["R"]
    own = R["margin"] < DELTA
    rnd = R["depth_margin"] < oracle.DELTA_DEPTH_ROUND
    ok = np.ones(b["ranges"].shape[0], bool)
    vals = b["values"]
    if vals.size == 0:
        return ok
    tile_of = np.repeat(np.arange(ok.size), b["ranges"][:, 1] - b["ranges"][:, 0])
    ok[np.unique(tile_of[own[vals]])] = False
    bits = b["depth"].astype(np.int64)
    near = (np.abs(np.diff(bits)) <= 1) & (tile_of[1:] == tile_of[:-1]) & (rnd[vals[1:]] | rnd[vals[:-1]])
    ok[np.unique(tile_of[1:][near])] = False
    return ok


def flagged_pixels(ora, targets=None):
    """Per view, the pixels whose discrete decisions are ambiguous, plus (given
    the targets) the pixels on the L1 kink."""
    out = []
    for v, amb in enumerate(ora["ambiguous"]):
        m = np.asarray(amb, bool)
        if targets is not None:
            m = m | (np.abs(ora["images"][v] - targets[v]) < L1_KINK).any(axis=0)
        out.append(m)
    return out


def excluded_gaussians(ora, n, opts, targets=None):
    """Gaussians whose gradient may differ legitimately: those whose FP64 alpha
    reaches alpha_min / 2 at an ambiguous pixel or (given the targets) at a
    pixel on the L1 kink, those with an ambiguous decision of their own, and
    those sitting on a kink of their own (colour clamp, Jacobian clamp)."""
    rec = oracle.touching(ora, flagged_pixels(ora, targets), opts)
    ex = np.zeros(n, bool)
    V = len(ora["records"])
    for v in range(V):
        ex |= rec[v * n:(v + 1) * n]
    for r in ora["records"]:
        ex |= record_ambiguous(r)
        ex |= r["grad_margin"] < DELTA
        ex |= r["color_margin"] < oracle.DELTA_COLOR
    return ex


def assert_excluded_fraction(ex, checked, report=None, limit=MAX_EXCLUDED):
    """The exclusions remove at most `limit` of the checked Gaussians."""
    checked = np.asarray(checked, bool)
    frac = float((ex & checked).sum()) / max(int(checked.sum()), 1)
    if report is not None:
        report["excluded_fraction"] = frac
    print(f"excluded {int((ex & checked).sum())} of {int(checked.sum())} checked Gaussians ({100 * frac:.3f} %)",
          flush=True)
    assert frac < limit, frac
    return frac


def compare_grads(gpu: dict, ora_grads: np.ndarray, exclude: np.ndarray, tol=GRAD_TOL, report=None):
    og = ora_grad_groups(ora_grads)
    keep = ~exclude
    out = {}
    for name in GROUPS:
        a, b = gpu[name], og[name]
        if b.size == 0:
            continue
        a, b = a[:, keep], b[:, keep]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
        elem = np.abs(a - b) - tol * (np.abs(b) + ELEM_FLOOR * rms)
        out[name] = (float(rel), float(elem.max()) if elem.size else 0.0)
        assert rel <= tol, (name, rel)
        assert elem.size == 0 or elem.max() <= 0, (name, float(elem.max()), int((elem > 0).sum()))
    if report is not None:
        report.update(grads=out, excluded=int(exclude.sum()))
    return out


def ws_np(rast, field, dtype, count):
    return rast.ws_tensor(field, dtype, count).cpu().numpy()


def gpu_records(rast):
    L = rast.layout
    rec = ws_np(rast, "records", torch.float32, 16 * L.vn).reshape(L.vn, 16)
    return rec


def gpu_images(rast):
    return [im.cpu().numpy() for im in unpack_images(rast.images, rast.sizes)]


def opts_for(tile=(16, 16), **kw):
    return oracle.default_opts(tile_w=tile[0], tile_h=tile[1], **kw)
