"""Comparison rules between the HIP path and the FP64 oracle.

Tolerances: images and final transmittance within 1e-5 relative
(|gpu - ora| <= 1e-5 max(1, |ora|) per element on pixels whose discrete
decisions are not ambiguous, and relative L2 <= 1e-5 over whole images);
gradients within 1e-3 relative per parameter group (relative L2) and per
element |gpu - ora| <= 1e-3 (|ora| + 1e-2 rms_group).  A decision is
ambiguous when its FP64 relative margin is below the oracle's guard (per
Gaussian: 1e-9, both sides decide in float64; per pair: 4e-6 for the alpha
thresholds and 2e-5 for the stop, bounds on the float32 error of alpha and
of the transmittance); another correct implementation may take it either
way, so such pixels (and the Gaussians touching them) are left out of the
per-element checks and counted.
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
    assert n_amb <= 1e-3 * n_pix + 200, (n_amb, n_pix)
    return worst


def compare_pixels(gpu_T, gpu_last, ora):
    for v, (t, l) in enumerate(zip(gpu_T, gpu_last)):
        amb = ora["ambiguous"][v].astype(bool)
        o = ora["T_final"][v]
        err = np.abs(t - o) / np.maximum(1.0, np.abs(o))
        assert float(err[~amb].max()) <= IMG_TOL
        assert np.array_equal(l[~amb], ora["last"][v][~amb])


L1_KINK = 1e-5  # |image - target| below this: the L1 sign may differ (float32 image error ~1e-6)


def excluded_gaussians(ora, n, opts, targets=None):
    """Gaussians whose gradient may differ legitimately: those listed in a tile
    that holds an ambiguous pixel or (given the targets) a pixel on the L1
    kink, those with an ambiguous decision of their own, and those sitting on
    a kink (colour clamp, Jacobian clamp)."""
    ex = np.zeros(n, bool)
    vals = ora["bins"]["values"]
    ranges = ora["bins"]["ranges"]
    for v, amb in enumerate(ora["ambiguous"]):
        if targets is not None:
            amb = amb.astype(bool) | (np.abs(ora["images"][v] - targets[v]) < L1_KINK).any(axis=0)
        if not amb.any():
            continue
        gx, gy = ora["grids"][v]
        H, W = amb.shape
        tw, th = opts.tile_w, opts.tile_h
        pad = np.zeros((gy * th, gx * tw), bool)
        pad[:H, :W] = amb
        tiles = np.nonzero(pad.reshape(gy, th, gx, tw).any(axis=(1, 3)).ravel())[0]
        for t in tiles:
            gt = ora["tile_base"][v] + t
            s, e = ranges[gt]
            ex[vals[s:e] % n] = True
    for r in ora["records"]:
        ex |= r["margin"] < DELTA
        ex |= r["grad_margin"] < DELTA
    return ex


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
        elem = np.abs(a - b) - tol * (np.abs(b) + 1e-2 * rms)
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
