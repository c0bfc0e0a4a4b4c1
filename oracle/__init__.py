"""FP64 CPU oracle of the differentiable Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the rasterizer library
and its Python binding never do.  It shares no code with the HIP path: the
arithmetic lives in ``gsr_oracle.c`` (plain C, double precision) and this
module only marshals NumPy arrays through ctypes and strings the stages
together in the order the method defines (project -> bin/order -> composite
-> L1 -> reverse compositing -> reverse projection).

Every scene input is float32 (as generated) and is upcast to float64 here.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libgsr_oracle.so")
_lib = None

GRAD_GROUPS = ("means", "log_scales", "quats", "logits", "sh_dc", "sh_rest")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        other = os.environ.get("GSR_ORACLE_LIBRARY")  # another build of this oracle (sanitizer runs)
        if other:
            _lib = ctypes.CDLL(other)
            _declare(_lib)
            return _lib
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


class Opts(ctypes.Structure):
    _fields_ = [
        ("near_plane", ctypes.c_double), ("far_plane", ctypes.c_double),
        ("eps2d", ctypes.c_double), ("sigma_extent", ctypes.c_double),
        ("jac_clamp", ctypes.c_double), ("alpha_min", ctypes.c_double),
        ("alpha_max", ctypes.c_double), ("T_min", ctypes.c_double),
        ("bg", ctypes.c_double * 3), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
    ]


class Cam(ctypes.Structure):
    _fields_ = [
        ("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3),
        ("fx", ctypes.c_double), ("fy", ctypes.c_double),
        ("cx", ctypes.c_double), ("cy", ctypes.c_double),
        ("W", ctypes.c_int32), ("H", ctypes.c_int32),
    ]


def default_opts(tile_w=16, tile_h=16, bg=(0.0, 0.0, 0.0), **kw) -> Opts:
    """Conventions of the vanilla 3DGS rasterizer that the paper trains with
    (App. A.1); each one is a named field."""
    o = Opts()
    o.near_plane = 0.01
    o.far_plane = 1e10
    o.eps2d = 0.3
    o.sigma_extent = 3.0
    o.jac_clamp = 1.3
    # the thresholds are the float32 values a float32 kernel compares against
    o.alpha_min = float(np.float32(1.0 / 255.0))
    o.alpha_max = float(np.float32(0.99))
    o.T_min = float(np.float32(1e-4))
    o.bg = (ctypes.c_double * 3)(*bg)
    o.tile_w = tile_w
    o.tile_h = tile_h
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def make_cam(c) -> Cam:
    cam = Cam()
    cam.R = (ctypes.c_double * 9)(*np.asarray(c["R"], np.float32).astype(np.float64).ravel())
    cam.t = (ctypes.c_double * 3)(*np.asarray(c["t"], np.float32).astype(np.float64))
    cam.fx, cam.fy = float(np.float32(c["fx"])), float(np.float32(c["fy"]))
    cam.cx, cam.cy = float(np.float32(c["cx"])), float(np.float32(c["cy"]))
    cam.W, cam.H = int(c["W"]), int(c["H"])
    return cam


_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)
_u32 = ctypes.POINTER(ctypes.c_uint32)
_u8 = ctypes.POINTER(ctypes.c_uint8)
_O = ctypes.POINTER(Opts)
_C = ctypes.POINTER(Cam)


def _declare(L):
    L.ora_sh_basis.argtypes = [ctypes.c_int, _d, _d, _d]
    L.ora_project.argtypes = [_O, _C, ctypes.c_int64, ctypes.c_int, _d, _d, _d, _d, _d, _u8,
                              _i32, _d, _d, _d, _d, _d, _d, _d, _i32, _i32, _i32, _d, _d, _d, _d]
    L.ora_bin.restype = ctypes.c_int64
    L.ora_bin.argtypes = [ctypes.c_int64, _i32, _i32, _u32, _i64, _i64, _i32, ctypes.c_int64,
                          ctypes.c_int64, _i64, _u32, _i64, _i64]
    L.ora_render.argtypes = [_O, ctypes.c_int32, ctypes.c_int32, _i64, _i64, ctypes.c_int64,
                             _d, _d, _d, _d, _d, _u8, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                             _d, _d, _i32, _d, _u8, _i64, _i32]
    L.ora_render_brute.argtypes = [_O, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _i32, _i32,
                                   _u32, _i64, _d, _d, _d, _d, _d, _d, _d, _i32]
    L.ora_render_bwd.argtypes = [_O, ctypes.c_int32, ctypes.c_int32, _i64, _i64, ctypes.c_int64,
                                 _d, _d, _d, _d, _d, _d, _d]
    L.ora_project_bwd.argtypes = [_O, _C, ctypes.c_int64, ctypes.c_int, _d, _d, _d, _d, _d, _u8,
                                  _d, ctypes.c_int64, ctypes.c_double, _d, _d, _i32]
    L.ora_l1.restype = ctypes.c_double
    L.ora_l1.argtypes = [ctypes.c_int64, _d, _d, ctypes.c_double, _d]


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def sh_basis(degree: int, direction) -> tuple[np.ndarray, np.ndarray]:
    d = np.ascontiguousarray(direction, np.float64)
    K = (degree + 1) ** 2
    Y = np.zeros(K)
    dY = np.zeros(3 * K)
    lib().ora_sh_basis(degree, _p(d, _d), _p(Y, _d), _p(dY, _d))
    return Y, dY.reshape(K, 3)


@dataclasses.dataclass
class Params:
    """FP64 copies of the Gaussian parameters (SoA planes)."""
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self):
        return self.means.shape[1]

    @staticmethod
    def from_scene(s) -> "Params":
        f = lambda a: np.ascontiguousarray(a, np.float64)
        return Params(f(s.means), f(s.log_scales), f(s.quats), f(s.opacity_logits), f(s.sh),
                      s.sh_degree)

    def flat(self) -> np.ndarray:
        return np.concatenate([self.means.ravel(), self.log_scales.ravel(), self.quats.ravel(),
                               self.logits.ravel(), self.sh.ravel()])

    def with_flat(self, v) -> "Params":
        n = self.n
        K3 = self.sh.shape[0]
        o = 0
        parts = []
        for rows in (3, 3, 4, 1, K3):
            parts.append(np.ascontiguousarray(v[o:o + rows * n].reshape(rows, n)))
            o += rows * n
        return Params(parts[0], parts[1], parts[2], parts[3][0].copy(), parts[4], self.sh_degree)

    def copy(self):
        return Params(self.means.copy(), self.log_scales.copy(), self.quats.copy(),
                      self.logits.copy(), self.sh.copy(), self.sh_degree)


def project(P: Params, cam: dict, opts: Opts, keep=None) -> dict:
    n = P.n
    out = dict(
        visible=np.zeros(n, np.int32), mean2d=np.zeros((2, n)), conic=np.zeros((3, n)),
        cov2d=np.zeros((3, n)), depth=np.zeros(n), opacity=np.zeros(n),
        color=np.zeros((3, n)), color_raw=np.zeros((3, n)), radius=np.zeros(n, np.int32),
        rect=np.zeros((4, n), np.int32), ntiles=np.zeros(n, np.int32),
        margin=np.zeros(n), grad_margin=np.zeros(n), depth_margin=np.zeros(n), color_margin=np.zeros(n),
    )
    c = make_cam(cam)
    kp = None if keep is None else np.ascontiguousarray(keep, np.uint8)
    lib().ora_project(ctypes.byref(opts), ctypes.byref(c), n, P.sh_degree,
                      _p(P.means, _d), _p(P.log_scales, _d), _p(P.quats, _d), _p(P.logits, _d),
                      _p(P.sh, _d), _p(kp, _u8),
                      *[_p(out[k], _i32 if out[k].dtype == np.int32 else _d) for k in (
                          "visible", "mean2d", "conic", "cov2d", "depth", "opacity", "color",
                          "color_raw", "radius", "rect", "ntiles", "margin", "grad_margin",
                          "depth_margin", "color_margin")])
    return out


def tile_grid(cam, opts):
    tx = (cam["W"] + opts.tile_w - 1) // opts.tile_w
    ty = (cam["H"] + opts.tile_h - 1) // opts.tile_h
    return tx, ty


def bin_records(rect, visible, depth_bits, tiebreak, tile_base, tiles_x, n_tiles_total):
    """Integer binning and ordering over concatenated records (see ora_bin)."""
    rect = np.ascontiguousarray(rect, np.int32)
    visible = np.ascontiguousarray(visible, np.int32)
    depth_bits = np.ascontiguousarray(depth_bits, np.uint32)
    tiebreak = np.ascontiguousarray(tiebreak, np.int64)
    tile_base = np.ascontiguousarray(tile_base, np.int64)
    tiles_x = np.ascontiguousarray(tiles_x, np.int32)
    nr = visible.shape[0]
    L = lib()
    args = (nr, _p(rect, _i32), _p(visible, _i32), _p(depth_bits, _u32), _p(tiebreak, _i64),
            _p(tile_base, _i64), _p(tiles_x, _i32), n_tiles_total)
    ranges = np.zeros((n_tiles_total, 2), np.int64)
    count = L.ora_bin(*args, 0, None, None, None, _p(ranges, _i64))
    tiles = np.zeros(max(count, 1), np.int64)
    depth = np.zeros(max(count, 1), np.uint32)
    values = np.zeros(max(count, 1), np.int64)
    got = L.ora_bin(*args, count, _p(tiles, _i64), _p(depth, _u32), _p(values, _i64),
                    _p(ranges, _i64))
    assert got == count
    return dict(count=count, tiles=tiles[:count], depth=depth[:count], values=values[:count],
                ranges=ranges)


def _records_view(recs):
    """Concatenate per-view record dicts into planes indexed by r = v*n + i."""
    cat = lambda k: np.ascontiguousarray(np.concatenate([r[k] for r in recs], axis=-1))
    return {k: cat(k) for k in ("mean2d", "conic", "opacity", "color", "depth", "visible",
                                "rect", "margin", "grad_margin", "depth_margin", "color_margin")}


DELTA_GAUSS = 1e-9   # per-Gaussian decisions: both sides evaluate them in float64
DELTA_ALPHA = 4e-6   # alpha thresholds: a float32 alpha carries <= ~1.5e-6 relative error
DELTA_T = 2e-5       # stop decision: float32 transmittance after ~1000 factors
# float32 rounding of a depth computed in float64 on both sides: the two
# float64 values differ by a few units of 1e-16, so only depths within 1e-12
# of a rounding boundary can round apart (a wider band would flag a few per
# cent of all records, the boundaries being 6e-8 apart)
DELTA_DEPTH_ROUND = 1e-12
# two consecutive entries that may blend into a pixel, with float64 depths
# this close, could be ordered the other way by another float64 evaluation
DELTA_DEPTH_GAP = DELTA_GAUSS
# colour clamp at 0: the colour is a float32 sum of up to 16 SH terms per
# channel, accurate to ~1e-7 of max(1, |sum|)
DELTA_COLOR = 1e-6


def forward(P: Params, cams: list, opts: Opts, keep=None, delta=DELTA_GAUSS, delta_alpha=DELTA_ALPHA,
            delta_T=DELTA_T, delta_depth_round=DELTA_DEPTH_ROUND, delta_depth_gap=DELTA_DEPTH_GAP) -> dict:
    """Full multi-view forward: records, binning, per-pixel compositing.

    delta* are the relative margins below which a discrete decision is called
    ambiguous (another correct implementation may take it the other way)."""
    n = P.n
    V = len(cams)
    recs = [project(P, c, opts, keep) for c in cams]
    R = _records_view(recs)
    grids = [tile_grid(c, opts) for c in cams]
    tiles_per_view = [a * b for a, b in grids]
    tile_base_v = np.concatenate([[0], np.cumsum(tiles_per_view)[:-1]]).astype(np.int64)
    T_total = int(sum(tiles_per_view))
    depth_bits = R["depth"].astype(np.float32).view(np.uint32)
    tiebreak = np.tile(np.arange(n, dtype=np.int64), V)
    tile_base = np.repeat(tile_base_v, n)
    tiles_x = np.repeat(np.array([g[0] for g in grids], np.int32), n)
    bins = bin_records(R["rect"], R["visible"], depth_bits, tiebreak, tile_base, tiles_x, T_total)
    # bit 0: a decision of the record's own may go the other way; bit 1: the
    # float32 rounding of its depth may (which matters only next to an entry
    # of the same or an adjacent float32 depth)
    rec_amb = np.ascontiguousarray((R["margin"] < delta).astype(np.uint8)
                                   | (2 * (R["depth_margin"] < delta_depth_round)).astype(np.uint8))
    nr = n * V
    images, Tf, last, D, amb, sigs, blended = [], [], [], [], [], [], []
    L = lib()
    for v, c in enumerate(cams):
        W, H = c["W"], c["H"]
        img = np.zeros((3, H, W))
        t = np.zeros((H, W))
        la = np.zeros((H, W), np.int32)
        d = np.zeros((H, W))
        a = np.zeros((H, W), np.uint8)
        sg = np.zeros((H, W), np.int64)
        nb = np.zeros((H, W), np.int32)
        rv = np.ascontiguousarray(bins["ranges"][tile_base_v[v]:tile_base_v[v] + tiles_per_view[v]])
        L.ora_render(ctypes.byref(opts), W, H, _p(rv, _i64), _p(bins["values"], _i64), nr,
                     _p(R["mean2d"], _d), _p(R["conic"], _d), _p(R["opacity"], _d),
                     _p(R["color"], _d), _p(R["depth"], _d), _p(rec_amb, _u8), delta_alpha, delta_T,
                     delta_depth_gap,
                     _p(img, _d), _p(t, _d), _p(la, _i32), _p(d, _d), _p(a, _u8), _p(sg, _i64), _p(nb, _i32))
        # A Gaussian whose own decisions are ambiguous may be listed in one
        # more tile row or column by another implementation: mark the pixels
        # of that enlarged area where it could contribute (alpha above half
        # the skip threshold), or the whole area when it has no 2D shape.
        idx = np.nonzero(recs[v]["margin"] < delta)[0]
        tw, th = opts.tile_w, opts.tile_h
        gx, gy = grids[v]
        rv = recs[v]
        for i in idx:
            if rv["radius"][i] == 0 and not rv["visible"][i]:
                continue
            x0, y0, x1, y1 = rv["rect"][:, i]
            x0, y0 = max(min(x0, gx - 1) - 1, 0), max(min(y0, gy - 1) - 1, 0)
            x1, y1 = min(max(x1, 0) + 1, gx - 1), min(max(y1, 0) + 1, gy - 1)
            ys, xs = np.mgrid[y0 * th:min((y1 + 1) * th, H), x0 * tw:min((x1 + 1) * tw, W)]
            A, B, Cc = rv["conic"][:, i]
            if A > 0 and Cc > 0:
                dx = xs + 0.5 - rv["mean2d"][0, i]
                dy = ys + 0.5 - rv["mean2d"][1, i]
                al = rv["opacity"][i] * np.exp(-0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy)
                a[ys[al >= 0.5 * opts.alpha_min], xs[al >= 0.5 * opts.alpha_min]] = 1
            else:
                a[ys, xs] = 1
        images.append(img)
        sigs.append(sg)
        blended.append(nb)
        Tf.append(t)
        last.append(la)
        D.append(d)
        amb.append(a)
    return dict(records=recs, R=R, bins=bins, images=images, T_final=Tf, last=last, depth=D,
                ambiguous=amb, signature=sigs, blended=blended, tile_base=tile_base_v, tiles_per_view=tiles_per_view, grids=grids,
                depth_bits=depth_bits)


def touching(fwd: dict, flagged: list, opts: Opts) -> np.ndarray:
    """Records whose FP64 alpha at a flagged pixel is at least alpha_min / 2.

    fwd: the output of forward(); flagged: one bool [H][W] mask per view of
    fwd's cameras.  Every entry of a flagged pixel's tile list is tested, past
    the stop too.  A record below alpha_min / 2 at a pixel stays below
    alpha_min under any float32 evaluation (relative error ~1e-6), so it takes
    no part in that pixel's compositing on any correct implementation; the
    others may.  Returns a bool array over record ids v * n + i."""
    R = fwd["R"]
    nr = R["visible"].shape[0]
    out = np.zeros(nr, bool)
    vals_all = fwd["bins"]["values"]
    ranges = fwd["bins"]["ranges"]
    thr = 0.5 * opts.alpha_min
    for v, mask in enumerate(flagged):
        ys, xs = np.nonzero(np.asarray(mask, bool))
        if ys.size == 0:
            continue
        gx, _ = fwd["grids"][v]
        t = (ys // opts.tile_h) * gx + xs // opts.tile_w
        order = np.argsort(t, kind="stable")
        t, ys, xs = t[order], ys[order], xs[order]
        cuts = np.flatnonzero(np.diff(t)) + 1
        for a, b in zip(np.concatenate([[0], cuts]), np.concatenate([cuts, [t.size]])):
            s, e = ranges[fwd["tile_base"][v] + t[a]]
            if e <= s:
                continue
            r = vals_all[s:e]
            dx = (xs[a:b] + 0.5)[None, :] - R["mean2d"][0, r][:, None]
            dy = (ys[a:b] + 0.5)[None, :] - R["mean2d"][1, r][:, None]
            A, B, Cc = R["conic"][0, r][:, None], R["conic"][1, r][:, None], R["conic"][2, r][:, None]
            p = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
            al = R["opacity"][r][:, None] * np.exp(np.minimum(p, 0.0))
            out[r[(al >= thr).any(axis=1)]] = True
    return out


def l1_loss(images, targets):
    """Mean over views of the per-view mean absolute error, and dL/dimage."""
    V = len(images)
    total = 0.0
    grads = []
    for img, tgt in zip(images, targets):
        cnt = img.size
        g = np.zeros_like(img)
        tg = np.ascontiguousarray(tgt, np.float64)
        s = lib().ora_l1(cnt, _p(np.ascontiguousarray(img), _d), _p(tg, _d), 1.0 / (cnt * V), _p(g, _d))
        total += s / cnt
        grads.append(g)
    return total / V, grads


def backward(P: Params, cams: list, opts: Opts, fwd: dict, dL_dimages: list, keep=None,
             stat_scale=None) -> dict:
    """Reverse mode: 2D gradients per record, then raw-parameter gradients and
    the densification statistics (stat_scale defaults to the view count so
    that S sums |dL_v/dmean2d| of the per-view loss L_v = V * L's share)."""
    n = P.n
    V = len(cams)
    nr = n * V
    R = fwd["R"]
    g2d = np.zeros((9, nr))
    L = lib()
    for v, c in enumerate(cams):
        rv = np.ascontiguousarray(
            fwd["bins"]["ranges"][fwd["tile_base"][v]:fwd["tile_base"][v] + fwd["tiles_per_view"][v]])
        gi = np.ascontiguousarray(dL_dimages[v], np.float64)
        L.ora_render_bwd(ctypes.byref(opts), c["W"], c["H"], _p(rv, _i64),
                         _p(fwd["bins"]["values"], _i64), nr, _p(R["mean2d"], _d),
                         _p(R["conic"], _d), _p(R["opacity"], _d), _p(R["color"], _d),
                         _p(R["depth"], _d), _p(gi, _d), _p(g2d, _d))
    K3 = P.sh.shape[0]
    grads = np.zeros((11 + K3, n))
    S = np.zeros(n)
    cnt = np.zeros(n, np.int32)
    kp = None if keep is None else np.ascontiguousarray(keep, np.uint8)
    scale = float(V if stat_scale is None else stat_scale)
    for v, c in enumerate(cams):
        cam = make_cam(c)
        gv = np.ascontiguousarray(g2d[:, v * n:(v + 1) * n])
        L.ora_project_bwd(ctypes.byref(opts), ctypes.byref(cam), n, P.sh_degree,
                          _p(P.means, _d), _p(P.log_scales, _d), _p(P.quats, _d),
                          _p(P.logits, _d), _p(P.sh, _d), _p(kp, _u8), _p(gv, _d), n, scale,
                          _p(grads, _d), _p(S, _d), _p(cnt, _i32))
    return dict(g2d=g2d, grads=grads, S=S, count=cnt)


def split_grads(grads: np.ndarray) -> dict:
    return dict(means=grads[0:3], log_scales=grads[3:6], quats=grads[6:10], logits=grads[10],
                sh_dc=grads[11:14], sh_rest=grads[14:])


def step_l1(P: Params, cams: list, targets: list, opts: Opts, keep=None, delta=DELTA_GAUSS) -> dict:
    """One fine-training step of the rasterizer: forward, L1, backward."""
    fwd = forward(P, cams, opts, keep, delta)
    loss, dimg = l1_loss(fwd["images"], targets)
    bwd = backward(P, cams, opts, fwd, dimg, keep)
    fwd.update(bwd)
    fwd["loss"] = loss
    fwd["dL_dimages"] = dimg
    return fwd


def loss_only(P: Params, cams: list, targets: list, opts: Opts, keep=None) -> float:
    fwd = forward(P, cams, opts, keep)
    return l1_loss(fwd["images"], targets)[0]


def visibility_mask(P: Params, cams: list, opts: Opts, aabb, keep=None):
    """Visibility cropping and the selective-densification region (Sec. 3.3):
    view_bits (bit v set when visible in view v), keep_b = OR over views, and
    in_block = mean inside the half-open box [min, max)."""
    n = P.n
    bits = np.zeros(n, np.uint32)
    for v, c in enumerate(cams):
        vis = project(P, c, opts, keep)["visible"].astype(bool)
        bits |= (vis.astype(np.uint32) << np.uint32(v))
    aabb = np.asarray(aabb, np.float64)
    inb = np.all((P.means >= aabb[:3, None]) & (P.means < aabb[3:, None]), axis=0)
    return bits, (bits != 0).astype(np.uint8), inb.astype(np.uint8)


ADAM_GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def adam_step(params: dict, grads: dict, m: dict, v: dict, lr, beta1: float, beta2: float, eps: float,
              step: int, visible=None):
    """One bias-corrected Adam step (Kingma & Ba, Alg. 1) on every parameter
    plane, the optimizer whose cost visibility cropping removes for unseen
    Gaussians (Sec. 3.3; Sparse Adam, App. A.1).  Written from the
    definition, in float64 on copies:

        m_t = b1 m_{t-1} + (1 - b1) g,   v_t = b2 v_{t-1} + (1 - b2) g^2,
        m^ = m_t / (1 - b1^t),           v^ = v_t / (1 - b2^t),
        p_t = p_{t-1} - lr m^ / (sqrt(v^) + eps)

    lr: six rates (means, log_scales, quats, opacity_logits, SH band 0 = the
    first three SH planes, the other SH planes).  visible: None (dense) or a
    [n] array; Gaussians with visible == 0 keep parameters and moments.
    Returns new (params, m, v) dicts of float64 arrays [rows][n]."""
    P, M, V = {}, {}, {}
    for k in ADAM_GROUPS:
        p = np.asarray(params[k], np.float64).reshape(-1, np.asarray(params[k]).shape[-1]).copy()
        g = np.asarray(grads[k], np.float64).reshape(p.shape)
        mk = np.asarray(m[k], np.float64).reshape(p.shape).copy()
        vk = np.asarray(v[k], np.float64).reshape(p.shape).copy()
        if k == "sh":
            rate = np.full((p.shape[0], 1), float(lr[5]))
            rate[:3] = float(lr[4])
        else:
            rate = np.full((p.shape[0], 1), float(lr[ADAM_GROUPS.index(k)]))
        upd = np.ones(p.shape[1], bool) if visible is None else (np.asarray(visible) != 0)
        m_new = beta1 * mk + (1.0 - beta1) * g
        v_new = beta2 * vk + (1.0 - beta2) * g * g
        m_hat = m_new / (1.0 - beta1 ** step)
        v_hat = v_new / (1.0 - beta2 ** step)
        p_new = p - rate * m_hat / (np.sqrt(v_hat) + eps)
        P[k] = np.where(upd, p_new, p)
        M[k] = np.where(upd, m_new, mk)
        V[k] = np.where(upd, v_new, vk)
    return P, M, V


def back_project(depth: np.ndarray, cam: dict) -> np.ndarray:
    """World points of a depth map (Sec. 3.2, fast camera selection): pixel
    (u, v) with composited depth D lies on its centre's ray at camera depth D,
    p = R^T (D ((u + 1/2 - cx)/fx, (v + 1/2 - cy)/fy, 1) - t).  [3][H][W]."""
    H, W = depth.shape
    R = np.asarray(cam["R"], np.float64).reshape(3, 3)
    t = np.asarray(cam["t"], np.float64)
    vs, us = np.mgrid[0:H, 0:W].astype(np.float64)
    D = np.asarray(depth, np.float64)
    xc = D * ((us + 0.5 - float(cam["cx"])) / float(cam["fx"]))
    yc = D * ((vs + 0.5 - float(cam["cy"])) / float(cam["fy"]))
    q = np.stack([xc - t[0], yc - t[1], D - t[2]])
    return np.einsum("ab,bhw->ahw", R.T, q)


def camera_coverage(depths: list, cams: list, blocks, tau: float = 0.1, margin_rel: float = 0.0,
                    ambiguous: list | None = None):
    """V_{c,b} = (1/N_p) sum_k 1[p_{c,k} in B_b] over the back-projected
    pixels of each view (N_p = W H), blocks half-open boxes [min, max), and
    the assignment C^(b) = {c | V_{c,b} >= tau} (Sec. 3.2).

    With margin_rel > 0 it also counts, per (view, block), the points whose
    membership could flip under a relative error margin_rel of their depth
    (within margin_rel * D * |ray| of a face) or whose pixel is listed in
    `ambiguous`; another correct depth map may count those either way."""
    blocks = np.asarray(blocks, np.float64).reshape(-1, 6)
    V, M = len(cams), blocks.shape[0]
    counts = np.zeros((V, M), np.int64)
    unsure = np.zeros((V, M), np.int64)
    for v, (D, c) in enumerate(zip(depths, cams)):
        p = back_project(D, c)
        H, W = D.shape
        fx, fy = float(c["fx"]), float(c["fy"])
        vs, us = np.mgrid[0:H, 0:W].astype(np.float64)
        ray = np.sqrt(((us + 0.5 - float(c["cx"])) / fx) ** 2 + ((vs + 0.5 - float(c["cy"])) / fy) ** 2 + 1.0)
        slack = margin_rel * np.abs(np.asarray(D, np.float64)) * ray
        amb = np.zeros((H, W), bool) if ambiguous is None else np.asarray(ambiguous[v], bool)
        for b in range(M):
            lo, hi = blocks[b, :3, None, None], blocks[b, 3:, None, None]
            inside = np.all((p >= lo) & (p < hi), axis=0)
            counts[v, b] = int(inside.sum())
            if margin_rel > 0 or ambiguous is not None:
                near = np.any((np.abs(p - lo) <= slack) | (np.abs(p - hi) <= slack), axis=0)
                unsure[v, b] = int((near | amb).sum())
    npix = np.array([c["W"] * c["H"] for c in cams], np.float64)[:, None]
    ratio = counts / npix
    # V >= tau with tau the float32 value: count >= tau N_p is exact in float64
    return dict(counts=counts, ratio=ratio, selected=counts >= float(np.float32(tau)) * npix, unsure=unsure)
