"""Small builders shared by the oracle pin tests (no rasterizer arithmetic)."""
import math

import numpy as np

import oracle

Y00 = 0.5 / math.sqrt(math.pi)


def _f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def cam(W=128, H=128, f=128.0, R=None, t=(0.0, 0.0, 4.0), cx=None, cy=None):
    """Camera whose values are float32-representable (cameras cross the
    boundary as float32)."""
    return dict(R=_f32(np.eye(3) if R is None else R), t=_f32(t), fx=float(_f32(f)),
                fy=float(_f32(f)), cx=float(_f32(W / 2.0 if cx is None else cx)),
                cy=float(_f32(H / 2.0 if cy is None else cy)), W=W, H=H)


def params(means, log_scales=None, quats=None, opacities=None, colors=None, sh_degree=0, sh=None):
    """Gaussians in FP64 from plain values; colours map to the DC coefficient."""
    means = np.asarray(means, np.float64).reshape(-1, 3).T.copy()
    n = means.shape[1]
    ls = np.full((3, n), math.log(0.05)) if log_scales is None else np.asarray(log_scales, np.float64).reshape(n, 3).T.copy()
    q = np.tile(np.array([[1.0], [0], [0], [0]]), (1, n)) if quats is None else np.asarray(quats, np.float64).reshape(n, 4).T.copy()
    o = np.full(n, 0.5) if opacities is None else np.asarray(opacities, np.float64)
    logits = np.log(o / (1 - o))
    K = (sh_degree + 1) ** 2
    if sh is None:
        shv = np.zeros((3 * K, n))
        c = np.full((n, 3), 0.5) if colors is None else np.asarray(colors, np.float64).reshape(n, 3)
        shv[0:3] = ((c - 0.5) / Y00).T
    else:
        shv = np.asarray(sh, np.float64)
    return oracle.Params(means, ls, q, logits, shv, sh_degree)


def tiny_scene(seed=3, n=40, sizes=((40, 32), (24, 36)), sh_degree=3, spread=0.6):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-spread, spread, (3, n))
    ls = rng.normal(-2.3, 0.4, (3, n))
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0)
    q *= rng.uniform(0.5, 2.0, n)  # unnormalised on purpose
    logits = rng.normal(0.0, 1.0, n)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((3 * K, n))
    sh[0:3] = (rng.uniform(0.2, 0.9, (3, n)) - 0.5) / Y00
    sh[3:] = rng.normal(0.0, 0.2, (3 * K - 3, n))
    P = oracle.Params(means, ls, q, logits, sh, sh_degree)
    cams = []
    for k, (W, H) in enumerate(sizes):
        a = 0.35 * k
        R = np.array([[math.cos(a), 0, -math.sin(a)], [0, 1, 0], [math.sin(a), 0, math.cos(a)]])
        cams.append(cam(W, H, 1.1 * W, R=R, t=(0.05 * k, -0.03, 3.0)))
    targets = [rng.uniform(0, 1, (3, H, W)) for (W, H) in sizes]
    return P, cams, targets
