"""Seeded synthetic scenes shaped like the city-block captures of LoBE-GS.

The paper trains on MatrixCity-Aerial, Mill19 and UrbanScene3D (Sec. 4.1,
"Datasets"); none of them is available here, so every workload is generated
from a seed.  The shapes follow the paper: 1600-px-wide views (Sec. 4.1),
millions of Gaussians per block (Tab. "comparison", #GS column), aerial oblique
cameras.

This module draws numbers only.  It holds none of the rasterizer's arithmetic
(no covariance, no projection of Gaussians, no compositing); both the HIP path
and the FP64 oracle consume exactly the float32 arrays produced here.  The only
geometry it does is camera placement (a look-at rotation) and, for the
rejection sampling of the batched workload, the fraction of Gaussian *centres*
that fall inside a camera's pyramid.

Layout (structure of arrays, float32, C-contiguous):
  means        [3][N]   world x, y, z (z up)
  log_scales   [3][N]   natural log of the per-axis standard deviation
  quats        [4][N]   (w, x, y, z), unit length as drawn
  opacity_logits [N]
  sh           [3K][N]  plane k*3 + c holds SH coefficient k of channel c
Cameras: dicts with R (3x3 world->camera, OpenCV axes x right, y down,
z forward), t (3,), fx, fy, cx, cy, W, H.
Targets: one float32 [3][H][W] image per view, U(0, 1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 20251001
Y00 = 0.28209479177387814  # constant real SH basis function 1/(2 sqrt(pi))


@dataclasses.dataclass
class Scene:
    name: str
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int
    cameras: list
    targets: list
    block_aabb: np.ndarray  # (6,) xmin ymin zmin xmax ymax zmax
    info: dict

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @property
    def n_views(self) -> int:
        return len(self.cameras)

    @property
    def pixels(self) -> int:
        return int(sum(c["W"] * c["H"] for c in self.cameras))

    def reordered(self, perm: np.ndarray) -> "Scene":
        """The same scene with its Gaussians stored in the order `perm`."""
        c = lambda a: np.ascontiguousarray(a[..., perm])
        return dataclasses.replace(self, means=c(self.means), log_scales=c(self.log_scales), quats=c(self.quats),
                                   opacity_logits=c(self.opacity_logits), sh=c(self.sh),
                                   name=self.name + "-reordered", info=dict(self.info, order="permuted"))


def morton_order(means: np.ndarray, bits: int = 10) -> np.ndarray:
    """Permutation sorting Gaussians by the Morton (Z-order) code of their
    means, quantised to 2^bits cells per axis of their bounding box (stable
    for equal codes).  Stored in this order, the Gaussians of one wavefront
    are spatial neighbours: they see the same views and touch the same tiles.
    Nothing the rasterizer computes depends on the order."""
    m = np.asarray(means, np.float64)
    lo = m.min(axis=1, keepdims=True)
    span = np.maximum(m.max(axis=1, keepdims=True) - lo, 1e-30)
    q = np.minimum((m - lo) / span * (1 << bits), (1 << bits) - 1).astype(np.uint64)
    code = np.zeros(m.shape[1], np.uint64)
    for b in range(bits):
        for a in range(3):
            code |= ((q[a] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + a)
    return np.argsort(code, kind="stable")


# --------------------------------------------------------------------------
# cameras


def look_at(eye, target, W, H, fx, fy=None, cx=None, cy=None):
    """World->camera pose (OpenCV axes) of a pinhole camera at `eye` looking
    at `target`, world z up."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    f = target - eye
    f /= np.linalg.norm(f)
    up = np.array([0.0, 0.0, 1.0])
    r = np.cross(f, up)
    if np.linalg.norm(r) < 1e-9:  # looking straight down
        r = np.array([1.0, 0.0, 0.0])
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ eye
    return dict(
        R=R.astype(np.float32),
        t=t.astype(np.float32),
        fx=np.float32(fx),
        fy=np.float32(fy if fy is not None else fx),
        cx=np.float32(cx if cx is not None else W / 2.0),
        cy=np.float32(cy if cy is not None else H / 2.0),
        W=int(W),
        H=int(H),
    )


def axis_camera(W, H, fx, z_dist, fy=None):
    """Camera at (0, 0, -z_dist) looking along +z with R = I."""
    return dict(
        R=np.eye(3, dtype=np.float32),
        t=np.array([0.0, 0.0, z_dist], np.float32),
        fx=np.float32(fx),
        fy=np.float32(fy if fy is not None else fx),
        cx=np.float32(W / 2.0),
        cy=np.float32(H / 2.0),
        W=int(W),
        H=int(H),
    )


def aerial_camera(target_xy, heading, pitch_deg, altitude, W, H, fx):
    """Oblique aerial view: the camera sits `altitude` above the ground, looks
    down at `pitch_deg` below the horizontal along `heading` (radians about
    world z) and aims at the ground point `target_xy`."""
    pitch = math.radians(pitch_deg)
    horiz = altitude / math.tan(pitch)
    dx, dy = math.cos(heading), math.sin(heading)
    eye = (target_xy[0] - horiz * dx, target_xy[1] - horiz * dy, altitude)
    return look_at(eye, (target_xy[0], target_xy[1], 0.0), W, H, fx)


def centre_in_view_fraction(cam, means, sample=200_000, seed=0):
    """Fraction of Gaussian centres inside the camera's pyramid (a cheap
    generator-side estimate used only to accept or reject random poses)."""
    n = means.shape[1]
    if n > sample:
        idx = np.random.default_rng(seed).choice(n, sample, replace=False)
        p = means[:, idx].astype(np.float64)
    else:
        p = means.astype(np.float64)
    c = cam["R"].astype(np.float64) @ p + cam["t"].astype(np.float64)[:, None]
    z = c[2]
    ok = z > 0.01
    zs = np.where(ok, z, 1.0)
    inside = (
        ok
        & (np.abs(c[0] / zs) < cam["W"] / (2.0 * float(cam["fx"])))
        & (np.abs(c[1] / zs) < cam["H"] / (2.0 * float(cam["fy"])))
    )
    return float(inside.mean())


# --------------------------------------------------------------------------
# Gaussian attributes


def _quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _attributes(rng, n, sh_degree, logit_mu=0.0, logit_sd=1.0):
    log_scales = rng.normal(-3.0, 0.5, (3, n))
    quats = _quats(rng, n)
    logits = rng.normal(logit_mu, logit_sd, n)
    K = (sh_degree + 1) ** 2
    sh = np.empty((3 * K, n))
    rgb = rng.uniform(0.0, 1.0, (3, n))
    sh[0:3] = (rgb - 0.5) / Y00
    if K > 1:
        sh[3:] = rng.normal(0.0, 0.2, (3 * (K - 1), n))
    return log_scales, quats, logits, sh


def _city_points(rng, n, half_extent, n_boxes):
    """60 % on a ground plane [-h, h]^2 with z ~ N(0, 0.05), 40 % uniform on
    the four sides and the roof of `n_boxes` random axis-aligned boxes."""
    n_ground = int(round(0.6 * n))
    n_box = n - n_ground
    pts = np.empty((3, n))
    pts[0, :n_ground] = rng.uniform(-half_extent, half_extent, n_ground)
    pts[1, :n_ground] = rng.uniform(-half_extent, half_extent, n_ground)
    pts[2, :n_ground] = rng.normal(0.0, 0.05, n_ground)
    inner = half_extent - 10.0
    cxy = rng.uniform(-inner, inner, (n_boxes, 2))
    hx = rng.uniform(2.0, 10.0, n_boxes)
    hy = rng.uniform(2.0, 10.0, n_boxes)
    hz = rng.uniform(5.0, 40.0, n_boxes)
    # faces: 0 +x, 1 -x, 2 +y, 3 -y, 4 roof
    areas = np.stack([2 * hy * hz, 2 * hy * hz, 2 * hx * hz, 2 * hx * hz, 4 * hx * hy], 1)
    flat = areas.ravel() / areas.sum()
    pick = rng.choice(flat.size, n_box, p=flat)
    b, face = pick // 5, pick % 5
    u = rng.uniform(-1.0, 1.0, n_box)
    v = rng.uniform(0.0, 1.0, n_box)
    x = np.empty(n_box)
    y = np.empty(n_box)
    z = np.empty(n_box)
    bx, by, bhx, bhy, bhz = cxy[b, 0], cxy[b, 1], hx[b], hy[b], hz[b]
    m = face == 0
    x[m], y[m], z[m] = bx[m] + bhx[m], by[m] + u[m] * bhy[m], v[m] * bhz[m]
    m = face == 1
    x[m], y[m], z[m] = bx[m] - bhx[m], by[m] + u[m] * bhy[m], v[m] * bhz[m]
    m = face == 2
    x[m], y[m], z[m] = bx[m] + u[m] * bhx[m], by[m] + bhy[m], v[m] * bhz[m]
    m = face == 3
    x[m], y[m], z[m] = bx[m] + u[m] * bhx[m], by[m] - bhy[m], v[m] * bhz[m]
    m = face == 4
    w = rng.uniform(-1.0, 1.0, n_box)
    x[m], y[m], z[m] = bx[m] + u[m] * bhx[m], by[m] + w[m] * bhy[m], bhz[m]
    pts[0, n_ground:], pts[1, n_ground:], pts[2, n_ground:] = x, y, z
    # interleave ground and box points so index order carries no structure
    perm = rng.permutation(n)
    return pts[:, perm]


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _targets(seed, cams):
    rng = np.random.default_rng([seed, 7])
    return [_f32(rng.uniform(0.0, 1.0, (3, c["H"], c["W"]))) for c in cams]


def _pack(name, means, attrs, sh_degree, cams, seed, aabb, info):
    log_scales, quats, logits, sh = attrs
    return Scene(
        name=name,
        means=_f32(means),
        log_scales=_f32(log_scales),
        quats=_f32(quats),
        opacity_logits=_f32(logits),
        sh=_f32(sh),
        sh_degree=sh_degree,
        cameras=cams,
        targets=_targets(seed, cams),
        block_aabb=np.asarray(aabb, np.float32),
        info=info,
    )


# --------------------------------------------------------------------------
# the five workloads


def config0(seed=SEED_BASE + 0):
    """Tiny single view: 2,000 Gaussians, SH degree 0, 128x128 camera at
    (0, 0, -4) looking along +z."""
    rng = np.random.default_rng(seed)
    n = 2000
    means = rng.uniform(-1.0, 1.0, (3, n))
    attrs = _attributes(rng, n, 0)
    cam = axis_camera(128, 128, 128.0, 4.0)
    return _pack("tiny-2k-sh0-128px", means, attrs, 0, [cam], seed,
                 [-1, -1, -1, 1, 1, 1], {})


def _aabb_of(means, half):
    return [-half, -half, float(means[2].min()), half, half, float(np.nextafter(means[2].max(), np.inf))]


def config1(seed=SEED_BASE + 1, n=1_000_000):
    """One 1920x1080 oblique view (45 deg pitch, 150 altitude, fx 1500) of a
    200x200 city block with 200 boxes, SH degree 3."""
    rng = np.random.default_rng(seed)
    means = _city_points(rng, n, 100.0, 200)
    attrs = _attributes(rng, n, 3)
    cam = look_at((0.0, -150.0, 150.0), (0.0, 0.0, 0.0), 1920, 1080, 1500.0)
    return _pack(f"city-block-{n // 1000}k-sh3-1view-1080p", means, attrs, 3, [cam], seed,
                 _aabb_of(means, 100.0), {})


BATCH_RES = [(1920, 1080)] * 6 + [(1600, 900)] * 6 + [(960, 540)] * 4


def _orbit_views(rng, means, resolutions, centre, jitter, pitch_rng, alt_rng,
                 frac_lo, frac_hi, heading_mode, look_half=None, max_tries=400):
    cams, fracs = [], []
    nv = len(resolutions)
    for k, (W, H) in enumerate(resolutions):
        fx = 1500.0 * W / 1920.0
        for attempt in range(max_tries):
            if heading_mode == "orbit":
                heading = 2 * math.pi * k / nv + rng.uniform(-0.2, 0.2)
                tgt = (centre[0] + rng.normal(0, jitter), centre[1] + rng.normal(0, jitter))
            else:
                heading = rng.uniform(0, 2 * math.pi)
                tgt = (rng.uniform(-look_half, look_half), rng.uniform(-look_half, look_half))
            pitch = rng.uniform(*pitch_rng)
            alt = rng.uniform(*alt_rng)
            cam = aerial_camera(tgt, heading, pitch, alt, W, H, fx)
            f = centre_in_view_fraction(cam, means, seed=k)
            if frac_lo <= f <= frac_hi:
                break
        cams.append(cam)
        fracs.append(f)
    return cams, fracs


def config2(seed=SEED_BASE + 2, n=3_000_000, resolutions=None):
    """16 views of uneven resolution (6x1080p, 6x1600x900, 4x960x540) on a
    jittered orbit around one 3M-Gaussian city block; each view keeps 5-40 %
    of the Gaussian centres."""
    rng = np.random.default_rng(seed)
    means = _city_points(rng, n, 100.0, 200)
    attrs = _attributes(rng, n, 3)
    res = resolutions if resolutions is not None else BATCH_RES
    cams, fracs = _orbit_views(rng, means, res, (0.0, 0.0), 20.0, (30.0, 60.0),
                               (30.0, 150.0), 0.05, 0.40, "orbit")
    return _pack(f"city-block-{n // 1000}k-sh3-{len(res)}views-uneven", means, attrs, 3, cams,
                 seed, _aabb_of(means, 100.0), {"centre_fraction": fracs})


def config3(seed=SEED_BASE + 3, n=8_000_000, n_views=32):
    """32 aerial 1080p views (pitch 30-60 deg, altitude 100-300) of an
    8M-Gaussian 1000x1000 city with 2,000 boxes."""
    rng = np.random.default_rng(seed)
    means = _city_points(rng, n, 500.0, 2000)
    attrs = _attributes(rng, n, 3)
    cams, fracs = _orbit_views(rng, means, [(1920, 1080)] * n_views, (0.0, 0.0), 0.0,
                               (30.0, 60.0), (100.0, 300.0), 0.0, 1.0, "random",
                               look_half=400.0, max_tries=1)
    return _pack(f"city-{n // 1000}k-sh3-{n_views}views-1080p", means, attrs, 3, cams, seed,
                 _aabb_of(means, 500.0), {"centre_fraction": fracs})


def config4(seed=SEED_BASE + 4, n=20_000_000, n_views=8, W=3840, H=2160, distance=140.0):
    """Depth-complexity stress: half the Gaussians in a volumetric cloud
    N(0, 20^2) per axis clipped to +-60 with low opacity, half on city
    surfaces; 8 views at 3840x2160 on an orbit of fixed distance."""
    rng = np.random.default_rng(seed)
    n_cloud = n // 2
    cloud = np.clip(rng.normal(0.0, 20.0, (3, n_cloud)), -60.0, 60.0)
    surf = _city_points(rng, n - n_cloud, 100.0, 200)
    means = np.concatenate([cloud, surf], 1)
    la, qa, la_logit, sha = _attributes(rng, n_cloud, 3, logit_mu=-2.0)
    lb, qb, lb_logit, shb = _attributes(rng, n - n_cloud, 3)
    attrs = (np.concatenate([la, lb], 1), np.concatenate([qa, qb], 1),
             np.concatenate([la_logit, lb_logit]), np.concatenate([sha, shb], 1))
    cams = []
    for k in range(n_views):
        heading = 2 * math.pi * k / n_views
        eye = (distance * math.cos(heading) * 0.8, distance * math.sin(heading) * 0.8, distance * 0.6)
        cams.append(look_at(eye, (0.0, 0.0, 0.0), W, H, 3000.0))
    return _pack(f"cloud-city-{n // 1000}k-sh3-{n_views}views-2160p", means, attrs, 3, cams, seed,
                 _aabb_of(means, 100.0), {})


def small_ragged(seed=SEED_BASE + 100, n=3000, sh_degree=3, sizes=((150, 97), (64, 40), (33, 71))):
    """Small multi-view scene for parity tests: uneven image sizes that are not
    multiples of any tile size, SH degree 3, a few thousand Gaussians in a
    unit cube seen from three directions."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (3, n))
    attrs = _attributes(rng, n, sh_degree)
    cams = []
    for k, (W, H) in enumerate(sizes):
        ang = 0.6 * k
        eye = (4.0 * math.sin(ang), -4.0 * math.cos(ang) * 0.3, -4.0 * math.cos(ang))
        cams.append(look_at(eye, (0.05 * k, 0.0, 0.0), W, H, 0.9 * W))
    return _pack(f"ragged-{n}-sh{sh_degree}-{len(sizes)}views", means, attrs, sh_degree, cams,
                 seed, [-0.5, -0.5, -1.0, 0.5, 0.5, 1.0], {})


def dense_cloud(seed=SEED_BASE + 101, n=400_000, sizes=((256, 256), (200, 136))):
    """Long tile lists for the sort: a Gaussian cloud N(0, 0.5^2) per axis
    (clipped to +-1.5) seen from distance 4 by two small views, so that the
    central tiles list tens of thousands of entries and the outer ones a
    few, covering every length class of the per-tile sort.  SH degree 0."""
    rng = np.random.default_rng(seed)
    means = np.clip(rng.normal(0.0, 0.5, (3, n)), -1.5, 1.5)
    attrs = _attributes(rng, n, 0)
    cams = []
    for k, (W, H) in enumerate(sizes):
        ang = 0.5 * k
        eye = (4.0 * math.sin(ang), 0.3 * k, -4.0 * math.cos(ang))
        cams.append(look_at(eye, (0.0, 0.0, 0.0), W, H, float(W)))
    return _pack(f"dense-cloud-{n // 1000}k-sh0-{len(sizes)}views", means, attrs, 0, cams, seed,
                 [-1.5, -1.5, -1.5, 1.5, 1.5, 1.5], {})


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}


@dataclasses.dataclass
class PartitionInput:
    """Inputs of the KD-tree partition: the scene box, coarse Gaussian
    centres [3][n] and each camera's back-projected pixels as points
    [3][total], camera v's at [offsets[v], offsets[v + 1])."""
    aabb: np.ndarray     # (6,) float32
    centers: np.ndarray  # [3][n] float32
    points: np.ndarray   # [3][total] float32
    offsets: np.ndarray  # [V + 1] int64


def partition_input(seed=SEED_BASE + 200, n=20_000, n_views=24, pixels=(24 * 16, 48 * 32), half=100.0,
                    hotspot=0.6):
    """A city block with an uneven camera distribution: the centres are the
    city points of the other workloads; each aerial camera sees a square
    footprint (side 30-90 % of the block's half extent) and its pixels are
    city points drawn from that footprint.  A fraction `hotspot` of the
    cameras look near one corner, the rest anywhere, so that the per-block
    camera counts are heterogeneous (the imbalance Sec. 3.1 addresses)."""
    rng = np.random.default_rng(seed)
    centres = _city_points(rng, n, half, max(4, n // 2000))
    hot = rng.uniform(-0.8 * half, -0.3 * half, 2)
    pts, offsets = [], [0]
    for v in range(n_views):
        c = hot + rng.normal(0.0, 0.15 * half, 2) if rng.uniform() < hotspot else rng.uniform(-0.8 * half, 0.8 * half, 2)
        r = rng.uniform(0.15, 0.45) * half
        inside = np.nonzero((np.abs(centres[0] - c[0]) < r) & (np.abs(centres[1] - c[1]) < r))[0]
        k = int(rng.integers(pixels[0], pixels[1] + 1))
        if inside.size == 0:
            inside = np.arange(n)
        pick = centres[:, rng.choice(inside, k)] + rng.normal(0.0, 0.2, (3, k))
        pts.append(pick)
        offsets.append(offsets[-1] + k)
    c32 = _f32(centres)
    c32[:2] = np.minimum(c32[:2], np.nextafter(np.float32(half), np.float32(-np.inf)))
    # a half-open box that holds every float32 centre
    aabb = np.array([-half, -half, c32[2].min(), half, half, np.nextafter(c32[2].max(), np.float32(np.inf))],
                    np.float32)
    assert np.all((c32 >= aabb[:3, None]) & (c32 < aabb[3:, None]))
    return PartitionInput(aabb=aabb, centers=c32,
                          points=_f32(np.concatenate(pts, axis=1)), offsets=np.asarray(offsets, np.int64))


def make_config(k: int, **kw) -> Scene:
    return CONFIGS[k](**kw)
