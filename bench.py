#!/usr/bin/env python3
"""Throughput of the differentiable Gaussian rasterizer on one MI355X.

Workload (default): 3M-Gaussian SH-3 city block, 16 views of uneven size
(6 x 1920x1080, 6 x 1600x900, 4 x 960x540), one fused forward + L1 + backward
step of all views per step, captured in one HIP graph (batched form).  The
same step is also timed as 16 plain per-view launch chains.  Inputs are
seeded synthetic data already resident in device memory; the Gaussians are
stored in Morton order of their means (the layout the framework keeps; the
generator's random order is timed too, for reference).

Prints one JSON line: Mpixels/s of the batched step (value), Gaussians/s,
the plain per-view rate and the ratio, the spread of single steps, device
memory, the roofline of the dominant kernel (the fused raster: algorithmic
HBM bytes over its time from device events on its stream over a second pass
of eager steps, the whole step's algorithmic bytes over the step time, and
the blended pairs' float operations), the timed outputs' parity against the
FP64 oracle on every view the oracle renders, and the oracle's own rate on
the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# Algorithmic float operations per blended (pixel, Gaussian) pair (alpha at
# least alpha_min, before the stop), counted from the method (not from the
# instructions): forward offset (2), quadratic
# form (6), exponent and opacity (2), threshold tests (2), transmittance
# update (2), colour accumulation (7) = 21; reverse pass: the same alpha (12),
# transmittance recovery (2), dL/dalpha over 3 channels (12), colour and
# suffix updates (9), opacity/mean/conic partials (14), 9-way reduction
# share (9) = 58.
FLOPS_FWD_PAIR = 21
FLOPS_BWD_PAIR = 58
RASTER_SOURCES = ["paper_2510_01767_amd/csrc/gsr_raster.hip", "paper_2510_01767_amd/csrc/gsr_device.h",
                  "paper_2510_01767_amd/csrc/gsr_internal.h", "paper_2510_01767_amd/csrc/gsr_cull.h"]
TRAFFIC_SUMMARY = "profiles/hbm_traffic_city-block-3000k-16views.md"


def fused_traffic(opt):
    """HBM bytes per launch of the fused raster kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), or None once the raster
    sources or the tuning differ from the ones the counters were taken with."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, TRAFFIC_SUMMARY)).read()
        meta = json.loads(text.split("```json")[1].split("```")[0])
    except (OSError, IndexError, ValueError):
        return None
    h = hashlib.sha256()
    for f in RASTER_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    same = (h.hexdigest()[:16] == meta["source_sha256_16"] and meta["tile"] == f"{opt.tile_w}x{opt.tile_h}"
            and meta["lds_batch"] == opt.lds_batch and meta["bwd_reduce"] == opt.bwd_reduce)
    return int(meta["traffic_bytes"]) if same else None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def b_alg_batched(n, U, K, F, vis, isect, pixels):
    """Algorithmic HBM bytes of one batched step (every view in one pass):
    geometry (means, log-scales, quaternions: 40 B) of every Gaussian once,
    opacity and SH (4 + 4K) of every Gaussian visible in some view once,
    per visible (view, Gaussian) 152 B (48 B record written, 32 B of scan and
    scatter, 36 B 2D gradient written and read back, 36 B of the reverse
    projection's per-view reads), per intersection 140 B (8 B key emitted, a
    two-pass sort at 2 x 24 B, a 40 B record gather forward and another
    backward), per pixel 52 B (colour, T and last written: 20 B; target,
    colour, T and last read: 32 B), and the gradients (read-modify-write of
    4F B) plus 16 B of densification statistics of every Gaussian visible in
    some view."""
    return 40 * n + (4 + 4 * K) * U + 152 * vis + 140 * isect + 52 * pixels + (2 * 4 * F + 16) * U


def b_alg_plain(n, K, F, n_views, vis, isect, pixels):
    """The same step as one pass per view: every view reads the means for its
    cull (12 B per Gaussian) and its visible Gaussians' parameters again;
    per visible (view, Gaussian) c_V = 200 + 4K + 12F bytes (the batched
    per-pair traffic plus that view's parameter reads and gradient
    read-modify-write)."""
    c_v = 200 + 4 * K + 12 * F
    return 12 * n * n_views + c_v * vis + 140 * isect + 52 * pixels


def b_alg_fused(vis, isect, pixels):
    """Algorithmic HBM bytes of the fused raster kernel (forward, L1 and
    reverse pass of every tile): a 40 B record gather per intersection in
    each direction, 52 B per pixel (image, T, last out; target in), and the
    36 B 2D gradient of every visible record written once."""
    return 80 * isect + 52 * pixels + 36 * vis


def slot_grad2d(slots, conic):
    """2D gradient (dmean 2, dconic 3, dopacity, dcolour 3) from GPU record
    slots, whose words 0..4 hold the moments of dL/dp over the pixel offsets
    d (gp dx, gp dy, gp dx^2, gp dx dy, gp dy^2; p = -d^T Q d / 2): with the
    conic Q = (A, B, C), dL/dmean2d = Q (m0, m1) and dL/dQ = -(m2/2, m3, m4/2)."""
    m = np.asarray(slots, np.float64)[:, :9]
    A, B, C = (np.asarray(conic, np.float64)[j] for j in range(3))
    out = m.copy()
    out[:, 0], out[:, 1] = A * m[:, 0] + B * m[:, 1], B * m[:, 0] + C * m[:, 1]
    out[:, 2], out[:, 3], out[:, 4] = -0.5 * m[:, 2], -m[:, 3], -0.5 * m[:, 4]
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-adam", action="store_true")
    ap.add_argument("--no-fcs", action="store_true")
    ap.add_argument("--no-partition", action="store_true")
    ap.add_argument("--no-densify", action="store_true")
    ap.add_argument("--tile", default=None, help="fixed tile shape WxH (with --no-autotune)")
    ap.add_argument("--lds-batch", type=int, default=256, help="with --no-autotune")
    ap.add_argument("--grid-per-cu", type=int, default=8, help="with --no-autotune")
    ap.add_argument("--bwd-reduce", type=int, default=0, help="with --no-autotune")
    ap.add_argument("--project-table", type=int, default=0, choices=[0, 1], help="with --no-autotune")
    ap.add_argument("--order", choices=["morton", "random"], default="morton",
                    help="storage order of the Gaussians: Morton order of their means (the layout the framework "
                         "keeps), or the generator's random order")
    ap.add_argument("--oracle-configs", default="",
                    help="comma-separated configs whose whole FP64 oracle step (0, 1) or one view of it (3, 4) "
                         "is also timed on the host cores")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (a kernel of known traffic, to scale "
                         "hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the framework has no multi-GPU path (blocks train independently, one "
              "GPU each); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_01767_amd import gsr as C
    from paper_2510_01767_amd import scenes
    from paper_2510_01767_amd.raster import (Rasterizer, camera_tensor, pack_images, partition_blocks_device,
                                             scene_tensors)

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    C.load(build_if_missing=False)
    t0 = time.time()
    scene = scenes.make_config(args.config)
    log(f"scene {scene.name}: {scene.n} Gaussians, {scene.n_views} views, {scene.pixels} pixels "
        f"({time.time() - t0:.1f} s)")
    scene_random = scene
    n_total = scene.n
    if args.order == "morton":
        scene = scene.reordered(scenes.morton_order(scene.means))
    sizes = [(c["W"], c["H"]) for c in scene.cameras]
    params = scene_tensors(scene)
    cams = camera_tensor(scene.cameras)
    targets = torch.from_numpy(pack_images(scene.targets)).cuda()
    torch.cuda.synchronize()

    if args.copy_mib:
        a = torch.empty(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    tile = tuple(int(x) for x in args.tile.split("x")) if args.tile else (16, 16)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    scene_bytes = sum(t.numel() * t.element_size() for t in params.values()) + cams.numel() * 4 + targets.numel() * 4
    torch.cuda.reset_peak_memory_stats()
    rb = Rasterizer(scene.n, scene.sh_degree, sizes, mode="batched", tile=tile, profile_stages=1,
                    lds_batch=args.lds_batch, grid_per_cu=args.grid_per_cu, bwd_reduce=args.bwd_reduce,
                    project_table=args.project_table)
    rb.step_l1(params, cams, targets, stats=True)
    counts = rb.counts()
    log(f"visible {counts.visible_total}, union {counts.visible_union}, intersections "
        f"{counts.intersections_total}, capacity {rb.layout.capacity}")
    if not args.no_autotune:
        best, ms = rb.autotune(params, cams, targets, reps=2)
        log(f"autotune: tile {best.tile_w}x{best.tile_h}, lds_batch {best.lds_batch}, grid/CU "
            f"{best.grid_per_cu}, bwd {best.bwd_variant}, reduction {best.bwd_reduce}, project table "
            f"{best.project_table}: {ms:.3f} ms")
    opt = rb.options

    # ---- timed region: K replays of the captured batched step
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        rb.capture(params, cams, targets, stats=True)
    stream.synchronize()
    for _ in range(args.warmup):
        rb.launch(stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        rb.launch(stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_batched = e0.elapsed_time(e1) / args.steps
    log(f"batched graph step {ms_batched:.3f} ms (wall {1000 * wall / args.steps:.3f} ms)")
    # the spread of single steps: each replay timed alone (after the timed region)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a, b in evs:
        a.record(stream)
        rb.launch(stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    single = np.array([a.elapsed_time(b) for a, b in evs])
    spread = {"median": round(float(np.median(single)), 4), "p10": round(float(np.percentile(single, 10)), 4),
              "p90": round(float(np.percentile(single, 90)), 4)}
    log(f"single steps: {spread}")
    free1 = torch.cuda.mem_get_info()[0]
    memory = {"workspace_bytes": int(rb.ws_bytes), "scene_bytes": int(scene_bytes),
              "torch_peak_allocated_bytes": int(torch.cuda.max_memory_allocated()),
              "device_bytes_taken_by_rasterizer": int(free0 - free1)}
    log(f"memory: {memory}")
    counts = rb.counts()
    images_gpu = rb.images.cpu().numpy()
    # the timed step's 2D gradients of every view, for the parity check (later stages
    # reuse the workspace)
    S_ = C.GSR_SLOT_FLOATS
    g2d_all = rb.ws_tensor("grad2d", torch.float32, S_ * rb.layout.vn).view(-1, S_)[:, :9].cpu().numpy()
    loss_gpu = float(rb.loss.item())
    last = rb.ws_tensor("pix_last", torch.int32, rb.pixels).cpu().numpy().astype(np.int64)
    walked = int(last.sum())

    # ---- per-kernel device time: the same step eagerly, stage events on its stream
    stage_tot = {}
    with torch.cuda.stream(stream):
        for _ in range(args.steps):
            rb.step_l1(params, cams, targets, stats=True, stream=stream)
            for name, (ms, k) in C.gsr_last_stage_times(rb.plan).items():
                a = stage_tot.setdefault(name, [0.0, 0])
                a[0] += ms
                a[1] += k
    torch.cuda.synchronize()
    stage_ms = {k: v[0] / args.steps for k, v in stage_tot.items()}
    log("stages (ms/step): " + ", ".join(f"{k} {v:.3f}" for k, v in sorted(stage_ms.items(), key=lambda x: -x[1])))
    dom = max(stage_ms, key=stage_ms.get)
    # profiling-only forward: pairs blended (alpha >= alpha_min before the stop) and pairs the
    # lanes evaluated after the sub-block culling
    pc_img = torch.empty_like(rb.images)
    bl, ev = rb.pair_counts(params, cams, images=pc_img, stream=stream)
    torch.cuda.synchronize()
    blended, evaluated = int(bl.to(torch.int64).sum().item()), int(ev.to(torch.int64).sum().item())
    del pc_img, bl, ev
    log(f"pairs: walked {walked}, evaluated {evaluated}, blended {blended}")

    # ---- plain per-view launches
    ms_plain = None
    if not args.no_plain:
        rp = Rasterizer(scene.n, scene.sh_degree, sizes, mode="plain", tile=(16, 16),
                        project_table=opt.project_table)
        rp.step_l1(params, cams, targets, stats=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(args.plain_steps):
            rp.step_l1(params, cams, targets, stats=True)
        torch.cuda.synchronize()
        ms_plain = 1000 * (time.perf_counter() - w0) / args.plain_steps
        log(f"plain per-view step {ms_plain:.3f} ms")
        del rp

    # ---- the same step with the Gaussians in the generator's random order
    ms_random = None
    if args.order == "morton" and not args.no_plain:
        pr = scene_tensors(scene_random)
        rr = Rasterizer(scene.n, scene.sh_degree, sizes, mode="batched", tile=(opt.tile_w, opt.tile_h),
                        lds_batch=opt.lds_batch, grid_per_cu=opt.grid_per_cu, bwd_reduce=opt.bwd_reduce,
                        project_table=opt.project_table)
        with torch.cuda.stream(stream):
            rr.capture(pr, cams, targets, stats=True)
        stream.synchronize()
        for _ in range(args.warmup):
            rr.launch(stream=stream)
        e0.record(stream)
        for _ in range(args.steps):
            rr.launch(stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_random = e0.elapsed_time(e1) / args.steps
        log(f"random-order graph step {ms_random:.3f} ms")
        del rr, pr

    # ---- the optimizer stage after the step: Adam over all parameter planes, dense and
    # visible-only (the step's view masks), on copies of the parameters
    adam = None
    if not args.no_adam:
        from paper_2510_01767_amd.raster import PARAM_NAMES
        pa = {k: params[k].clone() for k in PARAM_NAMES}
        ma = {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}
        va = {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}
        lr = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 1.25e-4)
        rb.step_l1(params, cams, targets, stats=True, stream=stream)
        res = {}
        for name, vis in (("dense", False), ("visible_only", True)):
            rb.adam_step(pa, rb.grads, ma, va, lr, 1, visible_only=vis, stream=stream)
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            for t in range(args.steps):
                rb.adam_step(pa, rb.grads, ma, va, lr, t + 2, visible_only=vis, stream=stream)
            a1.record(stream)
            torch.cuda.synchronize()
            res[name] = a0.elapsed_time(a1) / args.steps
        planes = 11 + 3 * (scene.sh_degree + 1) ** 2
        b_dense = 7 * 4 * planes * n_total
        b_vis = 7 * 4 * planes * counts.visible_union + 4 * n_total * planes
        gbs = b_dense / (res["dense"] * 1e-3) / 1e9
        adam = {"dense_ms": round(res["dense"], 4), "visible_only_ms": round(res["visible_only"], 4),
                "bytes_dense": b_dense, "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                                                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)},
                "visible_fraction": round(counts.visible_union / n_total, 4),
                "visible_only_GBps": round(b_vis / (res["visible_only"] * 1e-3) / 1e9, 1)}
        log(f"adam: {adam}")
        del pa, ma, va

    # ---- selective densification on the statistics of one step over the 16 views: threshold at
    # the 90th percentile of S / n, clone / split cut at the median largest scale, in-block only
    dens = None
    if not args.no_densify:
        from paper_2510_01767_amd.raster import PARAM_NAMES
        n = scene.n
        rb.S.zero_()
        rb.count.zero_()
        rb.step_l1(params, cams, targets, stats=True, stream=stream)
        torch.cuda.synchronize()
        seen = rb.count > 0
        thr = float(torch.quantile((rb.S[seen] / rb.count[seen].float())[: 1 << 24], 0.9))
        cut = float(torch.exp(params["log_scales"].max(dim=0).values).median())
        aabb = torch.from_numpy(np.asarray(scene.block_aabb, np.float32)).cuda()
        in_block = ((params["means"] >= aabb[:3, None]) & (params["means"] < aabb[3:, None])).all(0)
        in_block = in_block.to(torch.uint8).contiguous()
        gen = torch.Generator(device="cuda")
        gen.manual_seed(20251001)
        samples = torch.randn((2, 3, n), generator=gen, device="cuda")
        md = {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}
        vd = {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}
        opts_d = C.gsr_densify_opts(thr, cut, 0.005, 0.0, 1, 0)
        g_in = rb.gaussians(params)
        st = C.gsr_stats(rb.S.data_ptr(), rb.count.data_ptr())
        wsb = C.gsr_densify_workspace_size(n)
        wsd = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        sh_ = stream.cuda_stream
        count = lambda: C.gsr_densify_count(n, scene.sh_degree, opts_d, g_in, st, in_block.data_ptr(),
                                            wsd.data_ptr(), wsb, sh_)
        n_out = count()
        walls = []
        for _ in range(5):
            t0 = time.perf_counter()
            count()
            walls.append((time.perf_counter() - t0) * 1e3)
        new = lambda: {k: torch.empty((params[k].shape[0], n_out) if params[k].dim() == 2 else (n_out,),
                                      dtype=torch.float32, device="cuda") for k in PARAM_NAMES}
        out, mo, vo = new(), new(), new()
        parent = torch.empty(n_out, dtype=torch.int64, device="cuda")
        gs = lambda d: C.gsr_grads(*[d[k].data_ptr() for k in PARAM_NAMES])
        apply = lambda: C.gsr_densify_apply(n, scene.sh_degree, opts_d, g_in, gs(md), gs(vd), st,
                                            in_block.data_ptr(), samples.data_ptr(), n_out, gs(out), gs(mo),
                                            gs(vo), parent.data_ptr(), wsd.data_ptr(), wsb, sh_)
        apply()
        d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        d0.record(stream)
        for _ in range(args.steps):
            apply()
        d1.record(stream)
        torch.cuda.synchronize()
        ms_apply = d0.elapsed_time(d1) / args.steps
        # algorithmic bytes of the apply kernel: the decision inputs of every Gaussian (25 B),
        # the 59 planes (236 B) of every producing Gaussian plus its moments (472 B) or, for a
        # split, its 6 normal draws (24 B); per output 236 B of planes, 472 B of moments, 8 B
        # of parent index
        P = 4 * (11 + 3 * (scene.sh_degree + 1) ** 2)
        producing = torch.unique(parent).numel()
        child = (out["means"] != params["means"][:, parent]).any(0)
        n_split = int(child.sum().item()) // 2
        b_alg = (25 * n + producing * P + (producing - n_split) * 2 * P + n_split * 24 + n_out * (3 * P + 8))
        gbs = b_alg / (ms_apply * 1e-3) / 1e9
        dens = {"gaussians_in": n, "gaussians_out": n_out, "splits": n_split,
                "clones": n_out - producing - n_split, "grad_threshold": thr, "clone_max_scale": cut,
                "count_ms_wall": round(min(walls), 4), "apply_ms": round(ms_apply, 4), "bytes_apply": b_alg,
                "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbs / HBM_PEAK_GBS, 4)}}
        log(f"densify: {dens}")
        del out, mo, vo, md, vd, samples, parent

    # ---- fast camera selection: one depth-compositing pass over the views, then the
    # back-projected pixels counted into a 4 x 4 grid of blocks over the scene
    fcs = None
    if not args.no_fcs:
        m = scene.means.astype(np.float64)
        lo, hi = m.min(axis=1) - 1.0, m.max(axis=1) + 1.0
        xs, ys = np.linspace(lo[0], hi[0], 5), np.linspace(lo[1], hi[1], 5)
        blocks = torch.tensor([(xs[i], ys[j], lo[2], xs[i + 1], ys[j + 1], hi[2]) for i in range(4) for j in range(4)],
                              dtype=torch.float32, device="cuda")
        depth_img = torch.empty(3 * rb.pixels, dtype=torch.float32, device="cuda")
        _, depth = rb.render_depth(params, cams, images=depth_img, stream=stream)
        rb.camera_coverage(cams, depth, blocks, stream=stream)
        f0, f1, f2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        f0.record(stream)
        for _ in range(args.steps):
            _, depth = rb.render_depth(params, cams, images=depth_img, stream=stream)
        f1.record(stream)
        for _ in range(args.steps):
            counts_fcs, ratio, sel = rb.camera_coverage(cams, depth, blocks, stream=stream)
        f2.record(stream)
        torch.cuda.synchronize()
        ms_depth, ms_cov = f0.elapsed_time(f1) / args.steps, f1.elapsed_time(f2) / args.steps
        fcs = {"depth_render_ms": round(ms_depth, 4), "coverage_ms": round(ms_cov, 4), "blocks": 16,
               "views_selected": int(sel.sum().item()),
               "depth_mpixels_per_s": round(scene.pixels / (ms_depth * 1e-3) / 1e6, 1)}
        log(f"fcs: {fcs}")
        del depth_img

        # ---- scene partition (Alg. 1) into 8 blocks: the back-projected pixels stay in HBM
        # and every split counts them on the GPU; the host variant counts the same points
        if not args.no_partition:
            g0, g1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
            g0.record(stream)
            pts = rb.back_project(cams, depth, stream=stream)
            g1.record(stream)
            torch.cuda.synchronize()
            offsets = np.cumsum([0] + [c["W"] * c["H"] for c in scene.cameras]).astype(np.int64)
            ms_dev = []
            for _ in range(3):
                t0 = time.perf_counter()
                dev = partition_blocks_device(scene.block_aabb, scene.means, pts, offsets, 8, stream=stream)
                ms_dev.append((time.perf_counter() - t0) * 1e3)
            pts_host = pts.cpu().numpy()
            t0 = time.perf_counter()
            host = C.gsr_partition_blocks(scene.block_aabb, scene.means, pts_host, offsets, 8)
            ms_host = (time.perf_counter() - t0) * 1e3
            fcs["partition"] = {
                "blocks": 8, "refine_steps": 3, "back_project_ms": round(g0.elapsed_time(g1), 4),
                "device_ms": round(min(ms_dev), 3), "host_ms": round(ms_host, 1),
                "device_matches_host": bool(np.array_equal(dev[0], host[0]) and np.array_equal(dev[1], host[1])),
                "workloads": dev[2].tolist()}
            log(f"partition: {fcs['partition']}")
            del pts, pts_host

    # ---- roofline: algorithmic bytes (and blended-pair flops) against the measured times
    n, V = scene.n, scene.n_views
    P = scene.pixels
    I = counts.intersections_total
    vis = counts.visible_total
    U = counts.visible_union
    K = 3 * (scene.sh_degree + 1) ** 2
    F = 11 + K
    t_fused = stage_ms.get("fused raster")
    b_step = b_alg_batched(n, U, K, F, vis, I, P)
    b_fused = b_alg_fused(vis, I, P)
    gbs_step = b_step / (ms_batched * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": "k_fused", "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    if t_fused:
        gbs_fused = b_fused / (t_fused * 1e-3) / 1e9
        roof.update(achieved=round(gbs_fused, 1), frac=round(gbs_fused / HBM_PEAK_GBS, 4), bytes_alg=int(b_fused),
                    ms=round(t_fused, 4))
        flops = blended * (FLOPS_FWD_PAIR + FLOPS_BWD_PAIR)
        tf = flops / (t_fused * 1e-3) / 1e12
        roof["alu"] = {"blended_pairs": blended, "evaluated_pairs": evaluated, "walked_pairs": walked,
                       "flops_per_blended_pair": FLOPS_FWD_PAIR + FLOPS_BWD_PAIR, "achieved": round(tf, 3),
                       "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / FP32_PEAK_TFLOPS, 4)}
    roof["traffic"] = fused_traffic(opt) if args.config == 2 else None
    roof["step"] = {"bytes_alg": int(b_step), "ms": round(ms_batched, 4), "achieved": round(gbs_step, 1),
                    "frac": round(gbs_step / HBM_PEAK_GBS, 4)}
    if ms_plain:
        b_plain = b_alg_plain(n, K, F, V, vis, I, P)
        g = b_plain / (ms_plain * 1e-3) / 1e9
        roof["plain_step"] = {"bytes_alg": int(b_plain), "ms": round(ms_plain, 3), "achieved": round(g, 1),
                              "frac": round(g / HBM_PEAK_GBS, 4)}
    roof["stage_ms"] = {k: round(v, 4) for k, v in stage_ms.items()}
    log(f"roofline: {roof}")

    # ---- parity of the timed outputs on every view the oracle renders, and the oracle's own rate
    parity = None
    cpu = None
    if not (args.no_parity and args.no_cpu):
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        Pn = oracle.Params.from_scene(scene)
        o = oracle.default_opts(tile_w=opt.tile_w, tile_h=opt.tile_h)
        # views taken round-robin over the resolutions, so the sample mixes sizes like the batch
        groups = {}
        for v, wh in enumerate(sizes):
            groups.setdefault(wh, []).append(v)
        order = []
        while any(groups.values()):
            for wh in sorted(groups, key=lambda x: -x[0] * x[1]):
                if groups[wh]:
                    order.append(groups[wh].pop(0))
        done, t_ora, checks = [], 0.0, []
        for v in order:
            c = scene.cameras[v]
            W, H = c["W"], c["H"]
            t1 = time.time()
            fo = oracle.forward(Pn, [c], o)
            img_o = fo["images"][0]
            d = np.sign(img_o - scene.targets[v]) / (3.0 * W * H * V)
            bo = oracle.backward(Pn, [c], o, fo, [d])
            t_ora += time.time() - t1
            done.append(v)
            if not args.no_parity:
                off = 3 * sum(w * h for w, h in sizes[:v])
                img_g = images_gpu[off:off + 3 * W * H].reshape(3, H, W).astype(np.float64)
                amb = fo["ambiguous"][0].astype(bool)
                err = np.abs(img_g - img_o) / np.maximum(1.0, np.abs(img_o))
                rel_l2 = float(np.linalg.norm(img_g - img_o) / np.linalg.norm(img_o))
                # 2D gradients of the view's records, leaving out those whose alpha reaches
                # alpha_min / 2 at an ambiguous pixel or at a pixel on the L1 kink
                kink = (np.abs(img_o - scene.targets[v]) < 1e-5).any(axis=0)
                visv = fo["records"][0]["visible"].astype(bool)
                ex = oracle.touching(fo, [amb | kink], o)[:n] | (fo["records"][0]["margin"] < oracle.DELTA_GAUSS)
                sel = visv & ~ex
                g2d = slot_grad2d(g2d_all[v * n:(v + 1) * n][sel], fo["records"][0]["conic"][:, sel])
                go = bo["g2d"].T[sel]
                g_rel = float(np.linalg.norm(g2d - go) / np.linalg.norm(go))
                rms = np.sqrt(np.mean(go * go, axis=0))
                g_elem = float(np.max(np.abs(g2d - go) - 1e-3 * (np.abs(go) + 1e-2 * rms)))
                checks.append({"view": v, "image_max_rel": float(err[:, ~amb].max()), "image_rel_l2": rel_l2,
                               "ambiguous_pixels": int(amb.sum()), "grad2d_rel_l2": g_rel,
                               "grad2d_elem_excess": g_elem,
                               "excluded_fraction": float((ex & visv).sum() / max(visv.sum(), 1))})
                log(f"parity view {v}: {checks[-1]}")
            del fo, bo
            if t_ora >= 10.0:
                break
        if checks:
            ok = all(c_["image_max_rel"] <= 1e-5 and c_["image_rel_l2"] <= 1e-5 and c_["grad2d_rel_l2"] <= 1e-3
                     and c_["grad2d_elem_excess"] <= 0.0 and c_["excluded_fraction"] < 0.05 for c_ in checks)
            parity = {"views": [c_["view"] for c_ in checks],
                      "image_max_rel": max(c_["image_max_rel"] for c_ in checks),
                      "image_rel_l2": max(c_["image_rel_l2"] for c_ in checks),
                      "grad2d_rel_l2": max(c_["grad2d_rel_l2"] for c_ in checks),
                      "grad2d_elem_excess": max(c_["grad2d_elem_excess"] for c_ in checks),
                      "ambiguous_pixels": sum(c_["ambiguous_pixels"] for c_ in checks),
                      "pixels": sum(sizes[c_["view"]][0] * sizes[c_["view"]][1] for c_ in checks),
                      "excluded_fraction_max": max(c_["excluded_fraction"] for c_ in checks),
                      "pass": bool(ok)}
            log(f"parity: {parity}")
        if not args.no_cpu:
            px = sum(sizes[v][0] * sizes[v][1] for v in done)
            cpu = {"value": round(px / t_ora / 1e6, 5), "unit": "Mpixels/s", "cores": threads, "kind": "oracle",
                   "cpu": cpu_model(),
                   "sample": f"FP64 oracle forward + L1 + backward (projection of all {n} Gaussians per view) "
                             f"of {len(done)} of the {V} views, taken round-robin over the resolutions "
                             f"({px} pixels), {t_ora:.1f} s"}
            log(f"cpu baseline: {cpu}")

    # ---- the oracle on the other configurations (whole steps of the small ones, one view of the large)
    oracle_cfg = None
    if args.oracle_configs:
        import oracle
        oracle_cfg = {}
        for k in [int(x) for x in args.oracle_configs.split(",") if x]:
            sc = scenes.make_config(k)
            Pk = oracle.Params.from_scene(sc)
            ok_ = oracle.default_opts()
            views = list(range(sc.n_views)) if k in (0, 1) else [0]
            t1 = time.time()
            for v in views:
                c = sc.cameras[v]
                fo = oracle.forward(Pk, [c], ok_)
                d = np.sign(fo["images"][0] - sc.targets[v]) / (3.0 * c["W"] * c["H"] * sc.n_views)
                oracle.backward(Pk, [c], ok_, fo, [d])
                del fo
            dt = time.time() - t1
            px = sum(sc.cameras[v]["W"] * sc.cameras[v]["H"] for v in views)
            oracle_cfg[sc.name] = {"views": len(views), "of_views": sc.n_views, "s": round(dt, 2),
                                   "mpixels_per_s": round(px / dt / 1e6, 4)}
            log(f"oracle {sc.name}: {oracle_cfg[sc.name]}")
            del sc, Pk

    mpix = P / (ms_batched * 1e-3) / 1e6
    out = {
        "metric": "fwd+bwd Mpixels/s and Gaussians/s (batched vs per-view) at 1e-5 image tol",
        "value": round(mpix, 2),
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_batched, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": scene_random.name, "gaussians": n, "views": V, "pixels": P,
                   "form": "batched fused fwd+L1+bwd with SD statistics, one HIP graph",
                   "tile": f"{opt.tile_w}x{opt.tile_h}", "lds_batch": opt.lds_batch,
                   "grid_per_cu": opt.grid_per_cu, "bwd_variant": "stored" if counts.bwd_variant == 2 else "recompute",
                   "bwd_reduce": opt.bwd_reduce, "project_table": opt.project_table,
                   "gaussian_order": args.order},
        "gaussians_per_s": round(n * V / (ms_batched * 1e-3), 1),
        "visible_gaussian_views_per_s": round(vis / (ms_batched * 1e-3), 1),
        "plain_ms_per_step": None if ms_plain is None else round(ms_plain, 3),
        "plain_mpixels_per_s": None if ms_plain is None else round(P / (ms_plain * 1e-3) / 1e6, 2),
        "batched_vs_plain": None if ms_plain is None else round(ms_plain / ms_batched, 3),
        "random_order_ms_per_step": None if ms_random is None else round(ms_random, 4),
        "step_ms_single": spread,
        "memory": memory,
        "loss": loss_gpu,
        "counts": {"visible": vis, "union": counts.visible_union, "intersections": I, "walked_pairs": walked,
                   "evaluated_pairs": evaluated, "blended_pairs": blended},
        "roofline": roof,
        "adam": adam,
        "fcs": fcs,
        "densify": dens,
        "parity": parity,
        "cpu_baseline": cpu,
        "oracle_other_configs": oracle_cfg,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
