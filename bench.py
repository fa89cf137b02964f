#!/usr/bin/env python3
"""Render+backward throughput of the MI355X Gaussian-splatting path.

One step = the whole hot path over one batch: EWA projection, binning and
sort, forward compositing of RGB/depth/alpha, backward compositing,
projection backward and the per-view se(3) pose gradient, for every view of
the workload.  Inputs are seeded synthetic scenes already resident in HBM.

Default workload: the 1M-Gaussian corridor scene seen by 8 keyframes at
1200x680 (fx = fy = 600), all views forward+backward in one batched call.

Prints one JSON line (rank 0):
  value        views per second (whole job)
  roofline     the dominant kernel's achieved rate vs MI355X peak, from HIP
               events recorded on the launch stream inside the timed pass
  cpu_baseline the FP64 oracle on the host cores on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3

# Algorithmic work per unit (the derivation is in the design notes).
# Compositing, per (pixel, Gaussian) evaluation and per blend:
FWD_FLOP_PER_EVAL = 15.0     # offset, quadratic form, opacity, clamp, cutoff test (+ one exp)
FWD_FLOP_PER_BLEND = 12.0    # transmittance update and the four accumulations
BWD_FLOP_PER_BLEND = 60.0    # recomputed falloff, transmittance recovery, dL/dalpha, the 10 per-Gaussian
                             # partials and their share of the wavefront reduction (+ one exp, one reciprocal)
# HBM bytes: per pair staged (record line 48 B read once per tile, value 4 B),
# per pixel (5 planes + T_final + n_contrib), per visible record's gradient row
PAIR_STAGE_BYTES = 52.0
FWD_PIXEL_BYTES = 28.0
BWD_PIXEL_BYTES = 28.0       # 5 upstream planes, T_final, n_contrib read
ACC_ROW_BYTES = 40.0
# LDS bytes delivered to lanes per wavefront step (one wavefront of 64
# lanes taking one hit-list entry): the entry's index, position/opacity,
# pre-scaled conic and colour (forward); index, position and conic, plus
# colour and row offset on active steps (backward); and per staged entry its
# 56 B written once and 40 B read by each wavefront's quadrant test.
FWD_LDS_PER_STEP = 64 * (2 + 16 + 16 + 16)
BWD_LDS_PER_STEP = 64 * (2 + 16 + 16)
BWD_LDS_PER_ACTIVE = 64 * 16
LDS_PER_STAGED = 56.0
LDS_PER_STAGED_TEST = 40.0
SORT_BYTES_PER_PAIR_PASS = 20.0  # 32-bit keys and values: histogram read 4 B, scatter read 8 B + write 8 B

# HBM bytes per launch of the compositing kernels from rocprofv3 FETCH_SIZE /
# WRITE_SIZE passes over the default workload and configuration (the
# profiles directory holds the summary), scaled by what the same counters
# read for a 256 MiB device copy (FETCH_SIZE x 2, WRITE_SIZE x 1).  They hold
# only for the kernel sources they were taken with; after any change to
# those the traffic is reported as null until it is measured again.
MEASURED_TRAFFIC = {
    ("composite_backward", 32, 8, 0, 256): {"fetch_bytes": 1121201327.0, "write_bytes": 615417856.0,
                                            "sources_sha256": "585f2e632cd442233005dcbcf8e7891d9d7005037941c92a7a9e4fa64bba680d"},
    ("composite_forward", 32, 8, 0, 256): {"fetch_bytes": 1086211335.0, "write_bytes": 194673664.0,
                                           "sources_sha256": "585f2e632cd442233005dcbcf8e7891d9d7005037941c92a7a9e4fa64bba680d"},
}
TRAFFIC_SOURCES = ("paper_2505_18992_amd/csrc/composite.hip", "paper_2505_18992_amd/csrc/internal.h")


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, cfg):
    rec = MEASURED_TRAFFIC.get((kernel, cfg["tile_w"], cfg["tile_h"], cfg["persistent"], cfg["lds_batch"]))
    if rec is None or rec["sources_sha256"] != sources_sha256():
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name):
    import scenes
    if name == "c4-1200":
        sc = scenes.make_c4(sizes=(1200, 680))
        desc = "corridor scene, 1M Gaussians, 8 keyframes at 1200x680, batched forward+backward (params + pose)"
    elif name == "c4-mixed":
        sc = scenes.make_c4()
        desc = "corridor scene, 1M Gaussians, 8 keyframes of mixed resolution, batched forward+backward"
    elif name == "c2":
        sc = scenes.make_c2()
        desc = "room scene, 200k Gaussians, one 640x480 view, forward+backward (params + pose)"
    elif name == "c5":
        sc = scenes.make_c5()
        desc = "street scene, 4 submaps x 1.5M Gaussians, 16 keyframes at 1242x375, forward+backward"
    elif name == "c1":
        sc = scenes.make_c1()
        desc = "1000 random Gaussians, one 128x96 view"
    else:
        raise SystemExit(f"unknown workload {name}")
    return sc, desc


CPU_CROPS = 8  # seeded 128x128 gradient crops per view in the CPU baseline


def cpu_baseline(sc, fp32=False, views=None, crops=CPU_CROPS):
    """Time the oracle (FP64, or its FP32 build) on views of the workload
    (all by default): the full forward image, and the gradient over seeded
    128x128 crops scaled to the whole view."""
    import oracle
    rng = np.random.default_rng(7)
    t_total, blends, crop_px_total, t_fwd_total, t_grad_total = 0.0, 0.0, 0, 0.0, 0.0
    views = list(range(len(sc.cameras))) if views is None else list(views)
    for v in views:
        cam = sc.cameras[v]
        g = sc.sets[sc.view_set[v]]
        W, H = cam.width, cam.height
        t0 = time.perf_counter()
        ref = oracle.render(g, cam, fp32=fp32)
        t_fwd = time.perf_counter() - t0
        skip = np.ones((H, W), np.uint8)
        cw, ch = min(128, W), min(128, H)
        for _ in range(crops):
            x0 = int(rng.integers(0, W - cw + 1)); y0 = int(rng.integers(0, H - ch + 1))
            skip[y0:y0 + ch, x0:x0 + cw] = 0
        crop_px = int((skip == 0).sum())
        gr, gd, ga = (w.astype(np.float64) for w in sc.weights[v])
        t0 = time.perf_counter()
        oracle.grad(g, cam, gr, gd, ga, skip=skip, fp32=fp32)
        t_grad = time.perf_counter() - t0
        t_total += t_fwd + t_grad * (W * H) / crop_px
        blends += float(ref["n_blend"].sum())
        crop_px_total += crop_px
        t_fwd_total += t_fwd
        t_grad_total += t_grad
    nv = len(views)
    prec = "FP32" if fp32 else "FP64"
    return {"value": nv / t_total, "unit": "views/s", "cores": oracle.num_threads(), "kind": "oracle",
            "precision": prec,
            "sample": f"{nv} view(s) of the workload: {prec} forward on each full view ({t_fwd_total:.1f} s) and the "
                      f"gradient on {crops} seeded 128x128 crops per view ({crop_px_total} px, {t_grad_total:.1f} s), "
                      f"scaled by pixel count",
            "blends_per_sec": blends / t_total, "seconds_measured": t_fwd_total + t_grad_total}


def cpu_oracle_configs(names):
    """The oracle (FP64 and FP32 builds) on a bounded sample of each other
    workload: C1 and C2 (one view each), one view of each resolution of the
    mixed corridor, one street view."""
    out = {}
    for name in names:
        sc, _ = workload(name)
        if name == "c4-mixed":
            first = {}
            for v, c in enumerate(sc.cameras):
                first.setdefault((c.width, c.height), v)
            views = sorted(first.values())
        elif name == "c5":
            views = [9]
        else:
            views = [0]
        out[name] = {"fp64": cpu_baseline(sc, views=views), "fp32": cpu_baseline(sc, fp32=True, views=views)}
        log(f"[bench] CPU oracle {name}: FP64 {out[name]['fp64']['value']:.3f} views/s, "
            f"FP32 {out[name]['fp32']['value']:.3f} views/s")
    return out


LOSS_BYTES_PER_PIXEL = 52.0  # rendered colour+depth and target colour+depth read (32 B), 3+1+1 gradient planes written


def time_mapping_loss(win, cams, steps):
    """Mapping loss (eq. 7-8) of every view of the window against a
    perturbed copy of its rendered frame: ms per call over all views and the
    achieved rate of the algorithmic bytes (inputs read once, planes written
    once)."""
    import torch
    from paper_2505_18992_amd import mapping_loss
    gen = torch.Generator(device="cuda").manual_seed(11)
    ims, tgs = [], []
    for rgb, depth, _ in win.outputs:
        ims.append((rgb, depth))
        noise = torch.randn(rgb.shape, generator=gen, device=rgb.device) * 0.05
        tgs.append(((rgb + noise).clamp(0, 1).contiguous(), torch.where(depth > 0, depth * 1.02, depth).contiguous()))
    terms, _ = mapping_loss(ims, tgs, cams)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        mapping_loss(ims, tgs, cams)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    pixels = sum(c.width * c.height for c in cams)
    gbs = LOSS_BYTES_PER_PIXEL * pixels / (ms * 1e-3) / 1e9
    log(f"[bench] mapping loss: {ms:.3f} ms for {len(cams)} views ({gbs:.0f} GB/s of algorithmic bytes)")
    return {"ms_per_call": ms, "views": len(cams), "bytes_per_pixel": LOSS_BYTES_PER_PIXEL, "achieved_GBs": gbs,
            "peak_GBs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS,
            "loss_view0": [float(v) for v in terms[0].cpu().tolist()]}


ACCUM_BYTES_PER_GAUSSIAN = 36.0   # [n,4] accumulators read and written, opacity read
ANCHOR_BYTES_PER_GAUSSIAN = 16.0  # accumulator rows read once
ANCHOR_BYTES_PER_ANCHOR = 18.0    # statistics row and two flags written
EXPAND_BYTES_PER_PIXEL = 13.0     # rendered alpha and depth and target depth read, mask byte written
EXPAND_BYTES_PER_SAMPLE = 48.0    # uniform, target depth and colour read; pixel, point and colour written


def _stage_ms(ctx, stage, fn, steps):
    """Milliseconds per call of one library stage, from the HIP events the
    library records on its launch stream around the stage's kernels (the
    host-side argument marshalling of each call is outside them)."""
    import torch
    fn()
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    calls, tot = ctx.profile_read()[stage]
    ctx.profile(False)
    return tot / max(calls, 1)


def time_expansion(sets, gw, cams, vset, cfg, win, steps, k=10, n_samples=4096):
    """Submap-expansion statistics on the workload: the accumulators in the
    projection backward (its stage time with and without them), the anchor
    reduction over the accumulators of the whole set taken as anchors of k
    Gaussians, and the expansion sampler on the window's rendered frames
    (target depth = rendered depth x 1.02, n_samples draws per view)."""
    import torch
    from paper_2505_18992_amd import RenderWindow, anchor_stats, expansion_sample, get_context
    ctx = get_context(0)
    ewin = RenderWindow(sets, cams, vset, tile=(cfg["tile_w"], cfg["tile_h"]), persistent=cfg["persistent"],
                        use_graph=False, pair_capacity=cfg["pair_capacity"], lds_batch=cfg["lds_batch"])
    for v in range(len(cams)):
        for dst, src in zip(ewin.grad_out[v], gw[v]):
            dst.copy_(src)
    ewin.run()
    torch.cuda.synchronize()
    acc = [torch.zeros((s[0].shape[0], 4), dtype=torch.float32, device=s[0].device) for s in sets]
    pb = {}
    for mode in ("plain", "accum"):
        ewin.set_accum(acc if mode == "accum" else None)
        ewin.run(forward=False, backward=True)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(steps):
            ewin.run(forward=False, backward=True)
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
        calls, tot = prof["project_backward"]
        pb[mode] = tot / max(calls, 1)
    ewin.close()
    n = sum(s[0].shape[0] for s in sets)
    extra = pb["accum"] - pb["plain"]
    # anchor reduction over the first set's accumulators
    a0 = acc[0][: (acc[0].shape[0] // k) * k]
    m = a0.shape[0] // k
    ms_anchor = _stage_ms(ctx, "anchor_stats", lambda: anchor_stats(a0, k, 1e-3, 0.05), steps)
    gbs_anchor = (ANCHOR_BYTES_PER_GAUSSIAN * m * k + ANCHOR_BYTES_PER_ANCHOR * m) / (ms_anchor * 1e-3) / 1e9
    # expansion sampler on the rendered frames
    ims = [(None, d, a) for _, d, a in win.outputs]
    tgs = [(rgb, torch.where(d > 0, d * 1.02, d).contiguous()) for rgb, d, _ in win.outputs]
    gen = torch.Generator(device="cuda").manual_seed(12)
    u = torch.rand((len(cams), n_samples), generator=gen, device="cuda")
    res = expansion_sample(ims, tgs, cams, 0.5, 0.1, u)
    counts = res["counts"].cpu().tolist()
    ms_exp = _stage_ms(ctx, "expansion", lambda: expansion_sample(ims, tgs, cams, 0.5, 0.1, u), steps)
    pixels = sum(c.width * c.height for c in cams)
    gbs_exp = (EXPAND_BYTES_PER_PIXEL * pixels + EXPAND_BYTES_PER_SAMPLE * n_samples * len(cams)) / (ms_exp * 1e-3) / 1e9
    log(f"[bench] expansion: project_backward {pb['plain']:.3f} -> {pb['accum']:.3f} ms with accumulators; "
        f"anchor stats {ms_anchor:.4f} ms ({gbs_anchor:.0f} GB/s); sampler {ms_exp:.4f} ms ({gbs_exp:.0f} GB/s)")
    return {
        "accumulate": {"project_backward_ms": pb["plain"], "project_backward_ms_with_accum": pb["accum"],
                       "extra_ms": extra, "gaussians": n, "bytes_per_gaussian": ACCUM_BYTES_PER_GAUSSIAN,
                       "achieved_GBs_of_extra": ACCUM_BYTES_PER_GAUSSIAN * n / (extra * 1e-3) / 1e9
                       if extra > 0 else None},
        "anchor_stats": {"ms_per_call": ms_anchor, "anchors": m, "k": k, "achieved_GBs": gbs_anchor,
                         "frac": gbs_anchor / HBM_PEAK_GBS},
        "expansion_sample": {"ms_per_call": ms_exp, "views": len(cams), "pixels": pixels,
                             "samples_per_view": n_samples, "candidates": counts, "achieved_GBs": gbs_exp,
                             "frac": gbs_exp / HBM_PEAK_GBS},
    }


DISTILL_BYTES_PER_PIXEL = 72.0  # both renders' colour+depth read (32 B), both sides' gradient planes written (40 B)


def time_distillation(steps, m=4):
    """One submap-fusion iteration of eq. 14 on the street workload: two
    overlapping 1.5 M-Gaussian submaps rendered at m keyframes of their
    overlap in one window (2m views, one graph per part), the distillation
    loss writing both sides' upstream planes, and the backward."""
    import torch
    import scenes
    from paper_2505_18992_amd import RenderWindow, distill_loss, get_context
    ctx = get_context(0)
    sc = scenes.make_c5(submaps=2, weights=False)
    kf = [scenes.camera_look((52.0 + 16.0 * i / max(m - 1, 1), 1.0 - 2.0 * (i % 2), 1.7), 0.03 * (i % 3 - 1), 0.0,
                             0.0, 1242, 375, 720.0, 720.0, 621.0, 187.5) for i in range(m)]
    cams, vset = kf + kf, [0] * m + [1] * m
    sets = [tuple(torch.from_numpy(a).cuda() for a in g.arrays()) for g in sc.sets]
    win = RenderWindow(sets, cams, vset, tile=(32, 8), persistent=0)
    ia, ib = win.outputs[:m], win.outputs[m:]

    def iteration():
        win.run(forward=True, backward=False)
        distill_loss(ia, ib, kf, grad_a=win.grad_out[:m], grad_b=win.grad_out[m:])
        win.run(forward=False, backward=True)
    for _ in range(3):
        iteration()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        iteration()
    torch.cuda.synchronize()
    ms_iter = (time.perf_counter() - t0) * 1e3 / steps
    ms_loss = _stage_ms(ctx, "distillation",
                        lambda: distill_loss(ia, ib, kf, grad_a=win.grad_out[:m], grad_b=win.grad_out[m:]), steps)
    loss, _, _, _ = distill_loss(ia, ib, kf, grad_a=win.grad_out[:m], grad_b=win.grad_out[m:])
    st = win.stats()
    # stage times of the same iteration launched eagerly
    twin = RenderWindow(sets, cams, vset, tile=(32, 8), persistent=0, use_graph=False,
                        pair_capacity=win.config()["pair_capacity"])
    tia, tib = twin.outputs[:m], twin.outputs[m:]

    def eager_iteration():
        twin.run(forward=True, backward=False)
        distill_loss(tia, tib, kf, grad_a=twin.grad_out[:m], grad_b=twin.grad_out[m:])
        twin.run(forward=False, backward=True)
    eager_iteration()
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(steps):
        eager_iteration()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    twin.close()
    stage_ms = {k: v[1] / steps for k, v in prof.items() if v[0] > 0}
    win.close()
    pixels = m * 1242 * 375
    gbs = DISTILL_BYTES_PER_PIXEL * pixels / (ms_loss * 1e-3) / 1e9
    log(f"[bench] distillation: {ms_iter:.3f} ms per iteration ({2 * m} views of 2 x 1.5M-Gaussian submaps); "
        f"loss kernel {ms_loss:.4f} ms ({gbs:.0f} GB/s)")
    return {"ms_per_iteration": ms_iter, "keyframes": m, "views": 2 * m, "gaussians_per_submap": sc.sets[0].n,
            "resolution": "1242x375", "blends": st["n_blended"], "evaluated": st["n_evaluated"],
            "pairs": st["n_pairs"], "loss": float(loss[0]), "stage_ms": stage_ms,
            "loss_kernel": {"ms_per_call": ms_loss, "bytes_per_pixel": DISTILL_BYTES_PER_PIXEL, "achieved_GBs": gbs,
                            "frac": gbs / HBM_PEAK_GBS}}


def time_decode(steps):
    """The voxel-anchor decode of eq. 1-5 at the anchor workload (50 k
    anchors, k = 10, decoder width 64: 500 k neural Gaussians) inside one
    mapping iteration of the anchor representation: decode, render of one
    1200x680 view, render backward, decode backward."""
    import numpy as np
    import torch
    import scenes
    from paper_2505_18992_amd import decode_backward, decode_forward, get_context, render, render_backward
    ctx = get_context(0)
    sc = scenes.make_c3()
    a, d = sc.anchors, sc.decoder
    cam = sc.cameras[0]
    R, t = cam.world_to_cam[:, :3].astype(np.float64), cam.world_to_cam[:, 3].astype(np.float64)
    centre = (-R.T @ t).astype(np.float32)  # the camera centre, a constant of the decode
    anchors = tuple(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (a.xyz, a.feat, a.scale, a.offsets))
    mlp = tuple([torch.from_numpy(x).cuda() for x in lst] for lst in (d.W1, d.b1, d.W2, d.b2))
    wts = [tuple(torch.from_numpy(x).cuda() for x in sc.weights[0])]
    gen = torch.Generator(device="cuda").manual_seed(5)
    dec = decode_forward(anchors, mlp, centre)
    up = [torch.randn(t.shape, generator=gen, device="cuda") for t in dec]

    def iteration():
        g = decode_forward(anchors, mlp, centre)
        outs, saved = render([g], [cam], tile=(32, 8))
        grads, _ = render_backward(saved, wts)
        saved.close()
        decode_backward(anchors, mlp, centre, grads[0])
    for _ in range(3):
        iteration()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        iteration()
    torch.cuda.synchronize()
    ms_iter = (time.perf_counter() - t0) * 1e3 / steps
    ms_f = _stage_ms(ctx, "decode_forward", lambda: decode_forward(anchors, mlp, centre), steps)
    ms_b = _stage_ms(ctx, "decode_backward", lambda: decode_backward(anchors, mlp, centre, up), steps)
    m, k, width = a.xyz.shape[0], a.k, d.W1[0].shape[0]
    # two matrix products per head: [36 -> width] and [width -> k, 3k, 7k]
    flop_f = 2.0 * m * (3 * 36 * width + width * 11 * k)
    flop_b = 2.0 * flop_f  # input and weight gradients of both layers
    byts_f = m * (12 + 128 + 12 + 12 * k) + m * k * 56  # anchors read, Gaussians written
    log(f"[bench] decode (50k anchors, k={k}): forward {ms_f:.4f} ms, backward {ms_b:.4f} ms; "
        f"anchor mapping iteration {ms_iter:.3f} ms")
    return {"anchors": m, "k": k, "width": width, "gaussians": m * k,
            "forward": {"ms": ms_f, "flop": flop_f, "achieved_TFLOPs": flop_f / (ms_f * 1e-3) / 1e12,
                        "bytes": byts_f, "achieved_GBs": byts_f / (ms_f * 1e-3) / 1e9},
            "backward": {"ms": ms_b, "flop": flop_b, "achieved_TFLOPs": flop_b / (ms_b * 1e-3) / 1e12},
            "iteration_ms": ms_iter, "iteration": "decode, render 1200x680, render backward, decode backward"}


def time_registration(steps, voxel=1.0, cap=20, tau=3.0, sigma=1.0):
    """Frame-to-map registration (eq. 10-12) on the street LiDAR case: the
    voxel map of 1.5 M map points, then per frame the double downsampling of
    the 131 k-point sweep (0.5 and 1.5 voxels) and the Gauss-Newton
    registration from the perturbed pose; and the same registration on the
    whole sweep (every point a source point)."""
    import numpy as np
    import torch
    import scenes
    from paper_2505_18992_amd import VoxelMap, get_context, icp_register, voxel_downsample
    ctx = get_context(0)
    sc = scenes.make_street_scan()
    pts = torch.from_numpy(sc.map_points).cuda()
    scan = torch.from_numpy(sc.scan).cuda()
    VoxelMap(pts, voxel, cap).close()
    torch.cuda.synchronize()
    ctx.profile(True)
    vm = VoxelMap(pts, voxel, cap)
    torch.cuda.synchronize()
    ms_build = ctx.profile_read()["voxel_map"][1]
    ctx.profile(False)
    n_vox = vm.info()[1]

    def frame():
        a = voxel_downsample(scan, 0.5 * voxel)
        s1 = scan[a].contiguous()
        b = voxel_downsample(s1, 1.5 * voxel)
        src = s1[b].contiguous()
        return icp_register(vm, src, sc.pose_init, None, tau, sigma, 100, 1e-4), src.shape[0]
    frame()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        (pose, res), n_src = frame()
    ms_frame = (time.perf_counter() - t0) * 1e3 / steps
    err_t = float(np.abs(pose[:, 3] - sc.pose_gt[:, 3]).max())
    # the whole sweep as the source
    icp_register(vm, scan, sc.pose_init, None, tau, sigma, 100, 1e-4)
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(max(2, steps // 4)):
        dpose, dres = icp_register(vm, scan, sc.pose_init, None, tau, sigma, 100, 1e-4)
    ms_dense = (time.perf_counter() - t0) * 1e3 / max(2, steps // 4)
    calls, icp_ms = ctx.profile_read()["icp"]
    ctx.profile(False)
    vm.close()
    ms_iter = icp_ms / max(calls, 1) / max(dres["iterations"], 1)
    log(f"[bench] registration: map build {ms_build:.3f} ms ({sc.map_points.shape[0]} points, {n_vox} voxels); "
        f"frame {ms_frame:.3f} ms ({n_src} source points, {res['iterations']} steps, |dt| {err_t:.3f} m); "
        f"whole sweep {ms_dense:.3f} ms ({scan.shape[0]} points, {dres['iterations']} steps, "
        f"{ms_iter:.3f} ms per step)")
    return {"map_points": int(sc.map_points.shape[0]), "voxels": int(n_vox), "voxel": voxel,
            "max_per_voxel": cap, "map_build_ms": ms_build,
            "frame": {"ms": ms_frame, "scan_points": int(scan.shape[0]), "source_points": int(n_src),
                      "iterations": res["iterations"], "converged": res["converged"],
                      "translation_error_m": err_t},
            "whole_sweep": {"ms": ms_dense, "source_points": int(scan.shape[0]), "iterations": dres["iterations"],
                            "ms_per_iteration": ms_iter,
                            "queries_per_sec": scan.shape[0] / (ms_iter * 1e-3)}}


def stage_rooflines(st, stage_ms, n_gauss, nv, peaks):
    """Per stage of the step: algorithmic HBM bytes, FP32 FLOP, LDS bytes
    delivered to lanes and transcendental operations, from the counters of
    the timed pass, and t_roof = the largest of bytes / 8 TB/s, FLOP / 157.3
    TFLOP/s, LDS bytes / the measured broadcast LDS rate and transcendentals
    / the measured exp2 rate."""
    R, V, P = st["n_records"], st["n_visible"], st["n_pairs"]
    E, B, px, T = st["n_evaluated"], st["n_blended"], st["n_pixels"], st["n_tiles"]
    fs, bs, ba = st["n_fwd_steps"], st["n_bwd_steps"], st["n_bwd_active"]
    waves_per_tile = st["tile_w"] * st["tile_h"] // 64
    sort_passes = math.ceil(math.ceil(math.log2(max(T, 2))) / 8)
    work = {
        "project": {"hbm_bytes": 56.0 * n_gauss + 76.0 * V + 4.0 * R},
        "scan": {"hbm_bytes": 12.0 * R + 8.0 * V},
        "depth_order": {"hbm_bytes": (4 * 20.0 + 20.0 + 12.0) * V},
        "emit": {"hbm_bytes": 16.0 * V + 8.0 * P},
        "sort": {"hbm_bytes": SORT_BYTES_PER_PAIR_PASS * sort_passes * P},
        "ranges": {"hbm_bytes": 4.0 * P + 8.0 * T},
        "composite_forward": {"hbm_bytes": PAIR_STAGE_BYTES * P + FWD_PIXEL_BYTES * px,
                              "flop": FWD_FLOP_PER_EVAL * E + FWD_FLOP_PER_BLEND * B,
                              "lds_bytes": FWD_LDS_PER_STEP * fs + (LDS_PER_STAGED + LDS_PER_STAGED_TEST *
                                                                    waves_per_tile) * P,
                              "trans": float(E)},
        "composite_backward": {"hbm_bytes": PAIR_STAGE_BYTES * P + BWD_PIXEL_BYTES * px + ACC_ROW_BYTES * V,
                               "flop": BWD_FLOP_PER_BLEND * B,
                               "lds_bytes": BWD_LDS_PER_STEP * bs + BWD_LDS_PER_ACTIVE * ba + LDS_PER_STAGED * P,
                               "trans": 2.0 * B},
        "project_backward": {"hbm_bytes": 112.0 * n_gauss + 80.0 * V},
        "pose_reduce": {"hbm_bytes": 0.0},
    }
    out = {}
    for name, ms in stage_ms.items():
        if name not in work:
            continue
        w = dict(hbm_bytes=0.0, flop=0.0, lds_bytes=0.0, trans=0.0)
        w.update(work[name])
        t = {"hbm": w["hbm_bytes"] / (HBM_PEAK_GBS * 1e9), "alu": w["flop"] / (FP32_VECTOR_PEAK_TFLOPS * 1e12),
             "lds": w["lds_bytes"] / (peaks["lds_broadcast_GBs"] * 1e9), "trans": w["trans"] / (peaks["exp2_Tps"] * 1e12)}
        bound = max(t, key=t.get)
        t_roof = t[bound] * 1e3
        row = dict(w, ms=ms, bound=bound, t_roof_ms=t_roof, frac=t_roof / ms if ms > 0 else None,
                   hbm_GBs=w["hbm_bytes"] / (ms * 1e-3) / 1e9, lds_GBs=w["lds_bytes"] / (ms * 1e-3) / 1e9)
        out[name] = row
    return out


def measure_workload(sc, args, ctx, tile, steps, warmup, one_view=True):
    """One workload on the GPU: a searched, graph-captured window over all
    its views (the timed step), the per-stage HIP-event times of the same
    configuration launched without the graph, and the same views one per
    launch."""
    import torch
    from paper_2505_18992_amd import RenderWindow, render, render_backward
    dev = torch.device("cuda:0")
    sets = [tuple(torch.from_numpy(a).to(dev) for a in g.arrays()) for g in sc.sets]
    gw = [tuple(torch.from_numpy(w).to(dev) for w in ws) for ws in sc.weights]
    cams, vset = sc.cameras, sc.view_set
    nv = len(cams)
    # the mapping-window launch: all views bound, tuned, captured in HIP graphs
    t0 = time.perf_counter()
    win = RenderWindow(sets, cams, vset, tile=tile, persistent=args.persistent, use_graph=True,
                       lds_batch=args.lds_batch, tune_cache=args.tune_cache or None, count=False)
    cfg = win.config()
    t_tune = time.perf_counter() - t0
    log(f"[bench] window ready in {t_tune:.1f} s: tile {cfg['tile_w']}x{cfg['tile_h']}, "
        f"persistent {cfg['persistent']}, lds batch {cfg['lds_batch']}, pair capacity {cfg['pair_capacity']}")
    for v in range(nv):
        for dst, src in zip(win.grad_out[v], gw[v]):
            dst.copy_(src)
    for _ in range(warmup):
        win.run()
    torch.cuda.synchronize()

    # timed region: K whole steps (forward + backward of every view)
    t0 = time.perf_counter()
    for _ in range(steps):
        win.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / steps
    st = win.stats()
    if st["overflow"]:
        raise SystemExit("pair capacity overflow in the timed pass")
    log(f"[bench] {steps} steps: {ms_step:.3f} ms/step")
    # the timed pass does not count its evaluations and blends (that is
    # instrumentation): one eager pass of the same configuration with the
    # counters on gives them (the render is deterministic)
    cwin = RenderWindow(sets, cams, vset, tile=(cfg["tile_w"], cfg["tile_h"]), persistent=cfg["persistent"],
                        use_graph=False, pair_capacity=cfg["pair_capacity"], lds_batch=cfg["lds_batch"], count=True)
    for v in range(nv):
        for dst, src in zip(cwin.grad_out[v], gw[v]):
            dst.copy_(src)
    cwin.run()
    cst = cwin.stats()
    cwin.close()
    for k in ("n_evaluated", "n_blended", "n_fwd_steps"):
        st[k] = cst[k]
    assert cst["n_pairs"] == st["n_pairs"] and cst["n_bwd_steps"] == st["n_bwd_steps"]

    # per-stage HIP-event timing: the same configuration launched without the
    # graph (events recorded on the launch stream around every stage)
    twin = RenderWindow(sets, cams, vset, tile=(cfg["tile_w"], cfg["tile_h"]), persistent=cfg["persistent"],
                        use_graph=False, pair_capacity=cfg["pair_capacity"], lds_batch=cfg["lds_batch"], count=False)
    for v in range(nv):
        for dst, src in zip(twin.grad_out[v], gw[v]):
            dst.copy_(src)
    twin.run()
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        twin.run()
    torch.cuda.synchronize()
    ms_eager_window = (time.perf_counter() - t0) * 1e3 / steps
    prof = ctx.profile_read()
    ctx.profile(False)
    twin.close()
    stage_ms = {k: v[1] / max(v[0], 1) for k, v in prof.items() if v[0] > 0}
    # fills run in both halves: per step, not per launch sequence
    if "fill" in prof:
        stage_ms["fill"] = prof["fill"][1] / steps
    log("[bench] stage ms/step: " + ", ".join(f"{k}={v:.3f}" for k, v in sorted(stage_ms.items(), key=lambda x: -x[1])))

    # one view per launch: the same kernels, each view its own forward+backward call
    ms_per_view_launch = None
    per_view_caps = []

    def one_view_pass():
        for v in range(nv):
            outs, saved = render([sets[vset[v]]], [cams[v]], [0], tile=(cfg["tile_w"], cfg["tile_h"]),
                                 pair_capacity=per_view_caps[v], lds_batch=cfg["lds_batch"],
                                 grid_ctas=cfg["persistent"], count=False)
            render_backward(saved, [gw[v]])
            saved.close()
    if one_view:
        for v in range(nv):
            outs, saved = render([sets[vset[v]]], [cams[v]], [0], tile=(cfg["tile_w"], cfg["tile_h"]),
                                 lds_batch=cfg["lds_batch"], grid_ctas=cfg["persistent"])
            per_view_caps.append(int(saved.stats()["n_pairs"] * 1.25) + 4096)
            saved.close()
        one_view_pass()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = max(2, steps // 4)
        for _ in range(reps):
            one_view_pass()
        torch.cuda.synchronize()
        ms_per_view_launch = (time.perf_counter() - t0) * 1e3 / reps
        log(f"[bench] one view per launch: {ms_per_view_launch:.3f} ms for {nv} views; "
            f"eager window {ms_eager_window:.3f} ms")
    return {"win": win, "cfg": cfg, "stats": st, "stage_ms": stage_ms, "ms_step": ms_step, "sets": sets, "gw": gw,
            "n_gauss": sum(g.n for g in sc.sets), "ms_per_view_launch": ms_per_view_launch, "tune_seconds": t_tune,
            "ms_eager_window": ms_eager_window}


def config_line(name, sc, desc, m, peaks):
    """The summary of one workload measured in the same run."""
    st, ms, nv = m["stats"], m["ms_step"], len(sc.cameras)
    table = stage_rooflines(st, m["stage_ms"], m["n_gauss"], nv, peaks)
    dom = max(m["stage_ms"], key=m["stage_ms"].get)
    row = table.get(dom, {})
    t_roof = sum(r["t_roof_ms"] for r in table.values())
    out = {"workload": desc, "views": nv, "gaussians": m["n_gauss"],
           "resolutions": sorted({f"{c.width}x{c.height}" for c in sc.cameras}),
           "ms_per_step": ms, "views_per_sec": nv / (ms * 1e-3), "blends_per_sec": st["n_blended"] / (ms * 1e-3),
           "counts": {"pairs": st["n_pairs"], "evaluated": st["n_evaluated"], "blended": st["n_blended"]},
           "window": {k: m["cfg"][k] for k in ("tile_w", "tile_h", "persistent", "lds_batch")},
           "dominant_kernel": dom, "dominant_ms": m["stage_ms"].get(dom),
           "dominant_frac": (row["flop"] / (row["ms"] * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS
                             if row.get("flop") else row["hbm_bytes"] / (row["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS)
           if row else None,
           "step_roofline_frac": t_roof / ms}
    if m["ms_per_view_launch"] is not None:
        out["one_view_per_launch"] = {"ms_for_all_views": m["ms_per_view_launch"],
                                      "views_per_sec": nv / (m["ms_per_view_launch"] * 1e-3),
                                      "batched_speedup": m["ms_per_view_launch"] / ms}
    log(f"[bench] {name}: {ms:.3f} ms/step, {out['views_per_sec']:.0f} views/s, "
        f"{out['blends_per_sec'] / 1e9:.1f} G blends/s")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c4-1200")
    ap.add_argument("--tile", default="auto", help="WxH, or auto for the window's search over shapes")
    ap.add_argument("--persistent", type=int, default=-1,
                    help="persistent compositing workgroups: 0 one per tile, -1 search")
    ap.add_argument("--lds-batch", type=int, default=0, help="entries per compositing batch, 0 search")
    ap.add_argument("--tune-cache", default=os.path.join(os.environ.get("TMPDIR", "/tmp"), "vpgs_tune.json"),
                    help="JSON tuning cache of the window's search ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-one-view", action="store_true",
                    help="skip the one-view-per-launch comparison (profiling runs: it launches the same kernels)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mapping-loss, expansion, distillation, registration and decode measurements "
                         "(profiling runs of the step alone)")
    ap.add_argument("--extras", default="loss,expansion,distillation,registration,decode",
                    help="which of the extra measurements to run (comma list)")
    ap.add_argument("--configs", default="c1,c2,c4-mixed,c5",
                    help="other workloads measured in the same run (comma list, '' for none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        return 2

    import torch
    from paper_2505_18992_amd import _lib, get_context

    _lib.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = get_context(0)
    tile = None if args.tile == "auto" else tuple(int(x) for x in args.tile.split("x"))
    log(f"[bench] building workload {args.workload}")
    sc, desc = workload(args.workload)
    m = measure_workload(sc, args, ctx, tile, args.steps, args.warmup, one_view=not args.no_one_view)
    win, cfg, st, stage_ms, ms_step = m["win"], m["cfg"], m["stats"], m["stage_ms"], m["ms_step"]
    sets, gw, cams, vset, nv, n_gauss = m["sets"], m["gw"], sc.cameras, sc.view_set, len(sc.cameras), m["n_gauss"]
    ms_per_view_launch, t_tune = m["ms_per_view_launch"], m["tune_seconds"]

    loss_stage = expansion = distillation = registration = anchor_decode = None
    extras = set() if args.no_extras else {e for e in args.extras.split(",") if e}
    # the mapping loss of eq. 7-8 on the same views (rendered frames
    # against perturbed copies of themselves), timed on its own
    if "loss" in extras:
        loss_stage = time_mapping_loss(win, cams, args.steps)
    # the submap-expansion statistics of Section III-A on the same workload
    if "expansion" in extras:
        expansion = time_expansion(sets, gw, cams, vset, cfg, win, args.steps)
    # submap fusion (eq. 14) on two street submaps
    if "distillation" in extras:
        distillation = time_distillation(args.steps)
    # frame-to-map registration (eq. 10-12) on a street LiDAR sweep
    if "registration" in extras:
        registration = time_registration(args.steps)
    # the voxel-anchor decode (eq. 1-5) and its backward
    if "decode" in extras:
        anchor_decode = time_decode(args.steps)

    E, B, P = st["n_evaluated"], st["n_blended"], st["n_pairs"]
    peaks = ctx.measure_peaks()
    log("[bench] measured peaks: " + ", ".join(f"{k}={v:.1f}" for k, v in peaks.items()))
    table = stage_rooflines(st, stage_ms, n_gauss, nv, peaks)
    dom = max(stage_ms, key=stage_ms.get)
    row = table[dom]
    if dom in ("composite_forward", "composite_backward"):
        roof = {"bound": "alu", "achieved": row["flop"] / (row["ms"] * 1e-3) / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": row["hbm_bytes"] / (row["ms"] * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom, cfg)
    roof["kernel"] = dom
    roof["kernel_ms"] = row["ms"]
    roof["work_per_launch"] = row["flop"] if roof["unit"] == "TFLOP/s" else row["hbm_bytes"]
    roof["work_unit"] = ("FLOP: 60 per blend" if dom == "composite_backward" else
                         "FLOP: 15 per evaluation + 12 per blend" if dom == "composite_forward" else "HBM bytes")
    roof["frac_of_measured_fp32"] = (roof["achieved"] / peaks["fp32_fma_TFLOPs"]
                                     if roof["unit"] == "TFLOP/s" else None)
    t_roof = sum(r["t_roof_ms"] for r in table.values())
    step_roofline = {"t_roof_ms": t_roof, "t_measured_ms": ms_step, "frac": t_roof / ms_step,
                     "stage_sum_ms": sum(r["ms"] for r in table.values()), "stages": table,
                     "peaks_used": {"hbm_GBs": HBM_PEAK_GBS, "fp32_TFLOPs": FP32_VECTOR_PEAK_TFLOPS,
                                    "lds_broadcast_GBs": peaks["lds_broadcast_GBs"], "exp2_Tps": peaks["exp2_Tps"]}}
    log(f"[bench] step roofline: sum of per-stage t_roof {t_roof:.3f} ms of {ms_step:.3f} ms measured "
        f"({t_roof / ms_step:.1%})")

    # the other workloads, each a searched window over all its views
    others = {}
    for name in [c for c in args.configs.split(",") if c and c != args.workload]:
        log(f"[bench] building workload {name}")
        osc, odesc = workload(name)
        om = measure_workload(osc, args, ctx, None, max(5, args.steps // 2), 2, one_view=True)
        om["win"].close()
        others[name] = config_line(name, osc, odesc, om, peaks)
        del om, osc
        torch.cuda.empty_cache()

    views_per_s = nv / (ms_step * 1e-3)
    out = {
        "metric": "render+backward views/sec and Gaussian-pixel blends/sec at 1M Gaussians, 1200x680",
        "value": views_per_s,
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "gaussians": n_gauss, "views": nv,
                   "resolutions": sorted({f"{c.width}x{c.height}" for c in cams}),
                   "launch": "one HIP graph per forward and per backward over all views"},
        "blends_per_sec": B / (ms_step * 1e-3),
        "counts": {"pairs": P, "evaluated": E, "blended": B},
        "window": dict({k: cfg[k] for k in ("tile_w", "tile_h", "persistent", "lds_batch", "pair_capacity")},
                       tune_seconds=t_tune, tune_cache=args.tune_cache or None),
        "one_view_per_launch": None if ms_per_view_launch is None else
        {"ms_for_all_views": ms_per_view_launch, "views_per_sec": nv / (ms_per_view_launch * 1e-3),
         "batched_speedup": ms_per_view_launch / ms_step},
        "stage_ms": stage_ms,
        "mapping_loss": loss_stage,
        "expansion": expansion,
        "distillation": distillation,
        "registration": registration,
        "decode": anchor_decode,
        "roofline": roof,
        "step_roofline": step_roofline,
        "measured_peaks": peaks,
        "other_configs": others,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(sc)
        out["cpu_baseline_fp32"] = cpu_baseline(sc, fp32=True)
        out["cpu_oracle_configs"] = cpu_oracle_configs([c for c in args.configs.split(",") if c])
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
