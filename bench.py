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

# Algorithmic work per unit (see the design notes for the derivation).
FWD_FLOP_PER_EVAL = 16.0     # falloff: offset, quadratic form, exp, opacity, clamp, cutoff test
FWD_FLOP_PER_BLEND = 12.0    # transmittance update and four fused accumulations
BWD_FLOP_PER_EVAL = 16.0     # the same falloff, recomputed
BWD_FLOP_PER_BLEND = 40.0    # transmittance recovery, alpha gradient, 10 per-Gaussian partials
SORT_BYTES_PER_PAIR_PASS = 32.0  # histogram read 8 B, scatter read 12 B + write 12 B


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


def cpu_baseline(sc, budget_s=25.0):
    """Time the FP64 oracle on one view: the full forward image and the
    gradient over three seeded 128x128 crops, scaled to the whole view."""
    import oracle
    v = 0
    g = sc.sets[sc.view_set[v]]
    cam = sc.cameras[v]
    W, H = cam.width, cam.height
    t0 = time.perf_counter()
    ref = oracle.render(g, cam)
    t_fwd = time.perf_counter() - t0
    rng = np.random.default_rng(7)
    skip = np.ones((H, W), np.uint8)
    cw = min(128, W)
    ch = min(128, H)
    for _ in range(3):
        x0 = int(rng.integers(0, W - cw + 1)); y0 = int(rng.integers(0, H - ch + 1))
        skip[y0:y0 + ch, x0:x0 + cw] = 0
    crop_px = int((skip == 0).sum())
    gr, gd, ga = (w.astype(np.float64) for w in sc.weights[v])
    t0 = time.perf_counter()
    oracle.grad(g, cam, gr, gd, ga, skip=skip)
    t_grad = time.perf_counter() - t0
    t_view = t_fwd + t_grad * (W * H) / crop_px
    blends = float(ref["n_blend"].sum())
    return {"value": 1.0 / t_view, "unit": "views/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"view 0 ({W}x{H}) of the workload: FP64 forward on the full view ({t_fwd:.2f} s) and "
                      f"gradient on 3 seeded 128x128 crops ({crop_px} px, {t_grad:.2f} s) scaled by pixel count",
            "blends_per_sec": blends / t_view, "seconds_measured": t_fwd + t_grad}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c4-1200")
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        return 2

    import torch
    from paper_2505_18992_amd import _lib, get_context, render, render_backward

    _lib.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tw, th = (int(x) for x in args.tile.split("x"))
    log(f"[bench] building workload {args.workload}")
    sc, desc = workload(args.workload)
    sets = [tuple(torch.from_numpy(a).to(dev) for a in g.arrays()) for g in sc.sets]
    gw = [tuple(torch.from_numpy(w).to(dev) for w in ws) for ws in sc.weights]
    cams, vset = sc.cameras, sc.view_set
    nv = len(cams)
    n_gauss = sum(g.n for g in sc.sets)
    ctx = get_context(0)

    cap = 0

    def step(capacity):
        outs, saved = render(sets, cams, vset, tile=(tw, th), pair_capacity=capacity)
        render_backward(saved, gw)
        return saved

    # first call sizes the pair list; later calls run with a fixed capacity (no host sync)
    saved = step(0)
    st = saved.stats()
    saved.close()
    cap = int(math.ceil(st["n_pairs"] * 1.02)) + 1024
    log(f"[bench] pairs={st['n_pairs']} blended={st['n_blended']} evaluated={st['n_evaluated']} capacity={cap}")
    for _ in range(args.warmup):
        step(cap).close()
    torch.cuda.synchronize()

    # timed region
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(cap).close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step")

    # per-stage HIP-event timing over a second pass of the same steps
    ctx.profile(True)
    saved = None
    for _ in range(args.steps):
        if saved is not None:
            saved.close()
        saved = step(cap)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    st = saved.stats()
    saved.close()
    if st["overflow"]:
        raise SystemExit("pair capacity overflow in the timed pass")
    stage_ms = {k: v[1] / max(v[0], 1) for k, v in prof.items() if v[0] > 0}
    log("[bench] stage ms/step: " + ", ".join(f"{k}={v:.3f}" for k, v in sorted(stage_ms.items(), key=lambda x: -x[1])))

    E, B, P = st["n_evaluated"], st["n_blended"], st["n_pairs"]
    dom = max(stage_ms, key=stage_ms.get)
    t_dom = stage_ms[dom] * 1e-3
    if dom == "composite_forward":
        work = FWD_FLOP_PER_EVAL * E + FWD_FLOP_PER_BLEND * B
        roof = {"bound": "alu", "achieved": work / t_dom / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s"}
    elif dom == "composite_backward":
        work = BWD_FLOP_PER_EVAL * E + BWD_FLOP_PER_BLEND * B
        roof = {"bound": "alu", "achieved": work / t_dom / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s"}
    else:
        passes = math.ceil((32 + math.ceil(math.log2(max(st["n_tiles"], 2)))) / 8)
        work = SORT_BYTES_PER_PAIR_PASS * passes * P
        roof = {"bound": "hbm", "achieved": work / t_dom / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = dom
    roof["kernel_ms"] = stage_ms[dom]
    roof["traffic"] = None

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
                   "resolutions": sorted({f"{c.width}x{c.height}" for c in cams}), "tile": args.tile},
        "blends_per_sec": B / (ms_step * 1e-3),
        "counts": {"pairs": P, "evaluated": E, "blended": B},
        "stage_ms": stage_ms,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
