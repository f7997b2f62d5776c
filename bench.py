#!/usr/bin/env python3
"""Benchmark: forward + backward of the one-pixel point rasterizer on one GPU.

Workload (default): 100M points from the 64-cluster Gaussian mixture (sigma
0.5 m) in a 100 m box, 4 FP32 features, one 1920x1080 pinhole + distortion
camera, 5-layer pyramid, alpha = 0.01, upstream gradient of an L1 loss to a
seeded random target.  A step is one forward and one backward pass
(three passes over the points plus the per-pixel kernels); inputs are resident
in HBM before timing starts.

Prints one JSON line with points/s, the roofline of the dominant kernel
(algorithmic bytes / its average duration, measured with HIP events on the
launch stream during the timed steps) and the CPU oracle timed on a bounded
sample on the host.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(n, C, s, phi, P):
    """Bytes the method itself must move per kernel (one view).

    Points: positions 12 B read in each of the three point passes, features
    C*s B read for points that blend (fraction phi) in the accumulation and
    backward passes, FP32 dfeat (4C) and dpos (12) written once.
    Pixels: key init 8, sums+count init 4C+4, key read 8, normalize read
    4C+4 and image write 4C, backward reads of G 4C, I 4C, count 4, key 8."""
    return {
        "k_clear": P * (8 + 4 * C + 4),
        "k_depth": n * 12,
        "k_accum": n * (12 + C * s * phi) + P * 8,
        "k_normalize": P * (8 * C + 4),
        "k_pack": P * (8 * C + 12),
        "k_backward": n * (12 + C * s * phi + 4 * C + 12),
        "k_reduce": 0,
    }


def l1_grad(frame, target):
    """dL/dI of L = sum_l mean |I_l - T_l| (one view)."""
    import torch
    G = torch.empty_like(frame.images)
    C = frame.channels
    for l in range(frame.layers):
        o = int(frame.offsets[0, l])
        w, h = frame.cams[0].width >> l, frame.cams[0].height >> l
        sl = slice(C * o, C * (o + w * h))
        G[sl] = torch.sign(frame.images[sl] - target[sl]) / float(C * w * h)
    return G


def cpu_baseline(scene_np, n_sample):
    """The CPU oracle (single-threaded C) on an i.i.d. prefix of the scene."""
    import numpy as np
    from oracle import oracle as O
    from paper_2110_06635_amd import synth
    pos = np.ascontiguousarray(scene_np.pos[:n_sample])
    feat = np.ascontiguousarray(scene_np.feat[:n_sample])
    total = O.total_pixels(scene_np.cams, scene_np.layers)
    G = synth.upstream_grad(total * feat.shape[1], 99)
    t0 = time.perf_counter()
    O.forward(pos, feat, scene_np.cams, scene_np.layers, alpha=scene_np.alpha)
    O.backward(pos, feat, scene_np.cams, scene_np.layers, G, alpha=scene_np.alpha, want_abs=False)
    dt = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
            "seconds": dt,
            "sample": f"{n_sample} points (i.i.d. prefix of the same scene), 1920x1080, "
                      f"L={scene_np.layers}, forward + backward (the backward recomputes the "
                      f"forward), float64 oracle, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--variants", default="bf16,f16", help="extra feature storage types to time")
    ap.add_argument("--cpu-sample", type=int, default=4_000_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is described in DESIGN.md, not built)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2110_06635_amd import adop, synth

    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nb} bytes read, {nb} bytes written")
        del src, dst
    t0 = time.time()
    s = synth.config3(n=args.n)
    log(f"generated {s.name} in {time.time() - t0:.1f}s")
    ctx = adop.Context(0)
    dev = torch.device("cuda:0")
    C = s.c
    target = torch.from_numpy(synth.target_values(adop.views_layout(s.cams, s.layers)[0] * C)).to(dev)

    def run(dtype, steps, warmup, timing):
        code = adop.DTYPES[dtype]
        raw, _ = synth.storage(s.feat, dtype)
        pos = torch.from_numpy(s.pos).to(dev)
        if dtype == "f32":
            feat = torch.from_numpy(raw).to(dev)
        else:
            feat = torch.from_numpy(raw.view(np.int16)).to(dev).view(adop.TORCH_STORAGE[code])
        scene = adop.Scene.prepare(ctx, pos, feat, code)
        del pos, feat
        torch.cuda.synchronize()
        frame = adop.Frame(s.cams, s.layers, C, dev)
        ws = ctx.workspace(C, 1, frame.pixels)
        adop.render_forward(ctx, scene, frame.cams, s.layers, alpha=s.alpha, frame=frame, workspace=ws)
        G = l1_grad(frame, target)
        out = (torch.empty((scene.n, C), dtype=torch.float32, device=dev),
               torch.empty((3, scene.n), dtype=torch.float32, device=dev),
               torch.empty((1, 6), dtype=torch.float64, device=dev),
               torch.empty((1, 9), dtype=torch.float64, device=dev))

        def step():
            adop.render_forward(ctx, scene, frame.cams, s.layers, alpha=s.alpha, frame=frame, workspace=ws)
            adop.render_backward(ctx, scene, frame, G, alpha=s.alpha, out=out, workspace=ws)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        if timing:
            ctx.timing(True)
            ctx.timing_read()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        kern = None
        if timing:
            kern = ctx.timing_read()
            ctx.timing(False)
        nz = (out[0] != 0).any(dim=1)
        phi = float(nz.float().mean().item())
        res = dict(ms=ms, kern=kern, phi=phi, pixels=frame.pixels,
                   s=4 if dtype == "f32" else 2,
                   coverage=float((frame.counts > 0).float().mean().item()))
        del scene, frame, G, out
        torch.cuda.empty_cache()
        return res

    log(f"timing {args.dtype}: warmup {args.warmup}, steps {args.steps}")
    r = run(args.dtype, args.steps, args.warmup, timing=True)
    n = s.n
    value = n / (r["ms"] * 1e-3)
    ab = algorithmic_bytes(n, C, r["s"], r["phi"], r["pixels"])
    kern = {k: {"avg_ms": (v[0] / v[1]) if v[1] else 0.0, "launches": v[1]} for k, v in r["kern"].items()}
    dom = max(kern, key=lambda k: kern[k]["avg_ms"])
    achieved = ab[dom] / (kern[dom]["avg_ms"] * 1e-3) / 1e9
    step_bytes = sum(ab.values())
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "algorithmic_bytes": int(ab[dom])}
    variants = {}
    for vd in [v for v in args.variants.split(",") if v and v != args.dtype]:
        log(f"timing variant {vd}")
        rv = run(vd, max(3, args.steps // 2), 2, timing=False)
        abv = algorithmic_bytes(n, C, rv["s"], rv["phi"], rv["pixels"])
        variants[vd] = {"value": n / (rv["ms"] * 1e-3), "ms_per_step": round(rv["ms"], 4),
                        "step_frac_of_hbm_roofline": round(sum(abv.values()) / (rv["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    cpu = None
    if not args.no_cpu:
        log(f"cpu baseline on {args.cpu_sample} points")
        cpu = cpu_baseline(s, args.cpu_sample)
    line = {
        "metric": "points/sec fwd+bwd at 100M pts 1080p (% HBM roofline); p99 render latency",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": s.name, "points": n, "resolution": "1920x1080", "layers": s.layers,
                   "channels": C, "feature_storage": args.dtype, "alpha": s.alpha,
                   "loss": "L1 to seeded U[0,1] target", "views": 1},
        "step_frac_of_hbm_roofline": round(step_bytes / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "step_algorithmic_bytes": int(step_bytes),
        "phi": round(r["phi"], 5),
        "coverage": round(r["coverage"], 5),
        "kernels_ms": {k: round(v["avg_ms"], 4) for k, v in kern.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "precision_variants": variants,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
