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


KERNEL_SOURCES = ["paper_2110_06635_amd/csrc/render_impl.h", "paper_2110_06635_amd/csrc/render.hip",
                  "paper_2110_06635_amd/csrc/render_c1.hip", "paper_2110_06635_amd/csrc/device.h",
                  "paper_2110_06635_amd/csrc/launch.h"]
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_counters(kernel, workload, storage):
    """Counter record of `kernel` kept under profiles/: HBM bytes per launch
    from the FETCH_SIZE / WRITE_SIZE runs (each scaled by its copy-kernel
    factor) and VALU instructions per launch, or None when no record matches
    this workload or the kernel sources have changed since the counters were
    taken."""
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("workload") != workload or rec.get("feature_storage") != storage:
        return None
    if rec.get("sources_sha256") != sources_sha256():
        return None
    return rec.get("kernels", {}).get(kernel)


# one wave64 VALU instruction per CU per cycle: 256 CUs x 2.4 GHz
VALU_ISSUE_PEAK = 256 * 2.4e9


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
    """dL/dI of L = sum over views and layers of mean |I - T|."""
    import torch
    G = torch.empty_like(frame.images)
    C = frame.channels
    for v in range(len(frame.cams)):
        for l in range(frame.layers):
            o = int(frame.offsets[v, l])
            w, h = frame.cams[v].width >> l, frame.cams[v].height >> l
            sl = slice(C * o, C * (o + w * h))
            G[sl] = torch.sign(frame.images[sl] - target[sl]) / float(C * w * h)
    return G


def atomic_ceiling(ctx):
    """The device's atomic throughput for the two kinds the render passes use
    (u64 minimum: depth pass, FP32 add: accumulation), 2^28 ops each:
    scattered over a 1 GiB buffer one cache line per lane (what HBM-resident
    pixel buffers see), over 2 MiB (L2-resident), and on 64 words (heavy
    contention, as on the hot pixels of coarse layers).  Ops per second."""
    import torch
    from paper_2110_06635_amd import adop
    buf = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda:0")
    ops = 1 << 28
    out = {"ops_per_case": ops}
    for kind, name, word in ((0, "u64_min", 8), (1, "f32_add", 4)):
        stride = 128 // word
        cases = {"scattered_hbm": ((1 << 30) // word, stride), "scattered_l2": ((2 << 20) // word, stride),
                 "contended_64_words": (64, 1)}
        for case, (fp, sd) in cases.items():
            adop.atomic_probe(ctx, kind, ops >> 4, fp, sd, buf)          # warm-up
            ms = adop.atomic_probe(ctx, kind, ops, fp, sd, buf)
            out[f"{name}_{case}"] = round(ops / (ms * 1e-3), 1)
    del buf
    torch.cuda.empty_cache()
    return out


def atomic_sweep(ctx):
    """Atomic throughput against the spacing of consecutive lanes' words
    (1 GiB buffer, 2^28 ops per case): with a spacing below one 64-byte line
    several lanes share one L2 request, so ops/s divided by the lanes per
    request gives the L2's request rate for the kind."""
    import torch
    from paper_2110_06635_amd import adop
    buf = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda:0")
    ops = 1 << 28
    rows = []
    for kind, name, word in ((1, "f32_add", 4), (0, "u64_min", 8)):
        for stride in (1, 2, 4, 8, 16, 32):
            fp = (1 << 30) // word
            adop.atomic_probe(ctx, kind, ops >> 4, fp, stride, buf)      # warm-up
            ms = adop.atomic_probe(ctx, kind, ops, fp, stride, buf)
            per_req = max(1, 64 // (word * stride))
            rows.append({"kind": name, "stride_words": stride, "lanes_per_64B": per_req,
                         "ops_per_s": round(ops / (ms * 1e-3), 1),
                         "requests_per_s": round(ops / per_req / (ms * 1e-3), 1), "ms": round(ms, 4)})
    del buf
    torch.cuda.empty_cache()
    return rows


def multiview_leg(ctx, steps, warmup, n=30_000_000):
    """The batched training step of the 16-view workload (30M points, C = 8
    BF16 features, 1920x1080, L = 5, one fused launch per pass): forward with
    the blend-set bits, then backward, timed over `steps` steps."""
    import numpy as np
    import torch
    from paper_2110_06635_amd import adop, synth
    s = synth.config4(n=n)
    V, C = len(s.cams), s.c
    dev = torch.device("cuda:0")
    target = torch.from_numpy(synth.target_values(adop.views_layout(s.cams, s.layers)[0] * C)).to(dev)
    raw, _ = synth.storage(s.feat, "bf16")
    code = adop.DTYPES["bf16"]
    pos = torch.from_numpy(s.pos).to(dev)
    feat = torch.from_numpy(raw.view(np.int16)).to(dev).view(adop.TORCH_STORAGE[code])
    scene = adop.Scene.prepare(ctx, pos, feat, code)
    del pos, feat, raw
    s.pos, s.feat = s.pos[:0], s.feat[:0]
    frame = adop.Frame(s.cams, s.layers, C, dev)
    ws = ctx.workspace(C, V, frame.pixels)
    adop.render_forward(ctx, scene, frame.cams, s.layers, alpha=s.alpha, frame=frame, workspace=ws,
                        record_visibility=True)
    G = l1_grad(frame, target)
    out = (torch.empty((scene.n, C), dtype=torch.float32, device=dev),
           torch.empty((3, scene.n), dtype=torch.float32, device=dev),
           torch.empty((V, 6), dtype=torch.float64, device=dev),
           torch.empty((V, 9), dtype=torch.float64, device=dev))

    def step():
        adop.render_forward(ctx, scene, frame.cams, s.layers, alpha=s.alpha, frame=frame, workspace=ws,
                            record_visibility=True)
        adop.render_backward(ctx, scene, frame, G, alpha=s.alpha, out=out, workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_read()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kern = ctx.timing_read()
    ctx.timing(False)
    phi = float((out[0] != 0).any(dim=1).float().mean().item())
    ab = algorithmic_bytes(scene.n, C, 2, phi, frame.pixels)   # points read once per fused pass
    res = {"workload": s.name, "points": scene.n, "views": V, "channels": C, "feature_storage": "bf16",
           "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 4),
           "value": scene.n * V / (ms * 1e-3), "unit": "point-views/s",
           "step_frac_of_hbm_roofline": round(sum(ab.values()) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "kernels_ms": {k: round(v[0] / v[1], 4) for k, v in kern.items() if v[1]}}
    del scene, frame, G, out, ws
    torch.cuda.empty_cache()
    return res


def host_cpu():
    """Host CPU model name and logical CPU count."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(scene_np, n_sample, n_per_thread):
    """The CPU oracle (single-threaded C, unchanged) on the host: one thread
    on an i.i.d. prefix of the scene, then every usable core at once, each
    thread rendering (forward + backward) its own i.i.d. slice of the scene
    through the same oracle call (ctypes releases the interpreter lock), and
    the aggregate points/s."""
    import threading
    import numpy as np
    from oracle import oracle as O
    from paper_2110_06635_amd import synth
    total = O.total_pixels(scene_np.cams, scene_np.layers)
    G = synth.upstream_grad(total * scene_np.feat.shape[1], 99)

    def render(lo, hi):
        pos = np.ascontiguousarray(scene_np.pos[lo:hi])
        feat = np.ascontiguousarray(scene_np.feat[lo:hi])
        O.forward(pos, feat, scene_np.cams, scene_np.layers, alpha=scene_np.alpha)
        O.backward(pos, feat, scene_np.cams, scene_np.layers, G, alpha=scene_np.alpha, want_abs=False)

    t0 = time.perf_counter()
    render(0, n_sample)
    dt1 = time.perf_counter() - t0
    model, ncpu = host_cpu()
    threads = max(1, min(16, ncpu, scene_np.n // max(1, n_per_thread)))
    ths = [threading.Thread(target=render, args=(k * n_per_thread, (k + 1) * n_per_thread))
           for k in range(threads)]
    t0 = time.perf_counter()
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    dtm = time.perf_counter() - t0
    desc = (f"1920x1080, L={scene_np.layers}, forward + backward (the backward recomputes the "
            f"forward), float64 oracle")
    return {"value": threads * n_per_thread / dtm, "unit": "points/s", "cores": threads, "kind": "oracle",
            "seconds": dtm,
            "sample": f"{threads} threads at once, each {n_per_thread} points (its own i.i.d. slice of the "
                      f"same scene), {desc}; aggregate points/s",
            "single_thread": {"value": n_sample / dt1, "unit": "points/s", "cores": 1, "seconds": dt1,
                              "sample": f"{n_sample} points (i.i.d. prefix of the same scene), {desc}"},
            "cpu_model": model, "logical_cpus": ncpu}


def serving_leg(n_points, requests, warmup, rates, max_batch=4, budget_gib=96, seed_scene=1005,
                max_inflight=3, candidates=True):
    """Serving: a resident BF16 scene, Poisson arrivals of mixed-resolution
    novel views at each rate in `rates`; the continuous-batching graph server
    (mixed-class fused batches, slots counted against the memory budget) vs
    the plain unbatched FP32 renderer on the same trace.  Returns a dict per
    rate plus the workload description."""
    import itertools
    import numpy as np
    import torch
    from paper_2110_06635_amd import adop, serve, synth
    dev = torch.device("cuda:0")
    t0 = time.time()
    s = synth.config5_scene(n=n_points, seed=seed_scene)
    log(f"generated {s.name} in {time.time() - t0:.1f}s")
    ctx = adop.Context(0)
    pos = torch.from_numpy(s.pos).to(dev)
    raw, _ = synth.storage(s.feat, "bf16")
    scene16 = adop.Scene.prepare(ctx, pos, torch.from_numpy(raw.view(np.int16)).to(dev).view(torch.bfloat16),
                                 adop.BF16)
    scene32 = adop.Scene.prepare(ctx, pos, torch.from_numpy(s.feat).to(dev), adop.F32)
    del pos
    out = {"workload": s.name, "points": s.n, "layers": 4, "classes": synth.SERVE_CLASSES,
           "class_weights": synth.SERVE_WEIGHTS, "requests": requests, "warmup": warmup,
           "max_batch": max_batch, "max_inflight": max_inflight, "candidates": candidates,
           "budget_bytes": budget_gib << 30, "rates": {}}
    combos = [c for b in range(1, max_batch + 1)
              for c in itertools.combinations_with_replacement(synth.SERVE_CLASSES, b)]
    for rate in rates:
        trace = synth.config5_requests(warmup + requests, rate=rate)
        res = {}
        for name, scene, be_cls, kw in (
                ("batched", scene16, serve.GpuBackend, dict(max_batch=max_batch, max_inflight=max_inflight)),
                ("plain_fp32", scene32, serve.PlainBackend, dict(max_batch=1, max_inflight=1))):
            be = (serve.GpuBackend(ctx, scene, layers=4, candidates=candidates) if be_cls is serve.GpuBackend
                  else be_cls(ctx, scene, layers=4))
            torch.cuda.reset_peak_memory_stats(dev)
            base = torch.cuda.memory_allocated(dev)
            # frames are released once their completion is recorded, as a
            # client consuming the stream would
            srv = serve.Server(be, budget_gib << 30, keep_results=False, **kw)
            # capture a slot for every class multiset before the trace (the
            # server evicts idle slots if they outgrow the budget)
            for combo in (combos if kw["max_batch"] > 1 else [(k,) for k in synth.SERVE_CLASSES]):
                srv.prewarm(combo)
            torch.cuda.synchronize()
            srv.start()
            log(f"serving {name}: {len(trace)} requests at {rate}/s")
            reqs = serve.replay(srv, trace, warmup=warmup)
            srv.stop()
            measured = {r.rid for r in reqs}
            srv.completed = [r for r in srv.completed if r.rid in measured]
            st = srv.stats()
            st["device_peak_allocated_bytes"] = int(torch.cuda.max_memory_allocated(dev) - base)
            res[name] = st
            srv.close()
            del srv, be, reqs
            torch.cuda.empty_cache()
        b, p = res["batched"], res["plain_fp32"]
        res["p99_speedup_vs_plain"] = p["p99_ms"] / b["p99_ms"] if b["p99_ms"] > 0 else None
        res["p50_speedup_vs_plain"] = p["p50_ms"] / b["p50_ms"] if b["p50_ms"] > 0 else None
        out["rates"][f"{rate:g}_per_s"] = res
    del scene16, scene32
    torch.cuda.empty_cache()
    return out


def serve_bench(args):
    """The serving benchmark alone (--serve): full trace."""
    res = serving_leg(args.serve_points, args.serve_requests, args.serve_warmup,
                      [args.serve_rate] + ([args.serve_rate_high] if args.serve_rate_high > 0 else []),
                      max_batch=args.serve_batch, budget_gib=args.serve_budget_gib)
    first = res["rates"][f"{args.serve_rate:g}_per_s"]
    line = {
        "metric": f"p99 render latency, mixed-resolution novel views ({args.serve_points} points resident, "
                  f"{args.serve_rate:g} req/s)",
        "value": first["batched"]["p99_ms"], "unit": "ms", "higher_is_better": False, "n_gpus": 1,
        "data": "synthetic", "dtype": "bf16 features, f32 accumulation",
        "config": {k: v for k, v in res.items() if k != "rates"},
        "rates": res["rates"],
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gmm100m", choices=["gmm100m", "planes10m", "multiview30m"],
                    help="gmm100m: the headline workload; planes10m: 10M points on 200 planes; "
                         "multiview30m: 30M points x 16 views, 8 BF16 channels, one fused launch per pass")
    ap.add_argument("--n", type=int, default=0, help="override the point count")
    ap.add_argument("--dtype", default="", choices=["", "f32", "bf16", "f16"])
    ap.add_argument("--variants", default="bf16,f16", help="extra feature storage types to time")
    ap.add_argument("--cpu-sample", type=int, default=4_000_000)
    ap.add_argument("--cpu-sample-mt", type=int, default=1_000_000,
                    help="points per thread of the all-cores oracle run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve", action="store_true", help="run the serving benchmark instead")
    ap.add_argument("--serve-points", type=int, default=50_000_000)
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-warmup", type=int, default=500)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-rate-high", type=float, default=2000.0,
                    help="a second, saturating arrival rate (0: none)")
    ap.add_argument("--no-serve-leg", action="store_true",
                    help="skip the short serving leg of the default run")
    ap.add_argument("--no-multiview-leg", action="store_true",
                    help="skip the short 16-view leg of the default run")
    ap.add_argument("--multiview-steps", type=int, default=5)
    ap.add_argument("--leg-requests", type=int, default=1500, help="measured requests per rate in the serving leg")
    ap.add_argument("--leg-warmup", type=int, default=100)
    ap.add_argument("--serve-batch", type=int, default=4)
    ap.add_argument("--serve-budget-gib", type=int, default=96)
    ap.add_argument("--discard", action="store_true",
                    help="stochastic point discarding (gamma 1.5, 4-NN radius, seeded beta)")
    ap.add_argument("--cull", default="", choices=["", "backface", "printed"],
                    help="normal culling with seeded random unit normals")
    ap.add_argument("--log-features", action="store_true", help="features are logarithmic descriptors")
    ap.add_argument("--no-visibility", action="store_true",
                    help="the forward records no blend-set bits; the backward re-tests every point")
    ap.add_argument("--atomic-sweep", action="store_true",
                    help="only measure atomic throughput against lane spacing, one JSON line per case")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is not built)"}))
        sys.exit(2)

    if args.serve:
        serve_bench(args)
        return
    if args.atomic_sweep:
        from paper_2110_06635_amd import adop
        ctx = adop.Context(0)
        for row in atomic_sweep(ctx):
            print(json.dumps(row), flush=True)
        print(json.dumps({"atomic_ceiling": atomic_ceiling(ctx)}), flush=True)
        return

    import numpy as np
    import torch
    from paper_2110_06635_amd import adop, synth

    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)   # one elementwise kernel: reads nb bytes, writes nb bytes
        torch.cuda.synchronize()
        log(f"copy probe (torch.neg elementwise kernel): {nb} bytes read, {nb} bytes written")
        del src, dst
    t0 = time.time()
    if args.workload == "gmm100m":
        s = synth.config3(n=args.n or 100_000_000)
        args.dtype = args.dtype or "f32"
    elif args.workload == "planes10m":
        per = (args.n or 10_000_000) // 200
        s = synth.config2(per_plane=per)
        args.dtype = args.dtype or "f32"
    else:
        s = synth.config4(n=args.n or 30_000_000)
        args.dtype = args.dtype or "bf16"
    V = len(s.cams)
    log(f"generated {s.name} in {time.time() - t0:.1f}s")
    ctx = adop.Context(0)
    dev = torch.device("cuda:0")
    C = s.c
    target = torch.from_numpy(synth.target_values(adop.views_layout(s.cams, s.layers)[0] * C)).to(dev)

    flags = ((adop.FLAG_DISCARD if args.discard else 0) | (adop.FLAG_LOG_FEATURES if args.log_features else 0) |
             {"": 0, "backface": adop.FLAG_CULL_BACKFACE, "printed": adop.FLAG_CULL_PRINTED}[args.cull])
    options = [o for o, on in (("discard", args.discard), ("log_features", args.log_features),
                               (f"cull_{args.cull}", bool(args.cull)), ("no_visibility", args.no_visibility)) if on]

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
        pre = {}
        if args.cull:
            scene.set_normals(ctx, torch.from_numpy(synth.unit_vectors(s.n, 4001)).to(dev))
        if args.discard:
            scene.beta = scene.gather(ctx, torch.from_numpy(synth.uniform01(s.n, 4002)).to(dev))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            scene.radius = adop.knn_radius(ctx, scene)
            torch.cuda.synchronize()
            pre["knn_radius_s"] = round(time.perf_counter() - t0, 3)
        frame = adop.Frame(s.cams, s.layers, C, dev)
        ws = ctx.workspace(C, V, frame.pixels)
        rec = not args.no_visibility
        adop.render_forward(ctx, scene, frame.cams, s.layers, alpha=s.alpha, frame=frame, workspace=ws, flags=flags,
                            record_visibility=rec)
        G = l1_grad(frame, target)
        out = (torch.empty((scene.n, C), dtype=torch.float32, device=dev),
               torch.empty((3, scene.n), dtype=torch.float32, device=dev),
               torch.empty((V, 6), dtype=torch.float64, device=dev),
               torch.empty((V, 9), dtype=torch.float64, device=dev))

        def step():
            adop.render_forward(ctx, scene, frame.cams, s.layers, alpha=s.alpha, frame=frame, workspace=ws,
                                flags=flags, record_visibility=rec)
            adop.render_backward(ctx, scene, frame, G, alpha=s.alpha, out=out, workspace=ws, flags=flags)

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
                   coverage=float((frame.counts > 0).float().mean().item()),
                   blends=int(frame.counts.sum().item()), pre=pre)
        del scene, frame, G, out
        torch.cuda.empty_cache()
        return res

    log(f"timing {args.dtype}: warmup {args.warmup}, steps {args.steps}")
    r = run(args.dtype, args.steps, args.warmup, timing=True)
    n = s.n
    value = n * V / (r["ms"] * 1e-3)
    ab = algorithmic_bytes(n, C, r["s"], r["phi"], r["pixels"])
    kern = {k: {"avg_ms": (v[0] / v[1]) if v[1] else 0.0, "launches": v[1]} for k, v in r["kern"].items()}
    dom = max(kern, key=lambda k: kern[k]["avg_ms"])
    achieved = ab[dom] / (kern[dom]["avg_ms"] * 1e-3) / 1e9
    step_bytes = sum(ab.values())
    rec = recorded_counters(dom, s.name, args.dtype) if not options else None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": int(rec["bytes_per_launch"]) if rec and "bytes_per_launch" in rec else None,
                "traffic_unit": "HBM bytes per launch",
                "algorithmic_bytes": int(ab[dom])}
    alu_issue = None
    if rec and "valu_insts" in rec:
        t = kern[dom]["avg_ms"] * 1e-3
        alu_issue = {"kernel": dom, "valu_insts_per_launch": rec["valu_insts"],
                     "achieved": round(rec["valu_insts"] / t / 1e9, 1), "peak": VALU_ISSUE_PEAK / 1e9,
                     "unit": "G wave-instructions/s", "frac": round(rec["valu_insts"] / t / VALU_ISSUE_PEAK, 4)}
    variants = {}
    for vd in [v for v in args.variants.split(",") if v and v != args.dtype]:
        log(f"timing variant {vd}")
        rv = run(vd, max(3, args.steps // 2), 2, timing=True)
        abv = algorithmic_bytes(n, C, rv["s"], rv["phi"], rv["pixels"])
        variants[vd] = {"value": n * V / (rv["ms"] * 1e-3), "ms_per_step": round(rv["ms"], 4),
                        "step_frac_of_hbm_roofline": round(sum(abv.values()) / (rv["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "kernels_ms": {k: round(v[0] / v[1], 4) for k, v in rv["kern"].items() if v[1]}}
    atomics = atomic_ceiling(ctx) if (args.workload == "gmm100m" and not options) else None
    cpu = None
    if not args.no_cpu and V == 1 and not options:
        log(f"cpu baseline on {args.cpu_sample} points, then all cores")
        cpu = cpu_baseline(s, args.cpu_sample, args.cpu_sample_mt)
    serving = None
    if args.workload == "gmm100m" and not options and not args.no_serve_leg:
        s.pos, s.feat = s.pos[:0], s.feat[:0]   # free the 100M-point arrays; the line uses only names
        serving = serving_leg(args.serve_points, args.leg_requests, args.leg_warmup,
                              [args.serve_rate] + ([args.serve_rate_high] if args.serve_rate_high > 0 else []),
                              max_batch=args.serve_batch, budget_gib=args.serve_budget_gib)
    multiview = None
    if args.workload == "gmm100m" and not options and not args.no_multiview_leg:
        log("16-view leg: 30M points x 16 views, C = 8 BF16")
        multiview = multiview_leg(ctx, args.multiview_steps, 2)
    line = {
        "metric": ("points/sec fwd+bwd at 100M pts 1080p (% HBM roofline); p99 render latency"
                   if args.workload == "gmm100m" else f"point-views/sec fwd+bwd ({args.workload})"),
        "value": value,
        "unit": "points/s" if V == 1 else "point-views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "feature_storage": args.dtype,
        "data": "synthetic",
        "config": {"workload": s.name, "points": n, "resolution": "1920x1080", "layers": s.layers,
                   "channels": C, "feature_storage": args.dtype, "alpha": s.alpha,
                   "loss": "L1 to seeded U[0,1] target", "views": V},
        "step_frac_of_hbm_roofline": round(step_bytes / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "step_algorithmic_bytes": int(step_bytes),
        "phi": round(r["phi"], 5),
        "coverage": round(r["coverage"], 5),
        "kernels_ms": {k: round(v["avg_ms"], 4) for k, v in kern.items()},
        "roofline": roofline,
        "alu_issue": alu_issue,
        "cpu_baseline": cpu,
        "options": options,
        "blends": r["blends"],
        "preprocess": r["pre"],
        "precision_variants": variants,
        "serving": serving,
        "multiview": multiview,
        "atomic_ceiling": atomics,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
