"""Benchmark: shortest-path-map builds on one MI355X.

One step = one complete spm_build (device ingest, generator visibility,
relaxation, cost sort, inside mask and pixel propagation) of the 1024 x 1024
scene with 60 convex obstacles, 3 point sources and 2 segment sources, with
the scene already resident in device memory.

value = W * H * G / t_step / 1e6  (Mpixel*generator/s; G = point sources +
segment sources + corner generators, the dense pair count the paper's method
shades).

Prints one JSON line.  roofline.achieved = the pixel kernel's algorithmic
lane-ops per launch / its average launch time, against 256 CUs x 4 SIMDs x
16 lanes x 2.4 GHz.  Algorithmic work per unit (what the method computes,
not what culling avoids): 8 lane-ops per pixel-generator pair (the cone
bound of every pair), 20 more per pixel-segment pair (the closest point),
8 per accepted candidate and 9 per examined lane-edge visibility test; the
last two counted by one instrumented build outside the timed region.
executed_ops_frac gives the same ratio for the operations the kernel
actually executes after culling.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SPM build Mpixel·gen/s + % VALU roofline; batched & backward vs plain"
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9      # CUs x SIMDs x lanes x clock: one 32-bit VALU op per lane per cycle
# arithmetic lane-ops per counted unit of the instrumented pixel kernel
# algorithmic lane-ops per unit of the method
ALG = {
    "pair": 8,          # per (pixel, generator): the cone bound cost + |p - g| against the current value
    "segment_pair": 20, # per (pixel, segment source): the clamped closest point
    "accept": 8,        # per accepted candidate: square root, add, compare, select
    "lane_edge": 9,     # per examined (pixel, generator, edge): orientations and compares
}
# lane-ops per unit of what the culled kernel executes (instrumented counters)
OPS = {
    "tile_bound": 12,    # per generator per tile: box gap (4 sub/max), squares, sqrt, scale, add, compare
    "lane_bound": 9,     # per (pixel, generator): 2 sub, mul+mad, sub, cvt, 2 mul, compare
    "relevance": 30,     # per (tile, edge): facing test, box ranges of 3 affine forms, compares
    "lane_edge": 12,     # per (pixel, generator, edge): 4 mad (two orientations), 2 med3, mul, 2 mad, 3 compares
    "accept": 4,         # per accepted candidate: cvt, sqrt, mad, compare
}


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tile", default="8x8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and backward figures")
    ap.add_argument("--cpu-pixels", type=int, default=1 << 20, help="oracle pixel sample for the CPU baseline")
    ap.add_argument("--sweep", type=int, default=0, metavar="SOURCES",
                    help="only run the Profiling-style sweep (k x k squares on 1000^2, k in 2..20) with this many "
                         "random single sources per map, print its JSON line and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only run one plain device copy of this many bytes (HBM counter calibration) and exit")
    return ap.parse_args()


def _file_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(kernel_src_hash):
    """HBM bytes per k_pixel launch from the committed rocprofv3 counter summary, if the
    kernel source has not changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "k_pixel_convex1024_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_src_hash:
        return None
    return t.get("bytes_per_launch")


def _cpu_baseline(scene, G, npix):
    import numpy as np
    from oracle import oracle as O
    O.build()
    threads = O.max_threads()
    t0 = time.perf_counter()
    cost, _ = O.costs(scene, nthreads=threads)
    t1 = time.perf_counter()
    rng = np.random.default_rng(123)
    WH0 = scene.width * scene.height
    pix = np.arange(WH0, dtype=np.int64) if npix >= WH0 else np.unique(rng.integers(0, WH0, npix))
    t2 = time.perf_counter()
    O.pixels(scene, cost, pix, nthreads=threads)
    t3 = time.perf_counter()
    WH = scene.width * scene.height
    t_full = (t1 - t0) + (t3 - t2) * WH / len(pix)
    return {
        "value": WH * G / t_full / 1e6, "unit": "Mpixel·gen/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"generator costs ({t1 - t0:.2f} s) + {len(pix)} of {WH} pixels ({t3 - t2:.2f} s) of the same "
                   f"scene" + ("" if len(pix) == WH else ", extrapolated to all pixels")),
    }


def _batched(spm, torch, reps=10):
    """256 mixed scenes (sides 128-1024, 4-80 hulls, 1-5 points, 0-3 segments), one hipGraph replay
    per batched build.  Throughput = sum over scenes of W * H * G / t."""
    from scenegen import config4_list
    scenes = config4_list()
    bb = spm.BatchBuilder(scenes, check=False)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        bb.build(s)
    s.synchronize()
    pairs = bb.pairs
    g = bb.capture(s)
    g.launch(s)
    s.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        g.launch(s)
    e1.record(s)
    s.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"workload": "256 scenes, sides in {128,256,512,1024}, 4-80 convex hulls, 1-5 points, 0-3 segments, "
                        "seed 7; one hipGraph replay per build",
            "scenes": len(scenes), "pixels": int(sum(x.width * x.height for x in scenes)), "pairs": pairs,
            "ms_per_batch": ms, "value": pairs / (ms * 1e-3) / 1e6, "unit": "Mpixel·gen/s"}


def _backward(spm, torch, b, scene, reps=20):
    """4096 agents on the plain workload: map rebuild + agent distances (forward) and the adjoint."""
    from scenegen import config5_agents
    A = torch.from_numpy(config5_agents(scene, 4096, seed=11)).cuda()
    w = torch.full((A.shape[0],), 1.0 / A.shape[0], device="cuda")
    for _ in range(3):
        b.build()
        spm.agent_distance(b, A)
        spm.source_gradients(b, A, w)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        b.build()
        spm.agent_distance(b, A)
    e[1].record()
    for _ in range(reps):
        spm.source_gradients(b, A, w)
    e[2].record()
    torch.cuda.synchronize()
    fwd = e[0].elapsed_time(e[1]) / reps
    bwd = e[1].elapsed_time(e[2]) / reps
    return {"agents": int(A.shape[0]), "forward_ms": fwd, "backward_ms": bwd, "forward_plus_backward_ms": fwd + bwd,
            "backward_agents_per_s": A.shape[0] / (bwd * 1e-3)}


# The paper's own timings of its Profiling maps (Table 1: polygons, computation seconds; GTX 970),
# quoted as context next to the sweep, never as a target.
PAPER_PROFILING = {2: (4, 0.0014), 4: (16, 0.0054), 6: (36, 0.0456), 8: (64, 0.1251), 10: (100, 0.2701),
                   14: (196, 0.8564), 20: (400, 2.7371)}


def _sweep(n_sources):
    """Profiling-style maps: 1000 x 1000, k x k rows of squares (each half its cell's width), one random
    free source per build, n_sources builds per map.  Reports the mean whole-build time per map."""
    import torch

    import paper_1805_08500_amd as spm
    from scenegen import profiling_grid
    rows = []
    stream = torch.cuda.current_stream()
    for k, (polys, paper_s) in PAPER_PROFILING.items():
        builders = [spm.Builder(spm.DeviceScene(profiling_grid(k, seed=s), "cuda:0")) for s in range(n_sources)]
        for b in builders[:3]:
            b.build(stream)
        torch.cuda.synchronize()
        timer = spm.Timer()
        t0 = time.perf_counter()
        for b in builders:
            b.build(stream, timer=timer)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stages, nb = timer.elapsed()
        G = [int(b.map.n_gen.item()) for b in builders]
        ms = (t1 - t0) * 1e3 / n_sources
        rows.append({"k": k, "polygons": polys, "vertices": 4 * polys, "mean_G": sum(G) / len(G),
                     "ms_per_build": ms, "pixel_ms": stages["pixel"] / max(nb, 1),
                     "Mpixel_gen_per_s": 1e6 * (sum(G) / len(G)) / (ms * 1e-3) / 1e6,
                     "paper_comp_s_gtx970": paper_s})
        del builders
    return {"sweep": "profiling-style maps, 1000x1000, k x k squares, %d random single sources each" % n_sources,
            "rows": rows}


def main():
    args = _parse()
    if args.sweep:
        print(json.dumps(_sweep(args.sweep)), flush=True)
        return
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 4}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1805_08500_amd as spm
    from scenegen import config2

    tw, th = (int(x) for x in args.tile.split("x"))
    scene = config2(args.seed)
    ds = spm.DeviceScene(scene, "cuda:0")
    b = spm.Builder(ds, tile=(tw, th))
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        b.build(stream)
    torch.cuda.synchronize()
    G = int(b.map.n_gen.item())
    W, H = scene.width, scene.height

    # timed region: exactly K whole builds
    timer = spm.Timer()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.build(stream, timer=timer)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages, nb = timer.elapsed()
    ms_step = (t1 - t0) * 1e3 / args.steps
    stage_avg = {k: v / max(nb, 1) for k, v in stages.items()}

    # one instrumented build (outside the timed region) for the work counts
    stats = torch.zeros(8, dtype=torch.int64, device="cuda:0")
    b.build(stream, stats=stats)
    torch.cuda.synchronize()
    s = stats.cpu().numpy().astype(np.float64)
    executed = (s[1] * 64 * OPS["tile_bound"] + s[2] * OPS["lane_bound"] + s[4] * 64 * OPS["relevance"]
                + s[5] * OPS["lane_edge"] + s[7] * OPS["accept"])
    n_segs = 0 if scene.segs is None else len(scene.segs)
    ops = (W * H * G * ALG["pair"] + W * H * n_segs * ALG["segment_pair"] + s[7] * ALG["accept"]
           + s[5] * ALG["lane_edge"])
    t_pix = stage_avg["pixel"] * 1e-3
    achieved = ops / t_pix / 1e12
    peak = PEAK_LANE_OPS / 1e12
    src_hash = _file_hash(os.path.join(ROOT, "paper_1805_08500_amd", "csrc", "k_pixel.hip"))

    pairs = W * H * G
    out = {
        "metric": METRIC,
        "value": pairs / (ms_step * 1e-3) / 1e6,
        "unit": "Mpixel·gen/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "convex-1024: 1024x1024 grid, 60 convex hulls (6-10 seeded points in 20-80 px "
                               "boxes), 3 point sources, 2 segment sources, seed %d" % args.seed,
                   "W": W, "H": H, "G": G, "E": scene.n_vertices, "tile": args.tile},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TOP/s",
                     "frac": achieved / peak, "traffic": _traffic(src_hash), "kernel": "k_pixel",
                     "executed_ops_frac": executed / t_pix / 1e12 / peak,
                     "ops_per_launch": ops},
        "stages_ms": stage_avg,
        "k_pixel_Mpixel_gen_per_s": pairs / t_pix / 1e6,
        "work_counts": {k: int(v) for k, v in zip(
            ["tiles", "gen_batches", "lane_bound", "wave_vis", "relevance", "lane_edge", "occluded", "accept"], s)},
        "k_pixel_source_hash": src_hash,
    }
    if not args.no_extras:
        out["batched"] = _batched(spm, torch)
        out["backward"] = _backward(spm, torch, b, scene)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _cpu_baseline(scene, G, args.cpu_pixels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
