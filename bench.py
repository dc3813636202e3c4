"""Benchmark: shortest-path-map builds on one MI355X.

One step = one complete build (spm_build_ex: device ingest, generator
visibility, relaxation, cost sort, inside mask, pixel propagation) of the
headline workload, the 2048 x 2048 maze (randomized-DFS 64 x 64 cells of 32 px
with 4 px walls, 4 exit segment sources, seed 1), with the scene already
resident in device memory.  --workload convex1024 selects the 1024 x 1024
scene with 60 convex obstacles instead.

value = W * H * G / t_step / 1e6  (Mpixel*generator/s; G = point sources +
segment sources + corner generators, the dense pair count the paper's method
shades).

Prints one JSON line.  roofline: the pixel kernel (the dominant one), bound by
32-bit VALU issue.  achieved = the algorithmic lane-ops of one launch / its
average launch time (HIP events on the build stream, over the timed builds);
the algorithmic work is counted in the method's own units by one instrumented
build outside the timed region: 8 lane-ops per pixel-generator bound test
(the cone bound of Procedure 3), 8 per accepted candidate (square root, add,
compare, select), 9 per examined lane-edge visibility test (orientations and
compares) and 20 per pixel-segment closest point (Section 4).  peak = 256 CUs
x 4 SIMDs x 16 lanes x 2.4 GHz.  The issue counters of the same kernel
(VALU busy, lane utilisation, executed lane-op rate) come from the committed
rocprofv3 summary while the kernel source is unchanged since it was taken.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SPM build Mpixel·gen/s + % VALU roofline; batched & backward vs plain"
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9      # CUs x SIMDs x lanes x clock: one 32-bit VALU op per lane per cycle
# algorithmic lane-ops per unit of the method (counted by the instrumented pixel kernel)
ALG = {
    "bound": 8,          # per (pixel, generator) bound test: cost + |p - g| against the pixel's value
    "accept": 8,         # per accepted candidate: square root, add, compare, select
    "lane_edge": 9,      # per examined (pixel, generator, edge) visibility test
    "segment": 20,       # per (pixel, segment source) closest point q*
    # per (cached edge, candidate) shadow test against the whole tile (Procedure 2's shadow of one edge): the
    # candidate in the edge's umbra behind the tile, three exact half-planes (one lane per cached edge)
    "shadow_point": 8,   # a point or corner: 6 multiply-adds, a three-way max, a compare
    "shadow_box": 14,    # a cluster's box: per half-plane its largest value over the box (2 selects, 2 multiply-adds)
}
# instrumented counters (spm_build_opts.d_stats order)
STAT_NAMES = ["tiles", "walk_steps", "lane_bound", "wave_vis", "relevance", "lane_edge", "one_edge_hides", "accept",
              "occ_cache_tests", "occ_cache_hits", "segment_lanes", "cluster_members", "cluster_members_tried",
              "clusters_hidden", "cluster_members_umbra", "cluster_members_umbra_tested"]
WORKLOADS = {
    "maze2048": "maze-2048: 2048x2048 grid, randomized-DFS maze of 64x64 cells (32 px, 4 px walls, exact union "
                "boundary), 4 exit segment sources on the outer boundary, seed %d",
    "convex1024": "convex-1024: 1024x1024 grid, 60 convex hulls (6-10 seeded points in 20-80 px boxes), 3 point "
                  "sources, 2 segment sources, seed %d",
}


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="maze2048")
    ap.add_argument("--tile", default="8x8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary workload, the batched and backward figures and the host-scene build")
    ap.add_argument("--cpu-pixels", type=int, default=2048, help="oracle pixel sample per CPU-baseline run")
    ap.add_argument("--sweep", type=int, default=0, metavar="SOURCES",
                    help="only run the Profiling-style sweep (k x k squares on 1000^2, k in 2..20) with this many "
                         "random single sources per map, print its JSON line and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only run one plain device copy of this many bytes (HBM counter calibration) and exit")
    return ap.parse_args()


def _file_hash(*paths):
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _pixel_source_hash():
    """The pixel kernel's source: k_pixel.hip and the device header it includes."""
    csrc = os.path.join(ROOT, "paper_1805_08500_amd", "csrc")
    return _file_hash(os.path.join(csrc, "k_pixel.hip"), os.path.join(csrc, "spm_internal.hpp"))


def _profile(name, kernel_src_hash):
    """A committed rocprofv3 summary (profiles/<name>.json), if the pixel kernel's source is the one it was
    taken with; else None."""
    p = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    return t if t.get("source_hash") == kernel_src_hash else None


def _scene(workload, seed):
    from scenegen import config2, config3
    return config3(seed) if workload == "maze2048" else config2(seed)


def _time_builds(spm, torch, b, steps, warmup, events_in_region=True):
    """ms per whole build over `steps` timed builds, and the per-stage HIP-event times.  With events_in_region the
    stage timer records its events inside the timed builds (the headline: the pixel kernel's time comes from the
    same builds); else the timed builds run bare and the stage times come from as many builds after them (the
    timer's eight events per build cost about 25 us, which matters for a 0.2 ms build)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        b.build(stream)
    torch.cuda.synchronize()
    timer = spm.Timer()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.build(stream, timer=timer if events_in_region else None)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if not events_in_region:
        for _ in range(steps):
            b.build(stream, timer=timer)
        torch.cuda.synchronize()
    stages, nb = timer.elapsed()
    return (t1 - t0) * 1e3 / steps, {k: v / max(nb, 1) for k, v in stages.items()}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(scene, G, npix, gpu_map):
    """The oracle (plain C, OpenMP) on the host cores: generator costs over the whole scene plus a seeded pixel
    sample, extrapolated to all pixels; median of 3 runs on every thread, one run on 1 thread with a smaller
    sample.  The GPU map is compared with the oracle on the first sample (parity on the bench's own workload)."""
    import numpy as np
    from oracle import oracle as O
    O.build()
    threads = O.max_threads()
    WH = scene.width * scene.height

    def run(nthreads, n, seed):
        rng = np.random.default_rng(seed)
        pix = np.unique(rng.integers(0, WH, n))
        t0 = time.perf_counter()
        cost, _ = O.costs(scene, nthreads=nthreads)
        t1 = time.perf_counter()
        r = O.pixels(scene, cost, pix, nthreads=nthreads)
        t2 = time.perf_counter()
        return (t1 - t0) + (t2 - t1) * WH / len(pix), t1 - t0, t2 - t1, pix, r

    runs = [run(threads, npix, 100 + k) for k in range(3)]
    t_all = statistics.median(r[0] for r in runs)
    one = run(1, max(64, npix // 8), 200)
    pix, r = runs[0][3], runs[0][4]
    d = gpu_map["dist"].reshape(-1)[pix].astype(np.float64)
    p = gpu_map["parent"].reshape(-1)[pix]
    D = r["dist64"]
    fin = np.isfinite(D)
    with np.errstate(invalid="ignore"):
        amb = fin & ((r["second"] - D) <= 1e-5 * D + 1e-6)
    rel = np.abs(d[fin] - D[fin]) / np.maximum(D[fin], 1e-30)
    parity = {"pixels": int(len(pix)), "free": int(fin.sum()),
              "finite_masks_equal": bool(np.array_equal(np.isfinite(d), fin)),
              "max_rel_err": float(rel.max()) if rel.size else 0.0,
              "parent_differs_clear": int((fin & ~amb & (p != r["parent"])).sum()),
              "parent_differs_near_tie": int((amb & (p != r["parent"])).sum()),
              "ambiguous_frac": float(amb.sum()) / max(1, int(fin.sum()))}
    return {
        "value": WH * G / t_all / 1e6, "unit": "Mpixel·gen/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"median of 3 runs, each: generator costs of the whole scene + {npix} random pixels (seeds 100-102) "
                   f"extrapolated to all {WH} pixels; {threads} OpenMP threads"),
        "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
        "seconds_per_run": [round(x[0], 3) for x in runs],
        "costs_s": round(statistics.median(x[1] for x in runs), 4),
        "one_thread": {"value": WH * G / one[0] / 1e6, "costs_s": round(one[1], 3),
                       "sample": f"{len(one[3])} random pixels, extrapolated"},
        "parity_on_sample": parity,
    }


def _batched(spm, torch, reps=10):
    """256 mixed scenes (sides 128-1024, 4-80 hulls, 1-5 points, 0-3 segments), one hipGraph replay per batched
    build.  Throughput = sum over scenes of W * H * G / t."""
    from scenegen import config4_list
    scenes = config4_list()
    from paper_1805_08500_amd import autotune
    t0 = time.perf_counter()
    tuned = autotune.tune(scenes, cache_path=None)
    tune_s = time.perf_counter() - t0
    bb = spm.BatchBuilder(scenes, check=False, tuned=tuned)
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
            "tuned": {"tile_w": {str(k): v for k, v in tuned["tile_w"].items()}, "pixel_waves": tuned["pixel_waves"],
                      "walk": tuned["walk"], "tuning_s": round(tune_s, 2), "pixel_ms": tuned["times"]["batch"]},
            "scenes": len(scenes), "pixels": int(sum(x.width * x.height for x in scenes)), "pairs": pairs,
            "ms_per_batch": ms, "value": pairs / (ms * 1e-3) / 1e6, "unit": "Mpixel·gen/s"}


def _backward(spm, torch, reps=20):
    """4096 agents on the 1024 x 1024 convex-hull scene: map rebuild + agent distances (forward) and the adjoint."""
    from scenegen import config2, config5_agents
    scene = config2(1)
    b = spm.Builder(spm.DeviceScene(scene, "cuda:0"))
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


def _host_scene(spm, torch, b, scene, reps=10):
    """spm_build from the host scene (validation, pinned staging, upload, build): the rate with the PCIe copy and
    the host checks inside the timed region (never the headline value)."""
    for _ in range(2):
        b.build_host(scene)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.build_host(scene)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    G = int(b.map.n_gen.item())
    return {"ms_per_build": ms, "value": scene.width * scene.height * G / (ms * 1e-3) / 1e6, "unit": "Mpixel·gen/s"}


# The paper's own timings of its Profiling maps (Table 1: polygons, computation seconds; GTX 970),
# quoted as context next to the sweep, never as a target.
PAPER_PROFILING = {2: (4, 0.0014), 4: (16, 0.0054), 6: (36, 0.0456), 8: (64, 0.1251), 10: (100, 0.2701),
                   14: (196, 0.8564), 20: (400, 2.7371)}


def _sweep(n_sources):
    """Profiling-style maps: 1000 x 1000, k x k rows of squares (each half its cell's width), one random free
    source per build, n_sources builds per map.  Reports the mean whole-build time per map."""
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
        print(json.dumps({"sweep_row": rows[-1]}), file=sys.stderr, flush=True)
        del builders
    return {"sweep": "profiling-style maps, 1000x1000, k x k squares, %d random single sources each" % n_sources,
            "rows": rows}


def _measure(spm, torch, np, workload, seed, tile, steps, warmup, events_in_region=True):
    tw, th = (int(x) for x in tile.split("x"))
    scene = _scene(workload, seed)
    b = spm.Builder(spm.DeviceScene(scene, "cuda:0"), tile=(tw, th))
    ms_step, stage_avg = _time_builds(spm, torch, b, steps, warmup, events_in_region)
    G = int(b.map.n_gen.item())
    # one instrumented build (outside the timed region) for the work counts
    stats = torch.zeros(16, dtype=torch.int64, device="cuda:0")
    b.build(torch.cuda.current_stream(), stats=stats)
    torch.cuda.synchronize()
    s = stats.cpu().numpy().astype(np.float64)
    return scene, b, G, ms_step, stage_avg, {k: int(v) for k, v in zip(STAT_NAMES, s)}


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

    scene, b, G, ms_step, stage_avg, counts = _measure(spm, torch, np, args.workload, args.seed, args.tile,
                                                       args.steps, args.warmup)
    W, H = scene.width, scene.height
    # the cluster walk tests every cluster it takes, and the members of the open ones, against the 64 cached edges
    cluster_walk = counts["cluster_members"] > 0
    units = {"bound": counts["lane_bound"], "accept": counts["accept"], "lane_edge": counts["lane_edge"],
             "segment": counts["segment_lanes"],
             "shadow_point": 64 * counts["cluster_members_umbra_tested"],
             "shadow_box": 64 * counts["walk_steps"] if cluster_walk else 0}
    ops = sum(units[k] * ALG[k] for k in units)
    ops_pixel_only = sum(units[k] * ALG[k] for k in ("bound", "accept", "lane_edge", "segment"))
    t_pix = stage_avg["pixel"] * 1e-3
    achieved = ops / t_pix / 1e12
    peak = PEAK_LANE_OPS / 1e12
    src_hash = _pixel_source_hash()
    prof = _profile("k_pixel_%s_counters" % args.workload, src_hash)
    traffic = None
    counters = None
    if prof:
        traffic = prof.get("hbm_bytes_per_launch")
        counters = prof.get("derived")
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
        "config": {"workload": WORKLOADS[args.workload] % args.seed, "W": W, "H": H, "G": G,
                   "E": scene.n_vertices, "tile": args.tile},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TOP/s", "frac": achieved / peak,
                     "traffic": traffic, "kernel": "k_pixel",
                     "algorithmic_lane_ops_per_launch": ops,
                     "ops_per_unit": ALG,
                     "units_per_launch": units,
                     "frac_without_shadow_tests": ops_pixel_only / t_pix / 1e12 / peak,
                     "k_pixel_ms": stage_avg["pixel"],
                     "counters": counters},
        "stages_ms": stage_avg,
        "k_pixel_Mpixel_gen_per_s": pairs / t_pix / 1e6,
        "work_counts": counts,
        "k_pixel_source_hash": src_hash,
    }
    if not args.no_extras:
        other = "convex1024" if args.workload == "maze2048" else "maze2048"
        sc2, b2, G2, ms2, st2, c2 = _measure(spm, torch, np, other, args.seed, args.tile, max(args.steps, 50),
                                             args.warmup, events_in_region=False)
        out["secondary"] = {"workload": WORKLOADS[other] % args.seed, "ms_per_step": ms2, "G": G2,
                            "value": sc2.width * sc2.height * G2 / (ms2 * 1e-3) / 1e6, "unit": "Mpixel·gen/s",
                            "stages_ms": st2, "timing": "builds timed bare; stage times from as many builds after them"}
        del b2
        out["host_scene_build"] = _host_scene(spm, torch, b, scene)
        out["batched"] = _batched(spm, torch)
        out["backward"] = _backward(spm, torch)
    if not args.no_cpu_baseline:
        b.build()
        torch.cuda.synchronize()
        out["cpu_baseline"] = _cpu_baseline(scene, G, args.cpu_pixels, b.map.host())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
