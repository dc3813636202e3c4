"""Autotuner for batched builds.

Chooses, for a batch of scenes:
  * the pixel tile shape (8x8, 16x4 or 4x16) for each grid side that occurs,
    by timing the pixel stage of single builds of up to `per_class` scenes of
    that side with each shape;
  * the waves per SIMD of the persistent batched pixel launch (as many as fit,
    4 or 2) and its walk (by generator count, or the register-cached /
    refilled lower-bound walk where the batch's generator counts allow it), by
    timing the batched pixel stage of the whole batch with the chosen tiles.
Every candidate set contains the defaults, so the choice is never slower than
the defaults on the timings it was made from.

Results are cached in a JSON file keyed by the device name, the library
file's modification time and (for the batch-level choice) a signature of the
batch, so a rebuilt library, another GPU or another batch retunes.  The edge
chunk size (64 edges per chunk box) is a compile-time constant of the kernels
and is not tuned.
"""
from __future__ import annotations

import hashlib
import json
import os

TILE_WIDTHS = (8, 16, 4)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "spm_autotune.json")


def choose(candidates, measure):
    """The candidate with the least measure(candidate); ties keep the earlier one.
    Returns (best, {repr(candidate): time})."""
    best, best_t, times = None, float("inf"), {}
    for c in candidates:
        t = float(measure(c))
        times[repr(c)] = t
        if t < best_t:
            best, best_t = c, t
    return best, times


class Cache:
    """A JSON file of {key: value}; path None keeps nothing."""

    def __init__(self, path):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            try:
                with open(path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    def get(self, key):
        return self.data.get(key)

    def put(self, key, value):
        self.data[key] = value
        if self.path:
            os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
            tmp = self.path + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1)
            os.replace(tmp, self.path)

    def get_or(self, key, compute):
        v = self.get(key)
        if v is None:
            v = compute()
            self.put(key, v)
        return v


def batch_signature(scenes) -> str:
    items = sorted((s.width, s.height, s.n_vertices, len(s.points), len(s.segs)) for s in scenes)
    return hashlib.sha256(repr(items).encode()).hexdigest()[:16]


def _device_key():
    import torch

    from . import _lib as C
    return f"{torch.cuda.get_device_name(0)}|{int(os.path.getmtime(C.LIB_PATH))}"


def tune(scenes, per_class: int = 3, reps: int = 3, cache_path: str = DEFAULT_CACHE, force: bool = False) -> dict:
    """Returns {"tile_w": {side: tile width}, "pixel_waves": w, "walk": k} for the batch (pass it to
    BatchBuilder(..., tuned=...)); "times" holds the measured pixel-stage milliseconds."""
    import torch

    from .spm import BatchBuilder, Builder, DeviceScene, Timer

    cache = Cache(None if force else cache_path)
    if force and cache_path:
        cache.path = cache_path
    dev = _device_key()

    def pixel_ms(build, timer_builds):
        build(None)
        torch.cuda.synchronize()
        t = Timer()
        for _ in range(timer_builds):
            build(t)
        st, n = t.elapsed()
        return st["pixel"] / max(n, 1)

    classes = {}
    for s in scenes:
        classes.setdefault(max(s.width, s.height), []).append(s)
    tiles, times = {}, {}
    for side, group in sorted(classes.items()):
        def tile_time(tw, group=group):
            tot = 0.0
            for s in group[:per_class]:
                b = Builder(DeviceScene(s, check=False), tile=(tw, 64 // tw))
                tot += pixel_ms(lambda t, b=b: b.build(timer=t), reps)
            return tot

        def compute(side=side, tile_time=tile_time):
            best, tt = choose(TILE_WIDTHS, tile_time)
            return {"tile_w": best, "times": tt}
        r = cache.get_or(f"{dev}|tile|{side}", compute)
        tiles[side] = int(r["tile_w"])
        times[f"tile {side}"] = r["times"]

    bb = BatchBuilder(scenes, check=False, tile_w=tiles)
    gmax = max(s.n_vertices + len(s.points) + len(s.segs) for s in scenes)
    walks = [0] + ([1] if gmax <= 512 else []) + ([2] if gmax <= 8192 else [])
    cands = [(w, k) for w in (0, 4, 2) for k in walks]

    def batch_time(c):
        bb.set_options(pixel_waves=c[0], walk=c[1])
        return pixel_ms(lambda t: bb.build(timer=t), reps)

    def compute_batch():
        best, tt = choose(cands, batch_time)
        return {"pixel_waves": best[0], "walk": best[1], "times": tt}
    r = cache.get_or(f"{dev}|batch|{batch_signature(scenes)}|" + json.dumps(sorted(tiles.items())), compute_batch)
    times["batch"] = r["times"]
    del bb
    return {"tile_w": tiles, "pixel_waves": int(r["pixel_waves"]), "walk": int(r["walk"]), "times": times}
