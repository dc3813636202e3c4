"""Tile-shape autotuner for the pixel stage.

For each grid side that occurs in a set of scenes, times the pixel stage of
every supported tile shape (8x8, 16x4, 4x16) on up to `per_class` of those
scenes and keeps the fastest.  Results are cached in a JSON file keyed by the
device name and the library file's modification time, so a rebuilt library
or another GPU retunes.
"""
from __future__ import annotations

import json
import os

import torch

from . import _lib as C
from .spm import Builder, DeviceScene, Timer

TILE_WIDTHS = (8, 16, 4)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "spm_autotune.json")


def _key():
    return f"{torch.cuda.get_device_name(0)}|{int(os.path.getmtime(C.LIB_PATH))}"


def tune(scenes, per_class: int = 3, reps: int = 3, cache_path: str = DEFAULT_CACHE, force: bool = False) -> dict:
    """Returns {side: best tile width} for the sides of `scenes`."""
    cache = {}
    if cache_path and os.path.exists(cache_path) and not force:
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    entry = cache.get(_key(), {})
    classes = {}
    for s in scenes:
        classes.setdefault(max(s.width, s.height), []).append(s)
    out = {}
    for side, group in sorted(classes.items()):
        if str(side) in entry:
            out[side] = int(entry[str(side)])
            continue
        best, best_t = 8, float("inf")
        for tw in TILE_WIDTHS:
            t_tot = 0.0
            for s in group[:per_class]:
                b = Builder(DeviceScene(s, check=False), tile=(tw, 64 // tw))
                b.build()
                timer = Timer()
                for _ in range(reps):
                    b.build(timer=timer)
                st, n = timer.elapsed()
                t_tot += st["pixel"] / max(n, 1)
            if t_tot < best_t:
                best, best_t = tw, t_tot
        out[side] = best
        entry[str(side)] = best
    cache[_key()] = entry
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return out
