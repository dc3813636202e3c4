"""The autotuner's search and cache (CPU; the GPU timing test is in test_gpu_batch.py)."""
import json

from paper_1805_08500_amd.autotune import Cache, batch_signature, choose
from scenegen import random_small


def test_choose_takes_the_least_and_keeps_the_first_tie():
    best, times = choose([8, 16, 4], {8: 3.0, 16: 2.0, 4: 2.0}.__getitem__)
    assert best == 16 and times == {"8": 3.0, "16": 2.0, "4": 2.0}


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    calls = []

    def compute():
        calls.append(1)
        return {"tile_w": 16, "times": {"8": 1.0, "16": 0.5}}
    a = Cache(path).get_or("dev|tile|512", compute)
    b = Cache(path).get_or("dev|tile|512", compute)       # a fresh reader of the same file
    assert a == b and len(calls) == 1
    with open(path) as f:
        assert json.load(f)["dev|tile|512"]["tile_w"] == 16
    Cache(path).get_or("dev|tile|1024", compute)           # another key adds, keeps the first
    with open(path) as f:
        assert set(json.load(f)) == {"dev|tile|512", "dev|tile|1024"}
    assert len(calls) == 2
    assert Cache(None).get_or("k", compute) == a and len(calls) == 3   # no file: nothing kept


def test_batch_signature_depends_on_the_scenes_not_their_order():
    s = [random_small(k) for k in range(5)]
    assert batch_signature(s) == batch_signature(s[::-1])
    assert batch_signature(s) != batch_signature(s[:4])
