"""Pixel samples for parity checks on maps too large for a whole-map oracle run (tests only).

Every sample is chosen from seeded random numbers and the oracle's own results,
never from the GPU map under test.
"""
import numpy as np


def wide_sample(scene, cost, seed, n_random, n_rows=3, block=96):
    """Row-major pixel indices: n_rows whole pixel rows (every region border they cross is in the
    sample), a block x block square of pixels around the generator with the largest finite cost
    (the deepest part of the scene, where the most candidates compete), and n_random uniform
    pixels."""
    W, H = scene.width, scene.height
    rng = np.random.default_rng(seed)
    parts = []
    for j in rng.choice(H, min(n_rows, H), replace=False):
        parts.append(j * W + np.arange(W, dtype=np.int64))
    from oracle import oracle as O
    kind, ref, xy = O.generators(scene)
    fin = np.isfinite(cost)
    if fin.any():
        g = int(np.argmax(np.where(fin, cost, -1.0)))
        cx, cy = int(xy[g, 0]), int(xy[g, 1])
        x0 = min(max(cx - block // 2, 0), max(W - block, 0))
        y0 = min(max(cy - block // 2, 0), max(H - block, 0))
        jj, ii = np.mgrid[y0:min(y0 + block, H), x0:min(x0 + block, W)]
        parts.append((jj * W + ii).reshape(-1).astype(np.int64))
    parts.append(rng.integers(0, W * H, n_random).astype(np.int64))
    return np.unique(np.concatenate(parts))
