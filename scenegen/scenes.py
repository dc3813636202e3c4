"""Seeded scene construction for the five benchmark workloads and for fuzzing.

Every coordinate is an integer in domain units (1 unit = 1 pixel).  The domain
is [0, W] x [0, H]; pixel (i, j) has its centre at (i + 1/2, j + 1/2).
Obstacles are simple polygons given as counter-clockwise vertex loops (the
obstacle lies on the left of every directed edge) with no repeated or
collinear consecutive vertices; closed obstacles are pairwise disjoint.  Point
sources lie strictly outside every closed obstacle and each closed segment
source is disjoint from every closed obstacle.  These are the inputs the paper
works with (polygonal obstacles in a rectangular domain, point sources and
segment sources: Section 3 and Section 4).

Randomness: numpy PCG64 seeded per scene.  The recipes follow the workload
table of the design notes (rectangles, convex hulls of random points, a
randomized-DFS maze, a batch of mixed scenes, agents for the adjoint).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "config1", "config2", "config3", "config4_list", "config5_agents",
    "random_small", "profiling_grid", "scene_from_arrays", "save_scene", "load_scene",
]


# --------------------------------------------------------------------------
# scene container
# --------------------------------------------------------------------------
@dataclass
class Scene:
    width: int
    height: int
    polys: list = field(default_factory=list)      # list of (k, 2) int64 arrays, CCW
    points: np.ndarray = None                      # (n, 2) int64
    segs: np.ndarray = None                        # (m, 4) int64: ax, ay, bx, by
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.points is None:
            self.points = np.zeros((0, 2), np.int64)
        if self.segs is None:
            self.segs = np.zeros((0, 4), np.int64)
        self.points = np.asarray(self.points, np.int64).reshape(-1, 2)
        self.segs = np.asarray(self.segs, np.int64).reshape(-1, 4)
        self.polys = [np.asarray(p, np.int64).reshape(-1, 2) for p in self.polys]

    @property
    def n_vertices(self) -> int:
        return int(sum(len(p) for p in self.polys))

    @property
    def n_sources(self) -> int:
        return int(len(self.points) + len(self.segs))

    def flat(self) -> dict:
        """Flat int32 arrays: poly_start (n_polys+1), vx, vy, pts (n*2), segs (m*4)."""
        starts = [0]
        for p in self.polys:
            starts.append(starts[-1] + len(p))
        if self.polys:
            v = np.concatenate(self.polys, axis=0)
        else:
            v = np.zeros((0, 2), np.int64)
        return {
            "width": int(self.width),
            "height": int(self.height),
            "poly_start": np.asarray(starts, np.int32),
            "vx": np.ascontiguousarray(v[:, 0], np.int32),
            "vy": np.ascontiguousarray(v[:, 1], np.int32),
            "pts": np.ascontiguousarray(self.points.reshape(-1), np.int32),
            "segs": np.ascontiguousarray(self.segs.reshape(-1), np.int32),
        }


def scene_from_arrays(width, height, poly_start, vx, vy, pts, segs, meta=None) -> Scene:
    poly_start = np.asarray(poly_start, np.int64)
    vx = np.asarray(vx, np.int64)
    vy = np.asarray(vy, np.int64)
    polys = [np.stack([vx[a:b], vy[a:b]], axis=1) for a, b in zip(poly_start[:-1], poly_start[1:])]
    return Scene(int(width), int(height), polys, np.asarray(pts).reshape(-1, 2),
                 np.asarray(segs).reshape(-1, 4), dict(meta or {}))


def save_scene(path, scene: Scene) -> None:
    f = scene.flat()
    np.savez(path, **{k: np.asarray(v) for k, v in f.items()})


def load_scene(path) -> Scene:
    with np.load(path, allow_pickle=False) as z:
        return scene_from_arrays(int(z["width"]), int(z["height"]), z["poly_start"], z["vx"],
                                 z["vy"], z["pts"], z["segs"])


# --------------------------------------------------------------------------
# exact integer geometry used only to *construct* valid scenes
# --------------------------------------------------------------------------
def _cross(ax, ay, bx, by, cx, cy) -> int:
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)


def _hull(pts) -> list:
    """Strict convex hull (collinear points dropped), counter-clockwise."""
    p = sorted(set((int(x), int(y)) for x, y in pts))
    if len(p) < 3:
        return p

    def half(seq):
        out = []
        for q in seq:
            while len(out) >= 2 and _cross(*out[-2], *out[-1], *q) <= 0:
                out.pop()
            out.append(q)
        return out

    lower = half(p)
    upper = half(reversed(p))
    return lower[:-1] + upper[:-1]


def _seg_meet_closed(a, b, c, d) -> bool:
    """Closed segments [a,b] and [c,d] share at least one point."""
    d1 = _cross(*c, *d, *a)
    d2 = _cross(*c, *d, *b)
    d3 = _cross(*a, *b, *c)
    d4 = _cross(*a, *b, *d)
    if ((d1 > 0 and d2 < 0) or (d1 < 0 and d2 > 0)) and ((d3 > 0 and d4 < 0) or (d3 < 0 and d4 > 0)):
        return True

    def on(p, q, r):  # r on closed segment [p, q], given collinear
        return min(p[0], q[0]) <= r[0] <= max(p[0], q[0]) and min(p[1], q[1]) <= r[1] <= max(p[1], q[1])

    if d1 == 0 and on(c, d, a):
        return True
    if d2 == 0 and on(c, d, b):
        return True
    if d3 == 0 and on(a, b, c):
        return True
    if d4 == 0 and on(a, b, d):
        return True
    return False


def _point_in_closed_poly(p, poly) -> bool:
    """p inside or on the boundary of a simple polygon (exact)."""
    px, py = p
    n = len(poly)
    inside = False
    for i in range(n):
        ax, ay = int(poly[i][0]), int(poly[i][1])
        bx, by = int(poly[(i + 1) % n][0]), int(poly[(i + 1) % n][1])
        c = _cross(ax, ay, bx, by, px, py)
        if c == 0 and min(ax, bx) <= px <= max(ax, bx) and min(ay, by) <= py <= max(ay, by):
            return True
        if (ay > py) != (by > py):
            # crossing of the rightward ray from p; edge goes up iff by > ay
            if (c > 0) == (by > ay):
                inside = not inside
    return inside


def _polys_meet_closed(P, Q) -> bool:
    """Closed simple polygons P and Q share a point."""
    pb = (P[:, 0].min(), P[:, 1].min(), P[:, 0].max(), P[:, 1].max())
    qb = (Q[:, 0].min(), Q[:, 1].min(), Q[:, 0].max(), Q[:, 1].max())
    if pb[2] < qb[0] or qb[2] < pb[0] or pb[3] < qb[1] or qb[3] < pb[1]:
        return False
    n, m = len(P), len(Q)
    for i in range(n):
        a, b = tuple(P[i]), tuple(P[(i + 1) % n])
        for j in range(m):
            if _seg_meet_closed(a, b, tuple(Q[j]), tuple(Q[(j + 1) % m])):
                return True
    return _point_in_closed_poly(tuple(P[0]), Q) or _point_in_closed_poly(tuple(Q[0]), P)


def _seg_meets_poly_closed(a, b, P) -> bool:
    n = len(P)
    pb = (P[:, 0].min(), P[:, 1].min(), P[:, 0].max(), P[:, 1].max())
    if max(a[0], b[0]) < pb[0] or min(a[0], b[0]) > pb[2] or max(a[1], b[1]) < pb[1] or min(a[1], b[1]) > pb[3]:
        return False
    for i in range(n):
        if _seg_meet_closed(a, b, tuple(P[i]), tuple(P[(i + 1) % n])):
            return True
    return _point_in_closed_poly(a, P)


def _free_point(p, polys) -> bool:
    return not any(_point_in_closed_poly(p, P) for P in polys)


def _free_segment(a, b, polys) -> bool:
    return not any(_seg_meets_poly_closed(a, b, P) for P in polys)


def _signed_area2(P) -> int:
    x = P[:, 0]
    y = P[:, 1]
    return int(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


# --------------------------------------------------------------------------
# union boundary of a block occupancy grid (used for mazes and concave fuzz)
# --------------------------------------------------------------------------
def _trace_blocks(occ: np.ndarray, cell: int) -> list:
    """Boundary loops of the union of occupied cells, obstacle on the left.

    occ[by, bx] marks the closed square [cell*bx, cell*(bx+1)] x [cell*by, cell*(by+1)].
    Returns CCW loops with collinear runs merged.  Raises ValueError on a pinch
    (two cells touching only at a corner) or on a hole (a clockwise loop).
    """
    occ = np.asarray(occ, bool)
    ny, nx = occ.shape
    P = np.zeros((ny + 2, nx + 2), bool)
    P[1:-1, 1:-1] = occ
    # pinch check: 2x2 windows with a diagonal-only pattern
    a = P[:-1, :-1]
    b = P[:-1, 1:]
    c = P[1:, :-1]
    d = P[1:, 1:]
    if np.any((a & d & ~b & ~c) | (b & c & ~a & ~d)):
        raise ValueError("pinch vertex in block union")
    nxt = {}
    # vertical unit edges at lattice x = X (padded index), between P[Y, X-1] and P[Y, X]
    L = P[:, :-1]
    R = P[:, 1:]
    ys, xs = np.nonzero(L & ~R)           # obstacle left of x=X: go up
    for Y, X in zip(ys.tolist(), xs.tolist()):
        nxt[(X + 1, Y)] = (X + 1, Y + 1)
    ys, xs = np.nonzero(R & ~L)           # obstacle right: go down
    for Y, X in zip(ys.tolist(), xs.tolist()):
        nxt[(X + 1, Y + 1)] = (X + 1, Y)
    B = P[:-1, :]
    T = P[1:, :]
    ys, xs = np.nonzero(B & ~T)           # obstacle below y=Y: go -x
    for Y, X in zip(ys.tolist(), xs.tolist()):
        nxt[(X + 1, Y + 1)] = (X, Y + 1)
    ys, xs = np.nonzero(T & ~B)           # obstacle above: go +x
    for Y, X in zip(ys.tolist(), xs.tolist()):
        nxt[(X, Y + 1)] = (X + 1, Y + 1)
    loops = []
    seen = set()
    for start in sorted(nxt.keys(), key=lambda v: (v[1], v[0])):
        if start in seen:
            continue
        loop = []
        v = start
        while v not in seen:
            seen.add(v)
            loop.append(v)
            v = nxt[v]
        if v != start:
            raise ValueError("open boundary chain")
        # merge collinear runs
        n = len(loop)
        keep = []
        for i in range(n):
            p0, p1, p2 = loop[i - 1], loop[i], loop[(i + 1) % n]
            if _cross(*p0, *p1, *p2) != 0:
                keep.append(p1)
        arr = (np.asarray(keep, np.int64) - 1) * cell
        if _signed_area2(arr) <= 0:
            raise ValueError("hole in block union")
        # canonical start: lowest-then-leftmost vertex
        k = int(np.lexsort((arr[:, 0], arr[:, 1]))[0])
        loops.append(np.roll(arr, -k, axis=0))
    return loops


def _fill_holes(occ: np.ndarray) -> np.ndarray:
    """Mark every empty cell not 4-connected to the border as occupied."""
    occ = np.asarray(occ, bool).copy()
    ny, nx = occ.shape
    reach = np.zeros_like(occ)
    stack = [(y, x) for y in range(ny) for x in (0, nx - 1) if not occ[y, x]]
    stack += [(y, x) for x in range(nx) for y in (0, ny - 1) if not occ[y, x]]
    while stack:
        y, x = stack.pop()
        if reach[y, x] or occ[y, x]:
            continue
        reach[y, x] = True
        for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            yy, xx = y + dy, x + dx
            if 0 <= yy < ny and 0 <= xx < nx and not occ[yy, xx] and not reach[yy, xx]:
                stack.append((yy, xx))
    return occ | ~reach


def _fix_pinches(occ: np.ndarray) -> np.ndarray:
    """Resolve diagonal-only contacts by filling one empty cell of each such 2x2 window."""
    occ = np.asarray(occ, bool).copy()
    while True:
        a = occ[:-1, :-1]
        b = occ[:-1, 1:]
        c = occ[1:, :-1]
        d = occ[1:, 1:]
        p1 = a & d & ~b & ~c
        p2 = b & c & ~a & ~d
        if not (p1.any() or p2.any()):
            return occ
        ys, xs = np.nonzero(p1)
        occ[ys, xs + 1] = True
        ys, xs = np.nonzero(p2)
        occ[ys, xs] = True


# --------------------------------------------------------------------------
# workload 1: 256^2, eight axis-aligned rectangles, one point source
# --------------------------------------------------------------------------
def _rect_poly(x0, y0, x1, y1):
    return np.asarray([(x0, y0), (x1, y0), (x1, y1), (x0, y1)], np.int64)


def config1(seed: int = 1) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    W = H = 256
    rects = []
    tries = 0
    while len(rects) < 8:
        tries += 1
        if tries > 100000:
            raise RuntimeError("config1: could not place rectangles")
        w = int(rng.integers(8, 49))
        h = int(rng.integers(8, 49))
        x0 = int(rng.integers(0, W - w + 1))
        y0 = int(rng.integers(0, H - h + 1))
        r = (x0, y0, x0 + w, y0 + h)
        if any(r[0] <= q[2] and q[0] <= r[2] and r[1] <= q[3] and q[1] <= r[3] for q in rects):
            continue
        rects.append(r)
    polys = [_rect_poly(*r) for r in rects]
    while True:
        p = (int(rng.integers(0, 256)), int(rng.integers(0, 256)))
        if _free_point(p, polys):
            break
    return Scene(W, H, polys, np.asarray([p]), None,
                 {"name": "rectangles-256", "seed": seed, "recipe": "8 rects 8..48, 1 point"})


# --------------------------------------------------------------------------
# workload 2: 1024^2, sixty convex hulls, three points and two segments
# --------------------------------------------------------------------------
def _convex_obstacles(rng, W, H, n_obs, box_lo, box_hi, max_tries):
    polys = []
    tries = 0
    while len(polys) < n_obs and tries < max_tries:
        tries += 1
        s = int(rng.integers(box_lo, box_hi + 1))
        s = min(s, W, H)
        x0 = int(rng.integers(0, W - s + 1))
        y0 = int(rng.integers(0, H - s + 1))
        k = int(rng.integers(6, 11))
        pts = np.stack([rng.integers(x0, x0 + s + 1, k), rng.integers(y0, y0 + s + 1, k)], axis=1)
        hull = _hull(pts.tolist())
        if len(hull) < 3:
            continue
        P = np.asarray(hull, np.int64)
        if any(_polys_meet_closed(P, Q) for Q in polys):
            continue
        polys.append(P)
    return polys


def _free_points(rng, W, H, polys, n):
    out = []
    while len(out) < n:
        p = (int(rng.integers(0, W + 1)), int(rng.integers(0, H + 1)))
        if _free_point(p, polys):
            out.append(p)
    return out


def _free_segments(rng, W, H, polys, n, len_lo, len_hi):
    out = []
    while len(out) < n:
        a = (int(rng.integers(0, W + 1)), int(rng.integers(0, H + 1)))
        L = float(rng.uniform(len_lo, len_hi))
        th = float(rng.uniform(0.0, 2.0 * math.pi))
        b = (int(round(a[0] + L * math.cos(th))), int(round(a[1] + L * math.sin(th))))
        if not (0 <= b[0] <= W and 0 <= b[1] <= H) or a == b:
            continue
        if not _free_segment(a, b, polys):
            continue
        out.append((a[0], a[1], b[0], b[1]))
    return out


def config2(seed: int = 1) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    W = H = 1024
    polys = _convex_obstacles(rng, W, H, 60, 20, 80, 100000)
    if len(polys) < 60:
        raise RuntimeError("config2: could not place obstacles")
    pts = _free_points(rng, W, H, polys, 3)
    segs = _free_segments(rng, W, H, polys, 2, 40.0, 200.0)
    return Scene(W, H, polys, np.asarray(pts), np.asarray(segs),
                 {"name": "convex-1024", "seed": seed,
                  "recipe": "60 hulls of 6-10 pts in 20-80 boxes, 3 points, 2 segments 40-200"})


# --------------------------------------------------------------------------
# workload 3: 2048^2 randomized-DFS maze, union boundary, four exit segments
# --------------------------------------------------------------------------
def _maze_walls(rng, n):
    """Randomized depth-first maze on n x n cells.

    Returns (V, Hh): V[i, j] vertical wall at x-line i between rows j (i in 0..n),
    Hh[i, j] horizontal wall at y-line j over column i (j in 0..n).
    """
    V = np.ones((n + 1, n), bool)
    Hh = np.ones((n, n + 1), bool)
    seen = np.zeros((n, n), bool)
    start = (int(rng.integers(0, n)), int(rng.integers(0, n)))
    stack = [start]
    seen[start] = True
    while stack:
        cx, cy = stack[-1]
        nb = []
        if cx > 0 and not seen[cx - 1, cy]:
            nb.append((cx - 1, cy))
        if cx < n - 1 and not seen[cx + 1, cy]:
            nb.append((cx + 1, cy))
        if cy > 0 and not seen[cx, cy - 1]:
            nb.append((cx, cy - 1))
        if cy < n - 1 and not seen[cx, cy + 1]:
            nb.append((cx, cy + 1))
        if not nb:
            stack.pop()
            continue
        nx_, ny_ = nb[int(rng.integers(0, len(nb)))]
        if nx_ != cx:
            V[max(cx, nx_), cy] = False
        else:
            Hh[cx, max(cy, ny_)] = False
        seen[nx_, ny_] = True
        stack.append((nx_, ny_))
    return V, Hh


def config3(seed: int = 1, cells: int = 64, cell_px: int = 32, wall: int = 4) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    n = cells
    S = n * cell_px
    V, Hh = _maze_walls(rng, n)
    exits = {
        "bottom": int(rng.integers(0, n)),
        "top": int(rng.integers(0, n)),
        "left": int(rng.integers(0, n)),
        "right": int(rng.integers(0, n)),
    }
    Hh[exits["bottom"], 0] = False
    Hh[exits["top"], n] = False
    V[0, exits["left"]] = False
    V[n, exits["right"]] = False
    # rasterize onto a block lattice of half the wall thickness
    blk = wall // 2
    nb = S // blk
    per = cell_px // blk
    hw = wall // 2 // blk  # half wall in blocks
    occ = np.zeros((nb, nb), bool)  # occ[by, bx]
    for i in range(n + 1):
        for j in range(n):
            if V[i, j]:
                x0, x1 = i * per - hw, i * per + hw
                y0, y1 = j * per - hw, (j + 1) * per + hw
                occ[max(y0, 0):min(y1, nb), max(x0, 0):min(x1, nb)] = True
    for i in range(n):
        for j in range(n + 1):
            if Hh[i, j]:
                x0, x1 = i * per - hw, (i + 1) * per + hw
                y0, y1 = j * per - hw, j * per + hw
                occ[max(y0, 0):min(y1, nb), max(x0, 0):min(x1, nb)] = True
    polys = _trace_blocks(occ, blk)
    h = wall // 2
    lo, hi = h + 1, cell_px - h - 1
    segs = [
        (exits["bottom"] * cell_px + lo, 0, exits["bottom"] * cell_px + hi, 0),
        (exits["top"] * cell_px + lo, S, exits["top"] * cell_px + hi, S),
        (0, exits["left"] * cell_px + lo, 0, exits["left"] * cell_px + hi),
        (S, exits["right"] * cell_px + lo, S, exits["right"] * cell_px + hi),
    ]
    n_rects = int(V.sum() + Hh.sum())
    return Scene(S, S, polys, None, np.asarray(segs),
                 {"name": f"maze-{S}", "seed": seed, "wall_rectangles": n_rects,
                  "recipe": f"DFS maze {n}x{n} cells of {cell_px}px, {wall}px walls, union boundary"})


# --------------------------------------------------------------------------
# workload 4: a batch of 256 mixed scenes
# --------------------------------------------------------------------------
def _scaled_scene(seed, side):
    rng = np.random.Generator(np.random.PCG64(seed))
    W = H = side
    f = side / 1024.0
    lo = max(6, int(math.floor(20 * f)))
    hi = max(lo, int(math.floor(80 * f)))
    n_obs = int(rng.integers(4, 81))
    polys = _convex_obstacles(rng, W, H, n_obs, lo, hi, 40 * n_obs)
    n_pts = int(rng.integers(1, 6))
    n_seg = int(rng.integers(0, 4))
    pts = _free_points(rng, W, H, polys, n_pts)
    segs = _free_segments(rng, W, H, polys, n_seg, max(2.0, 40.0 * f), max(3.0, 200.0 * f))
    return Scene(W, H, polys, np.asarray(pts), np.asarray(segs).reshape(-1, 4),
                 {"name": f"batch-{side}", "seed": seed, "requested_obstacles": n_obs})


def config4_list(seed: int = 7, count: int = 256) -> list:
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.choice(np.asarray([128, 256, 512, 1024]), size=count)
    return [_scaled_scene(seed * 1000000 + k, int(sides[k])) for k in range(count)]


# --------------------------------------------------------------------------
# workload 5: agents in free space of the workload-2 scene
# --------------------------------------------------------------------------
def config5_agents(scene: Scene, n: int = 4096, seed: int = 11) -> np.ndarray:
    """Uniform continuous agent positions (float32) whose own point and whose
    pixel centre lie outside every closed obstacle."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    W, H = scene.width, scene.height
    polys = scene.polys
    bbs = [(P[:, 0].min(), P[:, 1].min(), P[:, 0].max(), P[:, 1].max()) for P in polys]

    def free_f(x, y):
        for P, b in zip(polys, bbs):
            if b[0] <= x <= b[2] and b[1] <= y <= b[3]:
                # exact test on a rational point with denominator 2^24
                q = (int(float(x) * 2.0 ** 40), int(float(y) * 2.0 ** 40))
                PP = [(int(a) << 40, int(c) << 40) for a, c in P]
                if _point_in_closed_poly(q, PP):
                    return False
        return True

    while len(out) < n:
        x = np.float32(rng.uniform(0.0, W))
        y = np.float32(rng.uniform(0.0, H))
        if not (0.0 <= x < W and 0.0 <= y < H):
            continue
        cx = math.floor(float(x)) + 0.5
        cy = math.floor(float(y)) + 0.5
        if free_f(float(x), float(y)) and free_f(cx, cy):
            out.append((x, y))
    return np.asarray(out, np.float32)


# --------------------------------------------------------------------------
# fuzzing scenes: small grids, rectangles / convex hulls / concave block shapes
# --------------------------------------------------------------------------
def _random_blob_occ(rng, nbx, nby, n_blobs, size_lo, size_hi):
    occ = np.zeros((nby, nbx), bool)
    for _ in range(n_blobs):
        target = int(rng.integers(size_lo, size_hi + 1))
        y = int(rng.integers(1, max(2, nby - 1)))
        x = int(rng.integers(1, max(2, nbx - 1)))
        cells = [(y, x)]
        blob = {(y, x)}
        while len(blob) < target:
            cy, cx = cells[int(rng.integers(0, len(cells)))]
            dy, dx = ((1, 0), (-1, 0), (0, 1), (0, -1))[int(rng.integers(0, 4))]
            yy, xx = cy + dy, cx + dx
            if 1 <= yy < nby - 1 and 1 <= xx < nbx - 1 and (yy, xx) not in blob:
                blob.add((yy, xx))
                cells.append((yy, xx))
            if len(cells) > 4 * target:
                break
        for (yy, xx) in blob:
            occ[yy, xx] = True
    return occ


def random_small(seed: int, kind: str = "mixed") -> Scene:
    """Small fuzz scene: side 16..128 (not always a multiple of 8), 1-6 obstacles.

    kind: 'rects', 'hulls', 'blocks' (concave orthogonal polygons), or 'mixed'.
    """
    rng = np.random.Generator(np.random.PCG64(1000003 * seed + 17))
    if kind == "mixed":
        kind = ("rects", "hulls", "blocks")[int(rng.integers(0, 3))]
    W = int(rng.integers(16, 129))
    H = int(rng.integers(16, 129))
    n_obs = int(rng.integers(1, 7))
    polys = []
    if kind == "rects":
        tries = 0
        while len(polys) < n_obs and tries < 2000:
            tries += 1
            w = int(rng.integers(2, max(3, W // 3)))
            h = int(rng.integers(2, max(3, H // 3)))
            x0 = int(rng.integers(0, W - w + 1))
            y0 = int(rng.integers(0, H - h + 1))
            P = _rect_poly(x0, y0, x0 + w, y0 + h)
            if any(_polys_meet_closed(P, Q) for Q in polys):
                continue
            polys.append(P)
    elif kind == "hulls":
        s_hi = max(6, min(W, H) // 2)
        tries = 0
        while len(polys) < n_obs and tries < 2000:
            tries += 1
            s = int(rng.integers(4, s_hi + 1))
            s = min(s, W, H)
            x0 = int(rng.integers(0, W - s + 1))
            y0 = int(rng.integers(0, H - s + 1))
            k = int(rng.integers(3, 11))
            pts = np.stack([rng.integers(x0, x0 + s + 1, k), rng.integers(y0, y0 + s + 1, k)], axis=1)
            hull = _hull(pts.tolist())
            if len(hull) < 3:
                continue
            P = np.asarray(hull, np.int64)
            if any(_polys_meet_closed(P, Q) for Q in polys):
                continue
            polys.append(P)
    else:
        cell = int(rng.integers(2, 7))
        nbx, nby = max(3, W // cell), max(3, H // cell)
        occ = _random_blob_occ(rng, nbx, nby, n_obs, 2, max(3, (nbx * nby) // 12))
        for _ in range(8):
            occ = _fix_pinches(_fill_holes(occ))
            if np.array_equal(occ, _fill_holes(occ)):
                break
        try:
            polys = _trace_blocks(occ, cell)
        except ValueError:
            polys = []
    n_pts = int(rng.integers(0, 4))
    n_seg = int(rng.integers(0, 3))
    if n_pts + n_seg == 0:
        n_pts = 1
    pts = _free_points(rng, W, H, polys, n_pts)
    segs = _free_segments(rng, W, H, polys, n_seg, 2.0, max(3.0, min(W, H) * 0.6))
    return Scene(W, H, polys, np.asarray(pts).reshape(-1, 2), np.asarray(segs).reshape(-1, 4),
                 {"name": f"fuzz-{kind}", "seed": seed})


# --------------------------------------------------------------------------
# the paper's "Profiling" family: uniform rows of square obstacles
# --------------------------------------------------------------------------
def profiling_grid(k: int, side: int = 1000, fill: float = 0.5, seed: int = 0) -> Scene:
    """k x k uniform grid of axis-aligned squares on a side x side domain with one
    random free integer source.  The paper does not give the square size or the
    spacing; here each square takes `fill` of its cell's width, centred."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cell = side / k
    sq = max(1, int(round(cell * fill)))
    polys = []
    for j in range(k):
        for i in range(k):
            cx = (i + 0.5) * cell
            cy = (j + 0.5) * cell
            x0 = int(round(cx - sq / 2))
            y0 = int(round(cy - sq / 2))
            polys.append(_rect_poly(x0, y0, x0 + sq, y0 + sq))
    pts = _free_points(rng, side, side, polys, 1)
    return Scene(side, side, polys, np.asarray(pts), None,
                 {"name": f"profiling-{k}x{k}", "seed": seed})
