"""Pins for the CPU oracle: closed forms, an independent exact method, invariants.

None of these tests retypes the oracle's formulas; each compares it with a
result reached another way (a different visibility algorithm, exhaustive path
enumeration, clipping against a box, coordinate rotation, lattice search) or
with a property the paper's definition fixes (Section 3: the map holds the
geodesic distance to the closest source and the first turn point).
"""
import math
from fractions import Fraction as F

import numpy as np
import pytest

from scenegen import Scene, config1, random_small, scene_from_arrays
from scenegen.scenes import _rect_poly
from oracle import mini


def _pix_centres(W, H):
    i, j = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    return i, j


# ---------------------------------------------------------------- free space
def test_free_space_single_point(oracle_mod):
    s = Scene(37, 29, [], np.asarray([[11, 4]]), None)
    m = oracle_mod.full_map(s)
    i, j = _pix_centres(37, 29)
    np.testing.assert_allclose(m["dist64"], np.hypot(i - 11, j - 4), rtol=0, atol=1e-12)
    assert (m["parent"] == 0).all()


def test_free_space_voronoi(oracle_mod):
    pts = np.asarray([[3, 3], [30, 7], [12, 25], [25, 26]])
    s = Scene(33, 31, [], pts, None)
    m = oracle_mod.full_map(s)
    i, j = _pix_centres(33, 31)
    d = np.stack([np.hypot(i - x, j - y) for x, y in pts])
    np.testing.assert_allclose(m["dist64"], d.min(0), atol=1e-12)
    srt = np.sort(d, 0)
    clear = srt[1] - srt[0] > 1e-9
    assert (m["parent"][clear] == d.argmin(0)[clear]).all()


def test_free_space_segment_by_rotation(oracle_mod):
    seg = np.asarray([[4, 5, 27, 19]])
    s = Scene(34, 26, [], None, seg)
    m = oracle_mod.full_map(s)
    i, j = _pix_centres(34, 26)
    a = complex(4, 5)
    e = complex(27 - 4, 19 - 5)
    L = abs(e)
    z = ((i + 1j * j) - a) * np.conj(e) / L          # segment lies on [0, L] of the real axis
    d_in = np.abs(z.imag)
    d_end = np.minimum(np.abs(z), np.abs(z - L))
    ref = np.where((z.real >= 0) & (z.real <= L), d_in, d_end)
    np.testing.assert_allclose(m["dist64"], ref, atol=1e-9)
    assert (m["parent"] == 0).all()


# ------------------------------------------------- one convex obstacle, by hand
def _clip_open_box(a, b, box):
    """True iff the closed segment [a,b] meets the open box (Liang-Barsky, exact)."""
    x0, y0, x1, y1 = (F(v) for v in box)
    lo, hi = F(0), F(1)
    lo_strict = hi_strict = False
    for p0, d, mn, mx in ((F(a[0]), F(b[0]) - F(a[0]), x0, x1), (F(a[1]), F(b[1]) - F(a[1]), y0, y1)):
        if d == 0:
            if not (mn < p0 < mx):
                return False
            continue
        t1, t2 = (mn - p0) / d, (mx - p0) / d
        if t1 > t2:
            t1, t2 = t2, t1
        if t1 >= lo:
            lo, lo_strict = t1, True
        if t2 <= hi:
            hi, hi_strict = t2, True
    if lo < hi:
        return True
    return lo == hi and not (lo_strict or hi_strict)


def _rect_geodesic(p, s, box):
    """Shortest path around one rectangle: direct, or hug the boundary."""
    x0, y0, x1, y1 = box
    C = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
    if not _clip_open_box(p, s, box):
        return math.dist(p, s)
    best = math.inf
    for a in range(4):
        if _clip_open_box(s, C[a], box):
            continue
        for b in range(4):
            if _clip_open_box(C[b], p, box):
                continue
            for step in (1, -1):
                L, k = 0.0, a
                while k != b:
                    k2 = (k + step) % 4
                    L += math.dist(C[k], C[k2])
                    k = k2
                best = min(best, math.dist(s, C[a]) + L + math.dist(C[b], p))
    return best


@pytest.mark.parametrize("box,src", [((10, 8, 22, 20), (3, 14)), ((5, 5, 9, 30), (20, 17)),
                                     ((12, 3, 30, 11), (21, 27))])
def test_single_rectangle_wraparound(oracle_mod, box, src):
    W, H = 36, 34
    s = Scene(W, H, [_rect_poly(*box)], np.asarray([src]), None)
    m = oracle_mod.full_map(s)
    for j in range(H):
        for i in range(W):
            p = (i + 0.5, j + 0.5)
            if box[0] <= p[0] <= box[2] and box[1] <= p[1] <= box[3]:
                assert np.isinf(m["dist64"][j, i]) and m["parent"][j, i] == -1
                continue
            assert abs(m["dist64"][j, i] - _rect_geodesic(p, src, box)) < 1e-9, (i, j)


# ------------------------------------------------ visibility against event sampling
def _to_h(pt):
    x, y = F(pt[0]), F(pt[1])
    d = math.lcm(x.denominator, y.denominator)
    return (int(2 * x * d), int(2 * y * d), d)


def _vis_cases(scene, rng, n):
    polys = scene.polys
    verts = [tuple(map(int, v)) for P in polys for v in P]
    out = []
    while len(out) < n:
        pts = []
        for _ in range(2):
            r = rng.integers(0, 4)
            if r == 0 and verts:
                pts.append(verts[int(rng.integers(0, len(verts)))])
            elif r == 1:
                pts.append((F(int(rng.integers(0, scene.width)) * 2 + 1, 2),
                            F(int(rng.integers(0, scene.height)) * 2 + 1, 2)))
            elif r == 2:
                pts.append((int(rng.integers(0, scene.width + 1)), int(rng.integers(0, scene.height + 1))))
            else:
                # a rational point: projection of a lattice point on a lattice segment
                A = np.asarray(rng.integers(0, [scene.width + 1, scene.height + 1]))
                B = np.asarray(rng.integers(0, [scene.width + 1, scene.height + 1]))
                if (A == B).all():
                    continue
                P = rng.integers(0, [scene.width + 1, scene.height + 1])
                e = B - A
                t = F(int((P - A) @ e), int(e @ e))
                t = min(max(t, F(0)), F(1))
                pts.append((A[0] + t * int(e[0]), A[1] + t * int(e[1])))
        if len(pts) < 2:
            continue
        if any(mini.strictly_inside(polys, (F(p[0]), F(p[1]))) for p in pts):
            continue
        out.append(tuple(pts))
    return out


@pytest.mark.parametrize("seed", range(8))
def test_visibility_matches_event_sampling(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    scene = random_small(seed + 500, kind=("rects", "hulls", "blocks")[seed % 3])
    E = mini._edges(scene.polys)
    for a, b in _vis_cases(scene, rng, 250):
        exp = mini.visible(scene.polys, a, b, E)
        got = oracle_mod.visible(scene, _to_h(a), _to_h(b))
        assert got == exp, (scene.meta, a, b)


def test_visibility_hand_degeneracies(oracle_mod):
    # square [10,20]^2 and an L-shaped (concave) polygon
    sq = _rect_poly(10, 10, 20, 20)
    L = np.asarray([(30, 10), (40, 10), (40, 14), (34, 14), (34, 20), (30, 20)])
    s = Scene(50, 30, [sq, L], np.asarray([[0, 0]]), None)
    cases = [
        ((0, 0), (30, 30), False),      # diagonal through two opposite corners: crosses interior
        ((0, 10), (30, 10), True),      # runs along the bottom edge (touching allowed)
        ((5, 0), (25, 20), False),      # passes through corner (20,20)? no: through (15,10)->interior
        ((0, 20), (10, 10), True),      # ends at a corner, grazing from outside
        ((0, 5), (25, 30), False),      # through corner (10,15)? enters interior
        ((9, 21), (21, 9), False),      # cuts the corner region (20,20)-(10,10) diagonal... crosses
        ((20, 0), (20, 30), True),      # along the right edge x=20
        ((21, 25), (29, 17), True),     # misses everything
        ((34, 14), (40, 20), True),     # from the reflex corner outward into the notch
        ((34, 14), (30, 10), False),    # from the reflex corner into the interior
        ((34, 20), (40, 14), True),     # across the notch, touching both corners
        ((32, 22), (36, 12), False),    # enters the L through its top
    ]
    for a, b, exp in cases:
        assert mini.visible(s.polys, a, b) == exp, (a, b)
        assert oracle_mod.visible(s, _to_h(a), _to_h(b)) == exp, (a, b)


# ------------------------------------------------ exhaustive enumeration (mini oracle)
def _tiny_scenes():
    out = []
    out.append(Scene(24, 20, [_rect_poly(8, 6, 14, 12)], np.asarray([[3, 9]]), None))
    out.append(Scene(26, 22, [np.asarray([(6, 6), (14, 6), (14, 9), (9, 9), (9, 16), (6, 16)])],
                     np.asarray([[20, 3]]), None))                       # concave L: reflex corner
    out.append(Scene(28, 22, [_rect_poly(10, 4, 13, 18)], None, np.asarray([[2, 2, 3, 19]])))
    out.append(Scene(30, 24, [_rect_poly(8, 8, 12, 12), np.asarray([(18, 5), (24, 9), (19, 14)])],
                     np.asarray([[27, 20]]), np.asarray([[2, 1, 6, 3]])))
    out.append(Scene(22, 22, [np.asarray([(5, 5), (17, 5), (17, 17), (13, 17), (13, 9), (9, 9), (9, 17), (5, 17)])],
                     None, np.asarray([[11, 20, 11, 13]])))                 # segment reaching into a U
    return out


@pytest.mark.parametrize("k", range(5))
def test_enumeration_matches_oracle(oracle_mod, k):
    scene = _tiny_scenes()[k]
    M = mini.Mini(scene, max_vertices=9)
    cost, gpar = oracle_mod.costs(scene)
    kind, ref, xy = oracle_mod.generators(scene)
    # every corner generator's cost equals the enumerated minimum
    for g in range(len(cost)):
        if kind[g] == oracle_mod.VERTEX:
            assert abs(cost[g] - M.cost[ref[g]]) < 1e-9 * max(1.0, cost[g]), (g, cost[g], M.cost[ref[g]])
    # reflex (non-generator) corners never beat the corners the oracle keeps
    m = oracle_mod.full_map(scene)
    for j in range(scene.height):
        for i in range(scene.width):
            D, knd, where = M.pixel(i, j)
            got = m["dist64"][j, i]
            if math.isinf(D):
                assert math.isinf(got)
                continue
            assert abs(got - D) < 1e-9 * max(1.0, D), (i, j, got, D)
            if m["second"][j, i] - got > 1e-7 * max(1.0, got):
                p = m["parent"][j, i]
                exp_kind = {"point": 0, "segment": 1, "vertex": 2}[knd]
                assert kind[p] == exp_kind and ref[p] == where, (i, j)


# ------------------------------------------------ runner-up D2 and single-generator values
def test_free_space_runner_up(oracle_mod):
    """Without obstacles every source is visible: D2 is the second smallest of the closed-form
    distances to the point sources and to the segment (rotated frame)."""
    pts = np.asarray([[3, 3], [30, 7], [12, 25], [25, 26]])
    seg = np.asarray([[4, 5, 27, 19]])
    s = Scene(34, 31, [], pts, seg)
    m = oracle_mod.full_map(s)
    i, j = _pix_centres(34, 31)
    dp = [np.hypot(i - x, j - y) for x, y in pts]
    e = complex(23, 14)
    L = abs(e)
    z = ((i + 1j * j) - complex(4, 5)) * np.conj(e) / L
    ds = np.where((z.real >= 0) & (z.real <= L), np.abs(z.imag), np.minimum(np.abs(z), np.abs(z - L)))
    srt = np.sort(np.stack(dp + [ds]), 0)
    np.testing.assert_allclose(m["dist64"], srt[0], atol=1e-9)
    np.testing.assert_allclose(m["second"], srt[1], atol=1e-9)


_KIND_NAME = {0: "point", 1: "segment", 2: "vertex"}
_mini_cache = {}


def _mini_values(O, k):
    """(scene, oracle map, oracle costs, generator table, mini's value matrix [pixels, G])."""
    if k not in _mini_cache:
        scene = _tiny_scenes()[k]
        M = mini.Mini(scene, max_vertices=9)
        cost, _ = O.costs(scene)
        kind, ref, xy = O.generators(scene)
        W, H, G = scene.width, scene.height, len(cost)
        vals = np.array([[M.generator_value(i, j, _KIND_NAME[int(kind[g])], int(ref[g])) for g in range(G)]
                         for j in range(H) for i in range(W)], np.float64).reshape(W * H, G)
        _mini_cache[k] = (scene, O.full_map(scene), cost, (kind, ref, xy), vals)
    return _mini_cache[k]


@pytest.mark.parametrize("k", range(5))
def test_runner_up_and_candidates_match_mini(oracle_mod, k):
    """Every (pixel, generator) value of the oracle, and its runner-up D2, against mini.py's
    brute force: its own visibility (event midpoints in Fraction arithmetic), its enumerated corner
    costs and its own clamped projection onto a segment source.  D2 is the second smallest value
    over the visible generators (Procedure 3 keeps the smallest; the next one decides which pixels
    are near-ties)."""
    scene, m, cost, (kind, ref, xy), vals = _mini_values(oracle_mod, k)
    W, H, G = scene.width, scene.height, len(cost)
    pix = np.repeat(np.arange(W * H, dtype=np.int64), G)
    gen = np.tile(np.arange(G, dtype=np.int32), W * H)
    got = oracle_mod.candidates(scene, cost, pix, gen).reshape(W * H, G)
    assert np.array_equal(np.isinf(got), np.isinf(vals)), np.argwhere(np.isinf(got) != np.isinf(vals))[:5]
    fin = np.isfinite(vals)
    np.testing.assert_allclose(got[fin], vals[fin], rtol=1e-12, atol=1e-12)
    srt = np.sort(vals, 1)
    d1 = srt[:, 0]
    d2 = srt[:, 1] if G > 1 else np.full(W * H, np.inf)
    for name, mine, ref_v in (("D", d1, m["dist64"].ravel()), ("D2", d2, m["second"].ravel())):
        assert np.array_equal(np.isinf(mine), np.isinf(ref_v)), name
        f = np.isfinite(mine)
        np.testing.assert_allclose(ref_v[f], mine[f], rtol=1e-12, atol=1e-12, err_msg=name)


def test_runner_up_pin_catches_plausible_mistakes(oracle_mod):
    """The pin above would fail for the mistakes a runner-up is prone to: taken over every other
    candidate whether visible or not, or counting the winner twice (D2 = D)."""
    over_invisible = 0
    winner_twice = 0
    for k in range(5):
        scene, m, cost, (kind, ref, xy), vals = _mini_values(oracle_mod, k)
        W, H, G = scene.width, scene.height, len(cost)
        if G < 2:
            continue
        i, j = _pix_centres(W, H)
        i, j = i.ravel(), j.ravel()
        blind = np.empty((W * H, G))
        for g in range(G):
            x0, y0, x1, y1 = (float(v) for v in xy[g])
            if kind[g] == oracle_mod.SEGMENT:
                ex, ey = x1 - x0, y1 - y0
                t = np.clip(((i - x0) * ex + (j - y0) * ey) / (ex * ex + ey * ey), 0, 1)
                blind[:, g] = np.hypot(i - x0 - t * ex, j - y0 - t * ey)
            else:
                blind[:, g] = cost[g] + np.hypot(i - x0, j - y0)
        free = np.isfinite(vals).sum(1) >= 2
        win = np.argmin(vals, 1)
        blind[np.arange(W * H), win] = np.inf
        wrong = blind.min(1)
        d2 = np.sort(vals, 1)[:, 1]
        over_invisible += int(np.sum(free & (wrong < d2 - 1e-6)))
        winner_twice += int(np.sum(free & (d2 > np.sort(vals, 1)[:, 0] + 1e-6)))
    assert over_invisible > 50 and winner_twice > 500, (over_invisible, winner_twice)


# ------------------------------------------------ invariants on larger scenes
def _check_invariants(O, scene):
    cost, gpar, Wm = O.costs(scene, weights=True)
    kind, ref, xy = O.generators(scene)
    G = len(cost)
    for v in range(G):
        if kind[v] != O.VERTEX:
            assert cost[v] == 0 and gpar[v] == v
            continue
        if not np.isfinite(cost[v]):
            assert gpar[v] == -1
            continue
        u = gpar[v]
        assert Wm[v, u] >= 0 and cost[u] + Wm[v, u] == cost[v]          # Bellman equality
        arcs = Wm[v] >= 0
        assert np.all(cost[arcs] + Wm[v, arcs] >= cost[v] - 1e-9 * cost[v])  # no better arc
        # chain ends at a source within G steps with strictly decreasing cost
        c, steps = v, 0
        while kind[c] == O.VERTEX:
            assert cost[gpar[c]] < cost[c]
            c = gpar[c]
            steps += 1
            assert steps <= G
    m = O.full_map(scene)
    D = m["dist64"]
    free = np.isfinite(D)
    # lower bound: never below the straight-line distance to the nearest source
    i, j = _pix_centres(scene.width, scene.height)
    lb = np.full(D.shape, np.inf)
    for x, y in scene.points:
        lb = np.minimum(lb, np.hypot(i - x, j - y))
    for ax, ay, bx, by in scene.segs:
        e = np.asarray([bx - ax, by - ay], float)
        t = np.clip(((i - ax) * e[0] + (j - ay) * e[1]) / (e @ e), 0, 1)
        lb = np.minimum(lb, np.hypot(i - ax - t * e[0], j - ay - t * e[1]))
    assert np.all(D[free] >= lb[free] - 1e-9)
    # 1-Lipschitz across neighbouring pixels that see each other
    H, Wd = D.shape
    for jj in range(0, H, 3):
        for ii in range(Wd - 1):
            if free[jj, ii] and free[jj, ii + 1]:
                a = (2 * ii + 1, 2 * jj + 1, 1)
                b = (2 * ii + 3, 2 * jj + 1, 1)
                if O.visible(scene, a, b):
                    assert abs(D[jj, ii] - D[jj, ii + 1]) <= 1 + 1e-9
    # the parent leg reproduces the distance
    for jj in range(0, H, 5):
        for ii in range(0, Wd, 5):
            if not free[jj, ii]:
                continue
            g = m["parent"][jj, ii]
            assert m["second"][jj, ii] >= D[jj, ii]
            assert np.isfinite(cost[g])
    return m


def test_invariants_config1(oracle_mod):
    _check_invariants(oracle_mod, config1(1))


@pytest.mark.parametrize("seed", [3, 7, 11])
def test_invariants_fuzz(oracle_mod, seed):
    _check_invariants(oracle_mod, random_small(seed))


def _mirror_x(scene):
    W = scene.width
    polys = [np.stack([W - P[::-1, 0], P[::-1, 1]], 1) for P in scene.polys]
    pts = np.stack([W - scene.points[:, 0], scene.points[:, 1]], 1) if len(scene.points) else None
    segs = scene.segs.copy()
    if len(segs):
        segs[:, 0] = W - segs[:, 0]
        segs[:, 2] = W - segs[:, 2]
    return Scene(W, scene.height, polys, pts, segs)


def test_mirror_and_translation(oracle_mod):
    s = random_small(21, kind="blocks")
    m0 = oracle_mod.full_map(s)
    m1 = oracle_mod.full_map(_mirror_x(s))
    np.testing.assert_allclose(m1["dist64"][:, ::-1], m0["dist64"], atol=1e-9)
    dx, dy = 6, 4
    t = Scene(s.width + 10, s.height + 9, [P + [dx, dy] for P in s.polys], s.points + [dx, dy],
              s.segs + [dx, dy, dx, dy] if len(s.segs) else None)
    m2 = oracle_mod.full_map(t)
    sub = m2["dist64"][dy:dy + s.height, dx:dx + s.width]
    np.testing.assert_allclose(sub, m0["dist64"], atol=1e-9)


def test_monotone_in_obstacles_and_sources(oracle_mod):
    base = Scene(48, 40, [_rect_poly(10, 10, 18, 30)], np.asarray([[4, 20]]), None)
    more_obs = Scene(48, 40, [_rect_poly(10, 10, 18, 30), _rect_poly(26, 4, 30, 26)], np.asarray([[4, 20]]), None)
    more_src = Scene(48, 40, [_rect_poly(10, 10, 18, 30)], np.asarray([[4, 20], [40, 35]]), None)
    d0 = oracle_mod.full_map(base)["dist64"]
    d1 = oracle_mod.full_map(more_obs)["dist64"]
    d2 = oracle_mod.full_map(more_src)["dist64"]
    both = np.isfinite(d0) & np.isfinite(d1)
    assert np.all(d1[both] >= d0[both] - 1e-9)
    assert np.all(d2 <= d0 + 1e-9)
    assert (d1[both] > d0[both] + 1e-6).any()   # the extra wall does lengthen some paths


# ------------------------------------------------ loose lattice cross-check
def test_sixteen_neighbour_lattice(oracle_mod):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import dijkstra
    scene = Scene(32, 28, [_rect_poly(8, 6, 14, 20), np.asarray([(18, 14), (26, 10), (24, 22)])],
                  np.asarray([[3, 3], [29, 25]]), None)
    h = 0.25
    nx, ny = int(scene.width / h) + 1, int(scene.height / h) + 1
    X, Y = np.meshgrid(np.arange(nx) * h, np.arange(ny) * h)

    def blocked(x, y):
        out = np.zeros(x.shape, bool)
        for P in scene.polys:
            n = len(P)
            inside = np.zeros(x.shape, bool)
            for k in range(n):
                ax, ay = P[k]
                bx, by = P[(k + 1) % n]
                c = (bx - ax) * (y - ay) - (by - ay) * (x - ax)
                on = (c == 0) & (x >= min(ax, bx)) & (x <= max(ax, bx)) & (y >= min(ay, by)) & (y <= max(ay, by))
                out |= on
                cross = ((ay > y) != (by > y)) & ((c > 0) == (by > ay))
                inside ^= cross
            out |= inside
        return out

    free = ~blocked(X, Y)
    idx = np.arange(nx * ny).reshape(ny, nx)
    moves = [(1, 0), (0, 1), (1, 1), (1, -1), (2, 1), (1, 2), (2, -1), (1, -2)]
    rows, cols, w = [], [], []
    for mx, my in moves:
        ys, xs = np.mgrid[max(0, -my):ny - max(0, my), 0:nx - mx]
        y2, x2 = ys + my, xs + mx
        mid = ~blocked((X[ys, xs] + X[y2, x2]) / 2, (Y[ys, xs] + Y[y2, x2]) / 2)
        ok = free[ys, xs] & free[y2, x2] & mid
        rows.append(idx[ys, xs][ok])
        cols.append(idx[y2, x2][ok])
        w.append(np.full(ok.sum(), h * math.hypot(mx, my)))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    ww = np.concatenate(w)
    A = coo_matrix((np.concatenate([ww, ww]), (np.concatenate([r, c]), np.concatenate([c, r]))),
                   shape=(nx * ny, nx * ny)).tocsr()
    srcs = [idx[int(y / h), int(x / h)] for x, y in scene.points]
    Dl = dijkstra(A, indices=srcs, min_only=True).reshape(ny, nx)
    m = oracle_mod.full_map(scene)["dist64"]
    ci = (np.arange(scene.width) * 4 + 2)
    cj = (np.arange(scene.height) * 4 + 2)
    Dg = Dl[np.ix_(cj, ci)]
    ok = np.isfinite(m) & np.isfinite(Dg)
    assert ok.sum() > 0.7 * m.size
    assert np.all(m[ok] <= Dg[ok] + 1.0)
    assert np.all(Dg[ok] <= 1.0275 * m[ok] + 1.0)


@pytest.mark.parametrize("seed", range(6))
def test_inside_matches_half_planes(oracle_mod, seed):
    """The inside mask (pixel centre in or on a closed obstacle) against the
    half-plane definition of a closed convex polygon: the centre lies on or to
    the left of every counter-clockwise edge.  The oracle decides it by
    crossing parity plus an on-boundary test, so the two share nothing."""
    from scenegen import random_small
    scene = random_small(seed, "hulls")
    W, H = scene.width, scene.height
    jj, ii = np.mgrid[0:H, 0:W]
    px = (2 * ii + 1).ravel().astype(np.int64)
    py = (2 * jj + 1).ravel().astype(np.int64)
    exp = np.zeros(W * H, bool)
    for P in scene.polys:
        P2 = 2 * np.asarray(P, np.int64)
        ok = np.ones(W * H, bool)
        for k in range(len(P2)):
            w, v = P2[k], P2[(k + 1) % len(P2)]
            ok &= (v[0] - w[0]) * (py - w[1]) - (v[1] - w[1]) * (px - w[0]) >= 0
        exp |= ok
    assert exp.any()
    got = oracle_mod.inside(scene, np.arange(W * H, dtype=np.int64))
    assert np.array_equal(got, exp)


# ------------------------------------------------ map values at rational points
QW = 256   # query points are numerators over 2 * QW domain units


def _rand_q(rng, W, H, n):
    return np.stack([rng.integers(0, 2 * W * QW + 1, n), rng.integers(0, 2 * H * QW + 1, n)], 1).astype(np.int64)


def test_points_free_space_closed_forms(oracle_mod):
    rng = np.random.default_rng(3)
    pts = np.asarray([[3, 3], [30, 7], [12, 25]])
    seg = np.asarray([[4, 5, 27, 19]])
    s = Scene(34, 31, [], pts, seg)
    cost, _ = oracle_mod.costs(s)
    q = _rand_q(rng, 34, 31, 400)
    r = oracle_mod.points(s, cost, q, QW)
    x, y = q[:, 0] / (2 * QW), q[:, 1] / (2 * QW)
    dp = np.stack([np.hypot(x - a, y - b) for a, b in pts])
    z = ((x + 1j * y) - complex(4, 5)) * np.conj(complex(23, 14)) / abs(complex(23, 14))
    L = abs(complex(23, 14))
    ds = np.where((z.real >= 0) & (z.real <= L), np.abs(z.imag), np.minimum(np.abs(z), np.abs(z - L)))
    ref = np.minimum(dp.min(0), ds)
    np.testing.assert_allclose(r["dist64"], ref, atol=1e-9)
    allc = np.vstack([dp, ds[None]])
    srt = np.sort(allc, 0)
    clear = srt[1] - srt[0] > 1e-9
    assert (r["parent"][clear] == allc.argmin(0)[clear]).all()


@pytest.mark.parametrize("box,src", [((10, 8, 22, 20), (3, 14)), ((12, 3, 30, 11), (21, 27))])
def test_points_rectangle_wraparound(oracle_mod, box, src):
    rng = np.random.default_rng(box[0])
    W, H = 36, 34
    s = Scene(W, H, [_rect_poly(*box)], np.asarray([src]), None)
    cost, _ = oracle_mod.costs(s)
    q = _rand_q(rng, W, H, 300)
    # a few points exactly on the rectangle's boundary and on its corner lines
    q = np.vstack([q, [[2 * QW * box[0], 2 * QW * 15], [2 * QW * 16, 2 * QW * box[3]], [2 * QW * box[2], 0]]])
    r = oracle_mod.points(s, cost, q, QW)
    for k, (X, Y) in enumerate(q):
        p = (F(int(X), 2 * QW), F(int(Y), 2 * QW))
        if box[0] <= p[0] <= box[2] and box[1] <= p[1] <= box[3]:
            assert np.isinf(r["dist64"][k]) and r["parent"][k] == -1
            continue
        assert abs(r["dist64"][k] - _rect_geodesic(p, src, box)) < 1e-9, (X, Y)


def test_points_agree_with_pixels_at_centres(oracle_mod):
    from scenegen import random_small
    for seed in range(4):
        s = random_small(seed)
        cost, _ = oracle_mod.costs(s)
        W, H = s.width, s.height
        pix = np.arange(W * H, dtype=np.int64)[:: max(1, (W * H) // 500)]
        q = np.stack([(2 * (pix % W) + 1) * QW, (2 * (pix // W) + 1) * QW], 1)
        a = oracle_mod.points(s, cost, q, QW)
        b = oracle_mod.pixels(s, cost, pix)
        assert np.array_equal(a["parent"], b["parent"])
        np.testing.assert_array_equal(a["dist64"], b["dist64"])
