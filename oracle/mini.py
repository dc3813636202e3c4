"""Exhaustive exact mini-oracle for tiny scenes -- TEST INFRASTRUCTURE ONLY.

Used to pin ``spm_oracle.c`` with an *independent* method, so that a plausible
mistake in the oracle (a wrong sign in an orientation, a mishandled grazing
contact, a wrong corner classification, a wrong reading of segment sources)
shows up as a disagreement:

* Visibility is decided by a different algorithm: every point where the
  closed segment meets an obstacle edge is an event; between consecutive
  events the segment is either inside an obstacle's open interior or not, so
  it suffices to test the midpoint of every gap (exact ``Fraction`` geometry).
* Generator costs come from enumerating every simple path through *all*
  obstacle vertices (convex and reflex corners alike), not from Dijkstra over
  the convex corners only.
* The distance from a point to a segment source is the minimum over the
  *whole visible part* of the segment (split at every ray through an obstacle
  vertex), not the distance to the clamped projection.

Paper: the map is the shortest-path distance to the closest source point or
segment point with the first turn point as parent (Section 3, Section 4);
shortest paths are found by search on a visibility graph (Section 2).
"""
from __future__ import annotations

import math
from fractions import Fraction as F
from itertools import permutations

import numpy as np


def _cross(o, a, b):
    return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])


def _edges(polys):
    out = []
    for P in polys:
        n = len(P)
        for i in range(n):
            out.append(((F(int(P[i][0])), F(int(P[i][1]))),
                        (F(int(P[(i + 1) % n][0])), F(int(P[(i + 1) % n][1])))))
    return out


def _on_segment(c, d, p):
    if _cross(c, d, p) != 0:
        return False
    return min(c[0], d[0]) <= p[0] <= max(c[0], d[0]) and min(c[1], d[1]) <= p[1] <= max(c[1], d[1])


def strictly_inside(polys, p) -> bool:
    """p in the open interior of some obstacle."""
    for P in polys:
        n = len(P)
        inside = False
        on = False
        for i in range(n):
            a = (F(int(P[i][0])), F(int(P[i][1])))
            b = (F(int(P[(i + 1) % n][0])), F(int(P[(i + 1) % n][1])))
            if _on_segment(a, b, p):
                on = True
                break
            if (a[1] > p[1]) != (b[1] > p[1]):
                xc = a[0] + (p[1] - a[1]) * (b[0] - a[0]) / (b[1] - a[1])
                if xc > p[0]:
                    inside = not inside
        if inside and not on:
            return True
    return False


def closed_inside(polys, p) -> bool:
    for P in polys:
        n = len(P)
        inside = False
        for i in range(n):
            a = (F(int(P[i][0])), F(int(P[i][1])))
            b = (F(int(P[(i + 1) % n][0])), F(int(P[(i + 1) % n][1])))
            if _on_segment(a, b, p):
                return True
            if (a[1] > p[1]) != (b[1] > p[1]):
                xc = a[0] + (p[1] - a[1]) * (b[0] - a[0]) / (b[1] - a[1])
                if xc > p[0]:
                    inside = not inside
        if inside:
            return True
    return False


def visible(polys, a, b, edges=None) -> bool:
    """Closed segment [a,b] avoids every open obstacle interior (event midpoints)."""
    a = (F(a[0]), F(a[1]))
    b = (F(b[0]), F(b[1]))
    if a == b:
        return not strictly_inside(polys, a)
    E = edges if edges is not None else _edges(polys)
    r = (b[0] - a[0], b[1] - a[1])
    rr = r[0] * r[0] + r[1] * r[1]
    ts = {F(0), F(1)}
    for c, d in E:
        s = (d[0] - c[0], d[1] - c[1])
        den = r[0] * s[1] - r[1] * s[0]
        ca = (c[0] - a[0], c[1] - a[1])
        if den != 0:
            t = (ca[0] * s[1] - ca[1] * s[0]) / den
            u = (ca[0] * r[1] - ca[1] * r[0]) / den
            if 0 <= t <= 1 and 0 <= u <= 1:
                ts.add(t)
        elif ca[0] * r[1] - ca[1] * r[0] == 0:
            for q in (c, d):
                t = ((q[0] - a[0]) * r[0] + (q[1] - a[1]) * r[1]) / rr
                if 0 <= t <= 1:
                    ts.add(t)
    ts = sorted(ts)
    for t0, t1 in zip(ts[:-1], ts[1:]):
        tm = (t0 + t1) / 2
        m = (a[0] + tm * r[0], a[1] + tm * r[1])
        if strictly_inside(polys, m):
            return False
    return True


def _dist(a, b) -> float:
    return math.sqrt(float((a[0] - b[0]) ** 2 + (a[1] - b[1]) ** 2))


def segment_reach(polys, p, seg, edges=None):
    """(distance, closest point) from p to the visible part of the segment, or (inf, None).

    The visible part is closed; it changes only where a ray from p through an
    obstacle vertex meets the segment, so the segment is split at those points
    and at its endpoints, each piece is tested at its midpoint, each split point
    on its own, and the nearest point of every visible piece is taken.
    """
    A = (F(int(seg[0])), F(int(seg[1])))
    B = (F(int(seg[2])), F(int(seg[3])))
    p = (F(p[0]), F(p[1]))
    e = (B[0] - A[0], B[1] - A[1])
    ts = {F(0), F(1)}
    for P in polys:
        for v in P:
            v = (F(int(v[0])), F(int(v[1])))
            dvec = (v[0] - p[0], v[1] - p[1])
            den = dvec[0] * e[1] - dvec[1] * e[0]
            if den == 0:
                continue
            ap = (A[0] - p[0], A[1] - p[1])
            # A + t e = p + s d  =>  t = -cross(d, A-p) / cross(d, e),  s = -cross(e, A-p) / cross(d, e)
            t = -(dvec[0] * ap[1] - dvec[1] * ap[0]) / den
            s = -(e[0] * ap[1] - e[1] * ap[0]) / den
            if 0 <= t <= 1 and s > 0:
                ts.add(t)
    ts = sorted(ts)
    best = (math.inf, None)

    def pt(t):
        return (A[0] + t * e[0], A[1] + t * e[1])

    for t in ts:
        q = pt(t)
        if visible(polys, p, q, edges):
            d = _dist(p, q)
            if d < best[0]:
                best = (d, q)
    ee = e[0] * e[0] + e[1] * e[1]
    tp = ((p[0] - A[0]) * e[0] + (p[1] - A[1]) * e[1]) / ee
    for t0, t1 in zip(ts[:-1], ts[1:]):
        if not visible(polys, p, pt((t0 + t1) / 2), edges):
            continue
        tc = min(max(tp, t0), t1)
        q = pt(tc)
        d = _dist(p, q)
        if d < best[0]:
            best = (d, q)
    return best


class Mini:
    """Brute-force exact map for a tiny scene (a handful of obstacle vertices)."""

    def __init__(self, scene, max_vertices: int = 9):
        self.scene = scene
        self.polys = scene.polys
        self.E = _edges(self.polys)
        self.V = [(F(int(x)), F(int(y))) for P in self.polys for (x, y) in P]
        if len(self.V) > max_vertices:
            raise ValueError("mini oracle: too many vertices for path enumeration")
        self.points = [(F(int(x)), F(int(y))) for x, y in scene.points]
        self.segs = [tuple(int(v) for v in s) for s in scene.segs]
        nV = len(self.V)
        self.vis = [[i == j or visible(self.polys, self.V[i], self.V[j], self.E) for j in range(nV)]
                    for i in range(nV)]
        # first leg from any source to each vertex
        self.src_leg = []
        for v in self.V:
            best = math.inf
            for s in self.points:
                if visible(self.polys, s, v, self.E):
                    best = min(best, _dist(s, v))
            for sg in self.segs:
                best = min(best, segment_reach(self.polys, v, sg, self.E)[0])
            self.src_leg.append(best)
        self.cost = self._enumerate()

    def _enumerate(self):
        """cost(v) = min over every simple vertex sequence ending at v of its length."""
        nV = len(self.V)
        best = [math.inf] * nV
        idx = list(range(nV))
        for k in range(1, nV + 1):
            for seq in permutations(idx, k):
                if not math.isfinite(self.src_leg[seq[0]]):
                    continue
                ok = True
                L = self.src_leg[seq[0]]
                for a, b in zip(seq[:-1], seq[1:]):
                    if not self.vis[a][b]:
                        ok = False
                        break
                    L += _dist(self.V[a], self.V[b])
                if ok and L < best[seq[-1]]:
                    best[seq[-1]] = L
        return best

    def pixel(self, i, j):
        """(D, kind, where) for pixel (i, j): kind 'point'/'segment'/'vertex', where = index."""
        p = (F(2 * i + 1, 2), F(2 * j + 1, 2))
        if closed_inside(self.polys, p):
            return math.inf, None, None
        best = (math.inf, None, None)
        for k, s in enumerate(self.points):
            if visible(self.polys, p, s, self.E):
                d = _dist(p, s)
                if d < best[0]:
                    best = (d, "point", k)
        for k, sg in enumerate(self.segs):
            d = segment_reach(self.polys, p, sg, self.E)[0]
            if d < best[0]:
                best = (d, "segment", k)
        for k, v in enumerate(self.V):
            if not math.isfinite(self.cost[k]):
                continue
            if visible(self.polys, p, v, self.E):
                d = _dist(p, v) + self.cost[k]
                if d < best[0] - 1e-12:
                    best = (d, "vertex", k)
        return best

    def generator_value(self, i, j, kind, ref):
        """What one generator offers pixel (i, j) when it is a candidate on its own: cost + distance
        when the pixel centre sees the generator's nearest point, +inf otherwise.  kind is
        'point' / 'segment' / 'vertex' and ref its index among the points, segments or all obstacle
        vertices.  A segment's nearest point is the clamped projection of the centre onto the
        whole segment (one candidate per segment source), computed here in Fraction arithmetic."""
        p = (F(2 * i + 1, 2), F(2 * j + 1, 2))
        if closed_inside(self.polys, p):
            return math.inf
        if kind == "point":
            q, c = self.points[ref], 0.0
        elif kind == "segment":
            ax, ay, bx, by = (F(v) for v in self.segs[ref])
            e = (bx - ax, by - ay)
            t = ((p[0] - ax) * e[0] + (p[1] - ay) * e[1]) / (e[0] * e[0] + e[1] * e[1])
            t = min(max(t, F(0)), F(1))
            q, c = (ax + t * e[0], ay + t * e[1]), 0.0
        else:
            q, c = self.V[ref], self.cost[ref]
            if not math.isfinite(c):
                return math.inf
        if not visible(self.polys, p, q, self.E):
            return math.inf
        return c + _dist(p, q)

    def grid(self):
        W, H = self.scene.width, self.scene.height
        D = np.full((H, W), np.inf)
        for j in range(H):
            for i in range(W):
                D[j, i] = self.pixel(i, j)[0]
        return D
