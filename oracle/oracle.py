"""CPU oracle for shortest path maps -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  The product library neither imports nor links it, and it
imports nothing from the product package.

Thin ctypes wrapper over ``spm_oracle.c`` (plain C, exact integer predicates,
IEEE double distances).  See that file's header for what is computed and which
parts of the paper each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spm_oracle.c")
_LIB = os.path.join(_HERE, "libspm_oracle.so")

POINT, SEGMENT, VERTEX = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP) into oracle/libspm_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-variable",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _CScene(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int), ("height", ctypes.c_int), ("n_polys", ctypes.c_int),
        ("poly_start", ctypes.POINTER(ctypes.c_int)), ("vx", ctypes.POINTER(ctypes.c_int)),
        ("vy", ctypes.POINTER(ctypes.c_int)), ("n_points", ctypes.c_int),
        ("pts", ctypes.POINTER(ctypes.c_int)), ("n_segs", ctypes.c_int),
        ("segs", ctypes.POINTER(ctypes.c_int)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        sp = ctypes.POINTER(_CScene)
        L.orc_num_generators.argtypes = [sp]
        L.orc_generators.argtypes = [sp, ip, ip, ip]
        L.orc_visible.argtypes = [sp] + [ctypes.c_int64] * 6
        L.orc_costs.argtypes = [sp, dp, ip, dp, ctypes.c_int]
        L.orc_pixels.argtypes = [sp, dp, ctypes.c_int, i64p, fp, ip, dp, dp, ctypes.c_int]
        L.orc_inside.argtypes = [sp, ctypes.c_int, i64p, ctypes.POINTER(ctypes.c_ubyte)]
        L.orc_candidates.argtypes = [sp, dp, ctypes.c_int, i64p, ip, dp, ctypes.c_int]
        L.orc_points.argtypes = [sp, dp, ctypes.c_int, i64p, ctypes.c_int64, dp, ip, dp, ctypes.c_int]
        L.orc_max_threads.argtypes = []
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class _Bound:
    """Keeps the flat arrays alive for the lifetime of the C struct."""

    def __init__(self, scene):
        f = scene.flat()
        self.arrs = {k: np.ascontiguousarray(v, np.int32) for k, v in f.items() if k not in ("width", "height")}
        for k in ("pts", "segs", "vx", "vy"):
            if self.arrs[k].size == 0:
                self.arrs[k] = np.zeros(1, np.int32)
        a = self.arrs
        self.c = _CScene(int(f["width"]), int(f["height"]), len(f["poly_start"]) - 1,
                         _ptr(a["poly_start"], ctypes.c_int), _ptr(a["vx"], ctypes.c_int),
                         _ptr(a["vy"], ctypes.c_int), len(scene.points), _ptr(a["pts"], ctypes.c_int),
                         len(scene.segs), _ptr(a["segs"], ctypes.c_int))

    @property
    def ref(self):
        return ctypes.byref(self.c)


def max_threads() -> int:
    return int(_load().orc_max_threads())


def generators(scene):
    """Canonical generator table: (kind[G], ref[G], xy4[G,4]) in domain units."""
    L = _load()
    b = _Bound(scene)
    G = L.orc_num_generators(b.ref)
    kind = np.zeros(max(G, 1), np.int32)
    ref = np.zeros(max(G, 1), np.int32)
    xy = np.zeros((max(G, 1), 4), np.int32)
    L.orc_generators(b.ref, _ptr(kind, ctypes.c_int), _ptr(ref, ctypes.c_int), _ptr(xy, ctypes.c_int))
    return kind[:G], ref[:G], xy[:G]


def visible(scene, a, b) -> bool:
    """Closed-segment visibility; a, b = (X, Y, w) rational points in doubled coordinates."""
    L = _load()
    bd = _Bound(scene)
    return bool(L.orc_visible(bd.ref, int(a[0]), int(a[1]), int(a[2]), int(b[0]), int(b[1]), int(b[2])))


def costs(scene, weights: bool = False, nthreads: int = 0):
    """Generator costs (float64) and generator parents; optionally the GxG arc matrix."""
    L = _load()
    b = _Bound(scene)
    G = L.orc_num_generators(b.ref)
    cost = np.zeros(max(G, 1), np.float64)
    par = np.zeros(max(G, 1), np.int32)
    W = np.zeros((G, G), np.float64) if weights else None
    L.orc_costs(b.ref, _ptr(cost, ctypes.c_double), _ptr(par, ctypes.c_int),
                _ptr(W, ctypes.c_double) if weights else None, int(nthreads))
    if weights:
        return cost[:G], par[:G], W
    return cost[:G], par[:G]


def pixels(scene, cost, pix, nthreads: int = 0) -> dict:
    """Per-pixel minimum for the listed row-major pixel indices."""
    L = _load()
    b = _Bound(scene)
    pix = np.ascontiguousarray(np.asarray(pix, np.int64).reshape(-1))
    n = pix.size
    cost = np.ascontiguousarray(np.asarray(cost, np.float64))
    if cost.size == 0:
        cost = np.zeros(1, np.float64)
    d32 = np.zeros(max(n, 1), np.float32)
    par = np.zeros(max(n, 1), np.int32)
    d64 = np.zeros(max(n, 1), np.float64)
    sec = np.zeros(max(n, 1), np.float64)
    if n:
        L.orc_pixels(b.ref, _ptr(cost, ctypes.c_double), n, _ptr(pix, ctypes.c_int64),
                     _ptr(d32, ctypes.c_float), _ptr(par, ctypes.c_int), _ptr(d64, ctypes.c_double),
                     _ptr(sec, ctypes.c_double), int(nthreads))
    return {"dist": d32[:n], "parent": par[:n], "dist64": d64[:n], "second": sec[:n]}


def points(scene, cost, qxy, qw: int, nthreads: int = 0) -> dict:
    """Map value at rational points: qxy (n, 2) int64 numerators of doubled coordinates over qw
    (so domain x = qxy[k, 0] / (2 qw)).  Returns dist64, parent, second."""
    L = _load()
    b = _Bound(scene)
    q = np.ascontiguousarray(np.asarray(qxy, np.int64).reshape(-1, 2))
    n = q.shape[0]
    cost = np.ascontiguousarray(np.asarray(cost, np.float64))
    if cost.size == 0:
        cost = np.zeros(1, np.float64)
    d64 = np.zeros(max(n, 1), np.float64)
    par = np.zeros(max(n, 1), np.int32)
    sec = np.zeros(max(n, 1), np.float64)
    if n:
        L.orc_points(b.ref, _ptr(cost, ctypes.c_double), n, _ptr(q, ctypes.c_int64), int(qw),
                     _ptr(d64, ctypes.c_double), _ptr(par, ctypes.c_int), _ptr(sec, ctypes.c_double),
                     int(nthreads))
    return {"dist64": d64[:n], "parent": par[:n], "second": sec[:n]}


def candidates(scene, cost, pix, gen, nthreads: int = 0) -> np.ndarray:
    """cost(g) + |p - x_g(p)| for each (pixel pix[k], generator gen[k]) pair when the pixel
    centre sees x_g(p), +inf otherwise (float64)."""
    L = _load()
    b = _Bound(scene)
    pix = np.ascontiguousarray(np.asarray(pix, np.int64).reshape(-1))
    gen = np.ascontiguousarray(np.asarray(gen, np.int32).reshape(-1))
    assert pix.size == gen.size
    cost = np.ascontiguousarray(np.asarray(cost, np.float64))
    if cost.size == 0:
        cost = np.zeros(1, np.float64)
    out = np.zeros(max(pix.size, 1), np.float64)
    if pix.size:
        L.orc_candidates(b.ref, _ptr(cost, ctypes.c_double), pix.size, _ptr(pix, ctypes.c_int64),
                         _ptr(gen, ctypes.c_int), _ptr(out, ctypes.c_double), int(nthreads))
    return out[:pix.size]


def inside(scene, pix) -> np.ndarray:
    L = _load()
    b = _Bound(scene)
    pix = np.ascontiguousarray(np.asarray(pix, np.int64).reshape(-1))
    out = np.zeros(max(pix.size, 1), np.uint8)
    if pix.size:
        L.orc_inside(b.ref, pix.size, _ptr(pix, ctypes.c_int64), _ptr(out, ctypes.c_ubyte))
    return out[:pix.size].astype(bool)


def full_map(scene, nthreads: int = 0) -> dict:
    """The whole map: dist/parent/dist64/second as (H, W) arrays plus the generator costs."""
    cost, gpar = costs(scene, nthreads=nthreads)
    n = scene.width * scene.height
    r = pixels(scene, cost, np.arange(n, dtype=np.int64), nthreads=nthreads)
    shp = (scene.height, scene.width)
    out = {k: v.reshape(shp) for k, v in r.items()}
    out["cost"] = cost
    out["gparent"] = gpar
    return out
