"""ctypes declarations for libspm.so (the C ABI in include/spm.h).

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspm.so")

SPM_OK = 0
SPM_ERR_INVALID_ARG = -1
SPM_ERR_GEOMETRY = -2
SPM_ERR_RANGE = -3
SPM_ERR_CAPACITY = -4
SPM_ERR_HIP = -5
SPM_ERR_UNREACHABLE = -6
SPM_N_STAGES = 8
SPM_MAX_SIDE = 8192
SPM_NOALLOC_MAX_WS = 16 << 20
SPM_N_STATS = 16
GEN_POINT, GEN_SEGMENT, GEN_VERTEX = 0, 1, 2

STAGES = ("ingest", "edge_sort", "gorder", "genvis", "relax", "gsort", "pixel", "total")

c_i32 = ctypes.c_int32
c_vp = ctypes.c_void_p


class SpmScene(ctypes.Structure):
    _fields_ = [("width", c_i32), ("height", c_i32), ("n_polys", c_i32), ("n_vertices", c_i32),
                ("n_points", c_i32), ("n_segs", c_i32), ("poly_start", c_vp), ("vx", c_vp), ("vy", c_vp),
                ("pts", c_vp), ("segs", c_vp)]


class SpmOut(ctypes.Structure):
    _fields_ = [("dist", c_vp), ("parent", c_vp), ("gen_kind", c_vp), ("gen_xy", c_vp), ("gen_cost", c_vp),
                ("gen_parent", c_vp), ("n_gen", c_vp)]


class SpmBuildOpts(ctypes.Structure):
    _fields_ = [("tile_w", c_i32), ("tile_h", c_i32), ("timer", c_vp), ("d_stats", c_vp), ("strip", c_i32),
                ("samples", c_i32), ("walk", c_i32)]


class SpmBatch(ctypes.Structure):
    _fields_ = [("n", c_i32), ("scenes", ctypes.POINTER(SpmScene)), ("outs", ctypes.POINTER(SpmOut)),
                ("tile_w", ctypes.POINTER(c_i32)), ("pixel_waves", c_i32), ("walk", c_i32)]


class SpmMapHost(ctypes.Structure):
    _fields_ = [("width", c_i32), ("height", c_i32), ("parent", c_vp), ("n_gen", c_i32), ("gen_kind", c_vp),
                ("gen_xy", c_vp), ("gen_parent", c_vp), ("gen_cost", c_vp)]


_lib = None


def lib():
    """Load libspm.so once.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1805_08500_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sp = ctypes.POINTER(SpmScene)
    op = ctypes.POINTER(SpmOut)
    P = ctypes.POINTER
    L.spm_last_error.restype = ctypes.c_char_p
    L.spm_last_error.argtypes = []
    L.spm_validate.argtypes = [sp]
    L.spm_query_sizes.argtypes = [sp, P(c_i32), P(ctypes.c_size_t)]
    L.spm_build.argtypes = [sp, op, c_vp, ctypes.c_size_t, c_vp]
    L.spm_build_ex.argtypes = [sp, op, c_vp, ctypes.c_size_t, c_vp, P(SpmBuildOpts)]
    L.spm_build_noalloc.argtypes = [sp, op, c_vp]
    L.spm_timer_create.argtypes = [P(c_vp)]
    L.spm_timer_destroy.argtypes = [c_vp]
    L.spm_timer_reset.argtypes = [c_vp]
    L.spm_timer_elapsed.argtypes = [c_vp, P(ctypes.c_float), P(c_i32)]
    L.spm_query_path.argtypes = [P(SpmMapHost), ctypes.c_float, ctypes.c_float, P(ctypes.c_float), c_i32,
                                 P(c_i32), P(ctypes.c_float)]
    fpp = P(ctypes.c_float)
    L.spm_agent_query_ws.argtypes = [sp, c_i32, P(ctypes.c_size_t)]
    L.spm_agent_distance.argtypes = [sp, op, c_i32, c_vp, c_vp, c_vp]
    L.spm_query_points.argtypes = [sp, op, c_i32, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp]
    L.spm_backward.argtypes = [sp, op, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]
    bp = P(SpmBatch)
    L.spm_batch_query_sizes.argtypes = [bp, P(ctypes.c_size_t)]
    L.spm_batch_prepare.argtypes = [bp, c_vp, ctypes.c_size_t]
    L.spm_build_batch.argtypes = [bp, c_vp, ctypes.c_size_t, c_vp, c_vp]
    L.spm_graph_capture_batch.argtypes = [bp, c_vp, ctypes.c_size_t, c_vp, P(c_vp)]
    L.spm_graph_launch.argtypes = [c_vp, c_vp]
    L.spm_graph_destroy.argtypes = [c_vp]
    for name in ("spm_validate", "spm_query_sizes", "spm_build", "spm_build_ex", "spm_build_noalloc", "spm_timer_create",
                 "spm_timer_destroy", "spm_timer_reset", "spm_timer_elapsed", "spm_query_path",
                 "spm_batch_query_sizes", "spm_batch_prepare", "spm_build_batch", "spm_graph_capture_batch",
                 "spm_graph_launch", "spm_graph_destroy", "spm_agent_query_ws", "spm_agent_distance",
                 "spm_backward"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class SpmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libspm error {code}: {msg}")
        self.code = code


def check(rc: int) -> None:
    if rc != SPM_OK:
        raise SpmError(rc, lib().spm_last_error().decode(errors="replace"))
