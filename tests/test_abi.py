"""CPU-only checks of the C ABI: symbols, host validation errors, sizes, path queries.

Nothing here launches device work: every call either is host-only
(spm_validate, spm_query_sizes, spm_query_path, spm_last_error) or fails its
argument checks before any HIP call.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from scenegen import Scene, config1, config2, random_small
from scenegen.scenes import _rect_poly

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def C():
    from paper_1805_08500_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import importlib
        importlib.import_module("paper_1805_08500_amd.build").build()
    _lib.lib()
    return _lib


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "spm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spm_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(C):
    names = _declared_functions()
    assert len(names) >= 10
    L = ctypes.CDLL(C.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_validate_accepts_generated_scenes(C):
    from paper_1805_08500_amd import validate
    validate(config1(1))
    validate(config2(1))
    for s in range(12):
        validate(random_small(s))


def _code(scene):
    from paper_1805_08500_amd import validate
    from paper_1805_08500_amd._lib import SpmError
    try:
        validate(scene)
    except SpmError as e:
        return e.code
    return 0


def test_validate_error_codes(C):
    ok = Scene(40, 40, [_rect_poly(10, 10, 20, 20)], np.asarray([[2, 2]]), None)
    assert _code(ok) == 0
    cw = Scene(40, 40, [_rect_poly(10, 10, 20, 20)[::-1]], np.asarray([[2, 2]]), None)
    assert _code(cw) == C.SPM_ERR_GEOMETRY
    overlap = Scene(40, 40, [_rect_poly(10, 10, 20, 20), _rect_poly(20, 12, 30, 18)], np.asarray([[2, 2]]), None)
    assert _code(overlap) == C.SPM_ERR_GEOMETRY              # touching counts as meeting
    nested = Scene(40, 40, [_rect_poly(5, 5, 35, 35), _rect_poly(10, 10, 20, 20)], np.asarray([[2, 2]]), None)
    assert _code(nested) == C.SPM_ERR_GEOMETRY
    bowtie = Scene(40, 40, [np.asarray([(10, 10), (20, 20), (20, 10), (10, 20)])], np.asarray([[2, 2]]), None)
    assert _code(bowtie) == C.SPM_ERR_GEOMETRY
    collinear = Scene(40, 40, [np.asarray([(10, 10), (15, 10), (20, 10), (20, 20), (10, 20)])], np.asarray([[2, 2]]),
                      None)
    assert _code(collinear) == C.SPM_ERR_GEOMETRY
    src_in = Scene(40, 40, [_rect_poly(10, 10, 20, 20)], np.asarray([[15, 15]]), None)
    assert _code(src_in) == C.SPM_ERR_GEOMETRY
    src_on = Scene(40, 40, [_rect_poly(10, 10, 20, 20)], np.asarray([[10, 15]]), None)
    assert _code(src_on) == C.SPM_ERR_GEOMETRY
    seg_hit = Scene(40, 40, [_rect_poly(10, 10, 20, 20)], None, np.asarray([[0, 15, 30, 15]]))
    assert _code(seg_hit) == C.SPM_ERR_GEOMETRY
    seg_zero = Scene(40, 40, [], None, np.asarray([[3, 3, 3, 3]]))
    assert _code(seg_zero) == C.SPM_ERR_GEOMETRY
    out_of_range = Scene(40, 40, [_rect_poly(10, 10, 50, 20)], np.asarray([[2, 2]]), None)
    assert _code(out_of_range) == C.SPM_ERR_RANGE
    too_big = Scene(9000, 10, [], np.asarray([[2, 2]]), None)
    assert _code(too_big) == C.SPM_ERR_RANGE
    no_source = Scene(40, 40, [_rect_poly(10, 10, 20, 20)], None, None)
    assert _code(no_source) == C.SPM_ERR_INVALID_ARG


def test_query_sizes_and_bad_counts(C):
    from paper_1805_08500_amd import query_sizes
    from paper_1805_08500_amd._lib import SpmError
    mg, ws = query_sizes(1024, 1024, 60, 336, 3, 2)
    assert mg == 341 and ws > 0
    mg2, ws2 = query_sizes(2048, 2048, 60, 336, 3, 2)
    assert ws2 > ws
    with pytest.raises(SpmError) as e:
        query_sizes(0, 10, 0, 0, 1, 0)
    assert e.value.code == C.SPM_ERR_RANGE
    with pytest.raises(SpmError) as e:
        query_sizes(10, 10, 1, 2, 1, 0)
    assert e.value.code == C.SPM_ERR_INVALID_ARG


def test_build_rejects_null_arguments_before_device_work(C):
    L = C.lib()
    s = C.SpmScene(10, 10, 0, 0, 1, 0, None, None, None, None, None)
    out = C.SpmOut()
    rc = L.spm_build(ctypes.byref(s), ctypes.byref(out), None, 0, None)
    assert rc == C.SPM_ERR_INVALID_ARG          # pts NULL with one point
    assert b"NULL" in L.spm_last_error()
    pts = (ctypes.c_int32 * 2)(1, 1)
    s.pts = ctypes.cast(pts, ctypes.c_void_p)
    rc = L.spm_build(ctypes.byref(s), ctypes.byref(out), None, 0, None)
    assert rc == C.SPM_ERR_INVALID_ARG          # outputs NULL
    rc = L.spm_build(None, ctypes.byref(out), None, 0, None)
    assert rc == C.SPM_ERR_INVALID_ARG


def test_host_build_error_codes_before_device_work(C):
    """spm_build takes a host scene and runs every check that can fail before any HIP call: each
    error code below comes back with the workspace and outputs never touched (their addresses are
    fake).  The HIP error is forced by the missing device, so that case only runs without a GPU."""
    from paper_1805_08500_amd.spm import _host_scene_struct
    L = C.lib()
    fake = 4096
    out = C.SpmOut(fake, fake, fake, fake, fake, fake, fake)
    big = ctypes.c_size_t(1 << 40)

    def rc_of(scene, ws=fake, nbytes=big, o=out):
        keep = []
        hs = _host_scene_struct(scene.flat(), keep)
        return L.spm_build(ctypes.byref(hs), ctypes.byref(o) if o is not None else None,
                           ctypes.c_void_p(ws) if ws else None, nbytes, None)

    ok = Scene(40, 40, [_rect_poly(10, 10, 20, 20)], np.asarray([[2, 2]]), np.asarray([[25, 30, 35, 22]]))
    cases = [
        (lambda: rc_of(ok, o=None), C.SPM_ERR_INVALID_ARG, b"NULL"),
        (lambda: rc_of(ok, o=C.SpmOut()), C.SPM_ERR_INVALID_ARG, b"NULL"),
        (lambda: rc_of(ok, ws=0), C.SPM_ERR_INVALID_ARG, b"workspace"),
        (lambda: rc_of(ok, nbytes=ctypes.c_size_t(100)), C.SPM_ERR_CAPACITY, b"needs"),
        (lambda: rc_of(Scene(40, 40, [_rect_poly(10, 10, 20, 20)[::-1]], np.asarray([[2, 2]]), None)),
         C.SPM_ERR_GEOMETRY, b"counter-clockwise"),
        (lambda: rc_of(Scene(40, 40, [_rect_poly(10, 10, 20, 20)], np.asarray([[15, 15]]), None)),
         C.SPM_ERR_GEOMETRY, b"inside"),
        (lambda: rc_of(Scene(40, 40, [_rect_poly(10, 10, 20, 20)], None, np.asarray([[0, 15, 30, 15]]))),
         C.SPM_ERR_GEOMETRY, b"meets"),
        (lambda: rc_of(Scene(40, 40, [_rect_poly(10, 10, 50, 20)], np.asarray([[2, 2]]), None)),
         C.SPM_ERR_RANGE, b"outside"),
        (lambda: rc_of(Scene(40, 40, [_rect_poly(10, 10, 20, 20)], np.asarray([[2, 41]]), None)),
         C.SPM_ERR_RANGE, b"outside"),
        (lambda: rc_of(Scene(9000, 40, [], np.asarray([[2, 2]]), None)), C.SPM_ERR_RANGE, b"outside"),
        (lambda: rc_of(Scene(40, 40, [_rect_poly(10, 10, 20, 20)], None, None)), C.SPM_ERR_INVALID_ARG, b"source"),
    ]
    for k, (call, code, what) in enumerate(cases):
        assert call() == code, (k, L.spm_last_error())
        assert what in L.spm_last_error(), (k, L.spm_last_error())
    import torch
    if not torch.cuda.is_available():
        assert rc_of(ok) == C.SPM_ERR_HIP, L.spm_last_error()


def test_build_rejects_bad_walk_before_device_work(C):
    """The walk option is checked on the host, before any device pointer is touched."""
    L = C.lib()
    n = 600   # point sources: up to 600 generators
    pts = (ctypes.c_int32 * (2 * n))(*([1, 1] * n))
    s = C.SpmScene(10, 10, 0, 0, n, 0, None, None, None, None, None)
    s.pts = ctypes.cast(pts, ctypes.c_void_p)
    fake = 4096   # never dereferenced: every check below fails first
    out = C.SpmOut(fake, fake, fake, fake, fake, fake, fake)
    for walk, what in [(7, b"outside"), (-1, b"outside"), (1, b"at most 512")]:
        opts = C.SpmBuildOpts(0, 0, None, None, 0, 0, walk)
        rc = L.spm_build_ex(ctypes.byref(s), ctypes.byref(out), ctypes.c_void_p(fake), ctypes.c_size_t(1 << 40), None,
                            ctypes.byref(opts))
        assert rc == C.SPM_ERR_INVALID_ARG, walk
        assert what in L.spm_last_error(), L.spm_last_error()


def _oracle_host_map(O, scene):
    m = O.full_map(scene)
    kind, ref, xy = O.generators(scene)
    return m, {"parent": m["parent"], "n_gen": len(kind), "gen_kind": kind, "gen_xy": xy,
               "gen_parent": m["gparent"], "gen_cost": m["cost"]}


def test_query_path_chain_invariants(oracle_mod, C):
    from paper_1805_08500_amd import query_path
    from paper_1805_08500_amd._lib import SpmError
    scene = random_small(4)
    m, hm = _oracle_host_map(oracle_mod, scene)
    H, W = m["dist"].shape
    checked = 0
    for j in range(0, H, 3):
        for i in range(0, W, 3):
            if not np.isfinite(m["dist64"][j, i]):
                with pytest.raises(SpmError) as e:
                    query_path(hm, i + 0.5, j + 0.5)
                assert e.value.code == C.SPM_ERR_UNREACHABLE
                continue
            pts, L = query_path(hm, i + 0.5, j + 0.5)
            assert abs(L - m["dist64"][j, i]) <= 1e-4 * max(1.0, m["dist64"][j, i])
            # every leg is visible
            for a, b in zip(pts[:-1], pts[1:]):
                ha = (int(round(2 * a[0] * 1024)), int(round(2 * a[1] * 1024)), 1024)
                hb = (int(round(2 * b[0] * 1024)), int(round(2 * b[1] * 1024)), 1024)
                if np.all(np.abs(np.asarray(a) * 1024 - np.round(np.asarray(a) * 1024)) < 1e-3) and \
                        np.all(np.abs(np.asarray(b) * 1024 - np.round(np.asarray(b) * 1024)) < 1e-3):
                    assert oracle_mod.visible(scene, ha, hb)
            checked += 1
    assert checked > 20


def test_query_path_errors(oracle_mod, C):
    from paper_1805_08500_amd import query_path
    from paper_1805_08500_amd._lib import SpmError
    scene = config1(1)
    m, hm = _oracle_host_map(oracle_mod, scene)
    with pytest.raises(SpmError) as e:
        query_path(hm, -1.0, 3.0)
    assert e.value.code == C.SPM_ERR_RANGE
    j, i = np.argwhere(np.isfinite(m["dist64"]))[0]
    with pytest.raises(SpmError) as e:
        query_path(hm, i + 0.5, j + 0.5, cap=1)
    assert e.value.code == C.SPM_ERR_CAPACITY


def test_batch_argument_errors(C):
    L = C.lib()
    rc = L.spm_batch_query_sizes(None, None)
    assert rc == C.SPM_ERR_INVALID_ARG
    sc = (C.SpmScene * 1)(C.SpmScene(10, 10, 0, 0, 1, 0, None, None, None, None, None))
    outs = (C.SpmOut * 1)()
    b = C.SpmBatch(1, sc, outs, None)
    assert L.spm_batch_query_sizes(ctypes.byref(b), None) == C.SPM_ERR_INVALID_ARG   # pts NULL
    pts = (ctypes.c_int32 * 2)(1, 1)
    sc[0].pts = ctypes.cast(pts, ctypes.c_void_p)
    assert L.spm_batch_query_sizes(ctypes.byref(b), None) == C.SPM_ERR_INVALID_ARG   # outputs NULL
    fake = ctypes.c_void_p(16)
    outs[0] = C.SpmOut(fake, fake, fake, fake, fake, fake, fake)
    ws = ctypes.c_size_t(0)
    assert L.spm_batch_query_sizes(ctypes.byref(b), ctypes.byref(ws)) == C.SPM_OK and ws.value > 0
    tiles = (ctypes.c_int32 * 1)(5)
    b.tile_w = tiles
    assert L.spm_batch_query_sizes(ctypes.byref(b), ctypes.byref(ws)) == C.SPM_ERR_INVALID_ARG
    b.tile_w = None
    assert L.spm_batch_prepare(ctypes.byref(b), None, 0) == C.SPM_ERR_INVALID_ARG
    assert L.spm_build_batch(ctypes.byref(b), fake, 1, None, None) == C.SPM_ERR_CAPACITY
    g = ctypes.c_void_p()
    assert L.spm_graph_capture_batch(ctypes.byref(b), fake, 1, None, ctypes.byref(g)) == C.SPM_ERR_INVALID_ARG



def test_build_entry_reaches_the_build_module():
    """__graft_entry__.build() must call the compiler module, not the package's build() function of
    the same name.  Runs in a fresh interpreter (where the package attribute is still the function)
    with both compilers replaced by stub modules: nothing is compiled."""
    import subprocess
    import sys
    script = (
        "import sys, types\n"
        "calls = []\n"
        "b = types.ModuleType('paper_1805_08500_amd.build')\n"
        "b.build = lambda verbose=False: calls.append(('lib', verbose))\n"
        "o = types.ModuleType('oracle.oracle')\n"
        "o.build = lambda force=False: calls.append(('oracle', force))\n"
        "sys.modules['paper_1805_08500_amd.build'] = b\n"
        "sys.modules['oracle.oracle'] = o\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import __graft_entry__\n"
        "__graft_entry__.build()\n"
        "assert calls == [('lib', True), ('oracle', True)], calls\n"
        "print('ok')\n"
    )
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-2000:]


def test_source_update_is_validated_before_rebuilding(C):
    """SPMDistance rebuilds through spm_build, whose host validation refuses a source moved onto or
    into an obstacle, out of the domain, or a segment made to touch an obstacle or shrink to a
    point; the builder keeps its scene.  (The builder here holds host buffers, which is enough to
    reach those checks; with no GPU a valid update fails at the first HIP call instead.)"""
    import torch
    import paper_1805_08500_amd as spm
    from paper_1805_08500_amd._lib import SpmError
    scene = Scene(40, 40, [_rect_poly(10, 10, 20, 20)], np.asarray([[2, 2], [30, 5]]),
                  np.asarray([[25, 30, 35, 22]]))
    b = spm.Builder(spm.DeviceScene(scene, device="cpu"))
    agents = torch.tensor([[5.5, 5.5]])
    segs = torch.tensor([[25.0, 30.0, 35.0, 22.0]])
    pts = torch.tensor([[2.0, 2.0], [30.0, 5.0]])
    bad = [
        (torch.tensor([[15.2, 14.9], [30.0, 5.0]]), segs, C.SPM_ERR_GEOMETRY),    # into the obstacle
        (torch.tensor([[10.4, 13.0], [30.0, 5.0]]), segs, C.SPM_ERR_GEOMETRY),    # rounds onto its edge
        (torch.tensor([[-0.7, 2.0], [30.0, 5.0]]), segs, C.SPM_ERR_RANGE),        # out of the domain
        (pts, torch.tensor([[5.0, 15.0, 30.0, 15.0]]), C.SPM_ERR_GEOMETRY),       # segment through it
        (pts, torch.tensor([[25.0, 30.0, 25.2, 29.9]]), C.SPM_ERR_GEOMETRY),      # segment of length 0
    ]
    for k, (p, s, code) in enumerate(bad):
        with pytest.raises(SpmError) as e:
            spm.SPMDistance.apply(p, s, agents, b)
        assert e.value.code == code, (k, str(e.value))
        assert np.array_equal(b.ds.scene.points, scene.points) and np.array_equal(b.ds.scene.segs, scene.segs)
    if not torch.cuda.is_available():
        with pytest.raises(SpmError) as e:
            spm.SPMDistance.apply(torch.tensor([[3.2, 2.0], [30.0, 5.0]]), segs, agents, b)
        assert e.value.code == C.SPM_ERR_HIP
        assert np.array_equal(b.ds.scene.points, scene.points)
