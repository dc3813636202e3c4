"""spm_build_noalloc (the library's static device workspace, for callers that cannot allocate)
against spm_build_ex with a caller workspace, through the C ABI."""
import ctypes
import sys

import numpy as np
import pytest

from scenegen import Scene, config1, config2, config3
from scenegen.scenes import _rect_poly

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_08500_amd as m
    return m


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(spm, scene):
    import torch
    ds = spm.DeviceScene(scene)
    a = spm.Builder(ds)
    a.build()
    torch.cuda.synchronize()
    return ds, a.map.host()


def _check(ref, got, label):
    for k in ("dist", "parent", "gen_kind", "gen_xy", "gen_cost", "gen_parent"):
        assert np.array_equal(ref[k], got[k]), (label, k)
    assert ref["n_gen"] == got["n_gen"], label


def test_noalloc_matches_workspace_build_twice(spm):
    """Two calls in a row, the second with a smaller scene: both equal the caller-workspace build bit
    for bit (the static workspace keeps the first call's contents, which the second must not see)."""
    import torch
    for label, scene in (("convex1024-s1", config2(1)), ("rect256-s1", config1(1))):
        _say(f"[noalloc] {label}")
        ds, ref = _pair(spm, scene)
        b = spm.Builder(ds)
        b.map.dist.fill_(-5.0)
        b.map.parent.fill_(-9)
        b.build_noalloc()
        torch.cuda.synchronize()
        _check(ref, b.map.host(), label)


def test_noalloc_largest_config_and_repeat(spm):
    """The 2048 x 2048 maze fits the static workspace; repeated calls on one stream stay exact."""
    import torch
    ds, ref = _pair(spm, config3(1))
    b = spm.Builder(ds)
    for rep in range(2):
        _say(f"[noalloc] maze rep {rep}")
        b.build_noalloc()
        torch.cuda.synchronize()
        _check(ref, b.map.host(), f"maze-{rep}")


def test_noalloc_rejects_oversized_scene(spm):
    from paper_1805_08500_amd._lib import SpmError, SPM_ERR_CAPACITY, SPM_NOALLOC_MAX_WS
    scene = Scene(4096, 4096, [_rect_poly(100, 100, 200, 300)], np.asarray([[5, 5]]), None)
    ds = spm.DeviceScene(scene)
    b = spm.Builder(ds)
    assert b.ws_bytes > SPM_NOALLOC_MAX_WS
    with pytest.raises(SpmError) as e:
        b.build_noalloc()
    assert e.value.code == SPM_ERR_CAPACITY
