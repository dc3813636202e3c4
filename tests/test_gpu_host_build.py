"""spm_build from host scenes (validated, staged through pinned memory) against the device-scene
build spm_build_ex, bit for bit."""
import sys

import numpy as np
import pytest

from scenegen import Scene, config1, config2, config3, random_small

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


def _copy(scene):
    return Scene(scene.width, scene.height, [p.copy() for p in scene.polys], scene.points.copy(), scene.segs.copy())


def _same(a, b):
    for k in ("dist", "parent", "gen_kind", "gen_xy", "gen_cost", "gen_parent"):
        assert np.array_equal(a[k], b[k]), k
    assert a["n_gen"] == b["n_gen"]


def test_host_build_matches_device_build(spm):
    import torch
    scenes = [config2(1), config1(2), random_small(3), Scene(37, 23, [], np.asarray([[5, 9]]), None), config3(2)]
    for sc in scenes:
        _say(f"[host-build] {sc.width}x{sc.height} V={sc.n_vertices}")
        ds = spm.DeviceScene(sc)
        a = spm.Builder(ds)
        a.build()
        b = spm.Builder(ds)
        tmp = _copy(sc)
        b.build_host(tmp)
        del tmp                      # the library staged its own copy before returning
        torch.cuda.synchronize()
        _same(a.map.host(), b.map.host())


def test_host_builds_cycle_the_staging_ring(spm):
    """More host builds in flight than staging slots, scenes of different sizes, no synchronisation
    in between: every map equals its device-scene build."""
    import torch
    scenes = [random_small(s) for s in range(40, 50)] + [config2(2)]
    ref, builders = [], []
    for sc in scenes:
        ds = spm.DeviceScene(sc)
        a = spm.Builder(ds)
        a.build()
        torch.cuda.synchronize()
        ref.append(a.map.host())
        builders.append(spm.Builder(ds))
    for rep in range(2):
        for b, sc in zip(builders, scenes):
            b.build_host(_copy(sc))
        torch.cuda.synchronize()
        for k, b in enumerate(builders):
            _same(ref[k], b.map.host())


def test_host_build_refuses_capture(spm):
    import torch
    from paper_1805_08500_amd._lib import SpmError, SPM_ERR_INVALID_ARG
    sc = random_small(7)
    b = spm.Builder(spm.DeviceScene(sc))
    x = torch.zeros(16, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    code = None
    with torch.cuda.graph(g, stream=s):
        x.add_(1.0)
        try:
            b.build_host(sc, stream=s)
        except SpmError as e:
            code = e.code
    assert code == SPM_ERR_INVALID_ARG
    g.replay()
    torch.cuda.synchronize()
    assert float(x[0]) == 1.0
