"""GPU parity: libspm (through its C ABI) against the CPU oracle, element by element."""
import sys

import numpy as np
import pytest

from scenegen import Scene, config1, config2, config3, profiling_grid, random_small
from scenegen.scenes import _rect_poly
from tests.samples import wide_sample
from tests.spm_compare import compare, compare_generators

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


def _gpu(spm, scene, tile=(8, 8)):
    import torch
    b = spm.Builder(spm.DeviceScene(scene), tile=tile)
    b.build()
    torch.cuda.synchronize()
    return b.map.host()


def _full(O, spm, scene, label, tile=(8, 8), max_ambiguous=0.05):
    _say(f"[parity] {label} {scene.width}x{scene.height} V={scene.n_vertices} tile={tile}")
    h = _gpu(spm, scene, tile)
    cost, gpar, wts = O.costs(scene, weights=True)
    ref = O.full_map(scene)
    st = compare(h["dist"], h["parent"], ref, label, O=O, scene=scene, cost=cost,
                 pix=np.arange(scene.width * scene.height), max_ambiguous=max_ambiguous)
    gs = compare_generators(h, cost, gpar, wts, label)
    _say(f"[parity] {label} ok ambiguous={st['ambiguous_frac']:.2e} alternatives={st['parent_alternatives']} "
         f"gen_parent_ties={gs['parent_ties']} max_rel={st['max_rel']:.2e}")
    return h, ref


def _sampled(O, spm, scene, label, pix, max_ambiguous, costs=None):
    """costs: the oracle's costs(scene, weights=True), when the caller already has them."""
    h = _gpu(spm, scene)
    if costs is None:
        _say(f"[parity] {label}: oracle costs")
        costs = O.costs(scene, weights=True)
    c, gpar, wts = costs
    gs = compare_generators(h, c, gpar, wts, label)
    _say(f"[parity] {label}: oracle on {pix.size} pixels")
    r = O.pixels(scene, c, pix)
    st = compare(h["dist"].reshape(-1)[pix], h["parent"].reshape(-1)[pix], r, label, O=O, scene=scene, cost=c,
                 pix=pix, max_ambiguous=max_ambiguous)
    _say(f"[parity] {label} ok pixels={pix.size} ambiguous={st['ambiguous_frac']:.2e} "
         f"alternatives={st['parent_alternatives']} gen_parent_ties={gs['parent_ties']} max_rel={st['max_rel']:.2e}")
    return h, st


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_config1_full(oracle_mod, spm, seed):
    _full(oracle_mod, spm, config1(seed), f"rect256-s{seed}", max_ambiguous=0.02)


@pytest.mark.parametrize("seed", range(0, 48))
def test_fuzz_small_full(oracle_mod, spm, seed):
    _full(oracle_mod, spm, random_small(seed), f"fuzz-{seed}", max_ambiguous=0.05)


def test_config2_full_seed1(oracle_mod, spm):
    _full(oracle_mod, spm, config2(1), "convex1024-s1", max_ambiguous=0.05)


@pytest.mark.parametrize("seed", [2, 3])
def test_config2_sampled(oracle_mod, spm, seed):
    scene = config2(seed)
    rng = np.random.default_rng(seed)
    pix = np.unique(rng.integers(0, scene.width * scene.height, 60000))
    _sampled(oracle_mod, spm, scene, f"convex1024-s{seed}", pix, max_ambiguous=0.05)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_config3_maze_wide(oracle_mod, spm, seed):
    """The 2048 x 2048 maze: three whole pixel rows, a 96 x 96 block around the costliest corner
    and 18000 random pixels (about 33000 in all) per seed."""
    scene = config3(seed)
    _say(f"[parity] maze2048-s{seed}: oracle costs")
    costs = oracle_mod.costs(scene, weights=True)
    pix = wide_sample(scene, costs[0], seed, 18000)
    _sampled(oracle_mod, spm, scene, f"maze2048-s{seed}", pix, max_ambiguous=0.08, costs=costs)


@pytest.mark.parametrize("k,seed", [(2, 0), (8, 1), (20, 2)])
def test_profiling_grid_sampled(oracle_mod, spm, k, seed):
    """The Profiling-style sweep maps (1000 x 1000, k x k squares, one random source)."""
    scene = profiling_grid(k, seed=seed)
    rng = np.random.default_rng(k)
    pix = np.unique(rng.integers(0, scene.width * scene.height, 40000))
    _sampled(oracle_mod, spm, scene, f"profiling-{k}x{k}-s{seed}", pix, max_ambiguous=0.08)


@pytest.mark.parametrize("k,side,seed", [(6, 192, 1), (12, 384, 2)])
def test_lattice_grid_full(oracle_mod, spm, k, side, seed):
    """Squares on a lattice: lines from pixel centres to corners often pass exactly through other
    corners, so the full visibility test's exact vertex rule decides many pixels.  The 12 x 12 map
    (577 generators) runs the refilled walk with its edges, boxes and costs staged in LDS."""
    _full(oracle_mod, spm, profiling_grid(k, side=side, seed=seed), f"lattice-{k}x{k}-{side}-s{seed}",
          max_ambiguous=0.08)


@pytest.mark.parametrize("tile", [(16, 4), (4, 16)])
def test_tile_shapes_bitwise(spm, tile):
    scene = config2(1)
    a = _gpu(spm, scene, (8, 8))
    b = _gpu(spm, scene, tile)
    assert np.array_equal(a["dist"], b["dist"]) and np.array_equal(a["parent"], b["parent"])


@pytest.mark.parametrize("make,walks", [(lambda: config2(1), (1, 2, 3, 4)), (lambda: profiling_grid(20, seed=2), (2, 3, 4)),
                                        (lambda: random_small(5), (1, 2, 3, 4)), (lambda: config3(1), (2, 3, 4)),
                                        (lambda: config3(3), (3, 4))])
def test_walk_modes_bitwise(spm, make, walks):
    """Every walk of the pixel stage gives the same map bit for bit (the (value, position) order decides)."""
    import torch
    scene = make()
    ds = spm.DeviceScene(scene)
    ref = None
    for w in (0,) + tuple(walks):
        b = spm.Builder(ds, walk=w)
        b.build()
        torch.cuda.synchronize()
        h = b.map.host()
        _say(f"[parity] walk {w} {scene.width}x{scene.height} G={h['n_gen']}")
        if ref is None:
            ref = h
        else:
            assert np.array_equal(ref["dist"], h["dist"]) and np.array_equal(ref["parent"], h["parent"]), f"walk {w}"


def test_deterministic(spm):
    scene = config2(2)
    a = _gpu(spm, scene)
    b = _gpu(spm, scene)
    for k in ("dist", "parent", "gen_cost", "gen_parent"):
        assert np.array_equal(a[k], b[k]), k


def test_edge_cases(oracle_mod, spm):
    cases = [
        ("free-point", Scene(37, 23, [], np.asarray([[5, 9]]), None)),
        ("free-segment", Scene(29, 31, [], None, np.asarray([[3, 3, 27, 20]]))),
        ("one-pixel", Scene(1, 1, [], np.asarray([[0, 0]]), None)),
        ("thin-strip", Scene(200, 3, [_rect_poly(50, 1, 60, 2)], np.asarray([[0, 0]]), None)),
        ("walled-off", Scene(40, 40, [np.asarray([(10, 0), (12, 0), (12, 40), (10, 40)])],
                              np.asarray([[2, 20]]), None)),
        ("pixel-on-segment", Scene(20, 20, [_rect_poly(12, 12, 16, 16)], None, np.asarray([[0, 0, 10, 10]]))),
        ("diagonal-edge", Scene(24, 24, [np.asarray([(4, 4), (14, 4), (14, 14)])], np.asarray([[20, 2]]), None)),
    ]
    # the strip behind its block is a near-tie almost everywhere: the routes above and below are mirror images
    bound = {"thin-strip": 0.2}
    for name, sc in cases:
        _full(oracle_mod, spm, sc, name, max_ambiguous=bound.get(name, 0.05))


def test_edge_cases_every_walk_bitwise(spm):
    """The edge-case scenes (ragged tiles, a single pixel, an empty cache, a source on the map's border,
    unreachable pixels) with every walk of the pixel stage forced: the same map bit for bit."""
    import torch
    cases = [
        Scene(37, 23, [], np.asarray([[5, 9]]), None),
        Scene(29, 31, [], None, np.asarray([[3, 3, 27, 20]])),
        Scene(1, 1, [], np.asarray([[0, 0]]), None),
        Scene(200, 3, [_rect_poly(50, 1, 60, 2)], np.asarray([[0, 0]]), None),
        Scene(40, 40, [np.asarray([(10, 0), (12, 0), (12, 40), (10, 40)])], np.asarray([[2, 20]]), None),
        Scene(20, 20, [_rect_poly(12, 12, 16, 16)], None, np.asarray([[0, 0, 10, 10]])),
        Scene(24, 24, [np.asarray([(4, 4), (14, 4), (14, 14)])], np.asarray([[20, 2]]), None),
        random_small(11, "blocks"),
    ]
    for sc in cases:
        ds = spm.DeviceScene(sc)
        ref = None
        for w in (0, 1, 2, 3, 4):
            b = spm.Builder(ds, walk=w)
            b.build()
            torch.cuda.synchronize()
            h = b.map.host()
            if ref is None:
                ref = h
            else:
                assert np.array_equal(ref["dist"], h["dist"]) and np.array_equal(ref["parent"], h["parent"]), \
                    f"walk {w} on {sc.width}x{sc.height}"
        _say(f"[parity] every walk {sc.width}x{sc.height}")


def test_max_side_sampled(oracle_mod, spm):
    scene = Scene(8192, 8192, [_rect_poly(4000, 100, 4100, 8100), _rect_poly(1000, 3000, 3900, 3050)],
                  np.asarray([[10, 10]]), np.asarray([[8000, 8000, 8190, 7000]]))
    costs = oracle_mod.costs(scene, weights=True)
    pix = wide_sample(scene, costs[0], 1, 12000, n_rows=2, block=64)
    _sampled(oracle_mod, spm, scene, "max-side-8192", pix, max_ambiguous=0.05, costs=costs)
