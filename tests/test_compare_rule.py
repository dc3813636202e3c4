"""CPU checks of the parity rule itself (tests/spm_compare.py), using the oracle's own maps as the
map under test and planting mistakes into copies of them."""
import numpy as np
import pytest

from scenegen import config1, random_small
from tests.spm_compare import compare, compare_generators


def _setup(O, scene):
    cost, gpar, wts = O.costs(scene, weights=True)
    ref = O.full_map(scene)
    return cost, gpar, wts, ref


def _cmp(O, scene, cost, ref, d, p, bound=1.0):
    return compare(d, p, ref, "planted", O=O, scene=scene, cost=cost, pix=np.arange(scene.width * scene.height),
                   max_ambiguous=bound)


def test_rule_accepts_the_oracle_and_valid_alternatives(oracle_mod):
    scene = config1(1)
    cost, gpar, wts, ref = _setup(oracle_mod, scene)
    st = _cmp(oracle_mod, scene, cost, ref, ref["dist"], ref["parent"])
    assert st["parent_alternatives"] == 0 and st["ambiguous"] > 0
    # at every ambiguous pixel, swap in the runner-up generator when it is a valid (visible, tied) choice
    d = ref["dist64"].reshape(-1)
    with np.errstate(invalid="ignore"):
        amb = np.flatnonzero(np.isfinite(d) & (ref["second"].reshape(-1) - d <= 1e-5 * d + 1e-6))
    kind, _, _ = oracle_mod.generators(scene)
    G = len(kind)
    p = ref["parent"].reshape(-1).copy()
    swapped = 0
    for k in amb[:200]:
        vals = oracle_mod.candidates(scene, cost, np.full(G, k), np.arange(G))
        alt = [g for g in np.argsort(vals) if g != p[k] and abs(vals[g] - d[k]) <= 1e-5 * d[k] + 1e-6]
        if alt:
            p[k] = alt[0]
            swapped += 1
    assert swapped > 0
    st = _cmp(oracle_mod, scene, cost, ref, ref["dist"], p.reshape(ref["parent"].shape))
    assert st["parent_alternatives"] == swapped


def test_rule_rejects_planted_mistakes(oracle_mod):
    scene = config1(2)
    cost, gpar, wts, ref = _setup(oracle_mod, scene)
    d = ref["dist64"].reshape(-1)
    fin = np.isfinite(d)
    with np.errstate(invalid="ignore"):
        amb = fin & (ref["second"].reshape(-1) - d <= 1e-5 * d + 1e-6)
    clear = np.flatnonzero(fin & ~amb)
    # a wrong parent at a clear pixel
    p = ref["parent"].copy().reshape(-1)
    p[clear[10]] = (p[clear[10]] + 1) % len(cost)
    with pytest.raises(AssertionError, match="clear pixels"):
        _cmp(oracle_mod, scene, cost, ref, ref["dist"], p)
    # a wrong parent at an ambiguous pixel: a generator the pixel does not see, or one far from D
    k = np.flatnonzero(amb)[0]
    kind, _, _ = oracle_mod.generators(scene)
    vals = oracle_mod.candidates(scene, cost, np.full(len(kind), k), np.arange(len(kind)))
    bad = [g for g in range(len(kind)) if not (abs(vals[g] - d[k]) <= 1e-5 * d[k] + 1e-6)]
    p = ref["parent"].copy().reshape(-1)
    p[k] = bad[0]
    with pytest.raises(AssertionError, match="not a valid"):
        _cmp(oracle_mod, scene, cost, ref, ref["dist"], p)
    # a distance off by more than the band, and a finite value where the oracle has +inf
    dd = ref["dist"].copy().reshape(-1)
    dd[clear[5]] *= 1.0 + 3e-5
    with pytest.raises(AssertionError, match="out of tolerance"):
        _cmp(oracle_mod, scene, cost, ref, dd, ref["parent"])
    dd = ref["dist"].copy().reshape(-1)
    dd[np.flatnonzero(~fin)[0]] = 1.0
    with pytest.raises(AssertionError, match="finite masks"):
        _cmp(oracle_mod, scene, cost, ref, dd, ref["parent"])
    # the ambiguous fraction above its bound
    with pytest.raises(AssertionError, match="above its bound"):
        _cmp(oracle_mod, scene, cost, ref, ref["dist"], ref["parent"], bound=1e-4)


def test_generator_rule(oracle_mod):
    scene = random_small(5)
    cost, gpar, wts = oracle_mod.costs(scene, weights=True)
    kind, _, _ = oracle_mod.generators(scene)
    h = {"n_gen": len(cost), "gen_cost": cost.copy(), "gen_parent": gpar.copy()}
    assert compare_generators(h, cost, gpar, wts, "same")["parent_ties"] == 0
    v = next(g for g in range(len(cost)) if kind[g] == oracle_mod.VERTEX and np.isfinite(cost[g]))
    # any other generator with an arc into v that does not attain its cost is rejected
    wrong = [u for u in range(len(cost)) if u != gpar[v] and not (wts[v, u] >= 0 and cost[u] + wts[v, u] == cost[v])]
    h2 = dict(h, gen_parent=gpar.copy())
    h2["gen_parent"][v] = wrong[0]
    with pytest.raises(AssertionError):
        compare_generators(h2, cost, gpar, wts, "wrong")
    h3 = dict(h, gen_cost=cost * (1 + 1e-8))
    with pytest.raises(AssertionError, match="cost rel err"):
        compare_generators(h3, cost, gpar, wts, "cost")
