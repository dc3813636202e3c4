"""Shared comparison rule between a GPU map and the oracle (tests only).

The rule (distances to 1e-5 relative, +inf/-1 exactly, parents bit-exact
except where the best two candidates are within 1e-5 relative):
  * dist is +inf exactly where the oracle's is;
  * |D_gpu - D| <= 1e-5 * D + 1e-6 elsewhere (the absolute floor covers a
    pixel centre lying on a segment source, where D = 0);
  * parent equal to the oracle's except at ambiguous pixels, second - D <=
    1e-5 * D + 1e-6.  Where several parents are correct only the unique part
    is compared: at an ambiguous pixel whose parent differs, the GPU's parent
    must itself be a valid choice, i.e. a generator the pixel centre sees whose
    value cost + distance (the oracle's, in FP64) lies within the same band of
    D.  So a wrong parent fails even at a near-tie;
  * the ambiguous fraction is bounded per workload (the bound is the caller's)
    and returned for the test output.

Generator parents follow the same pattern: equal to the oracle's, or (only
where exact FP64 ties make several predecessors correct) a predecessor whose
arc exists and attains the oracle's cost to 1e-12 relative.
"""
import numpy as np

RTOL = 1e-5
ATOL = 1e-6


def compare(d_gpu, p_gpu, ref, label, *, O, scene, cost, pix, max_ambiguous):
    """d_gpu/p_gpu: the GPU's values at the row-major pixels `pix` (any shape, same size);
    ref: the oracle's pixels() (or full_map()) result at the same pixels; cost: the oracle's
    generator costs.  Returns the statistics printed by the tests."""
    d_gpu = np.asarray(d_gpu).reshape(-1)
    p_gpu = np.asarray(p_gpu).reshape(-1)
    pix = np.asarray(pix, np.int64).reshape(-1)
    d_or = np.asarray(ref["dist64"]).reshape(-1)
    p_or = np.asarray(ref["parent"]).reshape(-1)
    second = np.asarray(ref["second"]).reshape(-1)
    assert d_gpu.size == d_or.size == pix.size, f"{label}: size mismatch"
    fin = np.isfinite(d_or)
    assert np.array_equal(np.isfinite(d_gpu), fin), \
        f"{label}: finite masks differ at pixels {pix[np.isfinite(d_gpu) != fin][:5]}"
    assert np.all(p_gpu[~fin] == -1), f"{label}: parent not -1 where dist is +inf"
    err = np.abs(d_gpu[fin].astype(np.float64) - d_or[fin])
    tol = RTOL * d_or[fin] + ATOL
    bad = err > tol
    if bad.any():
        k = np.argmax(err - tol)
        raise AssertionError(f"{label}: {int(bad.sum())} distances out of tolerance; worst gpu={d_gpu[fin][k]} "
                             f"oracle={d_or[fin][k]} at pixel {pix[fin][k]}")
    with np.errstate(invalid="ignore"):
        amb = fin & ((second - d_or) <= RTOL * d_or + ATOL)
    diff = fin & (p_gpu != p_or)
    pbad = diff & ~amb
    if pbad.any():
        raise AssertionError(f"{label}: {int(pbad.sum())} parent mismatches at clear pixels, e.g. pixels "
                             f"{pix[pbad][:5].tolist()} gpu={p_gpu[pbad][:5]} oracle={p_or[pbad][:5]}")
    alt = diff & amb
    if alt.any():
        v = O.candidates(scene, cost, pix[alt], p_gpu[alt])
        D = d_or[alt]
        valid = np.isfinite(v) & (np.abs(v - D) <= RTOL * D + ATOL)
        if not valid.all():
            raise AssertionError(f"{label}: {int((~valid).sum())} near-tie pixels whose GPU parent is not a valid "
                                 f"choice, e.g. pixels {pix[alt][~valid][:5].tolist()} gpu={p_gpu[alt][~valid][:5]} "
                                 f"value={v[~valid][:5]} D={D[~valid][:5]}")
    n_free = int(fin.sum())
    frac = float(amb.sum()) / max(1, n_free)
    assert frac <= max_ambiguous, f"{label}: ambiguous fraction {frac:.4f} above its bound {max_ambiguous}"
    return {"pixels": int(d_or.size), "free": n_free, "ambiguous": int(amb.sum()), "ambiguous_frac": frac,
            "parent_alternatives": int(alt.sum()),
            "max_rel": float(np.max(err / np.maximum(d_or[fin], 1e-30))) if fin.any() else 0.0}


def compare_generators(h, cost_or, gpar_or, weights, label):
    """Generator table of a GPU map (Map.host()) against the oracle's costs(scene, weights=True)."""
    G = h["n_gen"]
    assert G == len(cost_or), f"{label}: generator count {G} vs {len(cost_or)}"
    c = h["gen_cost"]
    assert np.array_equal(np.isinf(c), np.isinf(cost_or)), f"{label}: reached sets differ"
    f = np.isfinite(cost_or)
    rel = np.abs(c[f] - cost_or[f]) / np.maximum(cost_or[f], 1e-300)
    assert np.all(rel <= 1e-9), f"{label}: generator cost rel err {rel.max()}"
    gp = h["gen_parent"]
    diff = np.nonzero(gp != gpar_or)[0]
    for v in diff:
        u = int(gp[v])
        assert 0 <= u < G and np.isfinite(cost_or[v]) and gpar_or[v] != v, \
            f"{label}: generator {v} parent {u}, oracle {gpar_or[v]}"
        w = weights[v, u]
        assert w >= 0 and cost_or[u] < cost_or[v] and \
            abs(cost_or[u] + w - cost_or[v]) <= 1e-12 * cost_or[v], \
            f"{label}: generator {v} parent {u} is not a tied predecessor (oracle {gpar_or[v]})"
    return {"generators": int(G), "parent_ties": int(diff.size)}
