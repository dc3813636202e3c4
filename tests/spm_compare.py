"""Shared comparison rule between a GPU map and the oracle (tests only).

The rule (distances to 1e-5 relative, +inf/-1 exactly, parents bit-exact
except where the best two candidates are within 1e-5 relative):
  * dist is +inf exactly where the oracle's is;
  * |D_gpu - D| <= 1e-5 * D + 1e-6 elsewhere (the absolute floor covers a
    pixel centre lying on a segment source, where D = 0);
  * parent equal except at ambiguous pixels, second - D <= 1e-5 * D + 1e-6.
"""
import numpy as np

RTOL = 1e-5
ATOL = 1e-6


def compare(d_gpu, p_gpu, ref, label=""):
    d_or = ref["dist64"]
    fin = np.isfinite(d_or)
    assert np.array_equal(np.isfinite(d_gpu), fin), f"{label}: finite masks differ at {np.argwhere(np.isfinite(d_gpu) != fin)[:5]}"
    assert np.all(p_gpu[~fin] == -1), f"{label}: parent not -1 where dist is +inf"
    err = np.abs(d_gpu[fin].astype(np.float64) - d_or[fin])
    tol = RTOL * d_or[fin] + ATOL
    bad = err > tol
    if bad.any():
        k = np.argmax(err - tol)
        raise AssertionError(f"{label}: {int(bad.sum())} distances out of tolerance; worst gpu={d_gpu[fin][k]} "
                             f"oracle={d_or[fin][k]} at flat index {np.flatnonzero(fin)[k]}")
    with np.errstate(invalid="ignore"):
        amb = (ref["second"] - d_or) <= RTOL * d_or + ATOL
    pbad = fin & ~amb & (p_gpu != ref["parent"])
    if pbad.any():
        idx = np.argwhere(pbad)[:5]
        raise AssertionError(f"{label}: {int(pbad.sum())} parent mismatches, e.g. at {idx.tolist()} "
                             f"gpu={p_gpu[pbad][:5]} oracle={ref['parent'][pbad][:5]}")
    return {"pixels": int(d_or.size), "free": int(fin.sum()), "ambiguous": int((fin & amb).sum()),
            "ambiguous_frac": float((fin & amb).sum()) / max(1, int(fin.sum())),
            "max_rel": float(np.max(err / np.maximum(d_or[fin], 1e-30))) if fin.any() else 0.0}


def compare_generators(h, cost_or, gpar_or, label=""):
    G = h["n_gen"]
    assert G == len(cost_or), f"{label}: generator count {G} vs {len(cost_or)}"
    c = h["gen_cost"]
    assert np.array_equal(np.isinf(c), np.isinf(cost_or)), f"{label}: reached sets differ"
    f = np.isfinite(cost_or)
    rel = np.abs(c[f] - cost_or[f]) / np.maximum(cost_or[f], 1e-300)
    assert np.all(rel <= 1e-9), f"{label}: generator cost rel err {rel.max()}"
    same = h["gen_parent"] == gpar_or
    return float(same.mean()) if len(same) else 1.0
