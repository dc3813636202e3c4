"""Agent distances and the adjoint with respect to the sources (workload: the
1024^2 convex-hull scene, 4096 agents)."""
import math

import numpy as np
import pytest

from scenegen import config2, config5_agents

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup(oracle_mod):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_08500_amd as spm
    scene = config2(1)
    agents = config5_agents(scene, 4096, seed=11)
    b = spm.Builder(spm.DeviceScene(scene))
    b.build()
    torch.cuda.synchronize()
    cost, gpar = oracle_mod.costs(scene)
    kind, ref, xy = oracle_mod.generators(scene)
    pix = (np.floor(agents[:, 1]).astype(np.int64) * scene.width + np.floor(agents[:, 0]).astype(np.int64))
    r = oracle_mod.pixels(scene, cost, pix)
    return {"spm": spm, "scene": scene, "agents": agents, "b": b, "cost": cost, "gpar": gpar, "kind": kind,
            "xy": xy.astype(np.float64), "pix": r}


def _closest_on_seg(A, B, p):
    e = B - A
    t = np.clip(((p - A) @ e) / (e @ e), 0.0, 1.0)
    return A + t * e, t


def _chain(g, gpar, nsrc):
    """root and preroot of generator g (oracle parents)."""
    prev, cur = g, g
    if g < nsrc:
        return g, -1
    while cur >= nsrc:
        prev, cur = cur, gpar[cur]
    return cur, prev


def test_agent_distance_matches_oracle(setup):
    import torch
    spm, scene, agents = setup["spm"], setup["scene"], setup["agents"]
    D = spm.agent_distance(setup["b"], torch.from_numpy(agents).cuda()).cpu().numpy().astype(np.float64)
    par = setup["pix"]["parent"]
    amb = (setup["pix"]["second"] - setup["pix"]["dist64"]) <= 1e-5 * setup["pix"]["dist64"] + 1e-6
    ok = (par >= 0) & ~amb
    assert ok.sum() > 3800
    xy, kind, cost = setup["xy"], setup["kind"], setup["cost"]
    for i in np.nonzero(ok)[0]:
        g = par[i]
        a = agents[i].astype(np.float64)
        q = xy[g, :2] if kind[g] != 1 else _closest_on_seg(xy[g, :2], xy[g, 2:], a)[0]
        exp = math.dist(a, q) + cost[g]
        assert abs(D[i] - exp) <= 1e-5 * exp + 1e-6, (i, D[i], exp)


def _loss(pts, segs, agents, use, par, setup):
    """mean over the used agents of the distance along the oracle's fixed parent chain,
    with the sources at (pts, segs) -- FP64, function values only."""
    kind, xy, gpar = setup["kind"], setup["xy"], setup["gpar"]
    np_, ns = len(pts), len(segs)
    nsrc = np_ + ns

    def src_dist(r, v):
        if r < np_:
            return math.dist(v, pts[r])
        A, B = segs[r - np_, :2], segs[r - np_, 2:]
        return math.dist(v, _closest_on_seg(A, B, v)[0])

    tot = 0.0
    for i in use:
        g = par[i]
        a = agents[i].astype(np.float64)
        if g < nsrc:
            tot += src_dist(g, a)
            continue
        tot += math.dist(a, xy[g, :2])
        cur = g
        while gpar[cur] >= nsrc:
            tot += math.dist(xy[cur, :2], xy[gpar[cur], :2])
            cur = gpar[cur]
        tot += src_dist(gpar[cur], xy[cur, :2])
    return tot / len(agents)


def test_gradient_against_central_differences(setup):
    import torch
    spm, scene, agents = setup["spm"], setup["scene"], setup["agents"]
    n = len(agents)
    par = setup["pix"]["parent"]
    kind, xy, gpar = setup["kind"], setup["xy"], setup["gpar"]
    np_, ns = len(scene.points), len(scene.segs)
    nsrc = np_ + ns
    amb = (setup["pix"]["second"] - setup["pix"]["dist64"]) <= 1e-3
    # exclusions: no parent, near-tie at the pixel, or a segment closest point within 1e-3 of an end
    use = []
    for i in range(n):
        g = par[i]
        if g < 0 or amb[i]:
            continue
        root, pre = _chain(g, gpar, nsrc)
        if root >= np_:
            v = agents[i].astype(np.float64) if g < nsrc else xy[pre, :2]
            A, B = scene.segs[root - np_, :2].astype(np.float64), scene.segs[root - np_, 2:].astype(np.float64)
            e = B - A
            t_raw = ((v - A) @ e) / (e @ e)   # unclamped: the gradient switches form at 0 and 1
            if abs(t_raw) < 1e-3 or abs(t_raw - 1.0) < 1e-3:
                continue
        use.append(i)
    use = np.asarray(use)
    assert len(use) > 3800
    w = np.zeros(n, np.float32)
    w[use] = 1.0 / n
    gp, gs = spm.source_gradients(setup["b"], torch.from_numpy(agents).cuda(), torch.from_numpy(w).cuda())
    gp, gs = gp.cpu().numpy().astype(np.float64), gs.cpu().numpy().astype(np.float64)
    pts0 = scene.points.astype(np.float64)
    segs0 = scene.segs.astype(np.float64)
    h = 1e-3
    for k in range(np_):
        for c in range(2):
            P1, P2 = pts0.copy(), pts0.copy()
            P1[k, c] += h
            P2[k, c] -= h
            fd = (_loss(P1, segs0, agents, use, par, setup) - _loss(P2, segs0, agents, use, par, setup)) / (2 * h)
            assert abs(gp[k, c] - fd) <= 1e-4 * abs(fd) + 1e-6, ("pt", k, c, gp[k, c], fd)
    for k in range(ns):
        for c in range(4):
            S1, S2 = segs0.copy(), segs0.copy()
            S1[k, c] += h
            S2[k, c] -= h
            fd = (_loss(pts0, S1, agents, use, par, setup) - _loss(pts0, S2, agents, use, par, setup)) / (2 * h)
            assert abs(gs[k, c] - fd) <= 1e-4 * abs(fd) + 1e-6, ("seg", k, c, gs[k, c], fd)


def test_backward_deterministic_and_autograd(setup):
    import torch
    spm, scene, agents = setup["spm"], setup["scene"], setup["agents"]
    b = setup["b"]
    A = torch.from_numpy(agents).cuda()
    w = torch.full((len(agents),), 1.0 / len(agents), device="cuda")
    g1 = spm.source_gradients(b, A, w)
    g2 = spm.source_gradients(b, A, w)
    assert torch.equal(g1[0], g2[0]) and torch.equal(g1[1], g2[1])
    pts = torch.tensor(scene.points, dtype=torch.float32, device="cuda", requires_grad=True)
    segs = torch.tensor(scene.segs, dtype=torch.float32, device="cuda", requires_grad=True)
    D = spm.SPMDistance.apply(pts, segs, A, b)
    fin = torch.isfinite(D)
    loss = D[fin].sum() / len(agents)
    loss.backward()
    assert torch.allclose(pts.grad, g1[0], rtol=1e-6, atol=1e-7)
    assert torch.allclose(segs.grad, g1[1], rtol=1e-6, atol=1e-7)
