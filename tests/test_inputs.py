"""The seeded synthetic inputs (gen/): shapes, value ranges, determinism and
the load-factor scaling of the named workloads and of the 256-instance batch.
CPU only."""
from collections import deque

import numpy as np
import pytest

from gen.instance import load_instance, recipe_grid4_k8, recipe_grid100_k10000, \
    recipe_knn2500_k1000, recipe_small


def check_common(inst, u_range, d_range):
    n, m, K = inst.n, inst.m, inst.K
    rp, col = inst.row_ptr, inst.col
    assert rp[0] == 0 and rp[-1] == m and np.all(np.diff(rp) >= 0)
    tails = inst.tails()
    assert np.all((col >= 0) & (col < n)) and np.all(col != tails)  # no self-loops
    # CSR sorted by (tail, head), no duplicate arcs
    key = tails.astype(np.int64) * n + col
    assert np.all(np.diff(key) > 0)
    # every arc has its reverse (bidirectional graphs)
    assert np.array_equal(np.sort(key), np.sort(col.astype(np.int64) * n + tails))
    assert np.all(inst.s != inst.t)
    assert len(set(zip(inst.s.tolist(), inst.t.tolist()))) == K  # distinct OD pairs
    assert np.all(inst.u == np.round(inst.u))
    assert inst.u.min() >= u_range[0] and inst.u.max() <= u_range[1]
    assert np.all(inst.d == np.round(inst.d))
    assert inst.d.min() >= d_range[0] and inst.d.max() <= d_range[1]


def connected(inst):
    adj = [[] for _ in range(inst.n)]
    for a, b in zip(inst.tails().tolist(), inst.col.tolist()):
        adj[a].append(b)
        adj[b].append(a)
    seen = np.zeros(inst.n, bool)
    seen[0] = True
    q = deque([0])
    while q:
        v = q.popleft()
        for w in adj[v]:
            if not seen[w]:
                seen[w] = True
                q.append(w)
    return bool(seen.all())


def test_grid4_k8():
    inst = recipe_grid4_k8()
    assert (inst.n, inst.m, inst.K) == (16, 48, 8)
    check_common(inst, (5, 20), (1, 5))
    deg = np.bincount(inst.tails(), minlength=16) + np.bincount(inst.col, minlength=16)
    assert sorted(set(deg.tolist())) == [4, 6, 8]


def test_knn2500_k1000_unscaled_and_scaled():
    inst = recipe_knn2500_k1000()
    assert (inst.n, inst.m, inst.K) == (2500, 12198, 1000)
    check_common(inst, (500, 1500), (1, 50))
    assert connected(inst)
    sc = load_instance("knn2500_k1000")
    # demands scaled by LF / mu_hi of a certified bracket, capacities untouched
    alpha = 0.9 / sc.meta["mu_hi"]
    assert np.array_equal(sc.u, inst.u)
    assert np.allclose(sc.d, inst.d * alpha, rtol=1e-15, atol=0)
    lo, hi = sc.meta["lf_bracket"]
    assert hi == 0.9 and 0.9 * (1 - 1e-5) < lo <= hi


def test_grid100_k10000():
    inst = recipe_grid100_k10000()
    assert (inst.n, inst.m, inst.K) == (10000, 39600, 10000)
    check_common(inst, (1000, 3000), (1, 20))
    sc = load_instance("grid100_k10000")
    lo, hi = sc.meta["lf_bracket"]
    assert hi == 0.95 and 0.8 < lo < hi


def test_recipes_are_deterministic():
    a, b = recipe_small("knn", 300, 40, seed=7), recipe_small("knn", 300, 40, seed=7)
    for x, y in ((a.row_ptr, b.row_ptr), (a.col, b.col), (a.u, b.u), (a.s, b.s), (a.t, b.t),
                 (a.d, b.d)):
        assert np.array_equal(x, y)
    c = recipe_small("knn", 300, 40, seed=8)
    assert not np.array_equal(a.u, c.u) or not np.array_equal(a.col, c.col)


def test_batch_recipe_shapes_and_labels():
    from gen.batch import recipe_batch
    insts = recipe_batch(256, 4)
    assert len(insts) == 256
    ns = np.array([i.n for i in insts])
    Ks = np.array([i.K for i in insts])
    assert ns.min() >= 100 and ns.max() <= 5000
    assert Ks.min() >= 16 and Ks.max() <= 2000
    lfs = np.array([i.meta["load_factor"] for i in insts])
    assert lfs.min() >= 0.7 and lfs.max() <= 1.1
    labels = [i.meta["certified"] for i in insts]
    # a member is certified feasible exactly when its load factor is <= 1
    for lf, lab in zip(lfs, labels):
        assert (lab == "feasible") == (lf <= 1.0)
    assert labels.count("feasible") == 190
    for inst in insts[:8]:
        assert np.all(inst.s != inst.t)
        assert inst.u.min() >= 100 and inst.u.max() <= 1000
        assert connected(inst)


def _edge_lp_min_congestion(inst):
    """Minimum congestion mu* of the instance's demands from the arc-commodity
    LP (min mu s.t. conservation of every commodity at every vertex,
    sum_k f_ek <= mu u_e, f >= 0), solved directly with HiGHS: an independent
    reference for the path column generation of gen.loadfactor."""
    from scipy.optimize import linprog
    from scipy.sparse import coo_matrix
    n, m, K = inst.n, inst.m, inst.K
    tails = inst.tails().astype(np.int64)
    heads = inst.col.astype(np.int64)
    e = np.repeat(np.arange(m), K)
    k = np.tile(np.arange(K), m)
    var = e * K + k
    A_eq = coo_matrix((np.concatenate([np.ones(m * K), -np.ones(m * K)]),
                       (np.concatenate([tails[e] * K + k, heads[e] * K + k]),
                        np.concatenate([var, var]))), shape=(n * K, m * K + 1)).tocsr()
    b_eq = np.zeros(n * K)
    np.add.at(b_eq, inst.s.astype(np.int64) * K + np.arange(K), inst.d)
    np.add.at(b_eq, inst.t.astype(np.int64) * K + np.arange(K), -inst.d)
    A_ub = coo_matrix((np.concatenate([np.ones(m * K), -inst.u]),
                       (np.concatenate([e, np.arange(m)]),
                        np.concatenate([var, np.full(m, m * K)]))), shape=(m, m * K + 1)).tocsr()
    c = np.zeros(m * K + 1)
    c[-1] = 1.0
    res = linprog(c, A_ub=A_ub, b_ub=np.zeros(m), A_eq=A_eq, b_eq=b_eq, bounds=(0, None),
                  method="highs")
    assert res.status == 0
    return float(res.fun)


def test_congestion_bracket_contains_the_lp_optimum():
    """The certified bracket behind every load-factor scaling: on small
    instances the column-generation bracket mu_lo <= mu* <= mu_hi
    (gen.loadfactor) contains the minimum congestion of the arc-commodity LP
    and closes to its gap; the straight-cut bound of a grid is below it; and a
    demand scaling by LF / mu_hi (feasible label) or LF / mu_lo (infeasible
    label) puts the LP's minimum congestion on the labelled side of 1."""
    from gen.loadfactor import congestion_bracket, grid_cut_bound
    cases = [recipe_small("knn", 50, 12, seed=3, u_range=(5, 20), d_range=(1, 9)),
             recipe_small("knn", 80, 25, seed=4, u_range=(10, 40), d_range=(1, 20)),
             recipe_small("grid", 5, 10, seed=5, u_range=(5, 20), d_range=(1, 9))]
    for q, inst in enumerate(cases):
        mu = _edge_lp_min_congestion(inst)
        br = congestion_bracket(inst, gap=1e-6, max_iter=200)
        assert br["mu_lo"] <= mu * (1 + 1e-7) and mu <= br["mu_hi"] * (1 + 1e-7), (q, br, mu)
        assert br["mu_hi"] <= br["mu_lo"] * (1 + 1e-6), (q, br)
        if q == 2:
            assert grid_cut_bound(inst, 5, 5) <= mu * (1 + 1e-9)
        for lf in (0.9, 1.05):
            alpha = lf / (br["mu_hi"] if lf <= 1 else br["mu_lo"])
            mus = _edge_lp_min_congestion(inst.demand_scaled(alpha))
            assert (mus <= 1.0 + 1e-9) if lf <= 1 else (mus > 1.0), (q, lf, mus)


def test_knn_neighbours_equal_brute_force():
    """gen.graphs.knn_points: each point's 4 nearest neighbours (ties by index)
    equal a brute-force search over all pairwise distances of the same points."""
    from gen.graphs import knn_points
    for seed in (1, 2, 3):
        pts, nbrs = knn_points(300, np.random.default_rng(seed))
        d2 = ((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)
        np.fill_diagonal(d2, np.inf)
        idx = np.arange(len(pts))
        for i in range(len(pts)):
            want = np.lexsort((idx, d2[i]))[:4]
            assert np.array_equal(nbrs[i], want), (seed, i)
