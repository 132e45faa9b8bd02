"""Certified minimum-congestion bracket used to scale demands to a load factor.

For an instance with capacities u and demands d, the minimum congestion
mu* = min over all routings of max_e (flow_e / u_e) is the reciprocal of the
maximum concurrent flow. Scaling d by alpha = LF / mu* gives load factor LF:
the scaled instance is feasible iff LF <= 1 (Section 1's constraint system).

mu* is bracketed by path column generation on the path LP

    min mu  s.t.  sum_{p in P_k} x_p = d_k,  sum_{p ∋ e} x_p <= mu u_e,  x >= 0,

solved with HiGHS. mu_hi is the value of the restricted master (an explicit
routing), mu_lo = sum_k d_k dist_l(s_k, t_k) / sum_e u_e l_e for the master's
dual arc lengths l (weak duality), so mu_lo <= mu* <= mu_hi. Demands scaled by
LF / mu_hi are certified feasible for LF <= 1.

This is instance generation, not part of the PDR method.
"""
from __future__ import annotations

import time

import numpy as np
from scipy.optimize import linprog
from scipy.sparse import csc_matrix, csr_matrix
from scipy.sparse.csgraph import dijkstra


def _shortest_paths(n, tails, heads, lengths, s, t, chunk=512):
    """Shortest s_k -> t_k paths under positive arc lengths.

    Returns (dist[K], list of arc-id arrays).
    """
    m = len(heads)
    A = csr_matrix((lengths, (tails, heads)), shape=(n, n))
    keys = tails.astype(np.int64) * n + heads.astype(np.int64)
    order = np.argsort(keys, kind="stable")
    skeys = keys[order]
    K = len(s)
    dist = np.empty(K)
    paths = [None] * K
    srcs, inv = np.unique(s, return_inverse=True)
    for c0 in range(0, len(srcs), chunk):
        block = srcs[c0:c0 + chunk]
        D, P = dijkstra(A, directed=True, indices=block, return_predecessors=True)
        ks = np.nonzero((inv >= c0) & (inv < c0 + len(block)))[0]
        rows = inv[ks] - c0
        dist[ks] = D[rows, t[ks]]
        cur = t[ks].astype(np.int64)
        src = s[ks].astype(np.int64)
        arcs_rev = [[] for _ in range(len(ks))]
        active = np.nonzero(cur != src)[0]
        while active.size:
            prev = P[rows[active], cur[active]].astype(np.int64)
            if np.any(prev < 0):
                raise RuntimeError("unreachable commodity sink")
            pos = np.searchsorted(skeys, prev * n + cur[active])
            arc = order[pos]
            for a_i, arc_id in zip(active.tolist(), arc.tolist()):
                arcs_rev[a_i].append(arc_id)
            cur[active] = prev
            active = active[cur[active] != src[active]]
        for j, k in enumerate(ks.tolist()):
            paths[k] = np.array(arcs_rev[j][::-1], dtype=np.int64)
    assert m == len(tails)
    return dist, paths


def congestion_bracket(inst, gap: float = 1e-3, max_iter: int = 80, verbose: bool = False,
                       time_limit: float = 7200.0, kappa: float = 12.0, mu_lo0: float = 0.0,
                       on_iter=None):
    """Return dict(mu_hi, mu_lo, iters, columns) for the instance's demands.

    Columns come from two pricing rules per iteration: shortest paths under the
    master's dual arc lengths (classical column generation) and shortest paths
    under exponential congestion lengths exp(kappa * (load_e / u_e / mu - 1)) / u_e
    of the master's routing (the multiplicative-weights rule), which spreads
    flow over many bottlenecks at once. Both length vectors also give a weak
    duality lower bound; the larger is kept. Columns unused for three
    consecutive masters are dropped.
    """
    n, m, K = inst.n, inst.m, inst.K
    tails = inst.tails().astype(np.int64)
    heads = inst.col.astype(np.int64)
    u = inst.u.astype(np.float64)
    d = inst.d.astype(np.float64)
    s = inst.s.astype(np.int64)
    t = inst.t.astype(np.int64)
    t0 = time.time()

    # initial columns: fewest-hop paths
    _, paths = _shortest_paths(n, tails, heads, np.ones(m), s, t)
    col_k = list(range(K))
    col_arcs = list(paths)
    idle = [0] * K
    seen = set((k, tuple(p.tolist())) for k, p in enumerate(paths))

    def add_columns(newp, ks):
        added = 0
        for k in ks:
            key = (k, tuple(newp[k].tolist()))
            if key in seen:
                continue
            seen.add(key)
            col_k.append(k)
            col_arcs.append(newp[k])
            idle.append(0)
            added += 1
        return added

    mu_lo = float(mu_lo0)  # any valid lower bound known in advance (e.g. a cut bound)
    mu_hi = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        P = len(col_arcs)
        lens = np.array([len(a) for a in col_arcs], dtype=np.int64)
        rows = np.concatenate(col_arcs)
        cols = np.repeat(np.arange(1, P + 1), lens)
        A_ub = csc_matrix((np.concatenate([-u, np.ones(len(rows))]),
                           (np.concatenate([np.arange(m), rows]),
                            np.concatenate([np.zeros(m, dtype=np.int64), cols]))),
                          shape=(m, P + 1))
        A_eq = csc_matrix((np.ones(P), (np.array(col_k), np.arange(1, P + 1))), shape=(K, P + 1))
        c = np.zeros(P + 1)
        c[0] = 1.0
        res = linprog(c, A_ub=A_ub, b_ub=np.zeros(m), A_eq=A_eq, b_eq=d,
                      bounds=(0, None), method="highs-ipm")
        if res.status != 0:
            raise RuntimeError(f"master LP failed: {res.message}")
        mu_hi = min(mu_hi, float(res.fun))
        x = np.asarray(res.x[1:])
        load = np.bincount(rows, weights=np.repeat(x, lens), minlength=m)
        lam = np.maximum(0.0, -np.asarray(res.ineqlin.marginals))
        pi = np.asarray(res.eqlin.marginals)
        # strictly positive lengths keep Dijkstra well defined; the bound is valid for any l >= 0
        lp = lam + 1e-9 * max(lam.max(), 1e-300) + 1e-300
        dist, newp = _shortest_paths(n, tails, heads, lp, s, t)
        mu_lo = max(mu_lo, float(np.dot(d, dist) / np.dot(u, lp)))
        rho = load / u / max(float(res.fun), 1e-300)
        lx = np.exp(kappa * (rho - 1.0)) / u
        dist_x, newp_x = _shortest_paths(n, tails, heads, lx, s, t)
        mu_lo = max(mu_lo, float(np.dot(d, dist_x) / np.dot(u, lx)))
        if verbose:
            print(f"[cg] it {it} cols {P} mu_hi {mu_hi:.6g} mu_lo {mu_lo:.6g} "
                  f"gap {mu_hi / mu_lo - 1:.2e} t {time.time() - t0:.1f}s", flush=True)
        if on_iter is not None:
            on_iter(dict(mu_hi=mu_hi, mu_lo=mu_lo, iters=it, columns=P))
        if mu_hi <= mu_lo * (1.0 + gap) or time.time() - t0 > time_limit:
            break
        # drop columns idle for three masters
        keep = []
        for q in range(P):
            idle[q] = 0 if x[q] > 0 else idle[q] + 1
            if idle[q] < 3:
                keep.append(q)
        if len(keep) < P:
            col_k[:] = [col_k[q] for q in keep]
            col_arcs[:] = [col_arcs[q] for q in keep]
            idle[:] = [idle[q] for q in keep]
            seen.clear()
            seen.update((k, tuple(a.tolist())) for k, a in zip(col_k, col_arcs))
        added = add_columns(newp, np.nonzero(dist < pi - 1e-12 * np.maximum(1.0, np.abs(pi)))[0].tolist())
        added += add_columns(newp_x, range(K))
        if added == 0:
            break
    return dict(mu_hi=mu_hi, mu_lo=mu_lo, iters=it, columns=len(col_arcs),
                seconds=time.time() - t0)


def grid_cut_bound(inst, a: int, b: int) -> float:
    """Lower bound on the minimum congestion of an a x b grid instance from its
    straight cuts: every vertical or horizontal line splits the grid, and all
    demand from one side to the other must cross the arcs of the cut in that
    direction, so mu* >= demand / capacity for each cut and direction."""
    tails = inst.tails().astype(np.int64)
    heads = inst.col.astype(np.int64)
    rt, ct = np.divmod(tails, b)
    rh, ch = np.divmod(heads, b)
    rs, cs = np.divmod(inst.s.astype(np.int64), b)
    rk, ck = np.divmod(inst.t.astype(np.int64), b)
    best = 0.0
    for (pt, ph, ps, pk, size) in ((ct, ch, cs, ck, b), (rt, rh, rs, rk, a)):
        for c in range(size - 1):
            for sgn in (1, -1):
                side_t = (pt <= c) if sgn > 0 else (pt > c)
                side_h = (ph > c) if sgn > 0 else (ph <= c)
                cap = float(inst.u[side_t & side_h].sum())
                src = (ps <= c) if sgn > 0 else (ps > c)
                dst = (pk > c) if sgn > 0 else (pk <= c)
                dem = float(inst.d[src & dst].sum())
                if cap > 0:
                    best = max(best, dem / cap)
    return best
