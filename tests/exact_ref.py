"""Exact-rational references used to pin the FP64 oracle (test infrastructure).

None of this shares code with the oracle or with the GPU library. Everything
here runs in Python ``fractions.Fraction`` arithmetic on tiny inputs:

* ``qp_bruteforce``: the edge subproblem (Expression 14) solved by enumerating
  every candidate support set and congestion case of its KKT system and keeping
  the candidate with the smallest objective, evaluated directly.
* ``qp_threshold``: the same subproblem solved by Michelot's finite active-set
  threshold iteration (a different algorithm from the paper's sort-based
  Algorithm 2).
* ``edge_objective``: the subproblem objective of Expression 13 (edge
  subproblem in the step variable, slack r minimised out).
* ``exact_pdr``: PDR-ESO / AGD / GDM sweeps and the capacity-enforcing loop
  from the definitions (excess by in/out arc lists, QP by ``qp_threshold``,
  capped-simplex projection by ``cap_threshold``, AGD accept test by a direct
  difference of ``edge_objective``).
* ``cap_bruteforce`` / ``cap_threshold``: the capacity-enforcing edge step
  (projection onto {f >= 0, sum f <= u}) by support enumeration and by
  threshold iteration.
* ``lp_feasible``: feasibility of the constraint system of Section 1 by a
  Bland's-rule phase-1 simplex in exact arithmetic.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from itertools import combinations
from typing import List, Sequence

ZERO = Fr(0)


def fr(x) -> Fr:
    return x if isinstance(x, Fr) else Fr(x)


# --------------------------------------------------------------- edge QP
def qp_objective(fn: Sequence[Fr], c: Sequence[Fr], u: Fr) -> Fr:
    """Objective of the edge QP in f' up to a constant:
    1/2 (sum f' - u)_+^2 + sum_k (f'_k - c_k)^2 (r minimised out; the height terms
    of Expression 14 equal 2 sum (f'_k - c_k)^2 plus a constant, halved)."""
    over = sum(fn, ZERO) - u
    val = Fr(1, 2) * (over * over if over > 0 else ZERO)
    for a, b in zip(fn, c):
        val += (a - b) * (a - b)
    return val


def qp_bruteforce(c: Sequence, u) -> tuple:
    """Exact minimiser of the edge QP by enumerating KKT candidates.

    For every support A (f'_k > 0 exactly on A) and both congestion cases the
    stationarity equations have one solution; candidates that satisfy primal
    feasibility are evaluated and the smallest objective wins.
    Returns (f_new list, psi).
    """
    c = [fr(x) for x in c]
    u = fr(u)
    K = len(c)
    best = None
    for size in range(K + 1):
        for A in combinations(range(K), size):
            # uncongested: f'_k = c_k on A
            cand = [c[k] if k in A else ZERO for k in range(K)]
            if all(cand[k] > 0 for k in A) and sum(cand, ZERO) <= u:
                val = qp_objective(cand, c, u)
                if best is None or val < best[0]:
                    best = (val, cand, ZERO)
            # congested: f'_k = c_k - psi/2 on A, psi = sum_A f' - u
            psi = (sum((c[k] for k in A), ZERO) - u) / (1 + Fr(len(A), 2))
            if psi >= 0:
                cand = [c[k] - psi / 2 if k in A else ZERO for k in range(K)]
                if all(cand[k] > 0 for k in A):
                    val = qp_objective(cand, c, u)
                    if best is None or val < best[0]:
                        best = (val, cand, psi)
    assert best is not None
    return best[1], best[2]


def qp_threshold(c: Sequence, u) -> tuple:
    """Michelot-style threshold iteration for the edge QP (exact).

    A = {k: c_k > 0}; if sum_A c <= u the edge is uncongested. Otherwise repeat
    psi = (sum_A c - u) / (1 + |A|/2); A <- {k in A: c_k > psi/2} until A is
    unchanged. Returns (f_new, psi)."""
    c = [fr(x) for x in c]
    u = fr(u)
    A = [k for k in range(len(c)) if c[k] > 0]
    if sum((c[k] for k in A), ZERO) <= u:
        return [x if x > 0 else ZERO for x in c], ZERO
    while True:
        psi = (sum((c[k] for k in A), ZERO) - u) / (1 + Fr(len(A), 2))
        A2 = [k for k in A if c[k] > psi / 2]
        if A2 == A:
            break
        A = A2
    return [max(ZERO, x - psi / 2) for x in c], psi


def cap_objective(fn, c) -> Fr:
    return sum(((a - b) * (a - b) for a, b in zip(fn, c)), ZERO)


def cap_bruteforce(c: Sequence, u) -> tuple:
    """Exact projection of c onto {f >= 0, sum f <= u} (the capacity-enforcing
    edge step of Section 6's formulation) by enumerating supports A: the free
    candidate f = c on A, and the capped one f = c - lam on A with
    lam = (sum_A c - u) / |A| >= 0; feasible candidates are compared by
    sum (f - c)^2. Returns (f_new, lam)."""
    c = [fr(x) for x in c]
    u = fr(u)
    K = len(c)
    best = None
    for size in range(K + 1):
        for A in combinations(range(K), size):
            cand = [c[k] if k in A else ZERO for k in range(K)]
            if all(cand[k] > 0 for k in A) and sum(cand, ZERO) <= u:
                val = cap_objective(cand, c)
                if best is None or val < best[0]:
                    best = (val, cand, ZERO)
            if size:
                lam = (sum((c[k] for k in A), ZERO) - u) / size
                if lam >= 0:
                    cand = [c[k] - lam if k in A else ZERO for k in range(K)]
                    if all(cand[k] > 0 for k in A):
                        val = cap_objective(cand, c)
                        if best is None or val < best[0]:
                            best = (val, cand, lam)
    return best[1], best[2]


def cap_threshold(c: Sequence, u) -> tuple:
    """The same projection by Michelot's threshold iteration: A = {c > 0}; if
    sum_A c <= u the capacity is slack; else repeat lam = (sum_A c - u)/|A|,
    A <- {k in A: c_k > lam} until A is unchanged."""
    c = [fr(x) for x in c]
    u = fr(u)
    A = [k for k in range(len(c)) if c[k] > 0]
    if sum((c[k] for k in A), ZERO) <= u:
        return [x if x > 0 else ZERO for x in c], ZERO
    while True:
        lam = (sum((c[k] for k in A), ZERO) - u) / len(A)
        A2 = [k for k in A if c[k] > lam]
        if A2 == A or not A2:  # empty only when u = 0 and A's values all equal lam
            break
        A = A2
    return [max(ZERO, x - lam) for x in c], lam


# --------------------------------------------------------------- instances
class ExactInstance:
    """Instance data as Fractions with in/out arc lists per vertex."""

    def __init__(self, n, row_ptr, col, u, s, t, d):
        self.n = int(n)
        self.m = len(col)
        self.K = len(s)
        self.tail = []
        for i in range(self.n):
            self.tail += [i] * int(row_ptr[i + 1] - row_ptr[i])
        self.head = [int(x) for x in col]
        self.u = [fr(x) for x in u]
        self.s = [int(x) for x in s]
        self.t = [int(x) for x in t]
        self.d = [fr(x) for x in d]
        self.out_arcs = [[] for _ in range(self.n)]
        self.in_arcs = [[] for _ in range(self.n)]
        for e in range(self.m):
            self.out_arcs[self.tail[e]].append(e)
            self.in_arcs[self.head[e]].append(e)
        self.deg = [len(self.out_arcs[i]) + len(self.in_arcs[i]) for i in range(self.n)]

    @staticmethod
    def from_instance(inst, exact_values=True):
        conv = (lambda a: [Fr(float(x)).limit_denominator(10**12) for x in a])
        return ExactInstance(inst.n, inst.row_ptr, inst.col, conv(inst.u), inst.s, inst.t,
                             conv(inst.d))

    def heights(self, f):
        """h[i][k] from Expression 2-4 with in/out arc lists."""
        h = [[ZERO] * self.K for _ in range(self.n)]
        for i in range(self.n):
            for k in range(self.K):
                v = ZERO
                if self.s[k] == i:
                    v += self.d[k]
                if self.t[k] == i:
                    v -= self.d[k]
                for e in self.in_arcs[i]:
                    v += f[e][k]
                for e in self.out_arcs[i]:
                    v -= f[e][k]
                h[i][k] = v / self.deg[i] if self.deg[i] else ZERO
        return h

    def objective(self, f):
        """z of Expression 8 in the vertex form: 1/2 sum psi^2 + sum Delta^2/(2 delta)."""
        h = self.heights(f)
        z = ZERO
        for e in range(self.m):
            over = sum(f[e], ZERO) - self.u[e]
            if over > 0:
                z += over * over / 2
        for i in range(self.n):
            for k in range(self.K):
                z += self.deg[i] * h[i][k] * h[i][k] / 2
        return z


def edge_objective(F, dfs, hi, hj, u) -> Fr:
    """Expression 13 for one arc with the optimal slack r >= 0:
    1/2[(F + sum df - u)_+^2 + sum (h_i - df)^2 + sum (h_j + df)^2]."""
    over = F + sum(dfs, ZERO) - u
    v = over * over if over > 0 else ZERO
    for a, b, x in zip(hi, hj, dfs):
        v += (a - x) * (a - x) + (b + x) * (b + x)
    return v / 2


def exact_pdr(ex: ExactInstance, method: str, T: int, params=None):
    """T passes of Algorithm 1 ('eso'), Algorithm 3 ('agd'), Algorithm 4 ('gdm') or
    the capacity-enforcing loop ('cap') from f = 0 (and zero velocities).

    Returns (f, list of z values before each update)."""
    K, m = ex.K, ex.m
    f = [[ZERO] * K for _ in range(m)]
    vel = [[ZERO] * K for _ in range(m)]
    if params is None and method == "gdm":
        params = dict(beta_init=Fr(1, 10), beta_min=Fr(1, K), beta_max=Fr(1, 5),
                      alpha_inc=Fr(2), alpha_dec=Fr(1, 2), inc_period=10, gamma=Fr(9, 10))
    p = params or dict(beta_init=Fr(1, 4), beta_min=Fr(1, K), beta_max=Fr(1, 2),
                       alpha_inc=Fr(2), alpha_dec=Fr(1, 2), inc_period=10)
    beta = [fr(p["beta_init"])] * m
    zs = []
    for t in range(T):
        h = ex.heights(f)
        zs.append(ex.objective(f))
        fn = []
        for e in range(m):
            i, j = ex.tail[e], ex.head[e]
            if method in ("eso", "cap"):
                c = [(h[i][k] - h[j][k]) / 2 + f[e][k] for k in range(K)]
                new, _ = (qp_threshold if method == "eso" else cap_threshold)(c, ex.u[e])
                fn.append(new)
            else:
                F = sum(f[e], ZERO)
                psi = max(ZERO, F - ex.u[e])
                dfs = [max(-f[e][k], beta[e] * (h[i][k] - h[j][k] - psi)) for k in range(K)]
                dz = (edge_objective(F, dfs, h[i], h[j], ex.u[e])
                      - edge_objective(F, [ZERO] * K, h[i], h[j], ex.u[e]))
                b = beta[e]
                if dz <= 0 and method == "gdm":
                    g = fr(p["gamma"])
                    vel[e] = [g * vel[e][k] + dfs[k] for k in range(K)]
                    fn.append([max(ZERO, f[e][k] + vel[e][k]) for k in range(K)])
                elif dz <= 0:
                    fn.append([f[e][k] + dfs[k] for k in range(K)])
                else:
                    fn.append(list(f[e]))
                    b = max(fr(p["beta_min"]), b * fr(p["alpha_dec"]))
                if t % p["inc_period"] == 0:
                    b = min(fr(p["beta_max"]), b * fr(p["alpha_inc"]))
                beta[e] = b
        f = fn
    return f, zs


# --------------------------------------------------------------- exact LP
def lp_feasible(ex: ExactInstance) -> bool:
    """Feasibility of Section 1's constraints by an exact phase-1 simplex (Bland's rule).

    Variables: f_e,k >= 0 and capacity slacks s_e >= 0. Rows: sum_k f_e,k + s_e = u_e
    and, per (i, k), sum_out f - sum_in f = b_ik (d_k at s_k, -d_k at t_k)."""
    m, K, n = ex.m, ex.K, ex.n
    nv = m * K + m
    rows, rhs = [], []
    for e in range(m):
        r = [ZERO] * nv
        for k in range(K):
            r[e * K + k] = Fr(1)
        r[m * K + e] = Fr(1)
        rows.append(r)
        rhs.append(ex.u[e])
    for i in range(n):
        for k in range(K):
            r = [ZERO] * nv
            for e in ex.out_arcs[i]:
                r[e * K + k] += 1
            for e in ex.in_arcs[i]:
                r[e * K + k] -= 1
            b = ZERO
            if ex.s[k] == i:
                b += ex.d[k]
            if ex.t[k] == i:
                b -= ex.d[k]
            rows.append(r)
            rhs.append(b)
    R = len(rows)
    for q in range(R):  # make rhs >= 0
        if rhs[q] < 0:
            rows[q] = [-x for x in rows[q]]
            rhs[q] = -rhs[q]
    # tableau with artificials; objective = minimise sum of artificials
    ncol = nv + R
    T = [rows[q] + [Fr(1) if a == q else ZERO for a in range(R)] + [rhs[q]] for q in range(R)]
    basis = [nv + q for q in range(R)]
    obj = [ZERO] * (ncol + 1)
    for q in range(R):  # reduced costs: c_j - sum of rows (c = 1 on artificials)
        for j in range(ncol + 1):
            obj[j] -= T[q][j]
    for a in range(R):
        obj[nv + a] += 1
    while True:
        enter = next((j for j in range(ncol) if obj[j] < 0), None)
        if enter is None:
            break
        best, leave = None, None
        for q in range(R):
            if T[q][enter] > 0:
                ratio = T[q][-1] / T[q][enter]
                if best is None or ratio < best or (ratio == best and basis[q] < basis[leave]):
                    best, leave = ratio, q
        if leave is None:
            raise RuntimeError("phase 1 unbounded (impossible)")
        piv = T[leave][enter]
        T[leave] = [x / piv for x in T[leave]]
        for q in range(R):
            if q != leave and T[q][enter] != 0:
                fac = T[q][enter]
                T[q] = [a - fac * b for a, b in zip(T[q], T[leave])]
        if obj[enter] != 0:
            fac = obj[enter]
            obj = [a - fac * b for a, b in zip(obj, T[leave])]
        basis[leave] = enter
    return -obj[-1] == 0


# --------------------------------------------------------------- residual report
def exact_report(ex: ExactInstance, f) -> dict:
    """The residual report of a pseudo-flow f (m x K Fractions), in exact arithmetic.

    psi_e = max(0, sum_k f_ek - u_e) (Expression 5); phi_ek = h_ik - h_jk - psi_e
    (Section 3.3); rho_ek = phi_ek on used entries (f_ek > 0), else max(0, phi_ek);
    kkt = sum rho^2; z = 1/2 sum psi^2 + 1/2 sum_{i,k} Delta_ik^2 / delta_i
    (Expression 8); Farkas gap G = sum_k d_k (h_{s_k,k} - h_{t_k,k})
    - sum_e u_e max(0, max_k (h_ik - h_jk))."""
    h = ex.heights(f)
    psi = []
    for e in range(ex.m):
        over = sum(f[e], ZERO) - ex.u[e]
        psi.append(over if over > 0 else ZERO)
    kkt = ZERO
    cap_term = ZERO
    branches = dict(congested=False, used_negative=False, unused_positive=False)
    for e in range(ex.m):
        i, j = ex.tail[e], ex.head[e]
        lmax = ZERO
        if psi[e] > 0:
            branches["congested"] = True
        for k in range(ex.K):
            diff = h[i][k] - h[j][k]
            lmax = max(lmax, diff)
            phi = diff - psi[e]
            if f[e][k] > 0:
                rho = phi
                if phi < 0:
                    branches["used_negative"] = True
            else:
                rho = phi if phi > 0 else ZERO
                if phi > 0:
                    branches["unused_positive"] = True
            kkt += rho * rho
        cap_term += ex.u[e] * lmax
    z_psi = sum((p * p for p in psi), ZERO) / 2
    z_h = ZERO
    max_delta = ZERO
    for i in range(ex.n):
        for k in range(ex.K):
            delta = h[i][k] * ex.deg[i]
            z_h += delta * h[i][k] / 2
            max_delta = max(max_delta, abs(delta))
    gain = sum((ex.d[k] * (h[ex.s[k]][k] - h[ex.t[k]][k]) for k in range(ex.K)), ZERO)
    return dict(kkt_sq=kkt, z=z_psi + z_h, z_psi=z_psi, z_h=z_h, max_abs_excess=max_delta,
                max_congestion=max(psi) if psi else ZERO, farkas_gap=gain - cap_term,
                branches=branches)
