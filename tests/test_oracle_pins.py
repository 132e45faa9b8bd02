"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the pin it provides; together they are chosen so that a
plausible mistake in the oracle (a dropped term, a wrong sign or index, a
transposed operand, a wrong degree) fails at least one of them. None of these
tests uses the GPU library.
"""
import math
import os
import random
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from conftest import make_instance
from exact_ref import (ExactInstance, cap_bruteforce, cap_threshold, edge_objective, exact_pdr,
                       exact_report, lp_feasible, qp_bruteforce, qp_threshold)
from gen.instance import recipe_grid4_k8, recipe_small

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def two_vertex(d, u, K=1):
    """Arcs 0->1 and 1->0 with capacity u; K commodities 0 -> 1 with demand d."""
    return make_instance(2, [(0, 1), (1, 0)], u, [0] * K, [1] * K, [d] * K)


def read_golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = [p.strip() for p in line.split("|")]
            rows[parts[0]] = dict(d=Fr(parts[1]), u=Fr(parts[2]), K=int(parts[3]), method=parts[4],
                                  flows=[Fr(x) for x in parts[5].split()],
                                  flows1=[Fr(x) for x in parts[6].split()] if len(parts) > 6
                                  else None)
    return rows


# ------------------------------------------------------------------ P1: edge QP
def _rand_qp(rng, K):
    c = [Fr(rng.randint(-40, 40), rng.randint(1, 8)) for _ in range(K)]
    u = Fr(rng.randint(0, 60), rng.randint(1, 4))
    return c, u


def _qp_inputs_from_c(c):
    """Heights/flows giving potentials c under c_k = (h_i - h_j)/2 + f (f >= 0)."""
    fe = [Fr(abs(x.numerator) % 3, 2) for x in c]
    # choose h_i - h_j = 2 (c - f); split it as h_i = c - f, h_j = -(c - f)
    hi = [x - y for x, y in zip(c, fe)]
    hj = [-(x - y) for x, y in zip(c, fe)]
    return hi, hj, fe


def test_eso_edge_matches_bruteforce():
    """P1: Algorithm 2 in the oracle equals exact KKT enumeration of Expression 14."""
    rng = random.Random(11)
    for trial in range(400):
        K = rng.randint(1, 8)
        c, u = _rand_qp(rng, K)
        ref, psi_ref = qp_bruteforce(c, u)
        hi, hj, fe = _qp_inputs_from_c(c)
        out, psi, r, cong = oracle.eso_edge([float(x) for x in hi], [float(x) for x in hj],
                                            [float(x) for x in fe], float(u))
        scale = max(1.0, float(u), max(abs(float(x)) for x in c))
        assert np.max(np.abs(out - np.array([float(x) for x in ref]))) <= 1e-13 * scale
        assert abs(psi - float(psi_ref)) <= 1e-13 * scale
        # the slack: r = u - sum f' when uncongested, 0 when congested
        if psi_ref == 0:
            assert abs(r - max(0.0, float(u - sum(ref, Fr(0))))) <= 1e-12 * scale
        else:
            assert r == 0.0 and cong


def test_bruteforce_equals_threshold_method():
    """The two exact references (enumeration, threshold iteration) agree exactly."""
    rng = random.Random(5)
    for _ in range(300):
        c, u = _rand_qp(rng, rng.randint(1, 7))
        assert qp_bruteforce(c, u) == qp_threshold(c, u)


def test_eso_edge_special_cases():
    """P1 special cases: uncongested => max(0, c); K = 1 congested => (2c + u)/3;
    s == u exactly => psi = 0; u = 0."""
    # uncongested: s = 1 + 2 = 3 < 10
    out, psi, r, cong = oracle.eso_edge([1.0, 2.0, -3.0], [-1.0, -2.0, 3.0], [0.0, 0.0, 0.0], 10.0)
    assert np.array_equal(out, [1.0, 2.0, 0.0]) and psi == 0.0 and r == 7.0 and not cong
    # K = 1 congested: c = 9 > u = 3 -> f' = (2*9 + 3)/3 = 7, psi = 2 (9 - 3)/3 = 4
    out, psi, r, cong = oracle.eso_edge([9.0], [-9.0], [0.0], 3.0)
    assert out[0] == pytest.approx(7.0, abs=1e-14) and psi == pytest.approx(4.0, abs=1e-14)
    # boundary s == u: treated as uncongested, psi = 0 (reading of Algorithm 2)
    out, psi, r, cong = oracle.eso_edge([1.0, 2.0], [-1.0, -2.0], [0.0, 0.0], 3.0)
    assert np.array_equal(out, [1.0, 2.0]) and psi == 0.0 and r == 0.0
    # zero capacity, two equal potentials 3: psi = 6/2 = 3, f' = 3 - 3/2 = 3/2 each
    out, psi, r, cong = oracle.eso_edge([3.0, 3.0], [-3.0, -3.0], [0.0, 0.0], 0.0)
    assert np.allclose(out, [1.5, 1.5], atol=1e-14) and psi == pytest.approx(3.0)
    # all potentials non-positive: nothing flows
    out, psi, r, cong = oracle.eso_edge([-1.0, 0.0], [1.0, 0.0], [0.0, 0.0], 0.0)
    assert np.array_equal(out, [0.0, 0.0]) and psi == 0.0


def test_eso_edge_kkt_random_float():
    """P1 KKT check on FP inputs: f' = max(0, c - psi/2) and psi = max(0, sum f' - u)."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        K = int(rng.integers(1, 300))
        hi, hj = rng.normal(size=K) * 5, rng.normal(size=K) * 5
        fe = np.maximum(0, rng.normal(size=K) * 3)
        u = float(rng.uniform(0, 5 * K ** 0.5))
        out, psi, r, cong = oracle.eso_edge(hi, hj, fe, u)
        c = (hi - hj) / 2 + fe
        assert np.allclose(out, np.maximum(0, c - psi / 2), atol=1e-12, rtol=0)
        assert psi == pytest.approx(max(0.0, out.sum() - u), abs=1e-9 * max(1, u))


# ------------------------------------------------------------------ P2/P3: excess, z
def _random_flows(inst, seed, scale=3.0):
    rng = np.random.default_rng(seed)
    f = np.maximum(0.0, rng.normal(size=(inst.m, inst.K)) * scale)
    f[rng.random(size=f.shape) < 0.3] = 0.0
    return f


def test_excess_mass_conservation_and_initial_heights(grid4):
    """P2: sum_i Delta_ik = 0 for every k; at f = 0 Delta equals the injection of
    Expression 3 and z(0) = 1/2 sum_k d_k^2 (1/delta_s + 1/delta_t)."""
    inst = grid4
    Delta, h = oracle.excess(inst, _random_flows(inst, 1))
    assert np.max(np.abs(Delta.sum(axis=0))) < 1e-12
    Delta0, h0 = oracle.excess(inst, np.zeros((inst.m, inst.K)))
    hat = np.zeros((inst.n, inst.K))
    for k in range(inst.K):
        hat[inst.s[k], k] += inst.d[k]
        hat[inst.t[k], k] -= inst.d[k]
    assert np.array_equal(Delta0, hat)
    deg = oracle.degrees(inst)
    F, psi = oracle.congestion(inst, np.zeros((inst.m, inst.K)))
    z0 = oracle.objective(inst, h0, psi)[0]
    closed = 0.5 * sum(inst.d[k] ** 2 * (1 / deg[inst.s[k]] + 1 / deg[inst.t[k]])
                       for k in range(inst.K))
    assert z0 == pytest.approx(closed, rel=1e-14)


def test_degree_is_in_plus_out():
    """O1: grid degrees are 2 x (number of grid neighbours): 4 corners, 6 edges, 8 inner."""
    inst = recipe_small("grid", 4, 2, seed=3)
    deg = oracle.degrees(inst).reshape(4, 4)
    expect = np.array([[4, 6, 6, 4], [6, 8, 8, 6], [6, 8, 8, 6], [4, 6, 6, 4]])
    assert np.array_equal(deg, expect)


@pytest.mark.parametrize("kind,size,K", [("grid", 4, 8), ("knn", 30, 12)])
def test_objective_vertex_form_equals_edge_form(kind, size, K):
    """P3: z of Algorithm 1 (vertex form) equals the edge-sum form of Expression 8."""
    inst = recipe_small(kind, size, K, seed=4)
    f = _random_flows(inst, 2)
    _, h = oracle.excess(inst, f)
    _, psi = oracle.congestion(inst, f)
    z = oracle.objective(inst, h, psi)[0]
    assert z == pytest.approx(oracle.objective_edge_form(inst, h, psi), rel=1e-13)


def test_potential_difference_is_negative_gradient():
    """Remark 2: phi = h_i - h_j - psi equals -dz/df (central differences on z).
    Pins the signs and indices of the excess, height and congestion."""
    inst = recipe_small("knn", 12, 3, seed=9)
    rng = np.random.default_rng(0)
    f = rng.uniform(0.5, 2.0, size=(inst.m, inst.K))
    # make some arcs congested and others not (psi kinks are avoided by the margin)
    inst.u[: inst.m // 2] = f[: inst.m // 2].sum(axis=1) - 1.0
    inst.u[inst.m // 2:] = f[inst.m // 2:].sum(axis=1) + 1.0
    _, h = oracle.excess(inst, f)
    _, psi = oracle.congestion(inst, f)
    tails = inst.tails()

    def z_of(ff):
        _, hh = oracle.excess(inst, ff)
        _, pp = oracle.congestion(inst, ff)
        return oracle.objective(inst, hh, pp)[0]

    eps = 1e-6
    for e in range(inst.m):
        for k in range(inst.K):
            fp, fm = f.copy(), f.copy()
            fp[e, k] += eps
            fm[e, k] -= eps
            grad = (z_of(fp) - z_of(fm)) / (2 * eps)
            phi = h[tails[e], k] - h[inst.col[e], k] - psi[e]
            assert -grad == pytest.approx(phi, abs=1e-6)


# ------------------------------------------------------------------ P5: worked closed forms
@pytest.mark.parametrize("name", ["eso_infeasible", "eso_feasible", "agd_feasible", "agd_reject",
                                  "gdm_feasible", "cap_infeasible", "cap_feasible"])
def test_two_vertex_worked_examples(name):
    """P5: the oracle reproduces the hand-derived trajectories in tests/golden/two_vertex.txt."""
    g = read_golden("two_vertex.txt")[name]
    inst = two_vertex(float(g["d"]), float(g["u"]), g["K"])
    method = {"eso": oracle.ESO, "agd": oracle.AGD, "gdm": oracle.GDM,
              "cap": oracle.CAP}[g["method"]]
    st = oracle.State(inst, method)
    for step, expect in enumerate(g["flows"]):
        st.run(1)
        e0 = 0  # arc 0->1 is first in CSR order
        assert np.allclose(st.f[e0], float(expect), rtol=0, atol=1e-13 * float(g["d"])), (name, step)
        expect1 = 0.0 if g["flows1"] is None else float(g["flows1"][step])
        assert np.allclose(st.f[1], expect1, rtol=0, atol=1e-13 * float(g["d"])), (name, step)


def test_gdm_without_momentum_is_agd():
    """Algorithm 4 with gamma = 0 is Algorithm 3 (the step never drives f below 0,
    so max(0, f + df) = f + df)."""
    inst = recipe_small("knn", 30, 9, seed=6, u_range=(1, 6), d_range=(1, 6))
    prm = oracle.default_agd_params(inst.K)
    a, za = oracle.run(inst, oracle.AGD, 150, params=prm)
    b, zb = oracle.run(inst, oracle.GDM, 150, params=dict(prm, gamma=0.0))
    assert np.array_equal(a.f, b.f) and np.array_equal(a.beta, b.beta)
    assert np.array_equal(za, zb)


def test_two_vertex_fixed_point_and_farkas_gap():
    """P5: d = 10, u = 8 converges to f = (d + u)/2 = 9, z* = (d - u)^2/4 = 1, G = 2 z* = 2,
    and the verdict is infeasible; d = 6 converges to z -> 0 with verdict feasible."""
    inst = two_vertex(10.0, 8.0)
    st, zs = oracle.run(inst, oracle.ESO, 200)
    assert st.f[0, 0] == pytest.approx(9.0, abs=1e-12)
    rep = oracle.report(inst, st.f)
    assert rep["z"] == pytest.approx(1.0, abs=1e-12)
    assert rep["farkas_gap"] == pytest.approx(2.0, abs=1e-12)
    assert rep["verdict"] == "infeasible"
    inst = two_vertex(6.0, 8.0)
    st, zs = oracle.run(inst, oracle.ESO, 60)
    rep = oracle.report(inst, st.f)
    assert rep["z"] <= 1e-30 and rep["verdict"] == "feasible" and rep["farkas_gap"] <= 0


# ------------------------------------------------------------------ AGD step
def test_agd_objective_change_is_exact_subproblem_difference():
    """The oracle's AGD estimate of the objective change equals the exact difference
    of the edge subproblem objective (Expression 13, optimal slack) in rationals."""
    rng = random.Random(8)
    for _ in range(300):
        K = rng.randint(1, 6)
        hi = [Fr(rng.randint(-20, 20), 4) for _ in range(K)]
        hj = [Fr(rng.randint(-20, 20), 4) for _ in range(K)]
        fe = [Fr(rng.randint(0, 12), 2) for _ in range(K)]
        u = Fr(rng.randint(0, 30), 2)
        beta = Fr(1, 2 ** rng.randint(1, 4))
        F = sum(fe, Fr(0))
        psi = max(Fr(0), F - u)
        dfs = [max(-fe[k], beta * (hi[k] - hj[k] - psi)) for k in range(K)]
        exact = edge_objective(F, dfs, hi, hj, u) - edge_objective(F, [Fr(0)] * K, hi, hj, u)
        out, b, acc, dz = oracle.agd_edge([float(x) for x in hi], [float(x) for x in hj],
                                          [float(x) for x in fe], float(u), 1, float(beta))
        assert dz == pytest.approx(float(exact), abs=1e-12)
        assert acc == (exact <= 0)
        if acc:
            assert np.allclose(out, [float(x + y) for x, y in zip(fe, dfs)], atol=1e-14)
        else:
            assert np.array_equal(out, [float(x) for x in fe])
            assert b == max(1.0 / K, float(beta) / 2)


def test_gdm_step_is_exact_algorithm_4_step():
    """One GDM arc step of the oracle against Algorithm 4's step in exact
    rationals: the gradient step and its objective change are Algorithm 3's
    (Expression 13, optimal slack); an accepted step sets v' = gamma v + df and
    f' = max(0, f + v') (so momentum can carry a flow past its own step, down
    to zero), a rejected one keeps f and v and scales beta by alpha_dec
    (floored at beta_min), and every inc_period-th pass scales beta by
    alpha_inc (capped at beta_max). Dyadic inputs and gamma = 3/4 keep every
    binary64 operation exact; both decisions and both t cases occur."""
    rng = random.Random(44)
    seen = set()
    for _ in range(400):
        K = rng.randint(1, 6)
        hi = [Fr(rng.randint(-24, 24), 4) for _ in range(K)]
        hj = [Fr(rng.randint(-24, 24), 4) for _ in range(K)]
        fe = [Fr(rng.randint(0, 16), 2) for _ in range(K)]
        ve = [Fr(rng.randint(-16, 16), 4) for _ in range(K)]
        u = Fr(rng.randint(0, 40), 2)
        beta = Fr(1, 2 ** rng.randint(1, 5))
        t = rng.choice([3, 10, 20, 7])
        prm = dict(beta_init=0.1, beta_min=1.0 / 16, beta_max=0.25, alpha_inc=2.0,
                   alpha_dec=0.5, inc_period=10, gamma=0.75)
        F = sum(fe, Fr(0))
        psi = max(Fr(0), F - u)
        dfs = [max(-fe[k], beta * (hi[k] - hj[k] - psi)) for k in range(K)]
        dz = edge_objective(F, dfs, hi, hj, u) - edge_objective(F, [Fr(0)] * K, hi, hj, u)
        acc_x = dz <= 0
        if acc_x:
            v_x = [Fr(3, 4) * ve[k] + dfs[k] for k in range(K)]
            f_x = [max(Fr(0), fe[k] + v_x[k]) for k in range(K)]
            b_x = beta
        else:
            v_x, f_x = list(ve), list(fe)
            b_x = max(Fr(1, 16), beta / 2)
        if t % 10 == 0:
            b_x = min(Fr(1, 4), b_x * 2)
        fo, vo, b, acc, dzo = oracle.gdm_edge([float(x) for x in hi], [float(x) for x in hj],
                                              [float(x) for x in fe], [float(x) for x in ve],
                                              float(u), t, float(beta), prm)
        assert acc == acc_x
        assert dzo == float(dz)
        assert list(fo) == [float(x) for x in f_x]
        assert list(vo) == [float(x) for x in v_x]
        assert b == float(b_x)
        seen.add((acc_x, t % 10 == 0, any(fe[k] + v_x[k] < 0 for k in range(K)) if acc_x else None))
    assert {(True, True), (True, False), (False, True), (False, False)} <= {x[:2] for x in seen}
    assert (True, False, True) in seen or (True, True, True) in seen  # momentum clipped at zero


def test_agd_accept_decision_near_convergence():
    """Reading 12's factored congestion term, pinned where it decides: the two
    golden cases (tests/golden/agd_accept.txt) make the accept test of
    Algorithm 3 a small difference of large terms. The oracle's decision and
    objective change match exact rationals of the same binary64 inputs, and the
    difference of two squares evaluated in binary64 would decide each case the
    other way (so the pin discriminates between the two forms)."""
    rows = {}
    with open(os.path.join(GOLDEN, "agd_accept.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                p = [x.strip() for x in line.split("|")]
                rows[p[0]] = (float.fromhex(p[1]), float.fromhex(p[2]), float.fromhex(p[3]), p[4])
    assert set(rows) == {"reject", "accept"}
    u = 8.0
    for name, (hi, f, beta, decision) in rows.items():
        exact = (edge_objective(Fr(f), [max(-Fr(f), Fr(beta) * (Fr(hi) - (Fr(f) - Fr(u))))],
                                [Fr(hi)], [Fr(0)], Fr(u))
                 - edge_objective(Fr(f), [Fr(0)], [Fr(hi)], [Fr(0)], Fr(u)))
        assert (exact <= 0) == (decision == "accept"), name
        out, b, acc, dz = oracle.agd_edge([hi], [0.0], [f], u, 1, beta)
        assert acc == (decision == "accept"), name
        assert dz == pytest.approx(float(exact), rel=1e-6, abs=1e-12), name
        # the unfactored form, in binary64
        psi = f - u
        df = max(-f, beta * (hi - psi))
        after = f + df - u
        naive = 0.5 * (after * after - psi * psi) + df * (df - hi)
        assert (naive <= 0) != (decision == "accept"), name
    hi, f, beta, _ = rows["reject"]
    assert float(exact_ref_dz := (edge_objective(Fr(f), [Fr(1, 8)], [Fr(hi)], [Fr(0)], Fr(u))
                                  - edge_objective(Fr(f), [Fr(0)], [Fr(hi)], [Fr(0)], Fr(u)))) \
        == 2.0 ** -7, exact_ref_dz


# ------------------------------------------------------------------ residual report
def _read_report_golden():
    rows = {}
    with open(os.path.join(GOLDEN, "two_vertex_report.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                p = [x.strip() for x in line.split("|")]
                rows[p[0]] = [Fr(x) for x in p[1:]]
    return rows


def test_report_hand_derived_two_vertex():
    """The residual report (kkt of Section 3.3's stable-flow conditions, z,
    max |Delta|, max psi, Farkas gap) at hand-derived non-stationary pseudo-flows
    of the two-vertex instance (tests/golden/two_vertex_report.txt): unused arcs
    with phi > 0 and phi < 0, congested arcs, used arcs with phi < 0."""
    inst = two_vertex(10.0, 8.0)
    rows = _read_report_golden()
    assert set(rows) == {"f0", "f3", "f4", "r1", "r2"}
    for name, (a, b, kkt, z, zpsi, maxd, maxpsi, gap) in rows.items():
        f = np.array([[float(a)], [float(b)]])
        rep = oracle.report(inst, f)
        for key, want in (("kkt_sq", kkt), ("z", z), ("z_psi", zpsi), ("max_abs_excess", maxd),
                          ("max_congestion", maxpsi), ("farkas_gap", gap)):
            assert rep[key] == pytest.approx(float(want), rel=1e-14, abs=1e-14), (name, key)
        ex = exact_report(ExactInstance.from_instance(inst), [[Fr(a)], [Fr(b)]])
        assert ex["kkt_sq"] == kkt and ex["z"] == z and ex["farkas_gap"] == gap, name
    # the verdict: G > 0 certifies infeasibility already at f3 (Theorem 2's direction)
    assert oracle.report(inst, np.array([[8.5], [0.0]]))["verdict"] == "infeasible"


@pytest.mark.parametrize("method", [oracle.ESO, oracle.AGD, oracle.GDM])
@pytest.mark.parametrize("T", [2, 3, 11])
def test_report_matches_exact_rationals_at_non_stationary_iterates(grid4, method, T):
    """kkt_sq and the rest of the report at congested iterates away from a
    stationary point: the FP64 oracle's report of its own flows after T passes
    equals the exact-rational report of the same flows (independent code), on
    iterates where every branch of the kkt residual occurs (congested arcs,
    used entries with phi < 0, unused entries with phi > 0)."""
    import dataclasses
    inst = dataclasses.replace(grid4, d=grid4.d * 20.0)  # congested
    st, _ = oracle.run(inst, method, T)
    rep = oracle.report(inst, st.f)
    ex = ExactInstance.from_instance(inst)
    fx = [[Fr(float(x)) for x in row] for row in st.f]
    want = exact_report(ex, fx)
    assert want["branches"] == dict(congested=True, used_negative=True, unused_positive=True)
    assert want["kkt_sq"] > 0
    for key in ("kkt_sq", "z", "z_psi", "z_h", "max_abs_excess", "max_congestion"):
        assert rep[key] == pytest.approx(float(want[key]), rel=1e-12, abs=1e-12), key
    assert rep["farkas_gap"] == pytest.approx(float(want["farkas_gap"]),
                                              abs=1e-12 * float(np.max(inst.u)) * inst.m)


# ------------------------------------------------------------------ P4: exact sweeps
@pytest.mark.parametrize("method", ["eso", "agd", "gdm", "cap"])
def test_oracle_matches_exact_rational_sweeps(grid4, method):
    """P4: 60 sweeps in exact rationals (independent code: threshold QP, in/out arc
    lists, direct subproblem differences) match the FP64 oracle to 1e-12 max(u)."""
    inst = grid4
    ex = ExactInstance.from_instance(inst)
    f_ex, z_ex = exact_pdr(ex, method, 60)
    st, zs = oracle.run(inst, {"eso": oracle.ESO, "agd": oracle.AGD, "gdm": oracle.GDM,
                               "cap": oracle.CAP}[method], 60)
    f_ex = np.array([[float(x) for x in row] for row in f_ex])
    tol = 1e-12 * float(np.max(inst.u))
    assert np.max(np.abs(st.f - f_ex)) <= tol
    assert np.max(np.abs(zs - np.array([float(z) for z in z_ex]))) <= 1e-12 * max(1.0, zs[0])


# ------------------------------------------------------------------ P6: monotone z
@pytest.mark.parametrize("method", [oracle.ESO, oracle.AGD, oracle.CAP])
@pytest.mark.parametrize("kind,size,K,seed", [("grid", 4, 8, 1), ("knn", 40, 30, 2),
                                              ("grid", 5, 20, 3)])
def test_objective_monotone(method, kind, size, K, seed):
    """P6: z is non-increasing (convergence theorem of Section 4.3; AGD accepts only
    steps that do not increase the local objective, and the same Jensen step applies)."""
    inst = recipe_small(kind, size, K, seed=seed, u_range=(2, 10), d_range=(1, 8))
    st, zs = oracle.run(inst, method, 300)
    assert np.all(zs[1:] <= zs[:-1] * (1 + 1e-13) + 1e-300)


# ------------------------------------------------------------------ P7: optimality
def test_converged_eso_is_stable_pseudoflow(grid4):
    """P7: after convergence the flow satisfies the stable-flow optimality conditions
    (Section 3.3) and, on this feasible instance, is zero-stable (Definition 2)."""
    st, zs = oracle.run(grid4, oracle.ESO, 500)
    rep = oracle.report(grid4, st.f)
    assert rep["kkt_sq"] < 1e-20
    assert rep["max_abs_excess"] < 1e-9 and rep["max_congestion"] < 1e-9
    assert rep["verdict"] == "feasible" and rep["farkas_gap"] <= 0


def test_eso_fixed_point_characterisation():
    """P7: an ESO fixed point is stable: f = max(0, f + phi/2) on uncongested arcs."""
    inst = recipe_small("grid", 3, 4, seed=2, u_range=(50, 60), d_range=(1, 3))
    st, _ = oracle.run(inst, oracle.ESO, 3000)
    _, h = oracle.excess(inst, st.f)
    _, psi = oracle.congestion(inst, st.f)
    tails = inst.tails()
    phi = h[tails] - h[inst.col] - psi[:, None]
    assert np.all(np.abs(np.where(st.f > 1e-9, phi, np.maximum(phi, 0))) < 1e-9)


# ------------------------------------------------------------------ P8: verdicts
def _tiny_instances():
    rng = np.random.default_rng(42)
    out = []
    for trial in range(8):
        n = int(rng.integers(3, 6))
        pairs = [(i, j) for i in range(n) for j in range(n) if i != j]
        sel = rng.choice(len(pairs), size=min(len(pairs), int(rng.integers(n, 2 * n + 2))),
                         replace=False)
        arcs = [pairs[q] for q in sel]
        K = int(rng.integers(1, 4))
        st = []
        for _ in range(K):
            a, b = rng.choice(n, size=2, replace=False)
            st.append((int(a), int(b)))
        u = rng.integers(1, 6, size=len(arcs)).astype(float)
        d = rng.integers(1, 5, size=K).astype(float)
        out.append((n, arcs, u, [p[0] for p in st], [p[1] for p in st], d))
    return out


def test_verdict_matches_exact_lp_feasibility():
    """P8 (i): the oracle's verdict equals exact-rational LP feasibility on tiny graphs."""
    decided = 0
    for n, arcs, u, s, t, d in _tiny_instances():
        inst = make_instance(n, arcs, u, s, t, d)
        deg = oracle.degrees(inst)
        if np.any(deg[inst.s] == 0) or np.any(deg[inst.t] == 0):
            continue
        truth = lp_feasible(ExactInstance.from_instance(inst))
        st = oracle.State(inst, oracle.ESO)
        verdict = "undecided"
        for _ in range(200):
            st.run(500, record=False)
            verdict = oracle.report(inst, st.f)["verdict"]
            if verdict != "undecided":
                break
        if verdict == "undecided":
            continue
        decided += 1
        assert verdict == ("feasible" if truth else "infeasible"), (n, arcs, s, t, d)
    assert decided >= 6


def test_verdict_matches_maxflow_single_commodity():
    """P8 (ii): K = 1 is feasible iff max-flow(s, t) >= d (scipy maximum_flow)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_flow
    rng = np.random.default_rng(7)
    checked = 0
    for trial in range(10):
        inst = recipe_small("knn", 10, 1, seed=100 + trial, u_range=(1, 6), d_range=(1, 1))
        A = csr_matrix((inst.u.astype(np.int32), inst.col, inst.row_ptr), shape=(inst.n, inst.n))
        mf = maximum_flow(A, int(inst.s[0]), int(inst.t[0])).flow_value
        d = float(mf) * (0.7 if trial % 2 == 0 else 1.4)
        inst.d[:] = d
        st = oracle.State(inst, oracle.ESO)
        verdict = "undecided"
        for _ in range(100):
            st.run(500, record=False)
            verdict = oracle.report(inst, st.f)["verdict"]
            if verdict != "undecided":
                break
        assert verdict == ("feasible" if mf >= d else "infeasible")
        checked += 1
    assert checked == 10


# ------------------------------------------------------------------ P10/P11/P12
def test_scale_covariance_bitwise(grid4):
    """P10: (u, d) -> (4u, 4d) scales every iterate by 4 exactly (powers of two)."""
    for method in (oracle.ESO, oracle.AGD, oracle.GDM):
        a, za = oracle.run(grid4, method, 50)
        b, zb = oracle.run(grid4.scaled(4.0), method, 50)
        assert np.array_equal(b.f, 4.0 * a.f)
        assert np.array_equal(zb, 16.0 * za)
        assert np.array_equal(a.beta, b.beta)


def test_permutation_equivariance():
    """P11: relabelling commodities and vertices permutes the iterates."""
    inst = recipe_small("knn", 25, 6, seed=3)
    st, _ = oracle.run(inst, oracle.ESO, 80)
    # commodity permutation
    perm = np.random.default_rng(0).permutation(inst.K)
    inst2 = make_instance(inst.n, list(zip(inst.tails().tolist(), inst.col.tolist())), inst.u,
                          inst.s[perm], inst.t[perm], inst.d[perm])
    st2, _ = oracle.run(inst2, oracle.ESO, 80)
    assert np.allclose(st2.f, st.f[:, perm], atol=1e-12)
    # vertex relabelling: arcs are re-sorted into CSR order
    vp = np.random.default_rng(1).permutation(inst.n)
    arcs = [(int(vp[a]), int(vp[b])) for a, b in zip(inst.tails(), inst.col)]
    inst3 = make_instance(inst.n, arcs, inst.u, vp[inst.s], vp[inst.t], inst.d)
    st3, _ = oracle.run(inst3, oracle.ESO, 80)
    order = sorted(range(len(arcs)), key=lambda q: arcs[q])
    assert np.allclose(st3.f, st.f[order], atol=1e-12)


def test_zero_commodity_padding_is_exact(grid4):
    """P12: an extra commodity with zero demand never carries flow and leaves the
    other commodities' iterates unchanged."""
    inst = grid4
    s = np.append(inst.s, 0)
    t = np.append(inst.t, 5)
    d = np.append(inst.d, 0.0)
    inst2 = make_instance(inst.n, list(zip(inst.tails().tolist(), inst.col.tolist())), inst.u,
                          s, t, d)
    for method in (oracle.ESO,):
        a, _ = oracle.run(inst, method, 50)
        b, _ = oracle.run(inst2, method, 50)
        assert np.array_equal(b.f[:, -1], np.zeros(inst.m))
        assert np.array_equal(b.f[:, :-1], a.f)


# ------------------------------------------------------------------ run semantics
def test_resume_equals_single_run(grid4):
    """T sweeps then T' sweeps equal T + T' sweeps bitwise (state: f, beta, t, z_prev)."""
    for method in (oracle.ESO, oracle.AGD, oracle.GDM):
        a, _ = oracle.run(grid4, method, 37)
        b = oracle.State(grid4, method)
        b.run(20)
        b.run(17)
        assert np.array_equal(a.f, b.f) and np.array_equal(a.beta, b.beta) and a.t == b.t
        assert np.array_equal(a.v, b.v)


def test_stop_rule_is_checked_before_update(grid4):
    """Algorithm 1: the |z - z_prev| < eps test precedes the update, so a stop at pass p
    leaves f^(p) (p updates) and records z^(0..p)."""
    st, zs = oracle.run(grid4, oracle.ESO, 10_000, eps_obj=1e-6)
    assert st.stopped
    assert len(zs) == st.t + 1
    assert abs(zs[-1] - zs[-2]) < 1e-6 and np.all(np.abs(np.diff(zs[:-1])) >= 1e-6)


# ------------------------------------------------------------------ P13: forward-mode tangent
def test_eso_tangent_two_vertex_closed_forms():
    """d <= u: z_T = (d^2/2) 4^-T, so dz_T/dd = d 4^-T and dz_T/du = 0. d > u: the
    limit f* = (d+u)/2 has z* = (d-u)^2/4, so dz*/dd = (d-u)/2 and dz*/du_01 = -(d-u)/2
    (the reverse arc carries nothing)."""
    inst = two_vertex(6.0, 8.0)
    for T in (1, 2, 5, 9):
        z, gu, gd = oracle.eso_gradient(inst, T)
        assert z == pytest.approx(18.0 * 4.0 ** -T, rel=1e-14)
        assert gd[0] == pytest.approx(6.0 * 4.0 ** -T, rel=1e-14)
        assert np.all(gu == 0.0)
    inst = two_vertex(10.0, 8.0)
    z, gu, gd = oracle.eso_gradient(inst, 80)
    assert z == pytest.approx(1.0, abs=1e-12)
    assert gd[0] == pytest.approx(1.0, abs=1e-12)
    assert gu[0] == pytest.approx(-1.0, abs=1e-12) and gu[1] == 0.0


def _exact_z_after(ex, T):
    """z(f^T) in exact rationals: the objective evaluated before pass T + 1."""
    return exact_pdr(ex, "eso", T + 1)[1][T]


def test_eso_tangent_matches_exact_difference_quotients():
    """On a small congested instance the exact-rational difference quotient
    (z(theta + eps e_j) - z(theta)) / eps with eps = 1e-30 equals the derivative
    up to O(eps) away from kinks; the FP64 tangent must agree to 1e-9."""
    inst = recipe_small("grid", 3, 3, seed=7, u_range=(2, 5), d_range=(4, 9))
    T = 5
    z, gu, gd = oracle.eso_gradient(inst, T)
    ex = ExactInstance.from_instance(inst)
    z0 = _exact_z_after(ex, T)
    assert float(z0) == pytest.approx(z, rel=1e-12)
    assert np.any(gu != 0.0), "the instance should have congested arcs"
    eps = Fr(1, 10 ** 30)
    rng = random.Random(3)
    coords = rng.sample(range(inst.m), 6) + list(range(inst.m, inst.m + inst.K))
    for j in coords:
        u = list(ex.u)
        d = list(ex.d)
        if j < inst.m:
            u[j] += eps
        else:
            d[j - inst.m] += eps
        exj = ExactInstance(ex.n, inst.row_ptr, inst.col, u, inst.s, inst.t, d)
        quot = float((_exact_z_after(exj, T) - z0) / eps)
        tang = gu[j] if j < inst.m else gd[j - inst.m]
        assert abs(quot - tang) <= 1e-9 * max(1.0, abs(tang)), (j, quot, tang)


def test_eso_tangent_matches_central_differences():
    """The grid4_k8 instance with demands x20 (infeasible, many congested arcs),
    64 sweeps: forward-mode gradient vs central differences (h = 1e-6) of the
    FP64 oracle's own z(f^T) for every capacity and demand."""
    import dataclasses
    base = recipe_grid4_k8()
    inst = dataclasses.replace(base, d=base.d * 20.0)
    T, h = 64, 1e-6
    z, gu, gd = oracle.eso_gradient(inst, T)

    def zT(i2):
        return oracle.run(i2, oracle.ESO, T + 1)[1][T]

    scale = max(np.abs(gu).max(), np.abs(gd).max())
    for j in range(inst.m):
        up, um = inst.u.copy(), inst.u.copy()
        up[j] += h
        um[j] -= h
        fd = (zT(dataclasses.replace(inst, u=up)) - zT(dataclasses.replace(inst, u=um))) / (2 * h)
        assert abs(fd - gu[j]) <= 1e-5 * scale, j
    for k in range(inst.K):
        dp, dm = inst.d.copy(), inst.d.copy()
        dp[k] += h
        dm[k] -= h
        fd = (zT(dataclasses.replace(inst, d=dp)) - zT(dataclasses.replace(inst, d=dm))) / (2 * h)
        assert abs(fd - gd[k]) <= 1e-5 * scale, k


def test_violation_bounds_follow_from_z():
    """P9: z >= psi_e^2 / 2 and z >= Delta_ik^2 / (2 delta_i) term by term, so at
    every iterate max psi <= sqrt(2 z) and |Delta_ik| <= sqrt(2 z delta_i); the
    report's max congestion and max |excess| are the maxima of those terms."""
    inst = recipe_small("knn", 30, 12, seed=9, u_range=(1, 4), d_range=(2, 8))
    deg = oracle.degrees(inst)
    st = oracle.State(inst, oracle.ESO)
    done = 0
    for T in (0, 1, 5, 40):
        st.run(T - done)
        done = T
        rep = oracle.report(inst, st.f)
        Delta, _ = oracle.excess(inst, st.f)
        _, psi = oracle.congestion(inst, st.f)
        z = rep["z"]
        assert rep["max_congestion"] == pytest.approx(float(psi.max()), rel=1e-14, abs=0)
        assert rep["max_abs_excess"] == pytest.approx(float(np.abs(Delta).max()), rel=1e-14, abs=0)
        assert psi.max() <= math.sqrt(2 * z) * (1 + 1e-12)
        assert np.all(np.abs(Delta) <= np.sqrt(2 * z * deg)[:, None] * (1 + 1e-12))


# ------------------------------------------------------------------ capacity-enforcing loop (Section 6)
def test_cap_edge_matches_exact_projection():
    """The capacity-enforcing edge step equals the exact projection onto
    {f >= 0, sum f <= u} found by support enumeration, which equals the
    threshold iteration."""
    rng = random.Random(21)
    for _ in range(300):
        K = rng.randint(1, 7)
        c, u = _rand_qp(rng, K)
        ref, _ = cap_bruteforce(c, u)
        thr, lam = cap_threshold(c, u)  # lam: the smallest multiplier (unique unless u = 0)
        assert ref == thr
        hi, hj, fe = _qp_inputs_from_c(c)
        out, lam_o, binds = oracle.cap_edge([float(x) for x in hi], [float(x) for x in hj],
                                            [float(x) for x in fe], float(u))
        scale = max(1.0, float(u), max(abs(float(x)) for x in c))
        assert np.max(np.abs(out - np.array([float(x) for x in ref]))) <= 1e-13 * scale
        assert abs(lam_o - float(lam)) <= 1e-13 * scale
        assert binds == (sum((x for x in c if x > 0), Fr(0)) > u)


def test_cap_keeps_every_capacity():
    """Starting from f = 0 the loop never exceeds a capacity (each edge step is a
    projection onto the arc's capacity set) beyond the rounding of the sum, so
    the congestion term stays at the rounding level."""
    inst = recipe_small("knn", 40, 30, seed=2, u_range=(1, 4), d_range=(2, 9))
    st = oracle.State(inst, oracle.CAP)
    for _ in range(20):
        st.run(10)
        F, psi = oracle.congestion(inst, st.f)
        assert np.any(F >= inst.u * (1 - 1e-12))  # capacities do bind
        assert np.all(F <= inst.u * (1 + 1e-14))
        assert np.all(psi <= 1e-14 * inst.u)


def test_cap_fixed_point_meets_the_pipe_pressure_conditions():
    """Section 6's KKT conditions at convergence, with gamma_e the pipe pressure
    (0 on an unsaturated arc): a used commodity has h_i - h_j = gamma_e (so 0 on
    an unsaturated arc, and the same value for every used commodity of a
    saturated arc); an unused one has h_i - h_j <= gamma_e."""
    inst = recipe_small("grid", 4, 6, seed=5, u_range=(1, 3), d_range=(2, 6))
    st, zs = oracle.run(inst, oracle.CAP, 20000, eps_obj=1e-15)
    rep = oracle.report(inst, st.f)
    assert rep["z"] > 1e-3 and rep["verdict"] == "infeasible"  # capacities bind
    _, h = oracle.excess(inst, st.f)
    F, _ = oracle.congestion(inst, st.f)
    tails = inst.tails()
    tol = 1e-5 * float(np.max(np.abs(h)))
    saturated = 0
    for e in range(inst.m):
        diff = h[tails[e]] - h[inst.col[e]]
        used = st.f[e] > 1e-9 * float(np.max(inst.d))
        sat = F[e] >= inst.u[e] * (1 - 1e-9)
        if sat:
            saturated += 1
            gamma = float(diff[used].max()) if used.any() else max(0.0, float(diff.max()))
            assert gamma >= -tol
        else:
            gamma = 0.0
        assert np.all(np.abs(diff[used] - gamma) <= tol), e
        assert np.all(diff[~used] <= gamma + tol), e
    assert saturated > 0


def test_oracle_results_do_not_depend_on_its_thread_count():
    """The oracle parallelises only over outputs that are independent by
    definition (commodity ranges of the excess, arcs of the update) and sums
    serially, so runs with 1, 3 and 4 threads give the same bits (flows, z
    trajectory, learning rates, velocities, tangent). The instance is large
    enough (m K >= 65,536) for every parallel region to run threaded."""
    inst = recipe_small("knn", 300, 400, seed=31, u_range=(20, 90), d_range=(1, 6))
    assert inst.m * inst.K >= 65536
    nt0 = oracle.num_threads()
    out = {}
    try:
        for nt in (1, 3, 4):
            oracle.set_num_threads(nt)
            r = {}
            for name, meth in (("eso", oracle.ESO), ("agd", oracle.AGD), ("gdm", oracle.GDM),
                               ("cap", oracle.CAP)):
                st, zs = oracle.run(inst, meth, 12)
                r[name] = (st.f.copy(), zs.copy(), st.beta.copy(), st.v.copy())
            rng = np.random.default_rng(5)
            r["tangent"] = oracle.eso_tangent(inst, 6, rng.normal(size=inst.m),
                                              rng.normal(size=inst.K))
            out[nt] = r
    finally:
        oracle.set_num_threads(nt0)
    for nt in (3, 4):
        for name in ("eso", "agd", "gdm", "cap"):
            for a, b in zip(out[1][name], out[nt][name]):
                assert np.array_equal(a, b), (nt, name)
        f1, fd1, z1, zd1 = out[1]["tangent"]
        f2, fd2, z2, zd2 = out[nt]["tangent"]
        assert np.array_equal(f1, f2) and np.array_equal(fd1, fd2) and z1 == z2 and zd1 == zd2
