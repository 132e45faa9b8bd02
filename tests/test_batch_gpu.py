"""Batched sweeps (pdr_batch_*) through the C ABI.

A batch member runs the same per-arc and per-vertex code as a single context,
so its flows after T sweeps equal those of a single context of the same
instance bit for bit (the objective's partial sums are grouped differently, so
z agrees to rounding). Members are also checked against the FP64 oracle, for
per-instance stopping, graph replays and the autotuner.
"""
import functools
import sys

import numpy as np
import pytest

import oracle
import paper_2108_07549_amd as pdr
from conftest import make_instance
from gen.instance import recipe_grid4_k8, recipe_small

pytestmark = pytest.mark.gpu

METHODS = {"eso": (pdr.ESO, oracle.ESO), "agd": (pdr.AGD, oracle.AGD),
           "gdm": (pdr.GDM, oracle.GDM), "cap": (pdr.CAP, oracle.CAP)}


def say(*a):
    print("[gpu-batch]", *a, flush=True)
    sys.stdout.flush()


def flow_tol(inst):
    scale = float(np.max(inst.u)) if inst.m else 0.0
    if scale == 0.0:
        scale = float(np.max(inst.d))
    return 1e-9 * max(scale, 1e-300)


def mixed_batch():
    """Uneven sizes and commodity counts: several tiling buckets, ragged K."""
    return [recipe_grid4_k8(),
            recipe_small("knn", 60, 5, seed=11, u_range=(2, 9), d_range=(1, 6)),
            recipe_small("knn", 300, 61, seed=12, u_range=(5, 30), d_range=(1, 6)),
            recipe_small("grid", 9, 130, seed=13, u_range=(10, 60), d_range=(1, 5)),
            recipe_small("knn", 120, 257, seed=14, u_range=(20, 90), d_range=(1, 4)),
            recipe_small("grid", 6, 1, seed=15, u_range=(1, 3), d_range=(4, 4)),
            recipe_small("knn", 40, 700, seed=16, u_range=(50, 400), d_range=(1, 3))]


@pytest.mark.parametrize("precision", [pdr.FP64, pdr.FP32_BULK])
@pytest.mark.parametrize("method", list(METHODS))
def test_batch_members_equal_single_contexts(method, precision):
    gm, _ = METHODS[method]
    insts = mixed_batch()
    T = 40
    with pdr.Batch(insts, method=gm, precision=precision) as b:
        say("batch", method, precision, "buckets", b.buckets())
        b.sweep(T)
        got = []
        for q in range(len(insts)):
            c = b.member(q)
            got.append((c.flows(), c.z_log(0, T), c.learning_rates(),
                        c.velocities() if gm == pdr.GDM else None, c.residual()))
    for q, inst in enumerate(insts):
        with pdr.Context.from_instance(inst, method=gm, precision=precision) as c:
            c.sweep(T)
            f, zl = c.flows(), c.z_log(0, T)
            assert np.array_equal(got[q][0], f), q
            assert np.allclose(got[q][1], zl, rtol=1e-12, atol=0), q
            if gm != pdr.ESO:
                assert np.array_equal(got[q][2], c.learning_rates()), q
            if gm == pdr.GDM:
                assert np.array_equal(got[q][3], c.velocities()), q
            assert got[q][4]["sweeps_done"] == T


def oracle_perturbation_response(inst, om, T):
    """How far the oracle's own iterate moves after T sweeps when every capacity
    is changed by a relative 1e-15: the conditioning of the trajectory."""
    import dataclasses
    a, _ = oracle.run(inst, om, T)
    b, _ = oracle.run(dataclasses.replace(inst, u=inst.u * (1 + 1e-15)), om, T)
    return float(np.max(np.abs(a.f - b.f)))


@pytest.mark.parametrize("method", list(METHODS))
def test_batch_members_match_the_oracle(method):
    """GDM's momentum can amplify rounding-level differences (on grid9_k130 a
    1e-15 relative change of u moves the oracle's own flows by 4e-7 after 60
    sweeps), so GDM is compared at 30 sweeps, where the oracle's response to
    such a change is checked to stay far below the tolerance."""
    gm, om = METHODS[method]
    insts = mixed_batch()
    T = 30 if method == "gdm" else 60
    with pdr.Batch(insts, method=gm) as b:
        b.sweep(T)
        for q, inst in enumerate(insts):
            if method == "gdm":
                assert oracle_perturbation_response(inst, om, T) <= 1e-2 * flow_tol(inst), q
            st, zo = oracle.run(inst, om, T)
            c = b.member(q)
            assert np.max(np.abs(c.flows() - st.f)) <= flow_tol(inst), q
            assert np.allclose(c.z_log(0, T), zo, rtol=1e-9, atol=1e-12 * zo[0]), q
            assert c.residual()["verdict"] == oracle.report(inst, st.f)["verdict"], q


def converging_batch():
    """Members that reach z <= 1e-8 within a few thousand sweeps (171 to 3234)."""
    mb = mixed_batch()
    return [mb[0], mb[1], mb[3], mb[5]]


def test_batch_members_stop_on_their_own():
    """z_target and eps stop each member at the oracle's pass; the others go on."""
    insts = converging_batch()
    for eps, zt in ((0.0, 1e-8), (1e-6, 0.0)):
        with pdr.Batch(insts, method=pdr.ESO, graph_sweeps=8) as b:
            b.sweep(20_000, eps, zt)
            assert b.stopped() == len(insts)
            for q, inst in enumerate(insts):
                st, zo = oracle.run(inst, oracle.ESO, 20_000, eps_obj=eps, z_target=zt)
                res = b.member(q).residual()
                say("stop", eps, zt, q, res["sweeps_done"], st.t)
                assert res["stopped"] == 1 and res["sweeps_done"] == st.t, q
                assert np.max(np.abs(b.member(q).flows() - st.f)) <= flow_tol(inst), q


def test_batch_graph_replays_match_direct_launches():
    insts = mixed_batch()
    with pdr.Batch(insts, method=pdr.AGD, graph_sweeps=8) as g, \
            pdr.Batch(insts, method=pdr.AGD, graph_sweeps=-1) as d:
        for rep in range(4):
            g.sweep(8)
            d.sweep(8)
            for q in range(len(insts)):
                assert np.array_equal(g.member(q).flows(), d.member(q).flows()), (rep, q)
        g.sweep(19)
        d.sweep(19)
        for q in range(len(insts)):
            assert np.array_equal(g.member(q).flows(), d.member(q).flows()), q


@pytest.mark.parametrize("method", ["eso", "gdm"])
def test_tuner_keeps_the_state_and_picks_covering_tilings(method):
    gm, om = METHODS[method]
    insts = mixed_batch()
    with pdr.Batch(insts, method=gm, precision=pdr.FP64) as b:
        b.sweep(10)
        before = [b.member(q).flows() for q in range(len(insts))]
        t_before = [b.member(q).residual()["sweeps_done"] for q in range(len(insts))]
        buckets = b.tune(reps=3)
        say("tuned", method, buckets)
        for q in range(len(insts)):
            assert np.array_equal(b.member(q).flows(), before[q]), q
            assert b.member(q).residual()["sweeps_done"] == t_before[q], q
        assert sum(x["instances"] for x in buckets) == len(insts)
        for x in buckets:
            assert x["ms"] > 0.0
            assert x["lanes_per_arc"] * x["vec_per_lane"] * 2 >= x["max_K"]
        for q, inst in enumerate(insts):
            L, nv, Kp = b.member(q).tiling()
            assert L * nv * 2 >= Kp
        b.sweep(20)  # 30 sweeps in all: within GDM's well-conditioned horizon here
        for q, inst in enumerate(insts):
            st, _ = oracle.run(inst, om, 30)
            assert np.max(np.abs(b.member(q).flows() - st.f)) <= flow_tol(inst), q


def test_tuner_keeps_a_wrapped_z_log():
    """The tuner's timing passes write z-log entries; once the ring has wrapped
    those slots hold retained evaluations, which must read the same after."""
    insts = mixed_batch()[:4]
    with pdr.Batch(insts, method=pdr.ESO, precision=pdr.FP64, z_log_capacity=64) as b:
        b.sweep(150)
        before = [b.member(q).z_log(150 - 64, 64) for q in range(len(insts))]
        ctrl = [b.member(q).residual() for q in range(len(insts))]
        b.tune(reps=2)
        for q in range(len(insts)):
            assert np.array_equal(b.member(q).z_log(150 - 64, 64), before[q]), q
            res = b.member(q).residual()
            assert res["evaluations"] == ctrl[q]["evaluations"]
            assert res["sweeps_done"] == ctrl[q]["sweeps_done"]


def test_batch_members_are_owned_by_the_batch():
    insts = converging_batch()[:3]
    with pdr.Batch(insts, method=pdr.ESO, precision=pdr.FP32_BULK) as b:
        b.sweep(30)
        c = b.member(1)
        pdr.lib().pdr_destroy(c.handle)  # ignored for a member
        f32 = c.flows()
        with pytest.raises(pdr.PdrError) as ei:
            c.set_precision(pdr.FP64)
        assert ei.value.status == 4
        b.set_precision(pdr.FP64)  # the whole batch widens exactly
        assert np.array_equal(b.member(1).flows(), f32)
        b.sweep(5000, 0.0, 1e-8)
        for q in range(len(insts)):
            res = b.member(q).residual()
            assert res["z"] <= 1e-8 and res["verdict"] == "feasible", q


@pytest.mark.parametrize("precision", [pdr.FP64, pdr.FP32_BULK])
def test_member_groups_give_the_same_iterates(precision):
    """Members split into 1, 2, 3 or 4 groups, each running its passes on its
    own stream (in captured graphs and direct launches), end in the same state
    bit for bit, with the same per-member stop tests."""
    insts = mixed_batch()
    runs = []
    for groups in (1, 2, 3, 4):
        with pdr.Batch(insts, method=pdr.ESO, precision=precision, groups=groups,
                       graph_sweeps=8) as b:
            b.sweep(8 * 4 + 3)  # four graph replays and three direct passes
            b.sweep(10_000, 0.0, 1e-6 if precision == pdr.FP64 else 1e-4)
            runs.append([(b.member(q).flows(), b.member(q).residual()["sweeps_done"])
                         for q in range(len(insts))])
    for r in runs[1:]:
        for q in range(len(insts)):
            assert np.array_equal(r[q][0], runs[0][q][0]), q
            assert r[q][1] == runs[0][q][1], q


def test_batch_rejects_a_bad_instance():
    good = recipe_grid4_k8()
    bad = make_instance(3, [(0, 1), (1, 2), (2, 0)], 1.0, [0], [0], [1.0])  # s == t
    with pytest.raises(pdr.PdrError) as ei:
        pdr.Batch([good, bad])
    assert ei.value.status == 1 and "instance 1" in ei.value.message


@functools.lru_cache(maxsize=1)
def bench_batch():
    """The benchmark's 256-instance batch (seed 4), generated once per module."""
    from gen.batch import recipe_batch
    return tuple(recipe_batch(256, 4))


def sampled_members(insts, extra=5, seed=7):
    """Members of the benchmark batch checked against the oracle: the largest,
    smallest and median by work (m K), the most overloaded certified-infeasible
    member, and `extra` more drawn with a fixed seed."""
    work = np.array([i.m * i.K for i in insts])
    order = np.argsort(work, kind="stable")
    picks = [int(order[-1]), int(order[0]), int(order[len(order) // 2])]
    infeasible = [q for q, i in enumerate(insts) if i.meta.get("certified") == "infeasible"]
    assert infeasible
    worst = max(infeasible, key=lambda q: insts[q].meta["load_factor"])
    if worst not in picks:
        picks.append(worst)
    rest = [q for q in range(len(insts)) if q not in picks]
    picks += [int(q) for q in np.random.default_rng(seed).choice(rest, extra, replace=False)]
    return picks


@pytest.mark.parametrize("method", list(METHODS))
def test_full_batch_sampled_members_match_the_oracle(method):
    """The 256-instance batch the benchmark times (FP64; tuned for ESO, the
    benchmark's method): sampled members (largest, smallest, median, the most
    overloaded certified-infeasible one and five more) after 3 sweeps against
    the oracle."""
    gm, om = METHODS[method]
    insts = list(bench_batch())
    picks = sampled_members(insts)
    with pdr.Batch(insts, method=gm, precision=pdr.FP64) as b:
        if method == "eso":
            say("full batch buckets", b.tune(reps=2))
        b.sweep(3)
        for q in picks:
            inst = insts[q]
            say("full batch member", method, q, inst.n, inst.m, inst.K, inst.meta.get("certified"))
            st, zo = oracle.run(inst, om, 3)
            c = b.member(q)
            assert np.max(np.abs(c.flows() - st.f)) <= flow_tol(inst), q
            assert np.allclose(c.z_log(0, 3), zo, rtol=1e-11, atol=0), q


# FP32 bulk against the FP64 oracle: T passes round each stored flow and height
# once per pass (u32 = 2^-24), so with no error of the pass map's own they stay
# within T * u32 * max(u) (flow units) and z within T * u32 relative; the
# single-instance tests state the same bounds.
U32 = 2.0 ** -24


@pytest.mark.parametrize("method", ["eso", "agd", "gdm"])
def test_full_batch_fp32_sampled_members_within_the_fp32_bound(method):
    """The benchmark batch in FP32 bulk storage, 32 passes (one captured graph
    per member group): sampled members' flows, heights and z trajectories
    against the FP64 oracle of the same passes, within the stated FP32
    bounds."""
    gm, om = METHODS[method]
    T = 32
    insts = list(bench_batch())
    picks = sampled_members(insts)
    with pdr.Batch(insts, method=gm, precision=pdr.FP32_BULK) as b:
        b.sweep(T)
        for q in picks:
            inst = insts[q]
            st, zo = oracle.run(inst, om, T)
            _, ho = oracle.excess(inst, st.f)
            c = b.member(q)
            umax = float(np.max(inst.u))
            err = dict(flow=float(np.max(np.abs(c.flows() - st.f))),
                       height=float(np.max(np.abs(c.heights() - ho))),
                       z_rel=float(np.max(np.abs(c.z_log(0, T) - zo) / np.abs(zo))))
            say("fp32 batch member", method, q, inst.n, inst.K, inst.meta.get("certified"), err,
                "bound", T * U32 * umax)
            assert err["flow"] <= T * U32 * umax, (q, err)
            assert err["height"] <= T * U32 * umax, (q, err)
            assert err["z_rel"] <= T * U32, (q, err)


# Certified members of the benchmark batch that reach a decided verdict within
# 40,000 GDM passes (measured): feasible 38, 49, 71, 180 (n 752, 516, 973, 534)
# and infeasible 144, 227 (n 2,810, 532).
VERDICT_MEMBERS = (38, 49, 71, 180, 144, 227)


def test_certified_members_reach_their_certified_verdict():
    """Certified members of the benchmark batch (both labels, several sizes),
    swept together until every member's verdict is decided (Farkas gap > tau:
    infeasible, a proof by weak duality; z <= 1e-8: feasible) or a pass cap.
    Every decided verdict equals the member's certified label (Theorems 1-2)
    and the oracle's verdict of the same iterate."""
    insts = list(bench_batch())
    sub = [insts[q] for q in VERDICT_MEMBERS]
    labels = [i.meta["certified"] for i in sub]
    assert labels.count("feasible") == 4 and labels.count("infeasible") == 2
    say("verdict members", [(q, i.n, i.K, round(i.meta["load_factor"], 3), lab)
                            for q, i, lab in zip(VERDICT_MEMBERS, sub, labels)])
    cap, chunk = 120_000, 20_000
    done = 0
    with pdr.Batch(sub, method=pdr.GDM, precision=pdr.FP64) as b:
        while True:
            b.sweep(chunk)
            done += chunk
            res = [b.member(q).residual() for q in range(len(sub))]
            verdicts = [r["verdict"] for r in res]
            say("passes", done, "verdicts", verdicts)
            if all(v != "undecided" for v in verdicts) or done >= cap:
                break
        for q, (inst, r) in enumerate(zip(sub, res)):
            assert r["status"] == "PDR_OK"
            rep = oracle.report(inst, b.member(q).flows())
            assert rep["verdict"] == r["verdict"], (VERDICT_MEMBERS[q], rep["verdict"], r["verdict"])
            assert r["verdict"] == labels[q], (VERDICT_MEMBERS[q], r["verdict"], labels[q])
