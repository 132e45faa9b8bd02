"""Reverse-mode gradient of z(f^T) through T PDR-ESO passes (pdr_adjoint)
against the oracle's forward-mode tangent (pinned in test_oracle_pins.py).

The GPU computes the whole gradient in one reverse sweep; the oracle needs one
forward-mode run per capacity or demand. Both differentiate the branch the
forward pass takes, so away from ties they agree to rounding.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import paper_2108_07549_amd as pdr
from gen.instance import MissingLoadFactor, load_instance, recipe_grid4_k8, recipe_small

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-adjoint]", *a, flush=True)
    sys.stdout.flush()


def check(inst, T, checkpoint, rtol=1e-9):
    say("adjoint", inst.meta.get("recipe"), "n", inst.n, "m", inst.m, "K", inst.K, "T", T,
        "checkpoint", checkpoint)
    with pdr.Context.from_instance(inst, method=pdr.ESO) as c:
        z, gu, gd = c.adjoint(T, checkpoint)
        f_after = c.flows()
        res = c.residual()
    zo, gu_o, gd_o = oracle.eso_gradient(inst, T)
    scale = max(np.abs(gu_o).max() if inst.m else 0.0, np.abs(gd_o).max(), 1e-300)
    assert z == pytest.approx(zo, rel=1e-10, abs=1e-300)
    assert np.max(np.abs(gu - gu_o)) <= rtol * scale
    assert np.max(np.abs(gd - gd_o)) <= rtol * scale
    # the context ends where T ordinary sweeps end
    with pdr.Context.from_instance(inst, method=pdr.ESO) as c:
        c.sweep(T)
        assert np.array_equal(c.flows(), f_after)
    assert res["sweeps_done"] == T
    return gu, gd


def test_c1_instance_256_passes():
    """The correctness configuration: grid4_k8, 256 passes, a checkpoint every 16."""
    check(recipe_grid4_k8(), 256, 16)


def test_congested_instance_gradients():
    """Demands x20 make grid4_k8 infeasible: congested arcs, O(10) gradients."""
    base = recipe_grid4_k8()
    inst = dataclasses.replace(base, d=base.d * 20.0)
    gu, gd = check(inst, 64, 16)
    assert np.count_nonzero(gu) > 0


@pytest.mark.parametrize("T,checkpoint", [(0, 0), (1, 0), (37, 16), (37, 1), (37, 64), (40, 7)])
def test_checkpoint_layouts(T, checkpoint):
    base = recipe_grid4_k8()
    inst = dataclasses.replace(base, d=base.d * 12.0)
    check(inst, T, checkpoint)


def test_ragged_commodities_and_tilings():
    inst = recipe_small("knn", 40, 61, seed=8, u_range=(2, 9), d_range=(1, 6))
    check(inst, 30, 8)
    inst = recipe_small("grid", 5, 131, seed=5, u_range=(5, 40), d_range=(1, 5))
    check(inst, 20, 6)


def test_adjoint_needs_fp64_eso():
    inst = recipe_grid4_k8()
    for kw in (dict(method=pdr.AGD), dict(method=pdr.ESO, precision=pdr.FP32_BULK)):
        with pdr.Context.from_instance(inst, **kw) as c:
            with pytest.raises(pdr.PdrError) as ei:
                c.adjoint(4)
            assert ei.value.status == 4


def test_grid100_k10000_sampled_coordinates():
    """The benchmark workload at full size: 3 passes, a checkpoint every 2;
    sampled capacities and demands against single forward-mode runs."""
    try:
        inst = load_instance("grid100_k10000")
    except MissingLoadFactor as exc:
        pytest.skip(f"load factor not certified yet: {exc}")
    T = 3
    with pdr.Context.from_instance(inst, method=pdr.ESO) as c:
        z, gu, gd = c.adjoint(T, 2)
    rng = np.random.default_rng(1)
    coords = [int(np.argmax(np.abs(gu))), int(rng.integers(0, inst.m))] + \
             [inst.m + int(x) for x in rng.integers(0, inst.K, 2)]
    for j in coords:
        du, dd = np.zeros(inst.m), np.zeros(inst.K)
        if j < inst.m:
            du[j] = 1.0
        else:
            dd[j - inst.m] = 1.0
        _, _, zo, zdot = oracle.eso_tangent(inst, T, du, dd)
        got = gu[j] if j < inst.m else gd[j - inst.m]
        say("grid100 coordinate", j, got, zdot)
        assert z == pytest.approx(zo, rel=1e-10)
        assert abs(got - zdot) <= 1e-9 * max(abs(zdot), 1e-12 * abs(zo))
