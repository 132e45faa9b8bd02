"""pdr_set_state_noalloc (no device allocation) against pdr_set_state.

Two calls in a row through the C ABI, the second with a smaller instance:
the first state is larger than the 32 MiB staging array, so it is staged in
several chunks; the second reuses the array the first left behind. After
each, the context's flows, learning rates, velocities and the passes that
follow equal those of a context given the same state by pdr_set_state, bit
for bit.
"""
import sys

import numpy as np
import pytest

import paper_2108_07549_amd as pdr
from gen.instance import recipe_grid4_k8, recipe_small

pytestmark = pytest.mark.gpu

SCRATCH_DOUBLES = 1 << 22


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


def _state(inst, seed):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.0, 3.0, (inst.m, inst.K)) * (rng.random((inst.m, inst.K)) < 0.7)
    beta = rng.uniform(0.01, 0.5, inst.m)
    v = rng.normal(0.0, 0.5, (inst.m, inst.K))
    return f, beta, v


def _compare(inst, method, precision, seed):
    f, beta, v = _state(inst, seed)
    say("instance n", inst.n, "m", inst.m, "K", inst.K, "m*K", inst.m * inst.K,
        "chunks", -(-inst.m * inst.K // ((SCRATCH_DOUBLES // inst.K) * inst.K)),
        "method", method, "precision", precision)
    out = []
    for noalloc in (False, True):
        with pdr.Context.from_instance(inst, method=method, precision=precision) as c:
            c.sweep(3)  # state to be replaced
            if noalloc:
                c.set_state_noalloc(f, beta, t=17, z_prev=1e300, v=v)
            else:
                c.set_state(f, beta, t=17, z_prev=1e300, v=v)
            r = dict(f=c.flows(), beta=c.learning_rates(),
                     v=c.velocities() if method == pdr.GDM else None)
            c.sweep(5)
            r.update(f5=c.flows(), beta5=c.learning_rates(), res=c.residual(),
                     z=c.z_log(c.residual()["evaluations"] - 5, 5))
            out.append(r)
    a, b = out
    if precision == pdr.FP64:
        assert np.array_equal(a["f"], f)
    for key in ("f", "beta", "f5", "beta5", "z"):
        assert np.array_equal(a[key], b[key]), key
    if method == pdr.GDM:
        assert np.array_equal(a["v"], b["v"])
    assert a["res"]["sweeps_done"] == b["res"]["sweeps_done"] == 22
    assert a["res"]["z"] == b["res"]["z"]


def test_noalloc_state_equals_set_state_two_calls_second_smaller():
    big = recipe_small("knn", 500, 2000, seed=21, u_range=(50, 400), d_range=(1, 9))
    assert big.m * big.K > SCRATCH_DOUBLES  # staged in more than one chunk
    _compare(big, pdr.ESO, pdr.FP64, 1)
    small = recipe_grid4_k8()
    _compare(small, pdr.GDM, pdr.FP64, 2)
    _compare(small, pdr.AGD, pdr.FP32_BULK, 3)


def test_noalloc_state_rejects_bad_arguments_like_set_state():
    inst = recipe_grid4_k8()
    with pdr.Context.from_instance(inst, method=pdr.ESO) as c:
        f = np.ones((inst.m, inst.K))
        f[3, 2] = -1.0
        with pytest.raises(pdr.PdrError) as ei:
            c.set_state_noalloc(f)
        assert ei.value.status == 1 and "finite and >= 0" in ei.value.message
        st = pdr.lib().pdr_set_state_noalloc(c.handle, None, None, None, 0, 0.0)
        assert st == 1
        # the context is still usable and unchanged
        c.sweep(2)
        assert c.residual()["sweeps_done"] == 2
