"""A batch of uneven instances for the batched sweep.

``recipe_batch(B, seed)`` draws B instances shaped like the paper's planar
family (random geometric 4-NN graphs, Section 7.1) with uneven sizes:
n ~ U{100..5000}, K ~ U{16..2000} (at most n(n-1)/2), capacities U{100..1000},
integer demands U{1..20} scaled to a per-instance load factor LF ~ U[0.7, 1.1].

Scaling uses a congestion bracket [mu_lo, mu_hi] of the unscaled demands from
two Frank-Wolfe steps of ``gen.loadfactor.congestion_bracket_fw`` (an explicit
routing gives mu_hi, dual arc lengths give mu_lo; no LP). The bracket is loose,
so an instance with LF > 1 is usually uncertified, and one with LF <= 1 is
certified feasible but may be lightly loaded. With alpha = LF / mu_hi the scaled instance's
minimum congestion lies in [LF mu_lo / mu_hi, LF]: it is certified feasible if
LF <= 1, certified infeasible if LF mu_lo / mu_hi > 1, and uncertified
otherwise. The brackets are computed once by ``python -m gen.batch`` and kept in
``gen/batch_loadfactor.json``; this module holds no part of the PDR method's
arithmetic.

Instance b of batch seed S uses the sub-seed 100000 + 1000 S + b for its graph,
OD pairs, capacities and demands (the streams of ``gen.instance.stream``), so
each instance is reproducible on its own.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import graphs
from .instance import Instance, od_pairs, stream

_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_loadfactor.json")


def _sub_seed(seed: int, b: int) -> int:
    return 100000 + 1000 * int(seed) + int(b)


def batch_shapes(B: int, seed: int):
    """(n, K, LF) of each instance of the batch."""
    rng = stream(seed, "misc")
    n = rng.integers(100, 5001, size=B)
    K = rng.integers(16, 2001, size=B)
    K = np.minimum(K, n * (n - 1) // 2)
    lf = rng.uniform(0.7, 1.1, size=B)
    return n.astype(int), K.astype(int), lf


def unscaled_instance(seed: int, b: int, n: int, K: int) -> Instance:
    sb = _sub_seed(seed, b)
    rp, col, nres = graphs.knn(int(n), stream(sb, "graph"))
    m = len(col)
    s, t = od_pairs(int(n), int(K), stream(sb, "od"))
    u = stream(sb, "cap").integers(100, 1001, size=m).astype(np.float64)
    d = stream(sb, "dem").integers(1, 21, size=int(K)).astype(np.float64)
    return Instance(int(n), rp, col, u, s, t, d,
                    dict(recipe="batch", batch_seed=seed, index=b, seed=sb, resamples=nres))


def _table() -> dict:
    if os.path.exists(_FILE):
        with open(_FILE) as fh:
            return json.load(fh)
    return {}


def recipe_batch(B: int = 256, seed: int = 4, scale: bool = True):
    """The batch as a list of Instances (scaled when brackets are stored)."""
    n, K, lf = batch_shapes(B, seed)
    tab = _table()
    out = []
    for b in range(B):
        inst = unscaled_instance(seed, b, n[b], K[b])
        key = f"{seed}:{b}"
        if scale:
            if key not in tab:
                raise KeyError(f"batch instance {key} has no bracket in {_FILE}; "
                               f"run python -m gen.batch {B} {seed}")
            br = tab[key]
            inst = inst.demand_scaled(float(lf[b]) / br["mu_hi"])
            lo = float(lf[b]) * br["mu_lo"] / br["mu_hi"]
            inst.meta.update(load_factor=float(lf[b]), lf_bracket=[lo, float(lf[b])],
                             certified=("feasible" if lf[b] <= 1.0 else
                                        "infeasible" if lo > 1.0 else "uncertified"))
        out.append(inst)
    return out


def main(argv):
    from .loadfactor import congestion_bracket_fw
    B = int(argv[0]) if argv else 256
    seed = int(argv[1]) if len(argv) > 1 else 4
    iters = int(argv[2]) if len(argv) > 2 else 2
    n, K, _ = batch_shapes(B, seed)
    tab = _table()
    t0 = time.time()
    for b in range(B):
        key = f"{seed}:{b}"
        if key in tab:
            continue
        inst = unscaled_instance(seed, b, n[b], K[b])
        br = congestion_bracket_fw(inst, iters=iters, kappa=4.0)
        tab[key] = dict(mu_hi=br["mu_hi"], mu_lo=br["mu_lo"], iters=br["iters"])
        with open(_FILE, "w") as fh:
            json.dump(tab, fh, indent=0, sort_keys=True)
        print(f"{key} n {n[b]} K {K[b]} mu_hi {br['mu_hi']:.6g} mu_lo {br['mu_lo']:.6g} "
              f"t {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
