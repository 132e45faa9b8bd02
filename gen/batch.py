"""A batch of uneven instances for the batched sweep.

``recipe_batch(B, seed)`` draws B instances shaped like the paper's planar
family (random geometric 4-NN graphs, Section 7.1) with uneven sizes:
n ~ U{100..5000}, K ~ U{16..2000} (at most n(n-1)/2), capacities U{100..1000},
integer demands U{1..20} scaled to a per-instance load factor LF ~ U[0.7, 1.1].

Scaling uses a certified bracket mu_lo <= mu* <= mu_hi of the minimum
congestion mu* of the unscaled demands (mu* = 1 / maximum concurrent flow),
from path column generation on HiGHS (``gen.loadfactor.congestion_bracket``:
an explicit routing gives mu_hi, the master's dual arc lengths give mu_lo by
weak duality). A member with LF <= 1 is scaled by alpha = LF / mu_hi, so its
minimum congestion alpha mu* <= LF <= 1: certified feasible, true load factor
in [LF mu_lo / mu_hi, LF]. A member with LF > 1 is scaled by alpha = LF / mu_lo,
so alpha mu* >= LF > 1: certified infeasible, true load factor in
[LF, LF mu_hi / mu_lo]. The brackets are computed once by
``python -m gen.batch`` and kept in ``gen/batch_loadfactor.json``; this module
holds no part of the PDR method's arithmetic.

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
            target = float(lf[b])
            ratio = br["mu_hi"] / br["mu_lo"] if br["mu_lo"] > 0 else float("inf")
            if target <= 1.0:
                inst = inst.demand_scaled(target / br["mu_hi"])
                bracket, label = [target / ratio, target], "feasible"
            elif br["mu_lo"] > 0:
                inst = inst.demand_scaled(target / br["mu_lo"])
                bracket, label = [target, target * ratio], "infeasible"
            else:  # no lower bound: scaled as a feasible target, label unknown
                inst = inst.demand_scaled(target / br["mu_hi"])
                bracket, label = [0.0, target], "uncertified"
            inst.meta.update(load_factor=target, lf_bracket=bracket, certified=label,
                             mu_hi=br["mu_hi"], mu_lo=br["mu_lo"])
        out.append(inst)
    return out


def _bracket(args):
    from .loadfactor import congestion_bracket
    seed, b, n, K = args
    inst = unscaled_instance(seed, b, n, K)
    br = congestion_bracket(inst, gap=1e-4, max_iter=60, time_limit=1800.0)
    return f"{seed}:{b}", dict(mu_hi=br["mu_hi"], mu_lo=br["mu_lo"], iters=br["iters"],
                               method="column generation"), n, K, br["seconds"]


def main(argv):
    """python -m gen.batch [B] [seed] [workers]: the bracket of every member that
    has no column-generation bracket yet, written to gen/batch_loadfactor.json."""
    from multiprocessing import Pool
    B = int(argv[0]) if argv else 256
    seed = int(argv[1]) if len(argv) > 1 else 4
    workers = int(argv[2]) if len(argv) > 2 else 4
    n, K, _ = batch_shapes(B, seed)
    tab = _table()
    todo = [(seed, b, int(n[b]), int(K[b])) for b in range(B)
            if tab.get(f"{seed}:{b}", {}).get("method") != "column generation"]
    todo.sort(key=lambda a: -a[2] * a[3])  # largest first
    t0 = time.time()
    with Pool(workers) as pool:
        for key, entry, nb, kb, sec in pool.imap_unordered(_bracket, todo):
            tab[key] = entry
            with open(_FILE + ".tmp", "w") as fh:
                json.dump(tab, fh, indent=0, sort_keys=True)
            os.replace(_FILE + ".tmp", _FILE)
            print(f"{key} n {nb} K {kb} mu_hi {entry['mu_hi']:.9g} mu_lo {entry['mu_lo']:.9g} "
                  f"({sec:.0f} s; {time.time() - t0:.0f} s in all)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
