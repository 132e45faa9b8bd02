"""Multicommodity-flow feasibility instances (Section 1: graph, capacities u,
commodities (s_k, t_k, d_k) with s_k != t_k) and the seeded recipes used by the
tests and the benchmark.

Every random draw comes from ``stream(seed, name)``, a PCG64 generator keyed by
the instance seed and a fixed sub-stream id, so each part of an instance
(graph, OD pairs, capacities, demands) is reproducible on its own.

Load-factor scaling multiplies integer demands by ``alpha = LF / mu_hi``, where
``mu_hi`` is the congestion of an explicit routing of the unscaled demands
(see ``gen.loadfactor``). The factors for the large recipes are stored in
``gen/loadfactor.json`` by ``gen/certify.py`` so that no LP runs at benchmark
time; ``load_instance`` raises ``MissingLoadFactor`` when the file has no entry.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Optional

import numpy as np

from . import graphs

_STREAMS = {"graph": 1, "od": 2, "cap": 3, "dem": 4, "misc": 5}
_LF_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "loadfactor.json")


def stream(seed: int, name: str) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), _STREAMS[name]])))


@dataclasses.dataclass
class Instance:
    n: int
    row_ptr: np.ndarray  # int64 [n+1], out-adjacency CSR
    col: np.ndarray      # int32 [m], arc heads
    u: np.ndarray        # float64 [m], capacities
    s: np.ndarray        # int32 [K]
    t: np.ndarray        # int32 [K]
    d: np.ndarray        # float64 [K], demands
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    @property
    def K(self) -> int:
        return int(self.s.shape[0])

    def tails(self) -> np.ndarray:
        return graphs.csr_tails(self.row_ptr)

    def scaled(self, alpha: float) -> "Instance":
        """Same instance with (u, d) -> (alpha u, alpha d)."""
        return dataclasses.replace(self, u=self.u * alpha, d=self.d * alpha,
                                   meta=dict(self.meta, scale=alpha))

    def demand_scaled(self, alpha: float) -> "Instance":
        """Same graph and capacities with demands d -> alpha d."""
        return dataclasses.replace(self, d=self.d * alpha,
                                   meta=dict(self.meta, demand_scale=alpha))

    def save(self, path: str) -> None:
        np.savez(path, n=self.n, row_ptr=self.row_ptr, col=self.col, u=self.u,
                 s=self.s, t=self.t, d=self.d, meta=json.dumps(self.meta))

    @staticmethod
    def load(path: str) -> "Instance":
        z = np.load(path, allow_pickle=False)
        return Instance(int(z["n"]), z["row_ptr"], z["col"], z["u"], z["s"], z["t"], z["d"],
                        json.loads(str(z["meta"])))


def od_pairs(n: int, K: int, rng: np.random.Generator):
    """K distinct ordered pairs (s, t), s != t, uniform by rejection."""
    if K > n * (n - 1):
        raise ValueError("more commodities than ordered vertex pairs")
    seen = set()
    s = np.empty(K, dtype=np.int32)
    t = np.empty(K, dtype=np.int32)
    k = 0
    while k < K:
        need = K - k
        a = rng.integers(0, n, size=2 * need + 16)
        b = rng.integers(0, n, size=2 * need + 16)
        for x, y in zip(a.tolist(), b.tolist()):
            if x == y or (x, y) in seen:
                continue
            seen.add((x, y))
            s[k], t[k] = x, y
            k += 1
            if k == K:
                break
    return s, t


def random_instance(row_ptr, col, K, seed, u_range, d_range, meta=None) -> Instance:
    n = len(row_ptr) - 1
    m = len(col)
    s, t = od_pairs(n, K, stream(seed, "od"))
    u = stream(seed, "cap").integers(u_range[0], u_range[1] + 1, size=m).astype(np.float64)
    d = stream(seed, "dem").integers(d_range[0], d_range[1] + 1, size=K).astype(np.float64)
    return Instance(n, np.asarray(row_ptr, np.int64), np.asarray(col, np.int32), u, s, t, d,
                    dict(meta or {}, seed=seed, u_range=list(u_range), d_range=list(d_range)))


# ---------------------------------------------------------------- recipes
# Each recipe returns the unscaled instance; ``load_instance`` applies the
# load-factor scaling where the recipe asks for one.

def recipe_grid4_k8(seed: int = 1) -> Instance:
    """4x4 bidirectional grid (n 16, m 48), K 8, u U{5..20}, d U{1..5}, unscaled."""
    rp, col = graphs.grid(4, 4)
    return random_instance(rp, col, 8, seed, (5, 20), (1, 5), dict(recipe="grid4_k8"))


def recipe_knn2500_k1000(seed: int = 2) -> Instance:
    """Random geometric 4-NN graph, n 2500; K 1000; u U{500..1500}; d U{1..50}; LF 0.9."""
    rp, col, nres = graphs.knn(2500, stream(seed, "graph"))
    return random_instance(rp, col, 1000, seed, (500, 1500), (1, 50),
                           dict(recipe="knn2500_k1000", resamples=nres, load_factor=0.9))


def recipe_grid100_k10000(seed: int = 3) -> Instance:
    """100x100 bidirectional grid (n 10000, m 39600); K 10000; u U{1000..3000}; d U{1..20}; LF 0.95."""
    rp, col = graphs.grid(100, 100)
    return random_instance(rp, col, 10000, seed, (1000, 3000), (1, 20),
                           dict(recipe="grid100_k10000", load_factor=0.95))


def recipe_small(kind: str, size: int, K: int, seed: int, u_range=(5, 20), d_range=(1, 5)) -> Instance:
    """Small instances for tests: kind 'grid' (size x size) or 'knn' (size points)."""
    if kind == "grid":
        rp, col = graphs.grid(size, size)
    elif kind == "knn":
        rp, col, _ = graphs.knn(size, stream(seed, "graph"))
    else:
        raise ValueError(kind)
    return random_instance(rp, col, K, seed, u_range, d_range, dict(recipe=f"{kind}{size}_k{K}"))


def recipe_knn2500_k81430(seed: int = 6) -> Instance:
    """Random geometric 4-NN graph, n 2500; K 81,430 (the commodity count of the
    paper's largest planar instance, whose graph has 2,500 vertices and 12,990
    arcs); u U{500..1500}; d U{1..20}; LF 0.9. Rows of 81,430 commodities are
    longer than a register-resident arc kernel holds (the streamed kernels)."""
    rp, col, nres = graphs.knn(2500, stream(seed, "graph"))
    return random_instance(rp, col, 81430, seed, (500, 1500), (1, 20),
                           dict(recipe="knn2500_k81430", resamples=nres, load_factor=0.9))


RECIPES = {
    "grid4_k8": recipe_grid4_k8,
    "knn2500_k1000": recipe_knn2500_k1000,
    "grid100_k10000": recipe_grid100_k10000,
    "knn2500_k81430": recipe_knn2500_k81430,
}


def _lf_table() -> dict:
    if os.path.exists(_LF_FILE):
        with open(_LF_FILE) as fh:
            return json.load(fh)
    return {}


class MissingLoadFactor(KeyError):
    pass


def load_instance(name: str, seed: Optional[int] = None, scale: bool = True) -> Instance:
    """Build a named recipe and apply its load-factor scaling (if it has one)."""
    fn = RECIPES[name]
    inst = fn() if seed is None else fn(seed)
    lf = inst.meta.get("load_factor")
    if not scale or lf is None:
        return inst
    key = f"{name}:{inst.meta['seed']}"
    entry = _lf_table().get(key)
    if entry is None:
        raise MissingLoadFactor(f"{key} has no entry in {_LF_FILE}; run python -m gen.certify {name}")
    alpha = lf / entry["mu_hi"]
    out = inst.demand_scaled(alpha)
    out.meta.update(mu_hi=entry["mu_hi"], mu_lo=entry["mu_lo"],
                    lf_bracket=[lf * entry["mu_lo"] / entry["mu_hi"], lf])
    return out
