"""Seeded synthetic graphs shaped like the paper's benchmark families.

The paper evaluates on public planar, grid and telecom multicommodity-flow
instances (Section 7.1). Those files are not used here; these generators
produce graphs of the same shape instead:

* ``grid(a, b)``: an a x b grid with both arc directions between 4-neighbours,
  the shape of the "grid" family (vertex degree about four per direction).
* ``knn(n, rng)``: points uniform in the unit square, each linked in both
  directions to its 4 nearest neighbours, the shape of the "planar" family
  (random points, arcs to neighbouring points).

Graphs are returned as an out-adjacency CSR sorted by (tail, head): vertex i's
out-arcs are ``col[row_ptr[i]:row_ptr[i+1]]`` and the arc id is the CSR
position. This module holds no part of the PDR method's arithmetic.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree


def _csr_from_pairs(n: int, tails: np.ndarray, heads: np.ndarray):
    order = np.lexsort((heads, tails))
    tails = tails[order]
    heads = heads[order]
    counts = np.bincount(tails, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, heads.astype(np.int32)


def grid(a: int, b: int):
    """a x b grid, vertex r*b + c, arcs to right/down neighbours in both directions."""
    n = a * b
    r, c = np.divmod(np.arange(n, dtype=np.int64), b)
    right = np.nonzero(c + 1 < b)[0]
    down = np.nonzero(r + 1 < a)[0]
    t = np.concatenate([right, right + 1, down, down + b])
    h = np.concatenate([right + 1, right, down + b, down])
    return _csr_from_pairs(n, t, h)


def knn_points(n: int, rng: np.random.Generator, k: int = 4):
    """Points U[0,1)^2 and their exact k nearest neighbours (ties broken by index)."""
    pts = rng.random((n, 2))
    tree = cKDTree(pts)
    # ask for a few extra candidates so ties at the k-th distance are resolved by index
    kk = min(n, k + 4)
    dist, idx = tree.query(pts, k=kk)
    nbrs = np.empty((n, k), dtype=np.int64)
    for i in range(n):
        cand = [(float(dd), int(j)) for dd, j in zip(dist[i], idx[i]) if j != i]
        cand.sort()
        nbrs[i] = [j for _, j in cand[:k]]
    return pts, nbrs


def knn(n: int, rng: np.random.Generator, k: int = 4, max_resample: int = 64):
    """Bidirectional k-NN graph; resampled from the same stream until connected.

    Returns (row_ptr, col, n_resamples).
    """
    for attempt in range(max_resample):
        _, nbrs = knn_points(n, rng, k)
        t = np.repeat(np.arange(n, dtype=np.int64), k)
        h = nbrs.reshape(-1)
        tt = np.concatenate([t, h])
        hh = np.concatenate([h, t])
        key = np.unique(tt * n + hh)
        tt, hh = np.divmod(key, n)
        row_ptr, col = _csr_from_pairs(n, tt, hh)
        A = csr_matrix((np.ones(len(col)), col, row_ptr), shape=(n, n))
        ncomp, _ = connected_components(A, directed=True, connection="strong")
        if ncomp == 1:
            return row_ptr, col, attempt
    raise RuntimeError("knn: no connected sample within max_resample draws")


def csr_tails(row_ptr: np.ndarray) -> np.ndarray:
    """Tail vertex of every arc of an out-adjacency CSR."""
    n = len(row_ptr) - 1
    return np.repeat(np.arange(n, dtype=np.int32), np.diff(row_ptr))
