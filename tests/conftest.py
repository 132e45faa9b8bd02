import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def make_instance(n, arcs, u, s, t, d):
    """Instance from an explicit arc list (sorted into out-adjacency CSR order)."""
    from gen.instance import Instance
    arcs = list(arcs)
    order = sorted(range(len(arcs)), key=lambda q: arcs[q])
    tails = np.array([arcs[q][0] for q in order], np.int64)
    heads = np.array([arcs[q][1] for q in order], np.int32)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(tails, minlength=n), out=row_ptr[1:])
    uu = np.asarray(u, np.float64)
    if uu.ndim == 0:
        uu = np.full(len(arcs), float(uu))
    else:
        uu = uu[order]
    return Instance(n, row_ptr, heads, uu, np.asarray(s, np.int32), np.asarray(t, np.int32),
                    np.asarray(d, np.float64), {})


@pytest.fixture(scope="session")
def grid4():
    from gen.instance import recipe_grid4_k8
    return recipe_grid4_k8()
