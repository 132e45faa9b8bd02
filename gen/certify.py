"""Write gen/loadfactor.json: certified congestion brackets for the scaled recipes.

Usage: python -m gen.certify [recipe[:seed] ...]

Each entry holds mu_hi (congestion of an explicit routing of the unscaled
demands) and mu_lo (a weak-duality lower bound), so that the benchmark and the
tests can scale demands to their load factor without solving an LP.
"""
from __future__ import annotations

import json
import os
import sys

from .instance import RECIPES, _LF_FILE, _lf_table
from .loadfactor import congestion_bracket, grid_cut_bound

# grid recipes: (rows, columns) for the straight-cut lower bound
GRID_SHAPES = {"grid100_k10000": (100, 100), "grid4_k8": (4, 4)}


def main(argv):
    targets = argv or ["knn2500_k1000", "grid100_k10000"]
    table = _lf_table()
    for tgt in targets:
        name, _, seed = tgt.partition(":")
        inst = RECIPES[name]() if not seed else RECIPES[name](int(seed))
        key = f"{name}:{inst.meta['seed']}"
        lo0 = grid_cut_bound(inst, *GRID_SHAPES[name]) if name in GRID_SHAPES else 0.0

        def save(br):
            # every master gives a certified bracket: keep the lowest mu_hi so far
            old = table.get(key)
            if old is not None and old.get("mu_hi", float("inf")) <= br["mu_hi"]:
                return
            table[key] = dict(mu_hi=br["mu_hi"], mu_lo=br["mu_lo"], iters=br["iters"],
                              columns=br["columns"], gap=br["mu_hi"] / br["mu_lo"] - 1.0)
            with open(_LF_FILE + ".tmp", "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
            os.replace(_LF_FILE + ".tmp", _LF_FILE)
            print(key, table[key], flush=True)

        br = congestion_bracket(inst, verbose=True, mu_lo0=lo0, on_iter=save,
                                time_limit=float(os.environ.get("CERTIFY_TIME_LIMIT", "7200")))
        save(br)


if __name__ == "__main__":
    main(sys.argv[1:])
