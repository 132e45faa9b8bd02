"""Write gen/loadfactor.json: certified congestion brackets for the scaled recipes.

Usage: python -m gen.certify [recipe[:seed] ...]

Each entry holds mu_hi (congestion of an explicit routing of the unscaled
demands) and mu_lo (a weak-duality lower bound), so that the benchmark and the
tests can scale demands to their load factor without solving an LP.
"""
from __future__ import annotations

import json
import sys

from .instance import RECIPES, _LF_FILE, _lf_table
from .loadfactor import congestion_bracket


def main(argv):
    targets = argv or ["knn2500_k1000", "grid100_k10000"]
    table = _lf_table()
    for tgt in targets:
        name, _, seed = tgt.partition(":")
        inst = RECIPES[name]() if not seed else RECIPES[name](int(seed))
        key = f"{name}:{inst.meta['seed']}"
        br = congestion_bracket(inst, verbose=True)
        table[key] = dict(mu_hi=br["mu_hi"], mu_lo=br["mu_lo"], iters=br["iters"],
                          columns=br["columns"], gap=br["mu_hi"] / br["mu_lo"] - 1.0)
        with open(_LF_FILE, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        print(key, table[key], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
