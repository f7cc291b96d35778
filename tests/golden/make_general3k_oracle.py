"""Writes the FP64 oracle's solves of the 3,000 x 6,000 general sparse LPs of seeds 8, 9 and 10 to
relative KKT 1e-4 (attempts, objective, relative errors) to tests/golden/general3k_oracle.json.

Calls only oracle/ and the seeded generator. Run from the repository root:
    python tests/golden/make_general3k_oracle.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2503_10344_amd import generators as g  # noqa: E402

SEEDS = (8, 9, 10)
TOL = 1e-4
LIMIT = 2_000_000


def main():
    out = {"m": 3000, "n": 6000, "cap": 1000, "tol": TOL, "iteration_limit": LIMIT, "seeds": {}}
    for s in SEEDS:
        lp = g.general_sparse(s, m=3000, n=6000, cap=1000)
        r = oracle.solve(lp, tol=TOL, iter_limit=LIMIT)
        out["seeds"][str(s)] = {"status": int(r.status), "iterations": int(r.iterations), "pobj": r.pobj,
                                "dobj": r.dobj, "rel_p": r.rel_p, "rel_d": r.rel_d, "rel_gap": r.rel_gap}
        print(s, out["seeds"][str(s)], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "general3k_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
