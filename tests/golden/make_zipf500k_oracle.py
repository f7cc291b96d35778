"""Writes the FP64 oracle's solve of the 500,000 x 1,000,000 general sparse LP (generator seed 0) to
relative KKT 1e-4: objective, attempts and relative errors, one entry per tolerance in TOLS, in
tests/golden/zipf500k_seed0_oracle.json. Entries already in the file are kept (a solve takes about
20 minutes on 6 cores at 1e-4; tighter tolerances take hours).

Calls only oracle/ and the seeded generator. Run from the repository root:
    OMP_NUM_THREADS=<threads> python tests/golden/make_zipf500k_oracle.py
The oracle's result does not depend on the thread count (every sum is serial).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2503_10344_amd import generators as g  # noqa: E402

TOLS = (1e-4,)
LIMIT = 1_000_000
PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "zipf500k_seed0_oracle.json")


def main():
    lp = g.general_sparse(0)
    out = {"lp": lp.name, "nnz": int(lp.nnz), "solves": {}}
    if os.path.exists(PATH):
        with open(PATH) as f:
            old = json.load(f)
        out["solves"] = old.get("solves", {})
    for tol in TOLS:
        key = "%g" % tol
        if key in out["solves"]:
            continue
        t = time.time()
        r = oracle.solve(lp, tol=tol, iter_limit=LIMIT)
        out["solves"][key] = {
            "tol": tol, "iteration_limit": LIMIT, "status": int(r.status), "iterations": int(r.iterations),
            "restarts": int(r.restarts), "pobj": r.pobj, "dobj": r.dobj, "rel_p": r.rel_p, "rel_d": r.rel_d,
            "rel_gap": r.rel_gap, "seconds": round(time.time() - t, 1), "threads": oracle.num_threads()}
        with open(PATH, "w") as f:
            json.dump(out, f, indent=1)
        print(key, json.dumps(out["solves"][key]), flush=True)


if __name__ == "__main__":
    main()
