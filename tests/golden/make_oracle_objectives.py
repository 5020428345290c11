"""Writes oracle_objectives.json: the FP64 oracle's objective at relative KKT
1e-8 (App. B.4) on instances without a constructed optimum, for the
full-size tests and the benchmark's objective errors.

Runs only the oracle (oracle/) on the seeded generators (lpgen/):

    python tests/golden/make_oracle_objectives.py        # about 2 minutes
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lpgen   # noqa: E402
import oracle  # noqa: E402

INSTANCES = {"c2": lpgen.config2}


def main():
    out = {}
    for name, mk in INSTANCES.items():
        lp = mk()
        t0 = time.perf_counter()
        P = oracle.Problem(lp, oracle.Params(eps=1e-8))
        r = P.solve()
        out[name] = {"instance": f"{lp.name}: m={lp.m}, n={lp.n}, nnz={lp.nnz}",
                     "eps": 1e-8, "status": int(r["status"]), "iters": int(r["iters"]),
                     "r_primal": r["r_primal"], "r_dual": r["r_dual"], "r_gap": r["r_gap"],
                     "obj_primal": r["obj_p"], "obj_dual": r["obj_d"],
                     "oracle_seconds": round(time.perf_counter() - t0, 1),
                     "oracle_threads": oracle.num_threads()}
        print(name, out[name], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_objectives.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
