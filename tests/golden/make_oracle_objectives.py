"""Writes oracle_objectives.json: the FP64 oracle's solve of benchmark
instances to a relative KKT tolerance (App. B.4): c2 to 1e-8 (it has no
constructed optimum) and c1 to 1e-4 (the tolerance c1 is timed at), for the
full-size tests and the benchmark's objective errors.

Runs only the oracle (oracle/) on the seeded generators (lpgen/):

    python tests/golden/make_oracle_objectives.py [name ...]
        # c2: about 2 minutes on 8 threads; c1: about 15 minutes
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lpgen   # noqa: E402
import oracle  # noqa: E402

INSTANCES = {"c2": (lpgen.config2, 1e-8), "c1": (lpgen.config1, 1e-4)}


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_objectives.json")
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    for name in sys.argv[1:] or list(INSTANCES):
        mk, eps = INSTANCES[name]
        lp = mk()
        t0 = time.perf_counter()
        P = oracle.Problem(lp, oracle.Params(eps=eps))
        r = P.solve()
        out[name] = {"instance": f"{lp.name}: m={lp.m}, n={lp.n}, nnz={lp.nnz}",
                     "eps": eps, "status": int(r["status"]), "iters": int(r["iters"]),
                     "r_primal": r["r_primal"], "r_dual": r["r_dual"], "r_gap": r["r_gap"],
                     "obj_primal": r["obj_p"], "obj_dual": r["obj_d"],
                     "oracle_seconds": round(time.perf_counter() - t0, 1),
                     "oracle_threads": oracle.num_threads()}
        print(name, out[name], flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
