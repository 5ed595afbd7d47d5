"""Write tests/golden/random_tree256_converged.json with the FP64 oracle only.

The 256-node Pruefer tree (n in [256, 4096] on 2D grids, eps = 5e-3, leaves
observed with Dirichlet(1) weights) is run by the oracle's Bipartite Iterative
Scaling (message sums in C, oracle/lse.c, on every host thread) until its
stopping sum is <= 1e-9; the dual of that state is within 2 C_inf E = 4e-9 of
the optimum (Lemma f_upper_bound_tree).  About an hour on 8 host cores; no GPU
involved.

Usage: python tests/golden/make_tree_golden.py [threads]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.fast import FastTreeOracle  # noqa: E402
from workloads import make_config  # noqa: E402


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    p = make_config(3)
    o = FastTreeOracle(p, threads=threads)
    t0 = time.time()
    hist = []
    r = o.solve(tol=1e-9, max_steps=20000, history=hist)
    ev = o.evaluate()
    out = {"workload": "random-tree-256node-2d (make_config(3))", "tol": 1e-9, "oracle": r,
           "dual": ev["dual"], "primal": ev["primal"], "transport": ev["transport"], "scale": ev["scale"],
           "err_sum": ev["err_sum"], "err_max": ev["err_max"], "c_inf": o.c_inf(),
           "history_every_100": hist[::100], "cpu_seconds": time.time() - t0}
    with open(os.path.join(HERE, "random_tree256_converged.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "history_every_100"}))


if __name__ == "__main__":
    main()
