"""Write tests/golden/batched_stars_sample_converged.json with the FP64 oracle only.

Twelve instances of the 512 uneven barycenter stars (4-16 leaves, n in
[128, 2048], 1D/2D grids, eps = 1e-2), drawn with a seeded generator, each run
by the oracle's Bipartite Iterative Scaling (message sums in C, oracle/lse.c)
until its stopping sum is <= 1e-10; each dual is then within
2 C_inf E <= 4e-10 of its optimum (Lemma f_upper_bound_tree).  No GPU involved.

Usage: python tests/golden/make_batched_golden.py [threads]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.fast import FastTreeOracle  # noqa: E402
from workloads import make_batched_stars  # noqa: E402

SAMPLE_SEED = 2024
SAMPLE_SIZE = 12


def sample_indices(count=512):
    return sorted(int(i) for i in np.random.default_rng(SAMPLE_SEED).choice(count, size=SAMPLE_SIZE, replace=False))


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    out = {"workload": "batched-stars-512 (make_batched_stars(count=512)), sampled instances", "tol": 1e-10,
           "sample_seed": SAMPLE_SEED, "instances": []}
    t0 = time.time()
    for i in sample_indices():
        p = make_batched_stars(count=1, first_instance=i)[0]
        o = FastTreeOracle(p, threads=threads)
        t1 = time.time()
        r = o.solve(tol=1e-10, max_steps=100000)
        ev = o.evaluate()
        rec = {"index": i, "name": p.name, "oracle": r, "dual": ev["dual"], "primal": ev["primal"],
               "transport": ev["transport"], "scale": ev["scale"], "err_sum": ev["err_sum"], "c_inf": o.c_inf(),
               "cpu_seconds": time.time() - t1}
        out["instances"].append(rec)
        print(json.dumps(rec), flush=True)
    out["cpu_seconds"] = time.time() - t0
    with open(os.path.join(HERE, "batched_stars_sample_converged.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
