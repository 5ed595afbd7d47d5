"""Write tests/golden/chain32_n1024_converged.json with the FP64 oracle only.

The 32-node chain (n = 1024, eps = 1e-3, every 4th node observed) is run by
the oracle's Bipartite Iterative Scaling until its stopping sum is <= 1e-10;
the dual objective of that state is within 2 C_inf E = 4e-10 of the optimum
(Lemma f_upper_bound_tree), far inside the 1e-6 relative tolerance the GPU
test applies.  Takes about an hour on one core; no GPU involved.

Usage: python tests/golden/make_chain_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import TreeOracle  # noqa: E402
from workloads import make_config  # noqa: E402


def main():
    p = make_config(2)
    o = TreeOracle(p)
    t0 = time.time()
    hist = []
    r = o.solve(tol=1e-10, max_steps=20000, history=hist)
    ev = o.evaluate()
    out = {"workload": "chain-hmm-32node-n1024 (make_config(2))", "tol": 1e-10, "oracle": r,
           "dual": ev["dual"], "primal": ev["primal"], "transport": ev["transport"], "scale": ev["scale"],
           "err_sum": ev["err_sum"], "err_max": ev["err_max"], "c_inf": o.c_inf(),
           "history_every_100": hist[::100], "cpu_seconds": time.time() - t0}
    with open(os.path.join(HERE, "chain32_n1024_converged.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "history_every_100"}))


if __name__ == "__main__":
    main()
