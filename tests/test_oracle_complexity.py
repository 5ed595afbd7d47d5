"""The paper's delta-approximation protocol on its barycenter workload, run by
the FP64 oracle (CPU only).

With eps = delta / (4 |E| log d) and delta' = delta / (8 C_inf) (the parameter
choice stated before Theorem tree_local_reg_complexity), Algorithm
tree_local_reg stopped at the stopping sum delta' and followed by Algorithm
round gives feasible plans whose transport cost is within delta of the
unregularised optimum (Lemma round_applied), within the number of half-sweeps
of Theorem num_iter.  The optimum comes from HiGHS (brute.lp_coupled), the
rounding from oracle/rounding.py; the log-normal stars follow Section 5
(uniform grid of d points in [0, 1], squared-Euclidean cost, so C_inf = 1).
"""
import numpy as np
import pytest

from oracle import TreeOracle
from oracle.brute import lp_coupled
from oracle.rounding import rounded_transport
from workloads import make_lognormal_star

DELTA = 0.2


def protocol_params(n_edges: int, d: int, c_inf: float = 1.0, delta: float = DELTA):
    return delta / (4.0 * n_edges * np.log(d)), delta / (8.0 * c_inf)


@pytest.mark.parametrize("L,d,seed", [(2, 6, 0), (3, 8, 1), (3, 5, 2), (4, 6, 3), (6, 4, 4)])
def test_delta_approximation_within_theorem_bounds(L, d, seed):
    eps, tol = protocol_params(L, d)
    p = make_lognormal_star(L, d, eps, instance=seed)
    o = TreeOracle(p)
    c_inf = o.c_inf()
    assert c_inf <= 1.0
    r = o.solve(tol=tol, max_steps=10 ** 6)
    assert r["status"] == "converged"
    # Theorem num_iter: the stopping sum is below delta' within 2 + 88 |E| C_inf / (delta' eps) half-sweeps
    assert r["t"] <= 2 + 88 * p.n_edges * c_inf / (tol * eps)
    T_hat, plans = rounded_transport(o, o.current_side())
    # the rounded plans are feasible: every constrained node carries its marginal,
    # every free node one common marginal
    for e, G in plans.items():
        a, b = int(p.edges[e][0]), int(p.edges[e][1])
        assert abs(G.sum() - 1.0) < 1e-12
        leaf = b if p.is_fixed[b] else a
        q = G.sum(axis=0) if leaf == b else G.sum(axis=1)
        assert np.max(np.abs(q - p.node_marginal(leaf))) < 1e-12
    centre = [G.sum(axis=1) for G in plans.values()]
    for q in centre[1:]:
        assert np.max(np.abs(q - centre[0])) < 1e-12
    T_star = lp_coupled(p)
    assert T_hat >= T_star - 1e-9          # a feasible point costs at least the optimum
    assert T_hat - T_star <= DELTA         # the delta-approximation guarantee
