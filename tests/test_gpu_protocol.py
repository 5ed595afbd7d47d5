"""The paper's accuracy-delta protocol on the device against the FP64 oracle
(needs an MI355X): with eps = delta / (4 |E| log d) and stopping sum
delta' = delta / (8 C_inf), the device stops at the oracle's half-sweep
(within two: both take the decision in FP64, summed in different orders), its
rounded transport cost (Algorithm round, FP64 on the device) matches the
oracle's, and it lies within delta of the unregularised optimum (HiGHS)."""
import numpy as np
import pytest

from oracle import TreeOracle
from oracle.brute import lp_coupled
from oracle.rounding import rounded_transport
from workloads import make_lognormal_star

pytestmark = pytest.mark.gpu

DELTA = 0.2


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_10849_amd import Context
    return Context(0)


@pytest.mark.parametrize("L,d,seed", [(3, 10, 0), (3, 20, 1), (4, 10, 2), (8, 10, 3)])
def test_protocol_matches_oracle(ctx, L, d, seed):
    from paper_2406_10849_amd import Problem
    eps = DELTA / (4.0 * L * np.log(d))
    tol = DELTA / 8.0
    p = make_lognormal_star(L, d, eps, instance=seed)
    g = Problem(ctx, p)
    r = g.solve(tol=tol, max_steps=10 ** 6, precision="fp64", check_every=2)
    assert r["status"] == "converged"
    o = TreeOracle(p)
    ro = o.solve(tol=tol, max_steps=10 ** 6)
    assert abs(r["t"] - ro["t"]) <= 2
    rr = g.round()
    if r["t"] == ro["t"]:
        T_o, _ = rounded_transport(o, o.current_side())
        assert abs(rr["transport"] - T_o) <= 1e-10
    T_star = lp_coupled(p)
    assert T_star - 1e-9 <= rr["transport"] <= T_star + DELTA
