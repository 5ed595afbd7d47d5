"""Pins of the FP64 rounding reference (Algorithm "round", Lemmas "round" and
"round_applied", and the Altschuler-Weed-Rigollet rounding it calls)."""
import numpy as np
import pytest

from oracle.brute import lp_coupled
from oracle.rounding import awr_round, round_plans, rounded_transport
from oracle.tree_ot import TreeOracle
from workloads.gen import make_tree

TREES = [
    # (edges, sizes, fixed): leaves constrained, interior free
    ([(0, 1), (1, 2), (1, 3), (3, 4), (3, 5)], [5, 7, 6, 8, 5, 6], [1, 0, 1, 0, 1, 1]),
    ([(0, 1), (0, 2), (0, 3)], [6, 5, 7, 4], [0, 1, 1, 1]),
    ([(0, 1), (1, 2), (2, 3), (3, 4)], [4, 6, 5, 6, 4], [1, 0, 0, 0, 1]),
]


def _run(k, steps, eps=0.2, inst=3):
    edges, sizes, fixed = TREES[k]
    p = make_tree(edges, sizes, fixed, eps=eps, instance=inst)
    o = TreeOracle(p)
    for _ in range(steps):
        o.tstep()
    return p, o


def test_awr_polytope_and_distance():
    """AWR output lies in U(r, c) and moves F by at most 2(|r-F1| + |c-F^T 1|)
    in L1 (their Lemma 7)."""
    rng = np.random.default_rng(5)
    for trial in range(20):
        n, m = rng.integers(2, 9, size=2)
        F = rng.uniform(0, 1, size=(n, m))
        F /= F.sum() * rng.uniform(0.8, 1.2)
        r = rng.dirichlet(np.ones(n))
        c = rng.dirichlet(np.ones(m))
        G = awr_round(F, r, c)
        assert np.all(G >= -1e-15)
        np.testing.assert_allclose(G.sum(axis=1), r, atol=1e-14)
        np.testing.assert_allclose(G.sum(axis=0), c, atol=1e-14)
        bound = 2 * (np.abs(r - F.sum(1)).sum() + np.abs(c - F.sum(0)).sum())
        assert np.abs(G - F).sum() <= bound + 1e-14


def test_awr_identity_on_feasible():
    rng = np.random.default_rng(6)
    r = rng.dirichlet(np.ones(5))
    c = rng.dirichlet(np.ones(4))
    F = np.outer(r, c)
    np.testing.assert_allclose(awr_round(F, r, c), F, atol=1e-16)


@pytest.mark.parametrize("k", range(len(TREES)))
@pytest.mark.parametrize("steps", [1, 2, 5])
def test_rounded_plans_are_feasible(k, steps):
    """Lemma round: every node's rounded marginals agree (mu_j on constrained
    nodes), on both sides of every edge."""
    p, o = _run(k, steps)
    S = o.current_side()
    plans = round_plans(o, S)
    for j in range(p.n_nodes):
        margs = []
        for kk in o.nbrs[j]:
            e = o.edge_of[(j, kk)]
            G = plans[e]
            assert np.all(G >= -1e-15)
            margs.append(G.sum(axis=1) if int(p.edges[e][0]) == j else G.sum(axis=0))
        for mg in margs:
            np.testing.assert_allclose(mg, margs[0], atol=1e-13)
            assert abs(mg.sum() - 1.0) < 1e-12
        if p.is_fixed[j]:
            np.testing.assert_allclose(margs[0], o.mu[j], atol=1e-13)


@pytest.mark.parametrize("k", range(len(TREES)))
@pytest.mark.parametrize("steps", [1, 3, 8])
def test_lemma_round_cost_bound(k, steps):
    """|T(B) - T(B_hat)| <= 2 C_inf * (stopping sum of the mismatched side)."""
    p, o = _run(k, steps)
    S = o.current_side()
    T0 = o.evaluate()["transport"]
    T1, _ = rounded_transport(o, S)
    E_S, _ = o.side_error(S)
    assert abs(T1 - T0) <= 2 * o.c_inf() * E_S + 1e-13
    assert E_S > 1e-8          # the bound is exercised, not trivially met


@pytest.mark.parametrize("k", range(len(TREES)))
def test_lemma_round_applied_against_lp(k):
    """LP optimum <= T(B_hat) <= LP + 2 eps |E| log d + 4 C_inf E_S."""
    for eps, steps in [(0.2, 4), (0.05, 30), (0.01, 200)]:
        p, o = _run(k, steps, eps=eps)
        S = o.current_side()
        T1, _ = rounded_transport(o, S)
        E_S, _ = o.side_error(S)
        lp = lp_coupled(p)
        d = int(max(p.sizes))
        assert T1 >= lp - 1e-9
        assert T1 <= lp + 2 * eps * p.n_edges * np.log(d) + 4 * o.c_inf() * E_S + 1e-9


def test_rounding_needs_unit_mass():
    """Before the first update the plans do not carry unit mass (Lemma tree_mass
    holds from the first half-sweep on), so the rows of the result miss r."""
    p, o = _run(0, 0)
    plans = round_plans(o, o.current_side())
    bad = 0.0
    for e, G in plans.items():
        bad = max(bad, abs(G.sum() - 1.0))
    assert bad > 1e-3
