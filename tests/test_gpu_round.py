"""Rounding (Algorithm round) on the device against the FP64 reference.

Both sides run the same number of FP64 half-sweeps from the cold start, then
round.  The device pass is FP64 throughout, so rounded transport, per-edge
transport, the stopping-sum parenthesis of Lemma round and the rounded plans
agree to summation order: 1e-10 relative on sums, 1e-12 absolute on plan
entries (every entry is at most 1).  The rounded plans must also be feasible
on their own: every node's marginals agree across its edges and equal mu_j
where constrained (checked directly from the device plans).
"""
import numpy as np
import pytest

from oracle import TreeOracle
from oracle.rounding import round_plans, rounded_transport
from workloads import make_config, make_chain, make_tree, make_random_tree, COST_EXPLICIT

pytestmark = pytest.mark.gpu

TREES = [
    ([(0, 1), (1, 2), (1, 3), (3, 4), (3, 5)], [5, 7, 6, 8, 5, 6], [1, 0, 1, 0, 1, 1]),
    ([(0, 1), (0, 2), (0, 3)], [6, 5, 7, 4], [0, 1, 1, 1]),
    ([(0, 1), (1, 2), (2, 3), (3, 4)], [4, 6, 5, 6, 4], [1, 0, 0, 0, 1]),
    # constrained interior node (split reading) and ragged sizes above one row tile
    ([(0, 1), (1, 2), (1, 3), (2, 4)], [300, 257, 40, 513, 7], [0, 1, 1, 0, 1]),
]


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_10849_amd import Context
    return Context(0)


def _pair(ctx, p, steps):
    from paper_2406_10849_amd import Problem
    g = Problem(ctx, p)
    r = g.solve(tol=0.0, max_steps=steps, precision="fp64")
    assert r["steps"] == steps or (r["status"] == "converged" and r["err_sum"] == 0.0)
    o = TreeOracle(p)
    o.run_fixed(r["steps"])
    return g, o


def _check_feasible(p, o, plans):
    for j in range(p.n_nodes):
        margs = []
        for k in o.nbrs[j]:
            e = o.edge_of[(j, k)]
            G = plans[e]
            assert np.min(G) >= -1e-15
            margs.append(G.sum(axis=1) if int(p.edges[e][0]) == j else G.sum(axis=0))
        for m in margs:
            assert np.max(np.abs(m - margs[0])) <= 1e-12
        if p.is_fixed[j]:
            assert np.max(np.abs(margs[0] - o.mu[j])) <= 1e-12


@pytest.mark.parametrize("k", range(len(TREES)))
@pytest.mark.parametrize("steps", [1, 2, 7])
def test_round_small_trees(ctx, k, steps):
    edges, sizes, fixed = TREES[k]
    p = make_tree(edges, sizes, fixed, eps=0.1, instance=20 + k)
    g, o = _pair(ctx, p, steps)
    S = o.current_side()
    res = g.round()
    T_o, plans_o = rounded_transport(o, S)
    assert res["side"] == (0 if o.t % 2 == 1 else 1)
    assert abs(res["transport"] - T_o) <= 1e-10 * max(1.0, abs(T_o))
    E_o, _ = o.side_error(S)
    assert abs(res["err_side"] - E_o) <= 1e-10 * E_o + 1e-14
    assert abs(res["c_inf"] - o.c_inf()) <= 1e-14 * o.c_inf()
    plans_g = {}
    for e in range(p.n_edges):
        plans_g[e] = g.rounded_coupling(e)
        To_e = float(np.sum(o.cost(int(p.edges[e][0]), int(p.edges[e][1])) * plans_o[e]))
        assert abs(res["edge_transport"][e] - To_e) <= 1e-10 * max(1.0, abs(To_e))
        assert np.max(np.abs(plans_g[e] - plans_o[e])) <= 1e-12
    _check_feasible(p, o, plans_g)
    # Lemma round on the device quantities
    T_unrounded = g.evaluate()["transport"]
    assert abs(res["transport"] - T_unrounded) <= 2 * res["c_inf"] * res["err_side"] + 1e-12


def test_round_random_tree_2d_and_explicit(ctx):
    p = make_random_tree(n_nodes=12, n_lo=60, n_hi=300, instance=3)
    for q in [p, make_tree([(0, 1), (1, 2), (1, 3)], [70, 300, 9, 260], [1, 0, 1, 1], eps=0.05, instance=8)]:
        if q is not p:
            # explicit cost matrices: the squared distances, perturbed, as FP32
            rng = np.random.default_rng(4)
            o0 = TreeOracle(q)
            cost = [(o0.cost(int(a), int(b)) * rng.uniform(0.5, 1.5, size=o0.cost(int(a), int(b)).shape))
                    .astype(np.float32) for a, b in q.edges]
            q.cost_kind = COST_EXPLICIT
            q.cost = cost
        g, o = _pair(ctx, q, 5)
        S = o.current_side()
        res = g.round()
        T_o, plans_o = rounded_transport(o, S)
        assert abs(res["transport"] - T_o) <= 1e-10 * max(1.0, abs(T_o))
        for e in range(q.n_edges):
            assert np.max(np.abs(g.rounded_coupling(e) - plans_o[e])) <= 1e-12


def test_round_requires_a_half_sweep_and_tracks_state(ctx):
    from paper_2406_10849_amd import Problem, GmotError
    p = make_tree(*TREES[0], eps=0.1, instance=1)
    g = Problem(ctx, p)
    with pytest.raises(GmotError):
        g.round()
    g.solve(tol=0.0, max_steps=3, precision="fp64")
    with pytest.raises(GmotError):
        g.rounded_coupling(0)          # no rounding of this state yet
    g.round()
    g.rounded_coupling(0)
    g.solve(tol=0.0, max_steps=1, precision="fp64")
    with pytest.raises(GmotError):
        g.rounded_coupling(0)          # the state changed since


def test_round_full_size_chain(ctx):
    """32-node chain, n = 1024: 6 FP64 half-sweeps, then rounding; transport
    and sampled rounded plans against the reference."""
    p = make_config(2)
    g, o = _pair(ctx, p, 6)
    S = o.current_side()
    res = g.round()
    T_o, plans_o = rounded_transport(o, S)
    assert abs(res["transport"] - T_o) <= 1e-10 * max(1.0, abs(T_o))
    E_o, _ = o.side_error(S)
    assert abs(res["err_side"] - E_o) <= 1e-10 * E_o + 1e-14
    for e in [0, 15, 30]:
        assert np.max(np.abs(g.rounded_coupling(e) - plans_o[e])) <= 1e-12


def test_round_converged_fp32core_chain(ctx):
    """Converged FP32-core run: the rounded plans are feasible and the rounded
    transport stays within the bound of Lemma round of the unrounded one."""
    from paper_2406_10849_amd import Problem
    p = make_chain(n_nodes=12, n=200, eps=1e-2)
    g = Problem(ctx, p)
    r = g.solve(tol=1e-6, max_steps=100000)
    assert r["status"] == "converged"
    res = g.round()
    ev = g.evaluate()
    assert res["err_side"] <= 1e-6 + 1e-9
    assert abs(res["transport"] - ev["transport"]) <= 2 * res["c_inf"] * res["err_side"] + 1e-12
    o = TreeOracle(p)
    _check_feasible(p, o, {e: g.rounded_coupling(e) for e in range(p.n_edges)})
