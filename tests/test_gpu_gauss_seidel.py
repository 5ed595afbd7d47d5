"""The node-sequential (Gauss-Seidel) schedule through the C ABI
(gmot_opts.schedule = GMOT_SCHED_GAUSS_SEIDEL) against the FP64 oracle's
sweeps (TreeOracle.gs_sweep / solve_gauss_seidel; needs an MI355X): the
potentials after a fixed number of sweeps element by element, the stopping
sum over every node, and at convergence the sweep count and the dual."""
import copy

import numpy as np
import pytest

from oracle import TreeOracle
from workloads import make_tree, make_star, make_chain, make_random_tree, COST_EXPLICIT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_10849_amd import Context
    return Context(0)


def _explicit(p, seed):
    q = copy.deepcopy(p)
    q.cost_kind = COST_EXPLICIT
    rng = np.random.default_rng(seed)
    q.cost = []
    for a, b in p.edges:
        X, Y = p.node_support(int(a)), p.node_support(int(b))
        C = np.sum((X[:, None, :] - Y[None, :, :]) ** 2, axis=2) + rng.uniform(0, 0.2, size=(X.shape[0], Y.shape[0]))
        q.cost.append(C.astype(np.float32))
    return q


CASES = {
    "tree-1d": lambda: make_tree([(0, 1), (1, 2), (1, 3), (3, 4), (3, 5), (0, 6)], [50, 40, 60, 33, 51, 47, 66],
                                 [0, 0, 1, 0, 1, 1, 1], eps=0.05, instance=81),
    "star-2d-ragged": lambda: make_star(n=300, leaves=5, eps=0.02, dim=2, instance=82),
    "chain": lambda: make_chain(n_nodes=9, n=257, eps=1e-2, instance=83),
    "explicit": lambda: _explicit(make_tree([(0, 1), (1, 2), (1, 3)], [40, 300, 77, 260], [1, 0, 1, 1], eps=0.05,
                                            instance=84), 7),
}


@pytest.mark.parametrize("name", list(CASES))
def test_sweeps_match_oracle(ctx, name):
    from paper_2406_10849_amd import Problem
    p = CASES[name]()
    sweeps = 7
    o = TreeOracle(p)
    for _ in range(sweeps):
        o.gs_sweep()
    e_o = o.full_error()[0]
    g = Problem(ctx, p)
    r = g.solve(tol=0.0, max_steps=sweeps, schedule="gauss_seidel", check_every=sweeps)
    assert r["status"] == "not_converged" and r["steps"] == sweeps
    lo, lg = o.potentials(), g.potentials()
    assert np.max(np.abs(lg - lo)) <= 1e-9 * max(1.0, float(np.max(np.abs(lo))))
    assert abs(r["err_sum"] - e_o) <= 1e-8 * max(e_o, 1e-12)
    eg, eo = g.evaluate(), o.evaluate()
    assert abs(eg["dual"] - eo["dual"]) <= 1e-10 * max(1.0, eo["scale"])


def test_converges_where_the_oracle_does(ctx):
    from paper_2406_10849_amd import Problem
    p = CASES["tree-1d"]()
    o = TreeOracle(p)
    ro = o.solve_gauss_seidel(tol=1e-9, max_sweeps=100000, check_every=4)
    g = Problem(ctx, p)
    r = g.solve(tol=1e-9, max_steps=100000, schedule="gauss_seidel", check_every=4)
    assert r["status"] == "converged" == ro["status"]
    assert r["steps"] == ro["sweeps"]
    assert abs(g.evaluate()["dual"] - o.evaluate()["dual"]) <= 1e-10 * max(1.0, o.evaluate()["scale"])


def test_continues_from_a_bipartite_state(ctx):
    """restart = 0 takes the held state: a few bipartite half-sweeps, then
    sweeps from there, equal the oracle doing the same."""
    from paper_2406_10849_amd import Problem
    p = CASES["chain"]()
    o = TreeOracle(p)
    o.run_fixed(5)
    o.gs_sweep()
    o.gs_sweep()
    g = Problem(ctx, p)
    g.solve(tol=0.0, max_steps=5, precision="fp64")
    g.solve(tol=0.0, max_steps=2, schedule="gauss_seidel", check_every=2, restart=False)
    assert np.max(np.abs(g.potentials() - o.potentials())) <= 1e-9 * max(1.0, float(np.max(np.abs(o.potentials()))))


def test_batches_refuse_the_schedule(ctx):
    from paper_2406_10849_amd import Problem, Batch, GmotError, GMOT_ENOTSUP
    b = Batch(ctx, [Problem(ctx, make_star(n=20, leaves=2, eps=0.1))])
    with pytest.raises(GmotError) as ei:
        b.solve(tol=1e-6, schedule="gauss_seidel")
    assert ei.value.code == GMOT_ENOTSUP


def test_random_tree_256_nodes_converges(ctx):
    """The 256-node tree (n in [256, 4096], 2D grids, eps = 5e-3) to a stopping
    sum of 1e-6 over every node; the oracle re-measures that sum on the
    returned potentials."""
    from paper_2406_10849_amd import Problem
    p = make_random_tree()
    g = Problem(ctx, p)
    r = g.solve(tol=1e-6, max_steps=20000, schedule="gauss_seidel", check_every=8)
    assert r["status"] == "converged" and r["err_sum"] <= 1e-6
    ev = g.evaluate()
    assert abs(ev["err_sum"] - r["err_sum"]) <= 1e-12 + 1e-9 * r["err_sum"]
