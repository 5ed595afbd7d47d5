"""Coupled MOT on modified junction trees through the C ABI
(gmot_junction_create) against the FP64 junction-tree oracle, which updates
separators by the steps of Proposition general_algo on clique tensors (needs
an MI355X).  The library takes cost tensors as FP32, so the oracle is given
the same FP32-rounded tensors."""
import copy

import numpy as np
import pytest

from oracle.junction import JunctionOracle
from workloads import make_wls, make_random_junction

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_10849_amd import Context
    return Context(0)


def fp32_costs(jp):
    q = copy.deepcopy(jp)
    q.clique_cost = [np.asarray(c, dtype=np.float32).astype(np.float64) for c in jp.clique_cost]
    return q


CASES = {
    "wls-J3-n10": lambda: make_wls(J=3, n=10, eps=0.05, instance=11),
    "wls-J6-n16": lambda: make_wls(J=6, n=16, eps=0.05, instance=12),
    "random-7": lambda: make_random_junction(n_seps=7, max_vars=2, n_lo=2, n_hi=6, eps=0.1, instance=13),
}


@pytest.mark.parametrize("name", list(CASES))
def test_junction_iterates_match_oracle(ctx, name):
    from paper_2406_10849_amd import JunctionTree
    jp = fp32_costs(CASES[name]())
    steps = 10
    o = JunctionOracle(jp)
    hist = o.run_fixed(steps)
    eo = o.evaluate()
    for precision, tol in (("fp64", 1e-9), ("fp32core", 1e-6)):
        g = JunctionTree(ctx, jp)
        r = g.solve(tol=0.0, max_steps=steps, precision=precision)
        assert r["steps"] == steps
        lo, lg = o.potentials(), g.potentials()
        assert np.max(np.abs(lg - lo)) <= (1e-9 if precision == "fp64" else 1e-5) * max(1.0, np.max(np.abs(lo)))
        eg = g.evaluate()
        assert abs(eg["dual"] - eo["dual"]) <= tol * max(1.0, eg["scale"])
        assert abs(eg["transport"] - eo["transport"]) <= tol * max(1.0, abs(eo["transport"]))
        rel = 1e-8 if precision == "fp64" else 1e-3
        assert abs(r["err_sum"] - hist[-1][0]) <= rel * hist[-1][0] + 1e-10
        for c, (a, b) in enumerate(jp.cliques):
            B = o.plan(c).reshape(jp.sep_size(a), jp.sep_size(b))
            assert np.max(np.abs(g.coupling(c) - B)) <= tol


@pytest.mark.parametrize("name", ["wls-J6-n16", "random-7"])
def test_junction_converged(ctx, name):
    """A converged FP32-core solve (FP64-judged): the oracle re-measures the
    stopping sum of the returned potentials, the dual agrees with the oracle's
    converged dual, and constrained separators carry their marginals."""
    from paper_2406_10849_amd import JunctionTree
    jp = fp32_costs(CASES[name]())
    ref = JunctionOracle(jp)
    ref.solve(tol=1e-11, max_steps=200000)
    er = ref.evaluate()
    g = JunctionTree(ctx, jp)
    r = g.solve(tol=1e-6, max_steps=200000)
    assert r["status"] == "converged"
    o = JunctionOracle(jp)
    lu = o.set_potentials(g.potentials())
    assert o.full_error(lu)[0] <= 1e-6 + 1e-10
    eg = g.evaluate()
    assert abs(eg["dual"] - er["dual"]) <= 1e-6 * max(1.0, eg["scale"])
    for s in range(jp.n_separators):
        if jp.sep_fixed[s]:
            assert np.sum(np.abs(g.node_marginal(s) - np.asarray(jp.sep_marginal[s]).reshape(-1))) <= 1e-6


def test_junction_rejects_bad_descriptions(ctx):
    from paper_2406_10849_amd import JunctionTree, GmotError, GMOT_EINVAL
    jp = make_wls(J=2, n=4, instance=14)
    bad = copy.deepcopy(jp)
    bad.separators = [(0, 3), (1,), (1,)]        # variable 1 in two separators, 2 in none
    with pytest.raises(GmotError) as ei:
        JunctionTree(ctx, bad)
    assert ei.value.code == GMOT_EINVAL
    bad = copy.deepcopy(jp)
    bad.cliques = [(0, 1), (1, 0)][:1] + [(0, 1)]  # a repeated pair: not a tree
    with pytest.raises(GmotError):
        JunctionTree(ctx, bad)
