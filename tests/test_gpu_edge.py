"""Edge cases of the HIP path against the FP64 oracle, through the C ABI
(needs an MI355X).

* Nodes with more than 128 tile records: the loops over records in the
  normaliser and the finalise step run several rounds per lane.
* Zero entries in given marginals (log 0 = -inf): guarded sums and the
  limit value of the constrained update, in both precisions.
* A held state whose stopping sum is not finite: the solve reports
  GMOT_NONFINITE, keeps the state it was given, and the handle stays usable;
  in a batch the other instances are unaffected.
"""
import copy

import numpy as np
import pytest

from oracle import TreeOracle
from workloads import make_chain, make_tree, make_batched_stars

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_10849_amd import Context
    return Context(0)


def gpu_problem(ctx, p, first_color=-1):
    from paper_2406_10849_amd import Problem
    return Problem(ctx, p, first_color=first_color)


def _with_zeros(p, node, idx):
    q = copy.deepcopy(p)
    off, n = int(q.marginal_offsets()[node]), int(q.sizes[node])
    mu = q.marginal[off:off + n].copy()
    mu[list(idx)] = 0.0
    q.marginal = q.marginal.copy()
    q.marginal[off:off + n] = mu / mu.sum()
    return q


@pytest.mark.parametrize("path", ["grid", "general"])
@pytest.mark.parametrize("shape", ["8,1,2", "2,1,2", "16,2"])
def test_more_than_128_tile_records(ctx, shape, path, monkeypatch):
    """A free node of 4200 points has 132 records of 32 rows (8,1,2 and
    2,1,2) or 66 of 64 rows (16,2): every record loop runs more than one round
    per lane.  Fixed-step iterates and in-loop stopping sums against the oracle,
    FP64 and FP32 core, on the grid kernel (GMOT_GRID=1) and on the general
    node kernel (GMOT_GRID=0)."""
    monkeypatch.setenv("GMOT_NODE_SHAPE", shape)
    monkeypatch.setenv("GMOT_GRID", "1" if path == "grid" else "0")
    p = make_tree([(0, 1), (1, 2), (1, 3)], [700, 4200, 900, 4200], [1, 0, 1, 1], dim=1, eps=0.02,
                  instance=70, support="grid", marginals="gm")
    steps = 8
    o = TreeOracle(p)
    hist = o.run_fixed(steps)
    eo = o.evaluate()
    for precision, tol in (("fp64", 1e-9), ("fp32core", 1e-6)):
        g = gpu_problem(ctx, p)
        r = g.solve(tol=0.0, max_steps=steps, precision=precision)
        assert r["steps"] == steps
        assert abs(g.evaluate()["dual"] - eo["dual"]) <= tol * eo["scale"]
        lo, lg = o.potentials(), g.potentials()
        assert np.max(np.abs(lg - lo)) <= (1e-9 if precision == "fp64" else 1e-5) * max(1.0, np.max(np.abs(lo)))
        rel = 1e-8 if precision == "fp64" else 1e-3
        assert abs(r["err_sum"] - hist[-1][0]) <= rel * hist[-1][0] + 1e-10
        for j in (1, 3):
            assert np.max(np.abs(g.node_marginal(j) - o.node_marginal(j))) <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32core"])
def test_zero_mass_marginals(ctx, precision):
    """Zero entries in the marginals of a constrained leaf, a constrained
    interior node and both ends of a constrained-constrained edge: iterates
    after a fixed number of half-sweeps, then a converged solve whose state
    the oracle re-measures."""
    p = make_tree([(0, 1), (1, 2), (2, 3), (3, 4), (4, 5)], [90, 120, 150, 80, 100, 70], [1, 0, 1, 0, 1, 1],
                  dim=1, eps=0.02, instance=71, support="grid", marginals="gm")
    p = _with_zeros(_with_zeros(_with_zeros(_with_zeros(p, 0, range(0, 20)), 2, [5, 77, 149]), 4, [0, 99]),
                    5, range(50, 70))
    steps = 20
    o = TreeOracle(p)
    o.run_fixed(steps)
    eo = o.evaluate()
    assert np.isfinite(eo["dual"])
    g = gpu_problem(ctx, p)
    r = g.solve(tol=0.0, max_steps=steps, precision=precision)
    assert r["steps"] == steps
    tol = 1e-9 if precision == "fp64" else 1e-6
    eg = g.evaluate()
    assert abs(eg["dual"] - eo["dual"]) <= tol * eo["scale"]
    for e in range(p.n_edges):
        assert np.max(np.abs(g.coupling(e) - o.coupling(e))) <= tol
    # zero rows stay exactly zero
    assert np.all(g.coupling(0)[:20] == 0.0)
    r = g.solve(tol=1e-7, max_steps=50000, precision=precision)
    assert r["status"] == "converged"
    lam = o.set_potentials(g.potentials())
    assert np.all(np.isfinite(g.potentials()))
    e_sum, _ = o.full_error(lam)
    assert e_sum <= 1e-7 + 1e-10


def test_host_potentials_must_be_finite(ctx):
    """gmot_set_potentials refuses a non-finite entry and keeps the held state."""
    from paper_2406_10849_amd import GmotError, GMOT_EINVAL
    p = make_chain(n_nodes=6, n=150, eps=1e-2)
    g = gpu_problem(ctx, p)
    g.solve(tol=0.0, max_steps=5)
    before = g.potentials()
    lam = np.zeros(g.n_pot)
    lam[3] = np.nan
    with pytest.raises(GmotError) as ei:
        g.set_potentials(lam)
    assert ei.value.code == GMOT_EINVAL
    assert np.array_equal(g.potentials(), before)


@pytest.mark.parametrize("precision", ["fp64", "fp32core"])
@pytest.mark.parametrize("how", ["nan_dev", "inf_dev", "huge_host"])
def test_nonfinite_sum_is_reported_and_state_kept(ctx, precision, how):
    """A held state whose stopping sum is not finite: a NaN or an infinity
    given through the device-pointer setter (which does not inspect values),
    or a finite potential of 1e300 given through the host setter (its plan
    entries overflow, so the sum is +inf).  The solve stops with
    GMOT_NONFINITE before any update and keeps the state it was given; after
    finite potentials are set the same handle converges."""
    import torch
    p = make_chain(n_nodes=6, n=150, eps=1e-2)
    g = gpu_problem(ctx, p)
    lam = np.zeros(g.n_pot)
    lam[g.n_pot // 3] = {"nan_dev": np.nan, "inf_dev": np.inf, "huge_host": 1e300}[how]
    if how == "huge_host":
        g.set_potentials(lam)
    else:
        g.set_potentials_dev(torch.from_numpy(lam).cuda())
        torch.cuda.synchronize()
    r = g.solve(tol=1e-6, max_steps=1000, precision=precision, restart=False)
    assert r["status"] == "nonfinite"
    assert r["steps"] == 0
    assert np.array_equal(g.potentials(), lam, equal_nan=True)
    g.set_potentials(np.zeros(g.n_pot))
    r = g.solve(tol=1e-6, max_steps=20000, precision=precision, restart=False)
    assert r["status"] == "converged"
    o = TreeOracle(p)
    e_sum, _ = o.full_error(o.set_potentials(g.potentials()))
    assert e_sum <= 1e-6 + 1e-10


def test_nonfinite_instance_in_a_batch(ctx):
    """One instance of a batch holds a state whose stopping sum overflows; it
    stops as non-finite with its state kept, the others converge."""
    from paper_2406_10849_amd import Batch
    probs = make_batched_stars(count=4, l_lo=2, l_hi=4, n_lo=40, n_hi=200, first_instance=80)
    gps = [gpu_problem(ctx, p) for p in probs]
    lam = np.zeros(gps[2].n_pot)
    lam[7] = 1e300
    gps[2].set_potentials(lam)
    b = Batch(ctx, gps)
    rs = b.solve(tol=1e-6, max_steps=20000, restart=False)
    assert rs[2]["status"] == "nonfinite" and rs[2]["steps"] == 0
    assert np.array_equal(gps[2].potentials(), lam)
    for i in (0, 1, 3):
        assert rs[i]["status"] == "converged"
        o = TreeOracle(probs[i])
        e_sum, _ = o.full_error(o.set_potentials(gps[i].potentials()))
        assert e_sum <= 1e-6 + 1e-10
