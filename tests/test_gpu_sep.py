"""Separable messages on Cartesian grid supports against the FP64 oracle and
against the general message kernel, through the C ABI (needs an MI355X).

When every support of an instance is a row-major grid (D = 2, on-the-fly
squared-Euclidean cost), the library splits each message's log-sum-exp into
two one-dimensional passes.  The oracle sums every (x, y) pair, so agreement
checks the split itself.  GMOT_NO_SEP=1 (read at problem creation) sends the
same problem through the general kernel.
"""
import copy

import numpy as np
import pytest

from oracle import TreeOracle
from workloads import make_tree, make_random_tree, make_batched_stars, make_star, grid_2d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_10849_amd import Context
    return Context(0)


def gpu_problem(ctx, p, first_color=-1):
    from paper_2406_10849_amd import Problem
    return Problem(ctx, p, first_color=first_color)


def _cases():
    # ragged grids (partial last rows), a constrained interior node, a free
    # star centre of degree 5
    t = make_tree([(0, 1), (0, 2), (0, 3), (0, 4), (0, 5), (5, 6), (6, 7)], [300, 70, 129, 64, 3, 257, 190, 33],
                  [0, 1, 1, 1, 1, 1, 0, 1], dim=2, eps=0.02, instance=90, support="grid", marginals="gm")
    # random 2D grid tree, the 256-node workload's recipe at small sizes
    r = make_random_tree(n_nodes=20, n_lo=30, n_hi=700, eps=5e-3, dim=2, cfg_id=3, instance=91)
    # more than 16 edges at the centre (messages through the full-message buffer)
    s = make_tree([(0, k) for k in range(1, 21)], [150] + [37 + 11 * k for k in range(20)], [0] + [1] * 20, dim=2,
                  eps=0.05, instance=92, support="grid", marginals="gm")
    return [t, r, s]


@pytest.mark.parametrize("path", ["horner", "pass"])
@pytest.mark.parametrize("case", [0, 1, 2])
def test_separable_iterates_match_oracle_and_general_kernel(ctx, case, path, monkeypatch):
    """Both separable paths: Horner's rule on uniform grids (k_sep_horner, FP64
    in both precisions; GMOT_GRID=1) and the shifted exponential sums
    (k_sep_pass; GMOT_GRID=0)."""
    monkeypatch.setenv("GMOT_GRID", "1" if path == "horner" else "0")
    p = _cases()[case]
    # which separable kernel group the instance takes (5 x 6 grids at eps = 5e-3
    # lie outside the Horner passes' range and take k_sep_pass either way)
    t = gpu_problem(ctx, p)
    t.solve(tol=0.0, max_steps=2, timing=True)
    gp = t.stats()["group_pairs"]
    horner = gp[6] > 0
    assert (gp[4] > 0) != horner and (path == "horner" or not horner)
    steps = 12
    o = TreeOracle(p)
    hist = o.run_fixed(steps)
    eo = o.evaluate()
    for precision, tol in (("fp64", 1e-9), ("fp32core", 1e-9 if horner else 1e-6)):
        g = gpu_problem(ctx, p)
        r = g.solve(tol=0.0, max_steps=steps, precision=precision)
        assert r["steps"] == steps
        assert abs(g.evaluate()["dual"] - eo["dual"]) <= tol * eo["scale"]
        for e in range(p.n_edges):
            assert np.max(np.abs(g.coupling(e) - o.coupling(e))) <= tol
        rel = 1e-8 if tol < 1e-6 else 1e-3
        assert abs(r["err_sum"] - hist[-1][0]) <= rel * hist[-1][0] + 1e-10
        monkeypatch.setenv("GMOT_NO_SEP", "1")
        h = gpu_problem(ctx, p)
        monkeypatch.delenv("GMOT_NO_SEP")
        h.solve(tol=0.0, max_steps=steps, precision=precision)
        # the general kernel's own precision bounds this comparison
        tol_h = 1e-9 if precision == "fp64" else 1e-6
        for e in range(p.n_edges):
            assert np.max(np.abs(g.coupling(e) - h.coupling(e))) <= tol_h


@pytest.mark.parametrize("shape", ["8,1,2", "4,1,1", "16,2"])
def test_separable_records_follow_the_node_shape(ctx, shape, monkeypatch):
    """Tile records are kept per 32 rows (32-row node tiles) or per 64; the
    separable node stage writes them at the plan's granularity."""
    monkeypatch.setenv("GMOT_NODE_SHAPE", shape)
    p = _cases()[0]
    o = TreeOracle(p)
    o.run_fixed(9)
    eo = o.evaluate()
    g = gpu_problem(ctx, p)
    g.solve(tol=0.0, max_steps=9, precision="fp64")
    assert abs(g.evaluate()["dual"] - eo["dual"]) <= 1e-9 * eo["scale"]
    assert np.max(np.abs(g.potentials() - o.potentials())) <= 1e-9 * max(1.0, np.max(np.abs(o.potentials())))


def test_degenerate_grids(ctx):
    """One-point supports, single-row grids (n < 4 gives one grid row) and
    a single-column grid (points sharing the second coordinate)."""
    col = make_tree([(0, 1), (1, 2)], [5, 40, 7], [1, 0, 1], dim=2, eps=0.1, instance=93, support="grid")
    col.support = col.support.copy()
    off = col.offsets()
    col.support[off[0]:off[1]] = np.stack([np.linspace(0, 1, 5), np.zeros(5)], axis=1)  # one column, five rows
    for p in (make_tree([(0, 1), (1, 2)], [1, 3, 2], [1, 0, 1], dim=2, eps=0.1, instance=94, support="grid"), col):
        o = TreeOracle(p)
        o.run_fixed(10)
        g = gpu_problem(ctx, p)
        g.solve(tol=0.0, max_steps=10, precision="fp64")
        assert np.max(np.abs(g.potentials() - o.potentials())) <= 1e-9 * max(1.0, np.max(np.abs(o.potentials())))


def test_separable_converged_and_per_node_schedule(ctx):
    """A converged FP32-core solve re-measured by the oracle; the per-node
    schedule gives bit-identical iterates; the finalise step carried by the
    separable first pass stops where the separate finalise kernel does."""
    p = _cases()[1]
    ref = TreeOracle(p)
    ref.solve(tol=1e-11, max_steps=50000)
    er = ref.evaluate()
    g = gpu_problem(ctx, p)
    r = g.solve(tol=1e-6, max_steps=50000)
    assert r["status"] == "converged"
    o = TreeOracle(p)
    lam = o.set_potentials(g.potentials())
    assert o.full_error(lam)[0] <= 1e-6 + 1e-10
    assert abs(o.evaluate(lam)["dual"] - er["dual"]) <= 1e-6 * er["scale"]
    a, b = gpu_problem(ctx, p), gpu_problem(ctx, p)
    ra = a.solve(tol=0.0, max_steps=15)
    rb = b.solve(tol=0.0, max_steps=15, schedule="per_node")
    assert ra["steps"] == rb["steps"] == 15
    assert np.array_equal(a.potentials(), b.potentials())
    for kw in ({"tol": 1e-6, "max_steps": 100000}, {"tol": 0.0, "max_steps": 37}):
        g1, g2 = gpu_problem(ctx, p), gpu_problem(ctx, p)
        r1 = g1.solve(**kw)
        r2 = g2.solve(schedule="per_node", **kw)
        assert r1["status"] == r2["status"] and r1["t"] == r2["t"] and r1["err_sum"] == r2["err_sum"]
        assert np.array_equal(g1.potentials(), g2.potentials())


def test_mixed_batch(ctx):
    """One batch holding 1D instances, 2D grid instances (separable) and a 2D
    instance on scattered points (general kernel): every instance matches the
    oracle after the same half-sweeps, and all converge."""
    from paper_2406_10849_amd import Batch
    probs = make_batched_stars(count=6, l_lo=2, l_hi=5, n_lo=20, n_hi=300, first_instance=120)
    scattered = make_tree([(0, 1), (0, 2), (0, 3)], [90, 60, 70, 80], [0, 1, 1, 1], dim=2, eps=0.02, instance=95)
    probs.append(scattered)
    assert {p.dim for p in probs} == {1, 2}
    gps = [gpu_problem(ctx, p) for p in probs]
    b = Batch(ctx, gps)
    steps = 10
    b.solve(tol=0.0, max_steps=steps, precision="fp64")
    for p, g in zip(probs, gps):
        o = TreeOracle(p)
        o.run_fixed(steps)
        assert np.max(np.abs(g.potentials() - o.potentials())) <= 1e-9 * max(1.0, np.max(np.abs(o.potentials())))
    rs = b.solve(tol=1e-6, max_steps=20000)
    evs = b.evaluate()
    for p, g, r, ev in zip(probs, gps, rs, evs):
        assert r["status"] == "converged"
        o = TreeOracle(p)
        assert o.full_error(o.set_potentials(g.potentials()))[0] <= 1e-6 + 1e-10
        # the batched evaluation equals the instance's own, up to summation order
        own = g.evaluate()
        for key in ("dual", "primal", "transport", "err_sum", "mass_min", "mass_max", "scale"):
            assert abs(ev[key] - own[key]) <= 1e-12 * max(1.0, abs(own[key])), key
