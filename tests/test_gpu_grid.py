"""Messages from uniform one-dimensional grids (k_msg_grid: the message of
eq. q as a polynomial in each row's ratio, summed by Horner's rule), through
the C ABI (needs an MI355X).

A D = 1 problem whose supports are uniform grids takes this path when the
autotuner finds it faster, or untuned when its node stage has at least 1024
message waves; GMOT_GRID=1 forces it for a plan (these tests) and
GMOT_NO_GRID=1 (read at problem creation) keeps the general node kernel.
The grid path sums in FP64 in both precisions, so after
the same half-sweeps its potentials match the oracle to 1e-9 of their size,
couplings to 1e-9 and the dual to 1e-9 of the objective scale, FP32-core mode
included; converged solves are re-measured by the oracle.  Problems outside
the path (non-uniform supports, or powers of a row's ratio beyond the admitted
range) take the general kernel and still match the oracle.
"""
import copy

import numpy as np
import pytest

from oracle import TreeOracle
from workloads import make_chain, make_star, make_tree, make_batched_stars

pytestmark = pytest.mark.gpu

GRID_GROUP = 5  # kernel group of the grid path in the timing stats
SEP_HORNER_GROUP = 6  # separable passes by Horner's rule


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_10849_amd import Context
    return Context(0)


@pytest.fixture(autouse=True)
def grid_on(monkeypatch):
    """These problems are small: without GMOT_GRID=1 the untuned default keeps
    the node kernel for plans of fewer than 1024 message waves."""
    monkeypatch.setenv("GMOT_GRID", "1")


def gpu_problem(ctx, p):
    from paper_2406_10849_amd import Problem
    return Problem(ctx, p)


def grid_pairs(ctx, p, group=GRID_GROUP):
    """Terms a kernel group evaluated in one timed half-sweep pair."""
    g = gpu_problem(ctx, p)
    g.solve(tol=0.0, max_steps=2, timing=True)
    return g.stats()["group_pairs"][group]


def _reversed(p):
    """The same problem with every support listed in descending order (h < 0)."""
    q = copy.deepcopy(p)
    off = q.offsets()
    moff = q.marginal_offsets()
    for j in range(q.n_nodes):
        q.support[off[j]:off[j + 1]] = q.support[off[j]:off[j + 1]][::-1].copy()
        if moff[j] >= 0:
            n = int(q.sizes[j])
            q.marginal[moff[j]:moff[j] + n] = q.marginal[moff[j]:moff[j] + n][::-1].copy()
    return q


def _cases():
    # ragged sizes (not multiples of 64), a constrained interior node, a star
    # centre of degree 12 over supports of different sizes, single-point and
    # two-point nodes (h = 0 and one interval), a large node (32 column tiles)
    chain = make_chain(n_nodes=12, n=200, eps=1e-3)
    star = make_tree([(0, k) for k in range(1, 13)], [150] + [37 + 53 * k for k in range(12)], [0] + [1] * 12,
                     dim=1, eps=0.05, instance=120, support="grid", marginals="gm")
    tiny = make_tree([(0, 1), (1, 2), (1, 3), (3, 4)], [1, 70, 2, 129, 65], [1, 0, 1, 0, 1], dim=1, eps=0.5,
                     instance=121, support="grid", marginals="gm")
    big = make_star(n=2048, leaves=3, eps=0.01, instance=122)
    return {"chain": chain, "star12": star, "tiny": tiny, "big": big, "reversed": _reversed(chain)}


@pytest.mark.parametrize("rows", ["auto", "1"])
@pytest.mark.parametrize("name", ["chain", "star12", "tiny", "big", "reversed"])
def test_grid_iterates_match_oracle_and_general_kernel(ctx, name, rows, monkeypatch):
    """rows: two rows per lane where every message admits 128-row spans
    (star12, tiny, big), one otherwise; GMOT_GRID_ROWS=1 forces one."""
    if rows == "1":
        monkeypatch.setenv("GMOT_GRID_ROWS", "1")
    p = _cases()[name]
    assert grid_pairs(ctx, p) > 0
    steps = 12
    o = TreeOracle(p)
    o.run_fixed(steps)
    eo = o.evaluate()
    lo = o.potentials()
    scale = max(1.0, float(np.max(np.abs(lo))))
    for precision in ("fp64", "fp32core"):
        g = gpu_problem(ctx, p)
        r = g.solve(tol=0.0, max_steps=steps, precision=precision)
        assert r["steps"] == steps
        assert np.max(np.abs(g.potentials() - lo)) <= 1e-9 * scale, precision
        assert abs(g.evaluate()["dual"] - eo["dual"]) <= 1e-9 * eo["scale"], precision
        for e in range(p.n_edges):
            assert np.max(np.abs(g.coupling(e) - o.coupling(e))) <= 1e-9, (precision, e)
    # the general node kernel (FP64) on the same problem
    monkeypatch.setenv("GMOT_NO_GRID", "1")
    assert grid_pairs(ctx, p) == 0
    h = gpu_problem(ctx, p)
    assert h.solve(tol=0.0, max_steps=steps, precision="fp64")["steps"] == steps
    assert np.max(np.abs(h.potentials() - g.potentials())) <= 1e-9 * scale


def test_grid_per_node_schedule_gives_identical_iterates(ctx):
    """Per-node launches of the same items give bit-identical iterates."""
    p = _cases()["star12"]
    a, b = gpu_problem(ctx, p), gpu_problem(ctx, p)
    assert a.solve(tol=0.0, max_steps=15)["steps"] == 15
    assert b.solve(tol=0.0, max_steps=15, schedule="per_node")["steps"] == 15
    assert np.array_equal(a.potentials(), b.potentials())


def test_grid_converged_solves(ctx):
    """Converged solves (chain at eps = 1e-3, a batch of one-dimensional stars):
    the oracle re-measures the stopping sum of the returned potentials, and the
    dual matches the oracle's converged dual."""
    from paper_2406_10849_amd import Batch
    p = make_chain(n_nodes=12, n=200, eps=1e-3)
    ref = TreeOracle(p)
    ref.solve(tol=1e-11, max_steps=20000)
    er = ref.evaluate()
    g = gpu_problem(ctx, p)
    assert g.solve(tol=1e-6, max_steps=20000)["status"] == "converged"
    o = TreeOracle(p)
    lam = o.set_potentials(g.potentials())
    assert o.full_error(lam)[0] <= 1e-6 + 1e-10
    assert abs(o.evaluate(lam)["dual"] - er["dual"]) <= 1e-6 * er["scale"]
    probs = [q for q in make_batched_stars(count=40, l_lo=3, l_hi=8, n_lo=64, n_hi=700, first_instance=500)
             if q.dim == 1][:12]
    gps = [gpu_problem(ctx, q) for q in probs]
    rs = Batch(ctx, gps).solve(tol=1e-6, max_steps=20000)
    assert all(r["status"] == "converged" for r in rs)
    for q, gq in zip(probs, gps):
        oq = TreeOracle(q)
        assert oq.full_error(oq.set_potentials(gq.potentials()))[0] <= 1e-6 + 1e-10


def test_grid_eligibility(ctx):
    """A support moved off its grid, or powers of a row's ratio beyond the
    admitted range (a small eps on a coarse grid), take the general kernel;
    the iterates still match the oracle."""
    base = make_chain(n_nodes=6, n=150, eps=1e-2)
    off = copy.deepcopy(base)
    off.support = off.support.copy()
    off.support[3] += 1e-9
    coarse = make_chain(n_nodes=6, n=64, eps=1e-5)
    assert grid_pairs(ctx, base) > 0
    for p in (off, coarse):
        assert grid_pairs(ctx, p) == 0
        o = TreeOracle(p)
        o.run_fixed(8)
        g = gpu_problem(ctx, p)
        assert g.solve(tol=0.0, max_steps=8, precision="fp64")["steps"] == 8
        lo = o.potentials()
        assert np.max(np.abs(g.potentials() - lo)) <= 1e-9 * max(1.0, float(np.max(np.abs(lo))))


def test_grid_zero_mass_and_far_potentials(ctx):
    """Zero entries in a given marginal (log 0 = -inf columns) and potentials
    moved 300 nats away: the running maximum moves, and the partial sums are
    rescaled, within one call."""
    p = make_chain(n_nodes=8, n=200, eps=1e-2)
    q = copy.deepcopy(p)
    off, n = int(q.marginal_offsets()[0]), int(q.sizes[0])
    mu = q.marginal[off:off + n].copy()
    mu[:80] = 0.0
    q.marginal = q.marginal.copy()
    q.marginal[off:off + n] = mu / mu.sum()
    for prob, shift in ((q, 0.0), (p, 300.0), (p, -300.0)):
        o = TreeOracle(prob)
        o.run_fixed(6)
        lam = o.potentials() + shift
        g = gpu_problem(ctx, prob)
        g.solve(tol=0.0, max_steps=2)
        g.set_potentials(lam)
        o2 = TreeOracle(prob)
        o2.Lam = o2.set_potentials(lam)
        r = g.solve(tol=0.0, max_steps=4, restart=False, verify=False, precision="fp64")
        assert r["steps"] == 4
        o2.run_fixed(4)
        lo = o2.potentials()
        fin = np.isfinite(lo)
        assert np.array_equal(fin, np.isfinite(g.potentials()))
        assert np.max(np.abs(g.potentials()[fin] - lo[fin])) <= 1e-9 * max(1.0, float(np.max(np.abs(lo[fin]))))


def rect_grid_problem(rows, cols, eps, instance):
    """A three-node chain on one rows x cols Cartesian grid per node (row-major,
    uniform coordinates in [0, 1]), the middle node free."""
    p = make_tree([(0, 1), (1, 2)], [rows * cols] * 3, [1, 0, 1], dim=2, eps=eps, instance=instance,
                  support="grid", marginals="dirichlet")
    R = np.linspace(0.0, 1.0, rows) if rows > 1 else np.zeros(1)
    Cc = np.linspace(0.0, 1.0, cols) if cols > 1 else np.zeros(1)
    pts = np.stack(np.meshgrid(R, Cc, indexing="ij"), axis=-1).reshape(-1, 2)
    p.support = np.ascontiguousarray(np.concatenate([pts] * 3, axis=0))
    return p


@pytest.mark.parametrize("rows,cols", [(2, 100), (100, 2), (9, 70), (70, 9)])
def test_separable_horner_several_input_tiles(ctx, rows, cols, monkeypatch):
    """Grid lines of more than 64 points (several 64-input tiles per pass, Horner
    across tiles), both orientations: FP64 and FP32-core iterates to 1e-9 of
    the oracle and of the shifted-sum path (GMOT_NO_GRID=1, FP64); on the
    oracle's potentials the evaluation (whose transport cost comes from the
    passes' moments, with no pair pass) matches the oracle's objectives."""
    p = rect_grid_problem(rows, cols, eps=0.05, instance=130 + rows)
    assert grid_pairs(ctx, p, SEP_HORNER_GROUP) > 0
    steps = 10
    o = TreeOracle(p)
    o.run_fixed(steps)
    lo = o.potentials()
    scale = max(1.0, float(np.max(np.abs(lo))))
    for precision in ("fp64", "fp32core"):
        g = gpu_problem(ctx, p)
        assert g.solve(tol=0.0, max_steps=steps, precision=precision)["steps"] == steps
        assert np.max(np.abs(g.potentials() - lo)) <= 1e-9 * scale, precision
    g.set_potentials(lo)
    eg, eo = g.evaluate(), o.evaluate()
    for key in ["dual", "primal", "transport"]:
        assert abs(eg[key] - eo[key]) <= 1e-10 * max(1.0, eo["scale"]), key
    monkeypatch.setenv("GMOT_NO_GRID", "1")
    h = gpu_problem(ctx, p)
    assert h.solve(tol=0.0, max_steps=steps, precision="fp64")["steps"] == steps
    assert np.max(np.abs(h.potentials() - lo)) <= 1e-9 * scale


def test_separable_horner_fallback(ctx):
    """A coarse grid at a small eps (powers of an output's ratio beyond the
    admitted range) takes the shifted-sum passes: FP64 iterates still match the
    oracle; a uniform grid at the same size and a larger eps matches in FP32-core
    mode to 1e-9 (the Horner passes are FP64)."""
    coarse = rect_grid_problem(6, 7, eps=1e-4, instance=140)
    assert grid_pairs(ctx, coarse, SEP_HORNER_GROUP) == 0 and grid_pairs(ctx, coarse, 4) > 0
    o = TreeOracle(coarse)
    o.run_fixed(6)
    g = gpu_problem(ctx, coarse)
    assert g.solve(tol=0.0, max_steps=6, precision="fp64")["steps"] == 6
    lo = o.potentials()
    assert np.max(np.abs(g.potentials() - lo)) <= 1e-9 * max(1.0, float(np.max(np.abs(lo))))
    fine = rect_grid_problem(6, 7, eps=0.05, instance=141)
    assert grid_pairs(ctx, fine, SEP_HORNER_GROUP) > 0
    o = TreeOracle(fine)
    o.run_fixed(6)
    g = gpu_problem(ctx, fine)
    assert g.solve(tol=0.0, max_steps=6, precision="fp32core")["steps"] == 6
    lo = o.potentials()
    assert np.max(np.abs(g.potentials() - lo)) <= 1e-9 * max(1.0, float(np.max(np.abs(lo))))


def test_evaluation_on_uniform_grids_matches_oracle(ctx):
    """The FP64 evaluation pass takes the messages of uniform-grid plans from
    the Horner kernels (one-dimensional and separable): on given potentials,
    objectives, the stopping sum, node marginals and couplings agree with the
    oracle as for the general kernel; a batch mixing both kinds (and the
    general kernel) evaluates every instance the same way."""
    from paper_2406_10849_amd import Batch
    one = make_chain(n_nodes=7, n=150, eps=1e-2)
    two = make_tree([(0, 1), (1, 2), (1, 3)], [120, 300, 70, 200], [1, 0, 1, 1], dim=2, eps=0.05, instance=150,
                    support="grid", marginals="gm")
    scattered = make_tree([(0, 1), (0, 2)], [60, 50, 40], [0, 1, 1], dim=1, eps=0.05, instance=151)
    assert grid_pairs(ctx, one) > 0 and grid_pairs(ctx, two, SEP_HORNER_GROUP) > 0
    probs = [one, two, scattered]
    for p in probs:
        o = TreeOracle(p)
        o.run_fixed(7)
        g = gpu_problem(ctx, p)
        g.set_potentials(o.potentials())
        eg, eo = g.evaluate(), o.evaluate()
        for key in ["dual", "primal", "transport"]:
            assert abs(eg[key] - eo[key]) <= 1e-10 * max(1.0, eo["scale"]), key
        assert abs(eg["err_sum"] - eo["err_sum"]) <= 1e-10 + 1e-8 * eo["err_sum"]
        for j in range(p.n_nodes):
            assert np.max(np.abs(g.node_marginal(j) - o.node_marginal(j))) <= 1e-12
    gps = [gpu_problem(ctx, p) for p in probs]
    b = Batch(ctx, gps)
    b.solve(tol=0.0, max_steps=9)
    evs = b.evaluate()
    for p, g, ev in zip(probs, gps, evs):
        o = TreeOracle(p)
        eo = o.evaluate(o.set_potentials(g.potentials()))
        assert abs(ev["dual"] - eo["dual"]) <= 1e-10 * max(1.0, eo["scale"])
        assert abs(ev["err_sum"] - eo["err_sum"]) <= 1e-10 + 1e-8 * eo["err_sum"]
