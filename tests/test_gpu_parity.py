"""HIP path against the FP64 oracle, through the C ABI (needs an MI355X).

Tolerances
----------
* FP64 path (precision="fp64"): potentials and objectives within 1e-9 relative
  of the oracle after the same number of half-sweeps (only summation order
  differs).
* FP32-core path: dual objective within 1e-6 relative to the scale
  s = sum |eps <Lam, mu>| + sum |eps rho| + eps |E|, plans within 1e-6
  absolute, after the same half-sweeps; converged runs must show a stopping
  sum <= tol re-measured by the oracle in FP64 from the returned potentials,
  and a dual within 1e-6 (relative to s) of the oracle's converged dual.
"""
import copy

import numpy as np
import pytest

from oracle import TreeOracle
from workloads import (make_config, make_chain, make_star, make_tree, make_random_tree, make_batched_stars,
                       COST_EXPLICIT)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_10849_amd import Context
    return Context(0)


def gpu_problem(ctx, p, first_color=-1):
    from paper_2406_10849_amd import Problem
    return Problem(ctx, p, first_color=first_color)


def oracle_lam(o, flat):
    return o.set_potentials(flat)


def test_config1_star_fp64_1000_half_sweeps(ctx):
    p = make_config(1)
    g = gpu_problem(ctx, p)
    r = g.solve(tol=0.0, max_steps=1000, precision="fp64")
    # tol = 0 stops early only at an exact fixed point (stopping sum exactly 0),
    # where further half-sweeps leave the plans unchanged
    assert (r["steps"] == 1000 and r["t"] == 1001) or (r["status"] == "converged" and r["err_sum"] == 0.0)
    o = TreeOracle(p)
    o.run_fixed(1000)
    lo, lg = o.potentials(), g.potentials()
    assert np.max(np.abs(lo - lg)) <= 1e-9 * max(1.0, np.max(np.abs(lo)))
    eo, eg = o.evaluate(), g.evaluate()
    assert abs(eg["dual"] - eo["dual"]) <= 1e-10 * eo["scale"]
    assert abs(eg["primal"] - eo["primal"]) <= 1e-10 * eo["scale"]
    assert abs(eg["transport"] - eo["transport"]) <= 1e-10
    assert abs(eg["err_sum"] - eo["err_sum"]) <= 1e-12 + 1e-6 * eo["err_sum"]


@pytest.mark.parametrize("path", ["grid", "general"])
@pytest.mark.parametrize("precision", ["fp64", "fp32core"])
def test_small_chain_fixed_steps(ctx, precision, path, monkeypatch):
    """Both message paths of uniform one-dimensional grids: the grid kernel
    (GMOT_GRID=1) and the general node kernel (GMOT_GRID=0)."""
    monkeypatch.setenv("GMOT_GRID", "1" if path == "grid" else "0")
    p = make_chain(n_nodes=12, n=200, eps=1e-3)
    g = gpu_problem(ctx, p)
    steps = 40
    r = g.solve(tol=0.0, max_steps=steps, precision=precision)
    assert r["steps"] == steps
    o = TreeOracle(p)
    hist = o.run_fixed(steps)
    eo = o.evaluate()
    eg = g.evaluate()
    tol = 1e-9 if precision == "fp64" else 1e-6
    assert abs(eg["dual"] - eo["dual"]) <= tol * eo["scale"]
    for e in [0, 5, 10]:
        assert np.max(np.abs(g.coupling(e) - o.coupling(e))) <= tol
    # in-loop stopping sum of the last checked state vs the oracle's
    assert abs(r["err_sum"] - hist[-1][0]) <= 0.1 * hist[-1][0] + 1e-8


def converged_check(g, p, tol, dstar, scale):
    o = TreeOracle(p)
    lam = o.set_potentials(g.potentials())
    e_sum, e_max = o.full_error(lam)
    assert e_sum <= tol + 1e-10, e_sum
    ev = o.evaluate(lam)
    assert abs(ev["dual"] - dstar) <= 1e-6 * scale
    return e_sum


def test_small_chain_converged(ctx):
    p = make_chain(n_nodes=12, n=200, eps=1e-3)
    ref = TreeOracle(p)
    ref.solve(tol=1e-11, max_steps=20000)
    er = ref.evaluate()
    g = gpu_problem(ctx, p)
    r = g.solve(tol=1e-6, max_steps=20000)
    assert r["status"] == "converged"
    converged_check(g, p, 1e-6, er["dual"], er["scale"])


def test_random_tree_2d_ragged(ctx):
    p = make_random_tree(n_nodes=20, n_lo=30, n_hi=700, eps=5e-3, dim=2, cfg_id=3, instance=7)
    o = TreeOracle(p)
    o.run_fixed(12)
    g = gpu_problem(ctx, p)
    g.solve(tol=0.0, max_steps=12)
    eo, eg = o.evaluate(), g.evaluate()
    assert abs(eg["dual"] - eo["dual"]) <= 1e-6 * eo["scale"]
    for e in range(0, p.n_edges, 4):
        assert np.max(np.abs(g.coupling(e) - o.coupling(e))) <= 1e-6


def test_random_tree_converged(ctx):
    p = make_random_tree(n_nodes=16, n_lo=20, n_hi=300, eps=5e-3, dim=2, cfg_id=3, instance=8)
    ref = TreeOracle(p)
    ref.solve(tol=1e-11, max_steps=50000)
    er = ref.evaluate()
    g = gpu_problem(ctx, p)
    r = g.solve(tol=1e-6, max_steps=50000)
    assert r["status"] == "converged"
    converged_check(g, p, 1e-6, er["dual"], er["scale"])


def test_batched_stars_mixed_dims(ctx):
    from paper_2406_10849_amd import Batch
    probs = make_batched_stars(count=6, l_lo=2, l_hi=5, n_lo=20, n_hi=300)
    gps = [gpu_problem(ctx, p) for p in probs]
    b = Batch(ctx, gps)
    rs = b.solve(tol=1e-6, max_steps=20000)
    for p, g, r in zip(probs, gps, rs):
        assert r["status"] == "converged"
        ref = TreeOracle(p)
        ref.solve(tol=1e-11, max_steps=20000)
        er = ref.evaluate()
        converged_check(g, p, 1e-6, er["dual"], er["scale"])
        # same schedule as solving the instance alone (tiles may differ, so the
        # FP32 rounding and hence the stopping step may move by a half-sweep)
        solo = gpu_problem(ctx, p)
        rs1 = solo.solve(tol=1e-6, max_steps=20000)
        assert abs(rs1["t"] - r["t"]) <= 2


def test_batch_with_mixed_parities(ctx):
    from paper_2406_10849_amd import Batch
    probs = make_batched_stars(count=3, l_lo=2, l_hi=4, n_lo=40, n_hi=200, first_instance=50)
    gps = [gpu_problem(ctx, p) for p in probs]
    refs = [TreeOracle(p) for p in probs]
    for i, (g, o) in enumerate(zip(gps, refs)):   # instance i starts at half-sweep i + 1
        if i:
            g.solve(tol=0.0, max_steps=i, precision="fp64")
            o.run_fixed(i)
    b = Batch(ctx, gps)
    rs = b.solve(tol=0.0, max_steps=7, precision="fp64", restart=False)
    for g, o, r in zip(gps, refs, rs):
        o.run_fixed(7)
        assert r["steps"] == 7
        assert np.max(np.abs(g.potentials() - o.potentials())) <= 1e-9 * max(1.0, np.max(np.abs(o.potentials())))


@pytest.mark.parametrize("path", ["grid", "general"])
def test_timing_stats_count_working_half_sweeps(ctx, path, monkeypatch):
    monkeypatch.setenv("GMOT_GRID", "1" if path == "grid" else "0")
    p = make_chain(n_nodes=10, n=150, eps=1e-2)
    g = gpu_problem(ctx, p)
    g.stats(reset=True)
    r = g.solve(tol=1e-6, max_steps=5000, timing=True, verify=False)
    st = g.stats(reset=True)
    assert r["status"] == "converged"
    assert st["msg_launches"] == r["t"]          # half-sweeps 1..t computed messages
    assert abs(st["msg_pairs"] - r["t"] * p.pairs_per_tstep()) < 0.5
    assert st["msg_ms"] > 0
    # one kernel group does all of the stage: the uniform-grid group (5) with
    # GMOT_GRID=1, the D = 1 node-kernel group (1) with GMOT_GRID=0
    grp = 5 if path == "grid" else 1
    assert st["group_pairs"][grp] == st["msg_pairs"] and sum(st["group_pairs"]) == st["msg_pairs"]
    assert st["group_ms"][grp] > 0
    assert all(st["group_ms"][k] == 0.0 for k in range(7) if k != grp)


def test_evaluate_matches_oracle_on_given_potentials(ctx):
    p = make_tree([(0, 1), (1, 2), (1, 3), (3, 4), (3, 5)], [50, 300, 70, 260, 90, 33], [1, 0, 1, 0, 1, 1],
                  eps=0.05, instance=21, dim=2)
    o = TreeOracle(p)
    o.run_fixed(7)
    g = gpu_problem(ctx, p)
    g.set_potentials(o.potentials())
    eg, eo = g.evaluate(), o.evaluate()
    for key in ["dual", "primal", "transport"]:
        assert abs(eg[key] - eo[key]) <= 1e-10 * max(1.0, eo["scale"]), key
    assert abs(eg["err_sum"] - eo["err_sum"]) <= 1e-10 + 1e-8 * eo["err_sum"]
    assert abs(eg["mass_min"] - min(eo["masses"])) <= 1e-12
    for j in range(p.n_nodes):
        assert np.max(np.abs(g.node_marginal(j) - o.node_marginal(j))) <= 1e-12
    for e in range(p.n_edges):
        assert np.max(np.abs(g.coupling(e) - o.coupling(e))) <= 1e-12


def test_edge_cases(ctx):
    # two-node problems: fixed-fixed (Sinkhorn), fixed-free, one-point supports
    for sizes, fixed in [([37, 300], [1, 1]), ([260, 5], [1, 0]), ([1, 40], [1, 0]), ([1, 1], [1, 1])]:
        p = make_tree([(0, 1)], sizes, fixed, eps=0.1, instance=31)
        g = gpu_problem(ctx, p)
        r = g.solve(tol=1e-9, max_steps=5000, precision="fp64")
        assert r["status"] == "converged"
        o = TreeOracle(p)
        ro = o.solve(tol=1e-9, max_steps=5000)
        assert r["t"] == ro["t"]
        assert np.max(np.abs(g.coupling(0) - o.coupling(0))) <= 1e-12
        r = g.solve(tol=1e-9, max_steps=5000)
        assert r["status"] == "converged"
        assert np.max(np.abs(g.coupling(0) - o.coupling(0))) <= 1e-8
    # a single node: nothing to do
    p = make_tree(np.zeros((0, 2), dtype=np.int32), [5], [1], eps=0.1)
    g = gpu_problem(ctx, p)
    r = g.solve(tol=1e-6, max_steps=10)
    assert r["status"] == "converged" and r["steps"] == 0


def test_first_colour_and_restart(ctx):
    p = make_star(n=90, leaves=4, eps=0.02)
    g = gpu_problem(ctx, p, first_color=1)
    o = TreeOracle(p, first_color=1)
    g.solve(tol=0.0, max_steps=9)
    o.run_fixed(9)
    assert np.max(np.abs(g.coupling(2) - o.coupling(2))) <= 1e-6
    # continue without restart == one longer run
    g.solve(tol=0.0, max_steps=6, restart=False)
    o.run_fixed(6)
    assert np.max(np.abs(g.coupling(2) - o.coupling(2))) <= 1e-6
    # warm start from given potentials
    g2 = gpu_problem(ctx, p, first_color=1)
    g2.set_potentials(g.potentials())
    r2 = g2.solve(tol=1e-7, max_steps=5000, restart=False, precision="fp64")
    o2 = TreeOracle(p, first_color=1)
    o2.Lam = o2.set_potentials(g.potentials())
    ro2 = o2.solve(tol=1e-7, max_steps=5000)
    assert r2["t"] == ro2["t"]
    assert np.max(np.abs(g2.potentials() - o2.potentials())) <= 1e-9 * max(1.0, np.max(np.abs(o2.potentials())))


def test_explicit_cost(ctx):
    p = make_tree([(0, 1), (1, 2), (1, 3)], [40, 300, 77, 260], [1, 0, 1, 1], eps=0.05, instance=41)
    q = copy.deepcopy(p)
    q.cost_kind = COST_EXPLICIT
    rng = np.random.default_rng(5)
    q.cost = []
    for a, b in p.edges:
        X, Y = p.node_support(int(a)), p.node_support(int(b))
        C = np.sum((X[:, None, :] - Y[None, :, :]) ** 2, axis=2) + rng.uniform(0, 0.2, size=(X.shape[0], Y.shape[0]))
        q.cost.append(C.astype(np.float32))
    o = TreeOracle(q)
    o.run_fixed(10)
    g = gpu_problem(ctx, q)
    g.solve(tol=0.0, max_steps=10)
    eo, eg = o.evaluate(), g.evaluate()
    assert abs(eg["dual"] - eo["dual"]) <= 1e-6 * eo["scale"]
    for e in range(p.n_edges):
        assert np.max(np.abs(g.coupling(e) - o.coupling(e))) <= 1e-6


def test_invalid_inputs_rejected(ctx):
    from paper_2406_10849_amd import GmotError, GMOT_EINVAL, GMOT_EMARGINAL
    p = make_tree([(0, 1), (1, 2)], [4, 5, 6], [1, 0, 1], eps=0.1)
    bad = copy.deepcopy(p)
    bad.edges = np.array([[0, 1], [0, 1]], dtype=np.int32)
    with pytest.raises(GmotError) as ei:
        gpu_problem(ctx, bad)
    assert ei.value.code == GMOT_EINVAL
    bad = copy.deepcopy(p)
    bad.marginal = bad.marginal * 1.001
    with pytest.raises(GmotError) as ei:
        gpu_problem(ctx, bad)
    assert ei.value.code == GMOT_EMARGINAL
    g = gpu_problem(ctx, p)
    with pytest.raises(GmotError):
        g.solve(tol=-1.0)
    with pytest.raises(GmotError):
        g.solve(max_steps=0)


def test_full_size_chain_converges(ctx):
    """The benchmark workload (32-node chain, n = 1024, eps = 1e-3) with the
    benchmark's launch configuration; the oracle re-measures the stopping sum of
    the returned state in FP64."""
    p = make_config(2)
    g = gpu_problem(ctx, p)
    r = g.solve(tol=1e-6, max_steps=200000)
    assert r["status"] == "converged"
    o = TreeOracle(p)
    lam = o.set_potentials(g.potentials())
    e_sum, e_max = o.full_error(lam)
    assert e_sum <= 1e-6 + 1e-10, e_sum
    assert abs(e_sum - g.evaluate()["err_sum"]) <= 1e-9


def test_per_node_schedule_gives_identical_iterates(ctx):
    """The per-node schedule launches the tiles of each node of a half-sweep
    separately, node after node; the arithmetic per row is unchanged, so the
    iterates are bit-identical."""
    p = make_random_tree(n_nodes=12, n_lo=30, n_hi=400, eps=5e-3, dim=2, cfg_id=3, instance=9)
    a = gpu_problem(ctx, p)
    b = gpu_problem(ctx, p)
    ra = a.solve(tol=0.0, max_steps=15)
    rb = b.solve(tol=0.0, max_steps=15, schedule="per_node")
    assert ra["steps"] == rb["steps"] == 15
    assert np.array_equal(a.potentials(), b.potentials())


def test_one_pass_matches_two_pass(ctx, monkeypatch):
    """The one-pass message sums (shifted by the previous max of each row and
    column range) and the
    two-pass sums give the same FP32-core iterates within the FP32-core
    tolerance, and both match the oracle after the same half-sweeps (general
    node kernel: GMOT_NO_GRID=1 keeps the chain off the grid kernel)."""
    monkeypatch.setenv("GMOT_NO_GRID", "1")
    cases = [make_chain(n_nodes=12, n=200, eps=1e-3),
             make_random_tree(n_nodes=20, n_lo=100, n_hi=600, instance=5)]
    for p in cases:
        g1, g2 = gpu_problem(ctx, p), gpu_problem(ctx, p)
        steps = 60
        r1 = g1.solve(tol=0.0, max_steps=steps, passes="auto")
        r2 = g2.solve(tol=0.0, max_steps=steps, passes="two")
        assert r1["steps"] == r2["steps"] == steps
        o = TreeOracle(p)
        o.run_fixed(steps)
        eo = o.evaluate()
        for g in (g1, g2):
            assert abs(g.evaluate()["dual"] - eo["dual"]) <= 1e-6 * eo["scale"]
        for e in range(0, p.n_edges, 3):
            assert np.max(np.abs(g1.coupling(e) - g2.coupling(e))) <= 1e-6


SHAPES = ["2,1", "4,1", "8,1", "16,1", "2,2", "4,2", "8,2", "16,2", "2,2,2", "4,2,2", "8,2,2", "16,2,2",
          "2,1,2", "4,1,2", "8,1,2", "16,1,2"]


def _shape_cases():
    # a ragged 2D tree with a constrained interior node and a star centre of
    # degree 5, and a free star centre of degree 20 (more edges than the block
    # keeps in LDS: its messages go through the full-message buffer)
    edges = [(0, 1), (0, 2), (0, 3), (0, 4), (0, 5), (5, 6), (6, 7)]
    t = make_tree(edges, [300, 70, 129, 64, 1, 257, 190, 33], [0, 1, 1, 1, 1, 1, 0, 1], dim=2, eps=0.02,
                  instance=60)
    star = make_tree([(0, k) for k in range(1, 21)], [150] + [37 + 11 * k for k in range(20)],
                     [0] + [1] * 20, dim=1, eps=0.05, instance=62)
    # explicit FP32 costs (one row per lane, so every pinned shape runs with its
    # wave count only), ragged sizes for the tile-major copies
    ex = make_tree([(0, 1), (1, 2), (1, 3)], [70, 129, 33, 200], [1, 0, 1, 1], dim=1, eps=0.05, instance=63)
    rng = np.random.default_rng(63)
    ex.cost = []
    for a, b in ex.edges:
        X, Y = ex.node_support(int(a)), ex.node_support(int(b))
        C = np.sum((X[:, None, :] - Y[None, :, :]) ** 2, axis=2) * rng.uniform(0.5, 1.5, size=(X.shape[0], Y.shape[0]))
        ex.cost.append(C.astype(np.float32))
    ex.cost_kind = COST_EXPLICIT
    return [t, star, ex]


@pytest.mark.parametrize("shape", SHAPES)
def test_every_node_shape_matches_oracle(ctx, shape, monkeypatch):
    """Each node-kernel block shape (waves per block, rows per lane, lane
    groups per wave), pinned through GMOT_NODE_SHAPE: FP64 iterates to 1e-9
    of the oracle and FP32-core ones to 1e-6 (dual relative to the scale)."""
    monkeypatch.setenv("GMOT_NODE_SHAPE", shape)
    for p in _shape_cases():
        o = TreeOracle(p)
        o.run_fixed(12)
        eo = o.evaluate()
        for precision, tol in (("fp64", 1e-9), ("fp32core", 1e-6)):
            g = gpu_problem(ctx, p)
            r = g.solve(tol=0.0, max_steps=12, precision=precision)
            assert r["steps"] == 12
            assert abs(g.evaluate()["dual"] - eo["dual"]) <= tol * eo["scale"]
            for e in range(p.n_edges):
                assert np.max(np.abs(g.coupling(e) - o.coupling(e))) <= tol


def test_three_dimensional_supports(ctx):
    """D = 3 supports (random points) on a small tree: FP64 iterates and a
    converged FP32-core solve against the oracle."""
    p = make_tree([(0, 1), (1, 2), (1, 3)], [90, 200, 65, 140], [1, 0, 1, 1], dim=3, eps=0.05, instance=61)
    o = TreeOracle(p)
    o.run_fixed(20)
    g = gpu_problem(ctx, p)
    g.solve(tol=0.0, max_steps=20, precision="fp64")
    assert np.max(np.abs(g.potentials() - o.potentials())) <= 1e-9 * max(1.0, np.max(np.abs(o.potentials())))
    r = g.solve(tol=1e-6, max_steps=100000)
    assert r["status"] == "converged"
    ref = TreeOracle(p)
    ref.solve(tol=1e-10, max_steps=100000)
    er = ref.evaluate()
    converged_check(g, p, 1e-6, er["dual"], er["scale"])


def _shuffled(p, seed):
    """The same problem with every node's support points (and marginal) in a
    seeded random order."""
    q = copy.deepcopy(p)
    rng = np.random.default_rng(seed)
    off, moff = p.offsets(), p.marginal_offsets()
    for j in range(p.n_nodes):
        perm = rng.permutation(int(p.sizes[j]))
        q.support[off[j]:off[j + 1]] = p.support[off[j]:off[j + 1]][perm]
        if p.is_fixed[j]:
            m0, m1 = moff[j], moff[j] + int(p.sizes[j])
            q.marginal[m0:m1] = p.marginal[m0:m1][perm]
    return q


def test_scattered_one_dimensional_rows(ctx):
    """1D supports in a random order per node: a tile's rows spread over the
    whole support, so the one-pass sums keep a separate shift per row instead
    of the per-tile affine one; FP32-core iterates against the oracle and
    against two-pass sums after the same half-sweeps."""
    p = _shuffled(make_chain(n_nodes=8, n=300, eps=1e-3), 5)
    steps = 40
    o = TreeOracle(p)
    o.run_fixed(steps)
    eo = o.evaluate()
    g1, g2 = gpu_problem(ctx, p), gpu_problem(ctx, p)
    assert g1.solve(tol=0.0, max_steps=steps, passes="auto")["steps"] == steps
    assert g2.solve(tol=0.0, max_steps=steps, passes="two")["steps"] == steps
    for g in (g1, g2):
        assert abs(g.evaluate()["dual"] - eo["dual"]) <= 1e-6 * eo["scale"]
        for e in range(p.n_edges):
            assert np.max(np.abs(g.coupling(e) - o.coupling(e))) <= 1e-6


@pytest.mark.parametrize("offset", [300.0, -300.0])
def test_one_pass_far_from_stored_shifts(ctx, offset, monkeypatch):
    """One-pass sums from the first half-sweep (passes="one") on potentials
    moved 300 nats away from those the stored shifts were computed for: every
    row's max lies far above its shift (moved inside the kernel) or far below
    it (the wave falls back to two passes).  Iterates against the oracle run
    from the same potentials, sorted and shuffled 1D supports (general node
    kernel: GMOT_NO_GRID=1)."""
    monkeypatch.setenv("GMOT_NO_GRID", "1")
    for p in (make_chain(n_nodes=8, n=200, eps=1e-2), _shuffled(make_chain(n_nodes=8, n=200, eps=1e-2), 6)):
        g = gpu_problem(ctx, p)
        g.solve(tol=0.0, max_steps=6)
        o = TreeOracle(p)
        o.run_fixed(6)
        lam = o.potentials() + offset
        g.set_potentials(lam)
        o2 = TreeOracle(p)
        o2.Lam = o2.set_potentials(lam)
        steps = 4
        r = g.solve(tol=0.0, max_steps=steps, passes="one", restart=False, verify=False)
        assert r["steps"] == steps
        o2.run_fixed(steps)
        eo = o2.evaluate()
        assert abs(g.evaluate()["dual"] - eo["dual"]) <= 1e-6 * eo["scale"]
        for e in range(p.n_edges):
            assert np.max(np.abs(g.coupling(e) - o2.coupling(e))) <= 1e-6


def test_fused_finalise_stops_where_separate_one_does(ctx):
    """The finalise step carried by the next half-sweep's launch (layer
    schedule) and the separate finalise kernel (per-node schedule, the same
    arithmetic) stop at the same half-sweep with the same potentials and
    stopping sum: the speculative half-sweep after the decision leaves the kept
    state untouched.  Also for a fixed step budget."""
    p = make_chain(n_nodes=10, n=150, eps=5e-3)
    for kw in ({"tol": 1e-6, "max_steps": 100000}, {"tol": 0.0, "max_steps": 37}):
        g1, g2 = gpu_problem(ctx, p), gpu_problem(ctx, p)
        r1 = g1.solve(**kw)
        r2 = g2.solve(schedule="per_node", **kw)
        assert r1["status"] == r2["status"]
        assert r1["steps"] == r2["steps"] and r1["t"] == r2["t"]
        assert r1["err_sum"] == r2["err_sum"]
        assert np.array_equal(g1.potentials(), g2.potentials())


def test_compacted_batch_matches_uncompacted(ctx, monkeypatch):
    """A batch of 96 stars of mixed size and dimension, solved to 1e-6: once
    most instances have stopped the replays run on the work lists of the
    running ones (GMOT_COMPACT_RATIO=0 keeps the full lists); every instance
    ends at the same half-sweep with bit-identical potentials either way, and
    a sample agrees with the oracle's re-measured stopping sum."""
    from paper_2406_10849_amd import Batch
    monkeypatch.setenv("GMOT_NODE_SHAPE", "4,1,1")
    probs = make_batched_stars(count=96, l_lo=2, l_hi=9, n_lo=16, n_hi=400, first_instance=300)
    out = {}
    for ratio in ("0", "2"):
        monkeypatch.setenv("GMOT_COMPACT_RATIO", ratio)
        gps = [gpu_problem(ctx, p) for p in probs]
        b = Batch(ctx, gps)
        rs = b.solve(tol=1e-6, max_steps=20000, check_every=4)
        assert all(r["status"] == "converged" for r in rs)
        out[ratio] = (rs, [g.potentials() for g in gps])
    ts = [r["t"] for r in out["0"][0]]
    assert max(ts) >= 2 * min(ts)  # the batch does thin out
    for i in range(len(probs)):
        assert out["2"][0][i]["t"] == out["0"][0][i]["t"], i
        assert np.array_equal(out["2"][1][i], out["0"][1][i]), i
    for i in (0, 37, 95):
        o = TreeOracle(probs[i])
        assert o.full_error(o.set_potentials(out["2"][1][i]))[0] <= 1e-6 + 1e-10


def test_context_on_a_caller_stream(ctx):
    """A context ordered on a caller's stream (a torch stream) captures its
    graphs on that stream, with the separable group as a parallel branch:
    a batch mixing 1D and 2D-grid stars ends with bit-identical potentials and
    half-sweep counts to those of a context with its own stream."""
    import torch
    from paper_2406_10849_amd import Context, Batch
    probs = make_batched_stars(count=8, l_lo=2, l_hi=6, n_lo=40, n_hi=300, first_instance=500)
    assert {p.dim for p in probs} == {1, 2}
    outs = []
    stream = torch.cuda.Stream()
    for c in (ctx, Context(0, stream=stream)):
        gps = [gpu_problem(c, p) for p in probs]
        rs = Batch(c, gps).solve(tol=1e-6, max_steps=20000, check_every=4)
        assert all(r["status"] == "converged" for r in rs)
        outs.append(([r["t"] for r in rs], [g.potentials() for g in gps]))
    stream.synchronize()
    assert outs[0][0] == outs[1][0]
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b)
