"""The oracle's iterates against the invariants the paper proves.

* unit mass of every plan after each half-sweep (Lemma tree_mass)
* the updated side matches its constraints exactly (Section 3.1, after the
  algorithm)
* free-node constraint sum_k log u_(j,k) = rho_j 1 (eq. tree_dual_mass_consv)
* oscillation of every potential <= 2 C_inf (Lemma tree_dual_varia_bounds)
* sufficient dual increase eps E^2 / (22 |E|) (Lemma f_lower_bound_tree)
* D* - D_t <= 2 C_inf E_t (Lemma f_upper_bound_tree, scaled by eps)
* |P - D| <= C_inf E (duality gap through the same oscillation bound)
* convergence within 2 + 88 |E| C_inf / (delta' eps) half-sweeps (Theorem num_iter)
* Theorem and Algorithm forms of the update agree (Proposition equi)
"""
import numpy as np
import pytest

from oracle import TreeOracle
from workloads import make_tree, make_chain, make_random_tree, make_star

CASES = {
    "star": lambda: make_star(n=24, leaves=4, eps=0.05),
    "tree6": lambda: make_tree([(0, 1), (1, 2), (1, 3), (3, 4), (3, 5)], [5, 7, 6, 8, 5, 6],
                               [1, 0, 1, 0, 1, 1], eps=0.2, instance=11),
    "prufer": lambda: make_random_tree(n_nodes=14, n_lo=5, n_hi=20, eps=0.05, dim=2),
    "chain_split": lambda: make_chain(n_nodes=9, n=30, eps=0.05),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_invariants_along_iterates(name):
    p = CASES[name]()
    ref = TreeOracle(p)
    ref.solve(tol=1e-13, max_steps=50000)
    Dstar = ref.evaluate()["dual"]

    o = TreeOracle(p)
    cinf = o.c_inf()
    nE = p.n_edges
    prev_D = o.evaluate()["dual"]
    for t in range(1, 40):
        S = o.current_side()
        e_S, _, _ = o.tstep(check_equivalence=True)
        ev = o.evaluate()
        # unit mass on every edge after the first update
        assert max(abs(m - 1.0) for m in ev["masses"]) < 1e-12
        # the side just updated is exact
        assert o.side_error(S)[0] < 1e-12
        # free-node constraint: sum_k Lam_(j,k) is constant in x
        assert ev["rho_spread"] < 1e-9 * max(1.0, ev["scale"] / p.eps)
        # oscillation bound on the potentials lambda = eps * Lam
        for key, lam in o.Lam.items():
            assert p.eps * (lam.max() - lam.min()) <= 2 * cinf + 1e-9
        if t >= 2:
            # dual ascent with sufficient increase, driven by the error of the pre-update state
            assert ev["dual"] - prev_D >= p.eps * e_S ** 2 / (22 * nE) - 1e-12
            # suboptimality bounded by the error of the state it was measured on
            assert Dstar - prev_D <= 2 * cinf * e_S + 1e-12
        # duality gap bounded by the full stopping sum
        assert abs(ev["gap"]) <= cinf * ev["err_sum"] + 1e-12
        prev_D = ev["dual"]


@pytest.mark.parametrize("name", sorted(CASES))
def test_iteration_bound(name):
    p = CASES[name]()
    o = TreeOracle(p)
    tol = 1e-6
    r = o.solve(tol=tol, max_steps=100000)
    assert r["status"] == "converged"
    assert r["t"] <= 2 + 88 * p.n_edges * o.c_inf() / (tol * p.eps)


def test_other_side_error_is_zero_after_first_step():
    p = CASES["tree6"]()
    o = TreeOracle(p)
    o.tstep()
    for _ in range(6):
        other = o.S2 if o.current_side() is o.S1 else o.S1
        assert o.side_error(other)[0] < 1e-13
        o.tstep()


def test_check_then_update_returns_passing_state():
    p = CASES["star"]()
    o = TreeOracle(p)
    r = o.solve(tol=1e-8, max_steps=10000)
    assert r["status"] == "converged"
    assert o.full_error()[0] <= 1e-8 + 1e-15
    assert abs(o.full_error()[0] - r["err_sum"]) < 1e-14


def test_first_colour_does_not_change_fixed_point():
    p = CASES["tree6"]()
    a = TreeOracle(p)
    a.solve(tol=1e-13, max_steps=20000)
    b = TreeOracle(p, first_color=1)
    b.solve(tol=1e-13, max_steps=20000)
    for e in range(p.n_edges):
        assert np.max(np.abs(a.coupling(e) - b.coupling(e))) < 1e-10


def test_relabelled_and_reversed_tree_same_solution():
    p = CASES["tree6"]()
    a = TreeOracle(p)
    a.solve(tol=1e-13, max_steps=20000)
    Da = a.evaluate()["dual"]
    # relabel nodes by a permutation and reverse every edge's orientation
    perm = np.array([3, 5, 0, 1, 4, 2])      # new label of old node i
    inv = np.argsort(perm)
    import copy
    q = copy.deepcopy(p)
    q.edges = np.array([[perm[b], perm[a_]] for a_, b in p.edges], dtype=np.int32)
    q.sizes = p.sizes[inv].copy()
    q.is_fixed = p.is_fixed[inv].copy()
    q.support = np.concatenate([p.node_support(int(i)) for i in inv])
    q.marginal = np.concatenate([p.node_marginal(int(i)) for i in inv if p.is_fixed[int(i)]])
    b = TreeOracle(q)
    b.solve(tol=1e-13, max_steps=20000)
    assert abs(b.evaluate()["dual"] - Da) < 1e-11
    for e in range(p.n_edges):
        assert np.max(np.abs(b.coupling(e) - a.coupling(e).T)) < 1e-10


def test_reversed_support_order_reverses_plans():
    p = CASES["tree6"]()
    a = TreeOracle(p)
    a.solve(tol=1e-13, max_steps=20000)
    import copy
    q = copy.deepcopy(p)
    q.support = np.concatenate([p.node_support(j)[::-1] for j in range(p.n_nodes)])
    q.marginal = np.concatenate([p.node_marginal(j)[::-1] for j in range(p.n_nodes) if p.is_fixed[j]])
    b = TreeOracle(q)
    b.solve(tol=1e-13, max_steps=20000)
    for e in range(p.n_edges):
        assert np.max(np.abs(b.coupling(e) - a.coupling(e)[::-1, ::-1])) < 1e-10


@pytest.mark.parametrize("bad", ["cycle", "disconnected", "self_loop", "duplicate", "eps", "marginal", "size"])
def test_invalid_inputs_rejected(bad):
    import copy
    p = make_tree([(0, 1), (1, 2), (2, 3)], [3, 3, 3, 3], [1, 0, 0, 1], eps=0.1)
    q = copy.deepcopy(p)
    if bad == "cycle":
        q.edges = np.array([[0, 1], [1, 2], [2, 0]], dtype=np.int32)
    elif bad == "disconnected":
        q.edges = np.array([[0, 1], [1, 2], [0, 2]], dtype=np.int32)
    elif bad == "self_loop":
        q.edges = np.array([[0, 1], [1, 1], [2, 3]], dtype=np.int32)
    elif bad == "duplicate":
        q.edges = np.array([[0, 1], [1, 0], [2, 3]], dtype=np.int32)
    elif bad == "eps":
        q.eps = 0.0
    elif bad == "marginal":
        q.marginal = q.marginal * 1.01
    elif bad == "size":
        q.sizes = np.array([3, 0, 3, 3], dtype=np.int32)
    with pytest.raises(ValueError):
        TreeOracle(q)
