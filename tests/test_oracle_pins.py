"""The FP64 oracle against textbook algorithms, closed forms and brute force.

None of these re-types the oracle's update: each compares it with a different
published route to the same answer (see ``oracle.brute``)."""
import numpy as np
import pytest

import oracle_pins as P
from oracle import TreeOracle
from oracle.tree_ot import logsumexp


def test_single_edge_both_fixed_is_textbook_sinkhorn():
    assert P.single_edge_both_fixed(TreeOracle) < 1e-11


def test_single_edge_fixed_free_closed_form():
    assert P.single_edge_fixed_free(TreeOracle) < 1e-13


def test_star_matches_iterative_bregman_projections():
    assert P.star_vs_ibp(TreeOracle) < 1e-12


def test_fixed_point_maximises_dual_lbfgs():
    assert P.tiny_tree_dual(TreeOracle) < 1e-9


def test_local_vs_global_regularisation_brute_force():
    r = P.local_vs_global(TreeOracle)
    assert r["identity"] < 1e-12          # entropy factorisation on glued tree-Markov plans
    assert r["transport"] < 1e-12         # <C, glue(B)> = sum_e <C_e, B_e>
    assert r["mass"] < 1e-12
    assert r["sandwich_global"] <= 1e-12  # global optimum below glued local optimum (global objective)
    assert r["sandwich_local"] <= 1e-12   # local optimum below projected global optimum (local objective)
    assert r["distinct"] > 1e-4           # the two regularised problems really differ


def test_unregularised_lp_equivalence_and_small_eps_limit():
    r = P.lp_limit(TreeOracle)
    assert r["lp_gap"] < 1e-7             # coupled OT == MOT on a tree (unregularised)
    assert r["lo"] <= r["T"] <= r["hi"]


def test_unit_mass_after_every_half_sweep():
    assert P.mass_lemma(TreeOracle) < 1e-12


def test_stopping_sum_matches_dense_plans():
    # both classes and the class about to be updated, cold state and six half-sweeps
    assert P.stopping_sum_explicit_plans(TreeOracle) < 1e-12


def test_stopping_sum_node_identities():
    # degree-2 free node: sum_k |q_k - q_bar| = |q_1 - q_2| (arithmetic mean); constrained: |q - mu|
    assert P.stopping_sum_identities(TreeOracle) < 1e-12


def test_stopping_sum_is_textbook_sinkhorn_violation():
    assert P.stopping_sum_sinkhorn(TreeOracle) < 1e-12


def test_zero_mass_marginals():
    assert P.zero_mass(TreeOracle) < 1e-11


def test_logsumexp_special_cases():
    w = np.array([[0.0, -np.inf], [-np.inf, -np.inf], [1000.0, 1000.0]])
    out = logsumexp(w, axis=1)
    assert out[0] == 0.0
    assert out[1] == -np.inf
    assert abs(out[2] - (1000.0 + np.log(2.0))) < 1e-12


def test_c_message_oracle_passes_every_pin():
    """The oracle with its message sums in C (oracle/lse.c) is held to the same
    pins as the numpy one."""
    from oracle.fast import FastTreeOracle
    res = P.all_pins(FastTreeOracle)
    assert all(res.values()), res


def test_c_message_oracle_thread_count_does_not_change_results():
    from oracle.fast import FastTreeOracle
    from workloads import make_random_tree
    p = make_random_tree(n_nodes=14, n_lo=30, n_hi=200, eps=5e-3, dim=2, cfg_id=3, instance=12)
    a, b = FastTreeOracle(p, threads=1), FastTreeOracle(p, threads=4)
    a.run_fixed(6)
    b.run_fixed(6)
    assert np.array_equal(a.potentials(), b.potentials())
