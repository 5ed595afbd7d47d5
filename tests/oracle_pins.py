"""Pins of the FP64 oracle against results fixed by textbook algorithms and
closed forms (helper module; each pin returns an error measure).

Every pin runs a given oracle class, so the same pins can be aimed at a copy of
the oracle with a planted mistake to show that they catch it.
"""
from __future__ import annotations

import numpy as np

from oracle import brute
from workloads import make_tree


def _mx(*vals) -> float:
    """max() that reports a NaN as an infinite error (Python's max skips it)."""
    v = [float(x) for x in vals]
    return float("inf") if any(np.isnan(x) for x in v) else max(v)


def single_edge_both_fixed(cls) -> float:
    """Both ends constrained: the method reduces to entropic Sinkhorn (the
    marginal-product reference only shifts the objective by a constant)."""
    p = make_tree([(0, 1)], [7, 9], [1, 1], eps=0.3, instance=1)
    o = cls(p)
    o.solve(tol=1e-14, max_steps=4000)
    B = o.coupling(0)
    Bt = brute.sinkhorn_textbook(p.node_marginal(0), p.node_marginal(1), o.cost(0, 1), p.eps, iters=4000)
    return float(np.max(np.abs(B - Bt)))


def single_edge_fixed_free(cls) -> float:
    """Fixed node 0, free leaf 1: B(x, y) = mu(x) K(x, y) / sum_y K(x, y), and
    D = P = -eps sum_x mu(x) log sum_y K(x, y) - eps, reached after one half-sweep
    when the fixed node goes first and stays there."""
    p = make_tree([(0, 1)], [6, 8], [1, 0], eps=0.25, instance=2)
    o = cls(p)
    mu = p.node_marginal(0)
    C = brute._edge_cost(p, 0)
    K = np.exp(-C / p.eps)
    Bc = mu[:, None] * K / K.sum(axis=1, keepdims=True)
    Dc = -p.eps * float(mu @ np.log(K.sum(axis=1))) - p.eps
    Tc = float(np.sum(C * Bc))
    err = 0.0
    for _ in range(3):
        o.tstep()
        ev = o.evaluate()
        err = _mx(err, float(np.max(np.abs(o.coupling(0) - Bc))), abs(ev["dual"] - Dc), abs(ev["primal"] - Dc),
                  abs(ev["transport"] - Tc))
    return err


def star_vs_ibp(cls) -> float:
    """Star with leaves updated first: after every leaf half-sweep the plans
    equal those of equal-weight iterative Bregman projections."""
    p = make_tree([(0, 1), (0, 2), (0, 3)], [8, 6, 7, 9], [0, 1, 1, 1], eps=0.2, instance=3)
    o = cls(p, first_color=1)
    mus = [p.node_marginal(l) for l in (1, 2, 3)]
    Cs = [brute._edge_cost(p, e) for e in range(3)]
    ref = brute.ibp_barycenter(mus, Cs, p.eps, rounds=5)
    err = 0.0
    for r in range(5):
        o.tstep()   # leaves
        for e in range(3):
            err = _mx(err, float(np.max(np.abs(o.coupling(e) - ref[r][e]))))
        o.tstep()   # center
    return err


def tiny_tree_dual(cls) -> float:
    """Fixed point of the iteration maximises the dual: compare with a generic
    L-BFGS maximisation on a 6-node tree with free nodes of degree 3 and 2."""
    p = make_tree([(0, 1), (1, 2), (1, 3), (3, 4), (3, 5)], [3, 4, 5, 4, 3, 5], [1, 0, 1, 0, 1, 1],
                  eps=0.5, instance=4)
    o = cls(p)
    o.solve(tol=1e-13, max_steps=20000)
    ev = o.evaluate()
    Dstar, _ = brute.dual_lbfgs(p)
    return abs(ev["dual"] - Dstar) / ev["scale"]


def local_vs_global(cls) -> dict:
    """Brute-force full-tensor comparisons on a tiny tree (n <= 4 per node)."""
    p = make_tree([(0, 1), (1, 2), (1, 3), (3, 4)], [3, 4, 3, 4, 3], [1, 0, 1, 0, 1], eps=0.4, instance=5)
    o = cls(p)
    o.solve(tol=1e-14, max_steps=20000)
    plans = [o.coupling(e) for e in range(p.n_edges)]
    Bl = brute.glue(plans, p)
    Cfull = brute.full_cost_tensor(p)
    Pl = brute.local_objective(plans, p)
    Pg_glue = brute.global_objective(Bl, p)
    # entropy identity for tree-Markov joints
    deg = np.zeros(p.n_nodes, dtype=int)
    for a, b in p.edges:
        deg[a] += 1
        deg[b] += 1
    corr = 0.0
    for j in range(p.n_nodes):
        if not p.is_fixed[j]:
            q = brute._proj(Bl, j)
            corr += (deg[j] - 1) * float(q @ np.log(q))
    ident = abs(Pl - (Pg_glue + p.eps * (corr - (p.n_edges - 1))))
    transport = abs(float(np.sum(Cfull * Bl)) - sum(float(np.sum(brute._edge_cost(p, e) * plans[e]))
                                                     for e in range(p.n_edges)))
    Bg = brute.full_tensor_mot(p, iters=3000)
    Pg_star = brute.global_objective(Bg, p)
    proj = [brute.pairwise_marginal(Bg, int(a), int(b)) for a, b in p.edges]
    Pl_proj = brute.local_objective(proj, p)
    return {"identity": ident, "transport": transport, "mass": abs(float(Bl.sum()) - 1.0),
            "sandwich_global": Pg_star - Pg_glue, "sandwich_local": Pl - Pl_proj,
            "distinct": abs(Pg_star - Pg_glue)}


def lp_limit(cls) -> dict:
    """Unregularised optimum: coupled-edge LP equals full-tensor LP on a tree;
    the oracle's transport cost at small eps lies inside the rounding bounds of
    Lemmas round and round_applied."""
    p = make_tree([(0, 1), (1, 2), (1, 3)], [5, 4, 5, 4], [1, 0, 1, 1], eps=0.01, instance=6, support="grid",
                  marginals="gm")
    lp_c = brute.lp_coupled(p)
    lp_f = brute.lp_full_tensor(p)
    o = cls(p)
    o.solve(tol=1e-12, max_steps=200000)
    ev = o.evaluate()
    cinf = o.c_inf()
    E = ev["err_sum"]
    d = int(max(p.sizes))
    lo = lp_c - 2 * cinf * E
    hi = lp_c + 2 * p.eps * p.n_edges * np.log(d) + 6 * cinf * E
    return {"lp_gap": abs(lp_c - lp_f), "T": ev["transport"], "lo": lo, "hi": hi}


def mass_lemma(cls) -> float:
    """Lemma tree_mass: every plan has unit mass after every half-sweep."""
    p = make_tree([(0, 1), (1, 2), (1, 3), (3, 4), (3, 5)], [5, 7, 6, 8, 5, 6], [1, 0, 1, 0, 1, 1],
                  eps=0.2, instance=11)
    o = cls(p)
    worst = 0.0
    for _ in range(8):
        o.tstep()
        worst = _mx(worst, *[abs(float(o.coupling(e).sum()) - 1.0) for e in range(p.n_edges)])
    return worst


# ---- the stopping sum (Algorithm tree_local_reg while-condition; q_bar_j of
# Lemma f_upper_bound_tree) ------------------------------------------------------

def _split_tree():
    """7 nodes: free node 1 of degree 3, free node 4 of degree 2, constrained
    interior node 3 of degree 3 (read as three constrained leaves), constrained
    leaves 0, 2, 5, 6; random supports so no symmetry hides a term."""
    return make_tree([(0, 1), (1, 2), (1, 3), (3, 4), (3, 5), (4, 6)], [4, 5, 3, 6, 4, 5, 3],
                     [1, 0, 1, 1, 0, 1, 1], eps=0.3, instance=21)


def stopping_sum_explicit_plans(cls) -> float:
    """The oracle's stopping sum (both classes, and the class about to be
    updated as returned by a half-sweep) against the same sum read off dense
    plan matrices built from u = exp(Lam) (no messages, no log-sum-exp), at the
    cold state and after each of six half-sweeps."""
    p = _split_tree()
    o = cls(p)
    worst = 0.0
    for _ in range(7):
        plans = brute.plans_from_scalings(p, o.potentials())
        eb, mb = brute.stopping_sum_from_plans(p, plans)
        eo, mo = o.full_error()
        S = list(o.current_side())
        es_b, _ = brute.stopping_sum_from_plans(p, plans, nodes=S)
        es_o, _, _ = o.tstep()
        worst = _mx(worst, abs(eo - eb), abs(mo - mb), abs(es_o - es_b))
    return worst


def stopping_sum_identities(cls) -> float:
    """Node shares of the stopping sum from plan marginals given directly:
    a free node of degree 2 has sum_k ||q_k - q_bar||_1 = ||q_1 - q_2||_1
    exactly when q_bar is the arithmetic mean; a constrained node's share is
    sum_k ||q_k - mu||_1.  The marginals come from the dense plans, not from the
    oracle's messages."""
    p = make_tree([(0, 1), (1, 2), (2, 3)], [5, 6, 4, 5], [1, 0, 0, 1], eps=0.4, instance=22)
    o = cls(p)
    worst = 0.0
    for _ in range(5):
        marg = brute.plan_marginals(p, brute.plans_from_scalings(p, o.potentials()))
        for j in (1, 2):       # free, degree 2
            q = {k: np.log(v) for k, v in marg[j].items()}
            s, _ = o.node_error(j, q)
            k1, k2 = sorted(marg[j])
            worst = _mx(worst, abs(s - float(np.abs(marg[j][k1] - marg[j][k2]).sum())))
        for j in (0, 3):       # constrained
            q = {k: np.log(v) for k, v in marg[j].items()}
            s, _ = o.node_error(j, q)
            ref = sum(float(np.abs(v - p.node_marginal(j)).sum()) for v in marg[j].values())
            worst = _mx(worst, abs(s - ref))
        o.tstep()
    return worst


def stopping_sum_sinkhorn(cls) -> float:
    """Both ends constrained: the stopping sum checked before half-sweep t >= 2
    is the violation of the marginal that the previous half-sweep did not fit,
    which textbook Sinkhorn iterates (row scaling first) give directly."""
    p = make_tree([(0, 1)], [6, 8], [1, 1], eps=0.35, instance=23)
    o = cls(p)
    sums = [o.tstep()[0] for _ in range(12)]
    ref = brute.sinkhorn_violation_history(p.node_marginal(0), p.node_marginal(1), brute._edge_cost(p, 0), p.eps, 11)
    return _mx(*[abs(a - b) for a, b in zip(sums[1:], ref)])


def _with_zeros(p, node, idx):
    """Copy of p whose marginal of `node` has the entries idx set to 0 (renormalised)."""
    import copy
    q = copy.deepcopy(p)
    off = int(q.marginal_offsets()[node])
    n = int(q.sizes[node])
    mu = q.marginal[off:off + n].copy()
    mu[list(idx)] = 0.0
    q.marginal = q.marginal.copy()
    q.marginal[off:off + n] = mu / mu.sum()
    return q


def zero_mass(cls) -> float:
    """Given marginals with zero entries (log 0 = -inf in the log domain).
    (a) Constrained node 0, free leaf 1: the closed form B = mu(x) K / sum_y K
    with zero rows, D = P = -eps sum_{mu > 0} mu log sum_y K - eps, and a zero
    stopping sum, after every half-sweep (constrained node first).
    (b) Both ends constrained, zeros on both sides: textbook Sinkhorn plans and
    violation history (row scaling first)."""
    p = _with_zeros(make_tree([(0, 1)], [7, 6], [1, 0], eps=0.3, instance=24), 0, [1, 4])
    o = cls(p)
    mu = p.node_marginal(0)
    C = brute._edge_cost(p, 0)
    K = np.exp(-C / p.eps)
    Bc = mu[:, None] * K / K.sum(axis=1, keepdims=True)
    pos = mu > 0
    Dc = -p.eps * float(mu[pos] @ np.log(K.sum(axis=1)[pos])) - p.eps
    err = 0.0
    for _ in range(3):
        o.tstep()
        ev = o.evaluate()
        err = _mx(err, float(np.max(np.abs(o.coupling(0) - Bc))), abs(ev["dual"] - Dc), abs(ev["primal"] - Dc),
                  ev["err_sum"])
    q = _with_zeros(_with_zeros(make_tree([(0, 1)], [6, 7], [1, 1], eps=0.35, instance=25), 0, [2]), 1, [0, 5])
    o = cls(q)
    sums = [o.tstep()[0] for _ in range(12)]
    mu0, mu1, C = q.node_marginal(0), q.node_marginal(1), brute._edge_cost(q, 0)
    ref = brute.sinkhorn_violation_history(mu0, mu1, C, q.eps, 11)
    err = _mx(err, *[abs(a - b) for a, b in zip(sums[1:], ref)])
    o.solve(tol=1e-14, max_steps=4000)
    Bt = brute.sinkhorn_textbook(mu0, mu1, C, q.eps, iters=4000)
    return _mx(err, float(np.max(np.abs(o.coupling(0) - Bt))))


def all_pins(cls) -> dict:
    lg = local_vs_global(cls)
    lp = lp_limit(cls)
    return {
        "stopping_sum_explicit_plans": stopping_sum_explicit_plans(cls) < 1e-12,
        "stopping_sum_identities": stopping_sum_identities(cls) < 1e-12,
        "stopping_sum_sinkhorn": stopping_sum_sinkhorn(cls) < 1e-12,
        "zero_mass": zero_mass(cls) < 1e-11,
        "single_edge_both_fixed": single_edge_both_fixed(cls) < 1e-11,
        "single_edge_fixed_free": single_edge_fixed_free(cls) < 1e-13,
        "star_vs_ibp": star_vs_ibp(cls) < 1e-12,
        "tiny_tree_dual": tiny_tree_dual(cls) < 1e-9,
        "local_vs_global": (lg["identity"] < 1e-12 and lg["sandwich_global"] <= 1e-12
                            and lg["sandwich_local"] <= 1e-12),
        "lp_limit": lp["lo"] <= lp["T"] <= lp["hi"],
        "mass_lemma": mass_lemma(cls) < 1e-12,
    }
