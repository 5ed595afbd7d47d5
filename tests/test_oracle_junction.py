"""The FP64 junction-tree oracle (oracle/junction.py) against results fixed
by other routes (CPU only).

* A tree written as a junction tree (single-variable separators, one clique
  per edge): the separator updates of Proposition general_algo must give the
  tree oracle's iterates (messages and Theorem tree_dual_var there, tensor
  projections and the geometric-mean steps here).
* Wasserstein least squares and random junction trees: the converged dual
  equals a generic L-BFGS maximisation of the dual (eq. whole_dual, here with
  every intersection equal to the separator).
* The unregularised limit: at small eps the transport cost of the converged
  plans lies within the rounding bounds of the full-tensor MOT optimum (HiGHS),
  which equals the coupled-clique optimum on a junction tree.
* Lemma tree_mass carries over: every clique plan has unit mass after every
  class update.
* Planted mistakes in the oracle are each caught by one of these pins.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.sparse import coo_matrix

from oracle import TreeOracle, brute
from oracle.junction import JunctionOracle
from oracle.tree_ot import logsumexp
from workloads import make_tree, make_wls, make_random_junction, as_tree_problem, from_tree_problem


def _mx(*vals):
    v = [float(x) for x in vals]
    return float("inf") if any(np.isnan(x) for x in v) else max(v)


# ---------------------------------------------------------------- pins
def pin_tree_as_junction(cls) -> float:
    tp = make_tree([(0, 1), (1, 2), (1, 3), (3, 4), (3, 5)], [4, 5, 3, 6, 4, 5], [1, 0, 1, 0, 1, 1], eps=0.3,
                   instance=41)
    jo, to = cls(from_tree_problem(tp)), TreeOracle(tp)
    worst = 0.0
    for _ in range(9):
        a = jo.tstep()
        b = to.tstep()
        worst = _mx(worst, abs(a[0] - b[0]), float(np.max(np.abs(jo.potentials() - to.potentials()))))
    return worst


def pin_dual_lbfgs(cls, jp) -> float:
    o = cls(jp)
    o.solve(tol=1e-12, max_steps=50000)
    ev = o.evaluate()
    dstar, _ = brute.dual_lbfgs(as_tree_problem(jp))
    return abs(ev["dual"] - dstar) / max(1.0, abs(dstar))


def lp_full_tensor_junction(jp) -> float:
    """Unregularised MOT over the full tensor of all variables, cost the sum of
    the clique costs, joint marginals of the constrained separators fixed."""
    nv = len(jp.var_sizes)
    shape = tuple(int(n) for n in jp.var_sizes)
    C = np.zeros(shape)
    for c, (a, b) in enumerate(jp.cliques):
        vs = list(jp.separators[a]) + list(jp.separators[b])
        t = np.asarray(jp.clique_cost[c], dtype=np.float64)
        order = np.argsort(vs)
        t = np.transpose(t, order)
        sh = [1] * nv
        for v in vs:
            sh[v] = shape[v]
        C = C + t.reshape(sh)
    idx = np.arange(C.size).reshape(shape)
    rows, cols, rhs = [], [], []
    r = 0
    for s in range(jp.n_separators):
        if not jp.sep_fixed[s]:
            continue
        vs = list(jp.separators[s])
        mu = np.asarray(jp.sep_marginal[s])
        for st in itertools.product(*[range(shape[v]) for v in vs]):
            sl = [slice(None)] * nv
            for v, x in zip(vs, st):
                sl[v] = x
            ids = idx[tuple(sl)].ravel()
            rows += [r] * ids.size
            cols += ids.tolist()
            rhs.append(float(mu[st]))
            r += 1
    A = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(r, C.size)).tocsr()
    res = linprog(C.ravel(), A_eq=A, b_eq=np.array(rhs), bounds=(0, None), method="highs")
    assert res.status == 0, res.message
    return float(res.fun)


def pin_lp_limit(cls) -> dict:
    jp = make_wls(J=2, n=4, eps=0.01, instance=3)
    lp = lp_full_tensor_junction(jp)
    o = cls(jp)
    o.solve(tol=1e-12, max_steps=400000)
    ev = o.evaluate()
    cinf = max(float(np.max(np.abs(c))) for c in jp.clique_cost)
    E = ev["err_sum"]
    states = max(jp.sep_size(s) for s in range(jp.n_separators))
    lo = lp - 2 * cinf * E
    hi = lp + 2 * jp.eps * jp.n_cliques * np.log(states) + 6 * cinf * E
    return {"lp": lp, "T": ev["transport"], "lo": lo, "hi": hi}


def pin_mass(cls) -> float:
    o = cls(make_random_junction(n_seps=6, instance=5))
    worst = 0.0
    for _ in range(7):
        o.tstep()
        worst = _mx(worst, *[abs(m - 1.0) for m in o.evaluate()["masses"]])
    return worst


def all_junction_pins(cls) -> dict:
    lp = pin_lp_limit(cls)
    return {
        "tree_as_junction": pin_tree_as_junction(cls) < 1e-11,
        "wls_dual": pin_dual_lbfgs(cls, make_wls(J=3, n=4, eps=0.2, instance=1)) < 1e-9,
        "random_dual": pin_dual_lbfgs(cls, make_random_junction(n_seps=5, instance=2)) < 1e-9,
        "lp_limit": lp["lo"] <= lp["T"] <= lp["hi"],
        "mass": pin_mass(cls) < 1e-12,
    }


# ---------------------------------------------------------------- tests
def test_tree_as_junction_gives_tree_iterates():
    assert pin_tree_as_junction(JunctionOracle) < 1e-11


@pytest.mark.parametrize("jp", [make_wls(J=3, n=4, eps=0.2, instance=1), make_wls(J=4, n=3, eps=0.1, instance=4),
                                make_random_junction(n_seps=5, instance=2),
                                make_random_junction(n_seps=6, max_vars=3, instance=6)],
                         ids=["wls-J3", "wls-J4", "random-5", "random-6"])
def test_converged_dual_matches_lbfgs(jp):
    assert pin_dual_lbfgs(JunctionOracle, jp) < 1e-9


def test_unregularised_limit_within_rounding_bounds():
    r = pin_lp_limit(JunctionOracle)
    assert r["lo"] <= r["T"] <= r["hi"], r


def test_unit_mass_after_every_update():
    assert pin_mass(JunctionOracle) < 1e-12


def test_converged_plans_are_consistent():
    """At convergence neighbouring plans agree on their separator, constrained
    separators carry their marginal, free separators unit mass."""
    jp = make_random_junction(n_seps=6, max_vars=2, instance=8)
    o = JunctionOracle(jp)
    assert o.solve(tol=1e-13, max_steps=100000)["status"] == "converged"
    for s in range(jp.n_separators):
        ps = [np.exp(o.log_proj(c, s)) for c in o.nbr[s]]
        for q in ps[1:]:
            assert np.max(np.abs(q - ps[0])) < 1e-12
        if jp.sep_fixed[s]:
            assert np.max(np.abs(ps[0] - jp.sep_marginal[s])) < 1e-12
        else:
            assert abs(ps[0].sum() - 1.0) < 1e-12


# ---------------------------------------------------------------- mutants
class WrongRecursionExponent(JunctionOracle):
    """q_i = (q_{i-1}^(i-1) * k_i)^(1/(i-1)) instead of ^(1/i)."""
    def update_separator(self, s, lu=None):
        lu = self.lu if lu is None else lu
        cs = self.nbr[s]
        if len(cs) < 3:
            return super().update_separator(s, lu)
        lk = [self.log_m[s] + self.log_kbar(c, s, lu) for c in cs]
        lq = 0.5 * (lk[0] + lk[1])
        for i in range(3, len(cs) + 1):
            lq = ((i - 1) * lq + lk[i - 1]) / (i - 1)
        lnorm = self.log_m[s] - lq if self.prob.sep_fixed[s] else -float(logsumexp(lq.reshape(-1), axis=0))
        return {(s, c): np.broadcast_to(lnorm + lq - lk[i], self.prob.sep_shape(s)).copy() for i, c in enumerate(cs)}


class NoReferenceInK(JunctionOracle):
    """The other separator's reference m left out of k."""
    def log_kbar(self, c, s, lu=None):
        lu = self.lu if lu is None else lu
        o, first = self._sides(c, s)
        saved = self.log_m[o]
        self.log_m[o] = np.zeros_like(saved)
        try:
            return super().log_kbar(c, s, lu)
        finally:
            self.log_m[o] = saved


class FreeNotNormalised(JunctionOracle):
    """Free separators skip v_{ell+1} (no unit-mass scaling)."""
    def update_separator(self, s, lu=None):
        new = super().update_separator(s, lu)
        if self.prob.sep_fixed[s]:
            return new
        return {k: v + 0.3 for k, v in new.items()}


class ArithmeticQ(JunctionOracle):
    """q_ell as the arithmetic mean of the k_i."""
    def update_separator(self, s, lu=None):
        lu = self.lu if lu is None else lu
        cs = self.nbr[s]
        if len(cs) < 2:
            return super().update_separator(s, lu)
        lk = [self.log_m[s] + self.log_kbar(c, s, lu) for c in cs]
        with np.errstate(divide="ignore"):
            lq = np.log(sum(np.exp(x) for x in lk) / len(lk))
        lnorm = self.log_m[s] - lq if self.prob.sep_fixed[s] else -float(logsumexp(lq.reshape(-1), axis=0))
        return {(s, c): np.broadcast_to(lnorm + lq - lk[i], self.prob.sep_shape(s)).copy() for i, c in enumerate(cs)}


MUTANTS = [WrongRecursionExponent, NoReferenceInK, FreeNotNormalised, ArithmeticQ]


def test_real_junction_oracle_passes_every_pin():
    res = all_junction_pins(JunctionOracle)
    assert all(res.values()), res


@pytest.mark.parametrize("mut", MUTANTS, ids=lambda c: c.__name__)
def test_junction_mutant_is_caught(mut):
    with np.errstate(all="ignore"):
        try:
            res = all_junction_pins(mut)
        except Exception:
            return
    assert not all(res.values()), f"{mut.__name__} passed every pin: {res}"
