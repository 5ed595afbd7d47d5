"""The oracle's node-sequential (Gauss-Seidel) schedule against results fixed
by other routes (CPU only).

* One edge with both ends constrained: a sweep in the order (0, 1) is one
  row and one column scaling of textbook Sinkhorn started from the column
  scaling nu, so the stopping sum after sweep s is Sinkhorn's marginal
  violation after its (2s)-th half-step (oracle/brute.py, probability domain).
* A star whose centre is node 0: the sweep takes the centre and then the
  leaves, which depend only on the centre, so a sweep is two half-sweeps of
  Algorithm tree_local_reg starting with the centre's class.
* Every node update maximises the dual over that node's potentials (block
  coordinate ascent), so the dual never decreases along the updates.
* At convergence the dual equals a generic L-BFGS maximisation of the dual.
* Planted mistakes (stale messages within a sweep, leaves before the centre)
  are each caught by one of these pins.
"""
import numpy as np
import pytest

from oracle import TreeOracle, brute
from workloads import make_star, make_tree


def _two_node():
    return make_tree([(0, 1)], [7, 9], [1, 1], eps=0.2, instance=71)


def pin_sinkhorn(cls) -> float:
    p = _two_node()
    o = cls(p)
    mu, nu = p.node_marginal(0), p.node_marginal(1)
    C = o.cost(0, 1)
    hist = brute.sinkhorn_violation_history(mu, nu, C, p.eps, 12)
    worst = 0.0
    for s in range(6):
        o.gs_sweep()
        e = o.full_error()[0]
        worst = max(worst, abs(e - hist[2 * s + 1]) / max(hist[2 * s + 1], 1e-300))
    return worst


def pin_star_is_bipartite(cls) -> float:
    p = make_star(n=11, leaves=4, eps=0.15, instance=72)
    gs, bi = cls(p), TreeOracle(p, first_color=0)
    assert bi.S1 == [0]
    worst = 0.0
    for _ in range(5):
        gs.gs_sweep()
        bi.tstep()
        bi.tstep()
        worst = max(worst, float(np.max(np.abs(gs.potentials() - bi.potentials()))))
    return worst


def _tree():
    return make_tree([(0, 1), (1, 2), (1, 3), (3, 4), (3, 5), (0, 6)], [5, 4, 6, 3, 5, 4, 6],
                     [0, 0, 1, 0, 1, 1, 1], eps=0.25, instance=73)


def pin_dual_monotone(cls) -> float:
    """Largest decrease of the dual over single node updates (should be <= rounding)."""
    o = cls(_tree())
    last = o.evaluate()["dual"]
    worst = 0.0
    for _ in range(6):
        for j in o.gs_order():
            o.gs_update(j)
            d = o.evaluate()["dual"]
            worst = max(worst, last - d)
            last = d
    return worst


def pin_dual_lbfgs(cls) -> float:
    p = _tree()
    o = cls(p)
    if o.solve_gauss_seidel(tol=1e-13, max_sweeps=20000)["status"] != "converged":
        return float("inf")
    dstar, _ = brute.dual_lbfgs(p)
    return abs(o.evaluate()["dual"] - dstar) / max(1.0, abs(dstar))


def all_gs_pins(cls) -> dict:
    return {
        "sinkhorn": pin_sinkhorn(cls) < 1e-10,
        "star": pin_star_is_bipartite(cls) < 1e-12,
        "monotone": pin_dual_monotone(cls) < 1e-12,
        "lbfgs": pin_dual_lbfgs(cls) < 1e-9,
    }


def test_sweep_is_textbook_sinkhorn_on_one_edge():
    assert pin_sinkhorn(TreeOracle) < 1e-10


def test_star_sweep_is_two_bipartite_half_sweeps():
    assert pin_star_is_bipartite(TreeOracle) < 1e-12


def test_dual_never_decreases_along_node_updates():
    assert pin_dual_monotone(TreeOracle) < 1e-12


def test_converged_dual_matches_lbfgs():
    assert pin_dual_lbfgs(TreeOracle) < 1e-9


def test_order_is_breadth_first_from_node_0():
    o = TreeOracle(_tree())
    assert o.gs_order() == [0, 1, 6, 2, 3, 4, 5]


def test_stop_test_uses_every_node():
    o = TreeOracle(_tree())
    r = o.solve_gauss_seidel(tol=1e-8, max_sweeps=5000, check_every=3)
    assert r["status"] == "converged" and r["sweeps"] % 3 == 0
    assert r["err_sum"] == pytest.approx(o.full_error()[0], rel=0, abs=0)
    assert r["err_sum"] <= 1e-8


# ---------------------------------------------------------------- mutants
class StaleMessages(TreeOracle):
    """Jacobi within the sweep: every message taken from the sweep's start."""
    def gs_sweep(self):
        start = dict(self.Lam)
        new = {}
        for j in self.gs_order():
            msgs = {k: self.message(k, j, start) for k in self.nbrs[j]}
            logqs = {k: self.log_q(j, k, msgs[k], start) for k in self.nbrs[j]}
            saved = self.Lam
            self.Lam = start
            try:
                new.update(self.update_node_algorithm(j, logqs, msgs))
            finally:
                self.Lam = saved
        self.Lam.update(new)


class LeavesFirst(TreeOracle):
    """Breadth-first order reversed."""
    def gs_order(self):
        return list(reversed(super().gs_order()))


@pytest.mark.parametrize("mut", [StaleMessages, LeavesFirst], ids=lambda c: c.__name__)
def test_gs_mutant_is_caught(mut):
    with np.errstate(all="ignore"):
        try:
            res = all_gs_pins(mut)
        except Exception:
            return
    assert not all(res.values()), f"{mut.__name__} passed every pin: {res}"
