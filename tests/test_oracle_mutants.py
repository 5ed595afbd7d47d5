"""Planted mistakes in the oracle (CPU only) must be caught by the pins.

Each mutant is a subclass of the oracle with one plausible error: a dropped
term, a wrong sign, a transposed operand, a wrong mean, a missing
normalisation, a mis-scaled or incomplete stopping sum, or a missing
zero-mass limit.  At least one pin has to fail for every mutant."""
import numpy as np
import pytest

import oracle_pins as P
from oracle import TreeOracle
from oracle.tree_ot import logsumexp


class DropGamma(TreeOracle):
    def message(self, k, j, Lam=None):
        Lam = self.Lam if Lam is None else Lam
        w = Lam[(k, j)][None, :] - self.cost(j, k) / self.eps
        return logsumexp(w, axis=1)


class CostSign(TreeOracle):
    def message(self, k, j, Lam=None):
        Lam = self.Lam if Lam is None else Lam
        w = (Lam[(k, j)] + self.log_gamma[k])[None, :] + self.cost(j, k) / self.eps
        return logsumexp(w, axis=1)


class TransposedCost(TreeOracle):
    """Reads C_(k,j) where C_(j,k) belongs (only possible on square edges)."""
    def message(self, k, j, Lam=None):
        Lam = self.Lam if Lam is None else Lam
        C = self.cost(j, k)
        if C.shape[0] == C.shape[1]:
            C = self.cost(k, j)
        w = (Lam[(k, j)] + self.log_gamma[k])[None, :] - C / self.eps
        return logsumexp(w, axis=1)


class ArithmeticMeanUpdate(TreeOracle):
    def update_node_algorithm(self, j, logqs, msgs=None):
        if self.prob.is_fixed[j]:
            return super().update_node_algorithm(j, logqs, msgs)
        qj = np.mean(np.stack([np.exp(logqs[k]) for k in self.nbrs[j]]), axis=0)
        lqh = np.log(qj / qj.sum())
        return {(j, k): self.Lam[(j, k)] + lqh - logqs[k] for k in self.nbrs[j]}


class NoNormalisation(TreeOracle):
    def update_node_algorithm(self, j, logqs, msgs=None):
        if self.prob.is_fixed[j]:
            return super().update_node_algorithm(j, logqs, msgs)
        lqj = np.mean(np.stack([logqs[k] for k in self.nbrs[j]]), axis=0)
        return {(j, k): self.Lam[(j, k)] + lqj - logqs[k] for k in self.nbrs[j]}


class FixedSign(TreeOracle):
    def update_node_algorithm(self, j, logqs, msgs=None):
        if not self.prob.is_fixed[j]:
            return super().update_node_algorithm(j, logqs, msgs)
        return {(j, k): self.Lam[(j, k)] - self.log_gamma[j] + logqs[k] for k in self.nbrs[j]}


class WrongNeighbourPotential(TreeOracle):
    """Uses the target's own potential instead of the neighbour's in the message."""
    def message(self, k, j, Lam=None):
        Lam = self.Lam if Lam is None else Lam
        src = Lam[(k, j)]
        alt = Lam[(j, k)]
        v = alt if alt.shape == src.shape else src[::-1]
        w = (v + self.log_gamma[k])[None, :] - self.cost(j, k) / self.eps
        return logsumexp(w, axis=1)


# ---- mistakes in the stopping sum (Algorithm tree_local_reg while-condition) ----

class GeometricMeanError(TreeOracle):
    """q_bar_j as the normalised geometric mean instead of the arithmetic mean."""
    def node_error(self, j, logqs):
        if self.prob.is_fixed[j]:
            return super().node_error(j, logqs)
        lq = np.stack([logqs[k] for k in self.nbrs[j]])
        g = lq.mean(axis=0)
        qbar = np.exp(g - logsumexp(g, axis=0))
        terms = [float(np.sum(np.abs(np.exp(lq[i]) - qbar))) for i in range(lq.shape[0])]
        return float(sum(terms)), float(max(terms))


class HalfError(TreeOracle):
    def node_error(self, j, logqs):
        s, m = super().node_error(j, logqs)
        return 0.5 * s, 0.5 * m


class DoubleError(TreeOracle):
    def node_error(self, j, logqs):
        s, m = super().node_error(j, logqs)
        return 2.0 * s, 2.0 * m


class DropFixedTerm(TreeOracle):
    """Constrained nodes left out of the stopping sum."""
    def node_error(self, j, logqs):
        if self.prob.is_fixed[j]:
            return 0.0, 0.0
        return super().node_error(j, logqs)


class NoZeroMassLimit(TreeOracle):
    """Constrained update as Lam + log mu - log q everywhere (NaN where mu = 0)."""
    def update_node_algorithm(self, j, logqs, msgs=None):
        if not self.prob.is_fixed[j]:
            return super().update_node_algorithm(j, logqs, msgs)
        with np.errstate(invalid="ignore"):
            return {(j, k): self.Lam[(j, k)] + self.log_gamma[j] - logqs[k] for k in self.nbrs[j]}


MUTANTS = [DropGamma, CostSign, TransposedCost, ArithmeticMeanUpdate, NoNormalisation, FixedSign,
           WrongNeighbourPotential, GeometricMeanError, HalfError, DoubleError, DropFixedTerm, NoZeroMassLimit]


def test_real_oracle_passes_every_pin():
    res = P.all_pins(TreeOracle)
    assert all(res.values()), res


@pytest.mark.parametrize("mut", MUTANTS, ids=lambda c: c.__name__)
def test_mutant_is_caught(mut):
    with np.errstate(all="ignore"):
        try:
            res = P.all_pins(mut)
        except Exception:
            return   # crashing is also being caught
    assert not all(res.values()), f"{mut.__name__} passed every pin: {res}"
