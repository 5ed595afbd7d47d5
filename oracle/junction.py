"""FP64 CPU oracle for coupled MOT on a modified junction tree (test infrastructure).

Only the test suite, the smoke entry point and the benchmark's CPU-baseline leg
may import this module; the product library never does.  It shares no code
with the HIP path.

What it computes (Section 4 of the paper, "Generalized algorithm with local
regularization to general graphs"):

* Problem eq. ot_graph_local_reg on a modified junction tree (Definition
  jt_general): one plan tensor B_c per cost clique c, locally regularised with
  reference M_c = m_a (x) m_b over its two neighbouring separators a, b
  (m_s = the given marginal on constrained separators, ones elsewhere);
  neighbouring plans agree on their separator, constrained separators carry
  their marginal, free separators unit mass.
* Plans B_c = K_c * M_c * (u^a_c (x) 1) * (u^b_c (x) 1), K_c = exp(-C_c / eps)
  (Proposition local_reg_dual): every separator s holds one dual tensor
  u^s_i per neighbouring clique.
* Iteration: the separators, split into the two classes of the bipartite
  separator--clique tree, are updated class by class (the parallel update of
  Section 4.2); a separator's update solves its sub-dual problem eq. sub_dual
  by the steps of Proposition general_algo (geometric-mean tensors q_i,
  intermediate a_i and v_i, then u_i), or by u_1 = mu ./ k_1 when it has one
  neighbour.

Scope: each clique's variables are the disjoint union of its two separators'
variables, so every intersection of a separator with a neighbouring clique is
the separator itself (the inclusion sequence of Assumption inclusion is a
chain of equal sets and every projection P_{c cap c_i} is the identity); a
constraint, when present, fixes the joint marginal of all of a separator's
variables (gamma = the separator).  A free separator's constraint is unit
mass: v_{l+1} = exp(rho) is a scalar, mu_gamma = 1 and P_gamma sums every
entry (the special case the paper names after eq. sub_dual).

Everything is kept in the log domain: ``lu[(s, i)] = log u^s_i``.

Readings (listed in the design notes): one iteration = one class update;
the class of separator 0 (BFS over the separator--clique tree) goes first;
the stopping sum is that of Algorithm tree_local_reg with separators in place
of nodes -- for a constrained separator sum_i ||P_s(B_{c_i}) - mu_s||_1, for a
free one sum_i ||P_s(B_{c_i}) - mean_i P_s(B_{c_i})||_1.
"""
from __future__ import annotations

from collections import deque
from typing import Dict, List, Optional, Tuple

import numpy as np

from .tree_ot import logsumexp


def _lse_all(w: np.ndarray) -> float:
    """log of the sum of exp over every entry (-inf for an all -inf tensor)."""
    return float(logsumexp(w.reshape(-1), axis=0))


def validate_junction(prob) -> None:
    S = prob.n_separators
    if S < 1:
        raise ValueError("no separators")
    if prob.n_cliques != S - 1:
        raise ValueError("the separator--clique graph must be a tree (cliques = separators - 1)")
    seen_vars = set()
    for s, vs in enumerate(prob.separators):
        for v in vs:
            if v in seen_vars:
                raise ValueError("a variable may belong to one separator only (disjoint cliques)")
            seen_vars.add(v)
    adj = [[] for _ in range(S)]
    for c, (a, b) in enumerate(prob.cliques):
        if a == b or not (0 <= a < S and 0 <= b < S):
            raise ValueError("bad clique")
        adj[a].append(b)
        adj[b].append(a)
        want = prob.sep_shape(a) + prob.sep_shape(b)
        if tuple(np.shape(prob.clique_cost[c])) != want:
            raise ValueError(f"cost tensor of clique {c} must have shape {want}")
    reached, dq = {0}, deque([0])
    while dq:
        x = dq.popleft()
        for y in adj[x]:
            if y not in reached:
                reached.add(y)
                dq.append(y)
    if len(reached) != S:
        raise ValueError("separator--clique graph is not connected")
    for s in range(S):
        if prob.sep_fixed[s]:
            mu = np.asarray(prob.sep_marginal[s])
            if mu.shape != prob.sep_shape(s) or np.any(mu < 0) or abs(mu.sum() - 1.0) > 1e-9:
                raise ValueError(f"marginal of separator {s} must be a probability tensor of its shape")


class JunctionOracle:
    """Class-by-class separator updates of Proposition general_algo, FP64."""

    def __init__(self, prob, first_color: Optional[int] = None):
        validate_junction(prob)
        self.prob = prob
        self.eps = float(prob.eps)
        S = prob.n_separators
        # neighbouring cliques of each separator, in ascending clique order
        self.nbr: List[List[int]] = [[] for _ in range(S)]
        for c, (a, b) in enumerate(prob.cliques):
            self.nbr[a].append(c)
            self.nbr[b].append(c)
        colour = [-1] * S
        colour[0] = 0
        dq = deque([0])
        while dq:
            x = dq.popleft()
            for c in self.nbr[x]:
                a, b = prob.cliques[c]
                y = b if a == x else a
                if colour[y] < 0:
                    colour[y] = 1 - colour[x]
                    dq.append(y)
        fc = 0 if first_color is None else int(first_color)
        self.S1 = [s for s in range(S) if colour[s] == fc]
        self.S2 = [s for s in range(S) if colour[s] != fc]
        # log m_s: the given marginal on constrained separators, 0 elsewhere
        self.log_m: List[np.ndarray] = []
        for s in range(S):
            if prob.sep_fixed[s]:
                with np.errstate(divide="ignore"):
                    self.log_m.append(np.log(np.asarray(prob.sep_marginal[s], dtype=np.float64)))
            else:
                self.log_m.append(np.zeros(prob.sep_shape(s)))
        # u = 1 for every (separator, neighbouring clique)
        self.lu: Dict[Tuple[int, int], np.ndarray] = {(s, c): np.zeros(prob.sep_shape(s))
                                                       for s in range(S) for c in self.nbr[s]}
        self.t = 1

    # ------------------------------------------------------------ plans
    def _sides(self, c: int, s: int) -> Tuple[int, bool]:
        """The other separator of clique c seen from s, and whether s comes first."""
        a, b = self.prob.cliques[c]
        return (b, True) if a == s else (a, False)

    def log_plan(self, c: int, lu=None) -> np.ndarray:
        """log B_c = -C_c/eps + log m_a + log m_b + log u^a_c + log u^b_c, axes
        (variables of a) then (variables of b) (Proposition local_reg_dual)."""
        lu = self.lu if lu is None else lu
        a, b = self.prob.cliques[c]
        na, nb = len(self.prob.sep_shape(a)), len(self.prob.sep_shape(b))
        la = (self.log_m[a] + lu[(a, c)]).reshape(self.prob.sep_shape(a) + (1,) * nb)
        lb = (self.log_m[b] + lu[(b, c)]).reshape((1,) * na + self.prob.sep_shape(b))
        return -np.asarray(self.prob.clique_cost[c], dtype=np.float64) / self.eps + la + lb

    def plan(self, c: int, lu=None) -> np.ndarray:
        return np.exp(self.log_plan(c, lu))

    def log_proj(self, c: int, s: int, lu=None) -> np.ndarray:
        """log P_s(B_c): the plan summed over the other separator's variables."""
        lB = self.log_plan(c, lu)
        _, first = self._sides(c, s)
        ns = len(self.prob.sep_shape(s))
        axes = tuple(range(ns, lB.ndim)) if first else tuple(range(0, lB.ndim - ns))
        out = lB
        for ax in sorted(axes, reverse=True):
            out = logsumexp(out, axis=ax)
        return out

    def log_kbar(self, c: int, s: int, lu=None) -> np.ndarray:
        """log P_s(K_c * m_other * (u-bar (x) 1)): clique c projected onto
        separator s with the separator's own dual and reference left out."""
        lu = self.lu if lu is None else lu
        a, b = self.prob.cliques[c]
        o, first = self._sides(c, s)
        ns, no = len(self.prob.sep_shape(s)), len(self.prob.sep_shape(o))
        lo = self.log_m[o] + lu[(o, c)]
        lo = lo.reshape((1,) * ns + self.prob.sep_shape(o)) if first else lo.reshape(self.prob.sep_shape(o) + (1,) * ns)
        w = -np.asarray(self.prob.clique_cost[c], dtype=np.float64) / self.eps + lo
        axes = tuple(range(ns, ns + no)) if first else tuple(range(0, no))
        for ax in sorted(axes, reverse=True):
            w = logsumexp(w, axis=ax)
        return w

    # --------------------------------------------------------- the update
    def update_separator(self, s: int, lu=None) -> Dict[Tuple[int, int], np.ndarray]:
        """New log u^s_i for every neighbouring clique of separator s, from the
        sub-dual problem eq. sub_dual by the steps of Proposition general_algo
        (ell = 1: u_1 = v_2 = mu_gamma ./ k_1).  Here k_i = P_s(K * M * (u-bar (x) 1))
        carries the separator's own reference m_s, so that ||B_{c_i}||_1 =
        <k_i, u_i>.  All intersections equal the separator: every projection
        P_{s cap c_i} is the identity, and P_gamma is the identity (constrained)
        or the total sum (free: v_{ell+1} = exp(rho) is a scalar, mu_gamma = 1).
        Where a given marginal is 0, log k = -inf and the steps give -inf - (-inf);
        there u takes its limit 1 ./ (k_i ./ mu), from the projection without m_s."""
        lu = self.lu if lu is None else lu
        cs = self.nbr[s]
        ell = len(cs)
        fixed = bool(self.prob.sep_fixed[s])
        lkbar = [self.log_kbar(c, s, lu) for c in cs]
        lk = [self.log_m[s] + x for x in lkbar]           # log k_1 .. log k_ell

        def log_mu_over(lq):
            """log(mu_gamma ./ P_gamma(q))"""
            if fixed:
                with np.errstate(invalid="ignore"):
                    return self.log_m[s] - lq
            return np.asarray(-_lse_all(lq))

        new = {}
        with np.errstate(invalid="ignore"):
            if ell == 1:
                lu_new = [log_mu_over(lk[0]) + 0.0 * lk[0]]
            else:
                # step 1: geometric means from the largest intersection to the smallest
                lq = {2: 0.5 * (lk[0] + lk[1])}                      # q_2 = (k_1 * k_2)^(1/2)
                for i in range(3, ell + 1):
                    lq[i] = ((i - 1) * lq[i - 1] + lk[i - 1]) / i    # q_i = (P(q_{i-1})^(i-1) * k_i)^(1/i)
                # step 2: v_{ell+1}, then a_ell, v_ell, a_{ell-1}, ..., a_2
                lv = {ell + 1: ell * log_mu_over(lq[ell])}          # v_{ell+1} = (mu ./ P_gamma(q_ell))^ell
                la = {}
                for i in range(ell, 1, -1):
                    la[i] = lv[i + 1] / i + lq[i]                    # a_i = v_{i+1}^(1/i) * q_i
                    if i >= 3:
                        lv[i] = (i - 1) * (la[i] - lq[i - 1])        # v_i = (a_i ./ P(q_{i-1}))^(i-1)
                # step 3: u_1 = a_2 ./ k_1, u_i = a_i ./ k_i
                lu_new = [la[2] - lk[0]] + [la[i] - lk[i - 1] for i in range(2, ell + 1)]
        shape = self.prob.sep_shape(s)
        zero = ~np.isfinite(self.log_m[s]) if fixed else np.zeros(shape, dtype=bool)
        for i, c in enumerate(cs):
            v = np.broadcast_to(lu_new[i], shape).astype(np.float64)
            new[(s, c)] = np.where(zero, -lkbar[i], v)
        return new

    # ------------------------------------------------------- stopping sum
    def separator_error(self, s: int, lu=None) -> Tuple[float, float]:
        lu = self.lu if lu is None else lu
        qs = [np.exp(self.log_proj(c, s, lu)) for c in self.nbr[s]]
        if self.prob.sep_fixed[s]:
            mu = np.asarray(self.prob.sep_marginal[s], dtype=np.float64)
            terms = [float(np.abs(q - mu).sum()) for q in qs]
        else:
            qbar = sum(qs) / len(qs)
            terms = [float(np.abs(q - qbar).sum()) for q in qs]
        return float(sum(terms)), float(max(terms) if terms else 0.0)

    def side_error(self, S, lu=None) -> Tuple[float, float]:
        tot, mx = 0.0, 0.0
        for s in S:
            a, b = self.separator_error(s, lu)
            tot += a
            mx = max(mx, b)
        return tot, mx

    def full_error(self, lu=None) -> Tuple[float, float]:
        e1, m1 = self.side_error(self.S1, lu)
        e2, m2 = self.side_error(self.S2, lu)
        return e1 + e2, max(m1, m2)

    # ---------------------------------------------------------------- loop
    def current_side(self):
        return self.S1 if self.t % 2 == 1 else self.S2

    def tstep(self, stop_tol: Optional[float] = None):
        """One class update; returns (E_S, E_S max, stopped) of the state before it."""
        S = self.current_side()
        e_sum, e_max = self.side_error(S)
        if stop_tol is not None and self.t >= 2 and e_sum <= stop_tol:
            return e_sum, e_max, True
        new = {}
        for s in S:
            new.update(self.update_separator(s))
        self.lu.update(new)
        self.t += 1
        return e_sum, e_max, False

    def run_fixed(self, steps: int):
        return [self.tstep()[:2] for _ in range(steps)]

    def solve(self, tol: float = 1e-6, max_steps: int = 100000) -> dict:
        status, last, done = "not_converged", (float("inf"), float("inf")), 0
        while done < max_steps:
            e, m, stopped = self.tstep(stop_tol=tol)
            if stopped:
                return {"status": "converged", "t": self.t, "updates": done, "err_sum": e, "err_max": m}
            last = (e, m)
            done += 1
        return {"status": status, "t": self.t, "updates": done, "err_sum": last[0], "err_max": last[1]}

    # ------------------------------------------------------------ outputs
    def potentials(self, lu=None) -> np.ndarray:
        """Concatenated log u in clique order: for clique c = (a, b), log u^a_c
        flattened (C order) then log u^b_c."""
        lu = self.lu if lu is None else lu
        out = []
        for c, (a, b) in enumerate(self.prob.cliques):
            out.append(lu[(a, c)].reshape(-1))
            out.append(lu[(b, c)].reshape(-1))
        return np.concatenate(out) if out else np.zeros(0)

    def set_potentials(self, flat) -> Dict[Tuple[int, int], np.ndarray]:
        lu, o = {}, 0
        for c, (a, b) in enumerate(self.prob.cliques):
            for s in (a, b):
                n = self.prob.sep_size(s)
                lu[(s, c)] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(self.prob.sep_shape(s)).copy()
                o += n
        if o != len(flat):
            raise ValueError("potential vector has the wrong length")
        return lu

    def evaluate(self, lu=None) -> dict:
        """Objective values of the state: dual (eq. whole_dual, times eps, with
        log u in place of the Lagrange multipliers), primal (eq.
        ot_graph_local_reg, entropy with its -1 term), transport, plan masses,
        stopping sum."""
        lu = self.lu if lu is None else lu
        p, eps = self.prob, self.eps
        T = H = 0.0
        masses = []
        for c, (a, b) in enumerate(p.cliques):
            lB = self.log_plan(c, lu)
            B = np.exp(lB)
            na = len(p.sep_shape(a))
            lM = (self.log_m[a].reshape(p.sep_shape(a) + (1,) * len(p.sep_shape(b)))
                  + self.log_m[b].reshape((1,) * na + p.sep_shape(b)))
            with np.errstate(invalid="ignore"):
                H += float(np.sum(np.where(B > 0, B * (lB - lM - 1.0), 0.0)))
            T += float(np.sum(np.asarray(p.clique_cost[c]) * B))
            masses.append(float(B.sum()))
        lin = rho = 0.0
        for s in range(p.n_separators):
            tot = sum(lu[(s, c)] for c in self.nbr[s])
            if p.sep_fixed[s]:
                mu = np.asarray(p.sep_marginal[s])
                fin = np.isfinite(tot) & (mu > 0)
                lin += float(np.sum(tot[fin] * mu[fin]))
            else:
                rho += float(np.mean(tot))
        D = eps * (lin + rho - sum(masses))
        err_sum, err_max = self.full_error(lu)
        return {"dual": D, "primal": T + eps * H, "transport": T, "masses": masses, "err_sum": err_sum,
                "err_max": err_max}
