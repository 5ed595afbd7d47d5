"""FP64 CPU oracle for bipartite iterative scaling on a tree (test infrastructure).

This module is the correctness reference for the HIP path.  Only the test
suite, the smoke entry point and the CPU-baseline leg of the benchmark may
import it; the product library never calls it.  It shares no code with the HIP
path: its only common dependency is the seeded input generator package.

What it computes (Section 3 of the paper, "Tree-structured multi-marginal
optimal transport with local regularization"):

* Problem: coupled bi-marginal OT on a tree with a local entropy term per edge
  and reference measure ``M_(j,k) = gamma_j (x) gamma_k`` (eq. jointdist), where
  ``gamma_j`` is the given marginal on constrained nodes and the all-ones
  vector elsewhere; free nodes carry a unit-mass constraint
  (eq. ot_graph_pairwise_mass).
* Plans: ``B_(j,k) = diag(u_(j,k) * gamma_j) K diag(u_(k,j) * gamma_k)`` with
  ``K = exp(-C / eps)`` (eq. bi-marginal_B_sol).
* Iteration: Algorithm "Bipartite Iterative Scaling" — 2-colour the tree,
  start from ``u = 1``, and alternately update all scalings of one colour
  class with the multiplicative rules (eq. bipartite_tree_updates1/2) built
  from ``q_(j,k) = B_(j,k) 1`` and their geometric mean (eq. q), until the
  summed marginal error falls below the tolerance.
* A second, independent rendering of the same update — the closed form of
  Theorem "tree_dual_var" — is provided so that Proposition "equi" (the two
  forms agree) can be checked.

Everything is stored in the log domain: ``Lam[(j,k)] = log u_(j,k)``; the paper's
potentials are ``lambda = eps * Lam`` (Section 3.2).

Readings where the paper is silent (each is listed in the design notes):

* First colour class: the class of node 0 under BFS from node 0 unless
  ``first_color`` says otherwise (the paper only says "construct a bipartite
  graph").
* One iteration = one half-sweep (the paper increments t per half-sweep).
* The mean ``q_bar_j`` in the stopping sum is the arithmetic mean (it is
  defined that way in Lemma "f_upper_bound_tree"); the update uses the
  geometric mean ``q_j^{t+1}`` of eq. (q).
* A constrained node of degree r > 1 (the paper assumes constrained nodes are
  leaves and notes that such a node splits the tree) is read as r constrained
  leaves carrying the same marginal: each incident edge gets the fixed-node
  update and its own term in the stopping sum.
* The fixed-node rule is used in its general form with ``gamma_k`` inside the
  message (Algorithm form), which also covers edges whose both ends are fixed.
* Zero marginal entries: ``log 0 = -inf``; at those entries the fixed update
  takes the limit value ``Lam = -m_{k->j}`` (the closed form of Theorem
  "tree_dual_var", u = 1 / (K u')) from the message itself, since
  ``log q = -inf`` there.
* Stopping: check-then-update; the test is applied from the second
  half-sweep on (the first state has not been scaled anywhere yet) and the
  state returned is the one whose error passed the test.
* The node-sequential ("plain") schedule, which the paper does not state: a
  Gauss-Seidel sweep updates every node once, in breadth-first order from
  node 0, each with the same per-node rule from the latest potentials of its
  neighbours; after a sweep no class is exact, so its stop test uses the
  stopping sum over every node.
"""
from __future__ import annotations

from collections import deque
from typing import Dict, List, Optional, Tuple

import numpy as np

from workloads.problem import TreeProblem, COST_SQEUCLID, COST_EXPLICIT


# ----------------------------------------------------------------------------
# small numeric helpers
# ----------------------------------------------------------------------------

def logsumexp(w: np.ndarray, axis: int) -> np.ndarray:
    """Stabilised log(sum(exp(w))) along ``axis``; an all ``-inf`` slice gives -inf."""
    m = np.max(w, axis=axis, keepdims=True)
    m_safe = np.where(np.isfinite(m), m, 0.0)
    s = np.sum(np.exp(w - m_safe), axis=axis, keepdims=True)
    with np.errstate(divide="ignore"):
        out = np.log(s) + m_safe
    return np.squeeze(out, axis=axis)


def validate_tree(prob: TreeProblem) -> None:
    """Raise ValueError unless (nodes, edges) is a tree with valid data."""
    n = prob.n_nodes
    if n < 1:
        raise ValueError("empty tree")
    if prob.n_edges != n - 1:
        raise ValueError("a tree on N nodes has N-1 edges")
    if prob.eps <= 0 or not np.isfinite(prob.eps):
        raise ValueError("eps must be positive")
    if np.any(prob.sizes < 1):
        raise ValueError("every node needs at least one support point")
    seen = set()
    adj = [[] for _ in range(n)]
    for a, b in prob.edges:
        a, b = int(a), int(b)
        if not (0 <= a < n and 0 <= b < n) or a == b:
            raise ValueError("bad edge")
        key = (min(a, b), max(a, b))
        if key in seen:
            raise ValueError("duplicate edge")
        seen.add(key)
        adj[a].append(b)
        adj[b].append(a)
    # connected <=> BFS reaches everything (with N-1 edges this also rules out cycles)
    reached = {0}
    dq = deque([0])
    while dq:
        v = dq.popleft()
        for w in adj[v]:
            if w not in reached:
                reached.add(w)
                dq.append(w)
    if len(reached) != n:
        raise ValueError("graph is not connected")
    for j in range(n):
        if prob.is_fixed[j]:
            mu = prob.node_marginal(j)
            if np.any(mu < 0) or abs(mu.sum() - 1.0) > 1e-9:
                raise ValueError(f"marginal of node {j} must be a probability vector")


class TreeOracle:
    """Bipartite iterative scaling in float64 (Algorithm tree_local_reg)."""

    def __init__(self, prob: TreeProblem, first_color: Optional[int] = None):
        validate_tree(prob)
        self.prob = prob
        self.eps = float(prob.eps)
        n = prob.n_nodes
        self.nbrs: List[List[int]] = [[] for _ in range(n)]
        self.edge_of: Dict[Tuple[int, int], int] = {}
        for e, (a, b) in enumerate(prob.edges):
            a, b = int(a), int(b)
            self.nbrs[a].append(b)
            self.nbrs[b].append(a)
            self.edge_of[(a, b)] = e
            self.edge_of[(b, a)] = e
        for j in range(n):
            self.nbrs[j].sort()
        # bipartite split by BFS from node 0 (colour 0 = node 0's class)
        colour = [-1] * n
        colour[0] = 0
        dq = deque([0])
        while dq:
            v = dq.popleft()
            for w in self.nbrs[v]:
                if colour[w] < 0:
                    colour[w] = 1 - colour[v]
                    dq.append(w)
        self.colour = colour
        fc = 0 if first_color is None else int(first_color)
        self.S1 = [j for j in range(n) if colour[j] == fc]
        self.S2 = [j for j in range(n) if colour[j] != fc]
        # gamma_j: the marginal on constrained nodes, ones elsewhere (eq. jointdist)
        self.log_gamma: List[np.ndarray] = []
        self.mu: List[Optional[np.ndarray]] = []
        for j in range(n):
            if prob.is_fixed[j]:
                mu = np.asarray(prob.node_marginal(j), dtype=np.float64)
                with np.errstate(divide="ignore"):
                    self.log_gamma.append(np.log(mu))
                self.mu.append(mu)
            else:
                self.log_gamma.append(np.zeros(int(prob.sizes[j])))
                self.mu.append(None)
        # u^0 = 1  <=>  Lam = 0 on every directed edge
        self.Lam: Dict[Tuple[int, int], np.ndarray] = {}
        for j in range(n):
            for k in self.nbrs[j]:
                self.Lam[(j, k)] = np.zeros(int(prob.sizes[j]))
        self.t = 1
        self._cost_cache: Dict[Tuple[int, int], np.ndarray] = {}

    # ---------------------------------------------------------------- cost
    def cost(self, j: int, k: int) -> np.ndarray:
        """C_(j,k) as an n_j x n_k matrix (C_(j,k) = C_(k,j)^T)."""
        key = (j, k)
        if key in self._cost_cache:
            return self._cost_cache[key]
        p = self.prob
        if p.cost_kind == COST_SQEUCLID:
            X = p.node_support(j)
            Y = p.node_support(k)
            C = np.zeros((X.shape[0], Y.shape[0]))
            for d in range(p.dim):
                C += (X[:, d][:, None] - Y[:, d][None, :]) ** 2
        elif p.cost_kind == COST_EXPLICIT:
            e = self.edge_of[(j, k)]
            a, b = int(p.edges[e][0]), int(p.edges[e][1])
            Ce = np.asarray(p.cost[e], dtype=np.float64)
            C = Ce if (a, b) == (j, k) else Ce.T
        else:
            raise ValueError("unknown cost kind")
        if C.size <= 4_000_000:
            self._cost_cache[key] = C
        return C

    def c_inf(self) -> float:
        return max(float(np.max(np.abs(self.cost(int(a), int(b))))) for a, b in self.prob.edges)

    # ------------------------------------------------------------- messages
    def message(self, k: int, j: int, Lam=None) -> np.ndarray:
        """m_{k->j} = log( K_(j,k) (u_(k,j) * gamma_k) ), a vector over supp(j)."""
        Lam = self.Lam if Lam is None else Lam
        w = (Lam[(k, j)] + self.log_gamma[k])[None, :] - self.cost(j, k) / self.eps
        return logsumexp(w, axis=1)

    def log_q(self, j: int, k: int, m: np.ndarray, Lam=None) -> np.ndarray:
        """log q_(j,k) = log(B_(j,k) 1) = Lam_(j,k) + log gamma_j + m_{k->j} (eq. q)."""
        Lam = self.Lam if Lam is None else Lam
        return Lam[(j, k)] + self.log_gamma[j] + m

    # ---------------------------------------------------------------- error
    def node_error(self, j: int, logqs: Dict[int, np.ndarray]) -> Tuple[float, float]:
        """Node j's share of the stopping sum (and its largest single term).

        Constrained node: ||q_(j,k) - mu_j||_1 per incident edge.  Free node:
        sum_k ||q_(j,k) - q_bar_j||_1 with q_bar_j the arithmetic mean of the
        q_(j,k) (Lemma f_upper_bound_tree)."""
        if self.prob.is_fixed[j]:
            terms = [float(np.sum(np.abs(np.exp(logqs[k]) - self.mu[j]))) for k in self.nbrs[j]]
        else:
            qs = np.stack([np.exp(logqs[k]) for k in self.nbrs[j]])
            qbar = qs.mean(axis=0)
            terms = [float(np.sum(np.abs(qs[i] - qbar))) for i in range(qs.shape[0])]
        return float(sum(terms)), float(max(terms) if terms else 0.0)

    def side_error(self, S: List[int], Lam=None) -> Tuple[float, float]:
        Lam = self.Lam if Lam is None else Lam
        tot, mx = 0.0, 0.0
        for j in S:
            logqs = {k: self.log_q(j, k, self.message(k, j, Lam), Lam) for k in self.nbrs[j]}
            s, m = self.node_error(j, logqs)
            tot += s
            mx = max(mx, m)
        return tot, mx

    def full_error(self, Lam=None) -> Tuple[float, float]:
        """Stopping sum over every node (both colour classes)."""
        e1, m1 = self.side_error(self.S1, Lam)
        e2, m2 = self.side_error(self.S2, Lam)
        return e1 + e2, max(m1, m2)

    # --------------------------------------------------------------- update
    def update_node_algorithm(self, j: int, logqs: Dict[int, np.ndarray],
                              msgs: Optional[Dict[int, np.ndarray]] = None) -> Dict[Tuple[int, int], np.ndarray]:
        """New Lam_(j,k) for all k in N(j) by eq. bipartite_tree_updates1/2.

        ``msgs`` (the messages m_{k->j} behind ``logqs``) is needed only where
        a constrained node's marginal has zero entries: there log q = -inf
        carries no information and the update takes its limit value
        Lam = -m_{k->j} (Lam + log mu - log q = -m wherever mu > 0)."""
        new = {}
        if self.prob.is_fixed[j]:
            # u <- u * mu ./ q   (per incident edge)
            lg = self.log_gamma[j]
            zero = ~np.isfinite(lg)
            for k in self.nbrs[j]:
                with np.errstate(invalid="ignore"):
                    upd = self.Lam[(j, k)] + lg - logqs[k]
                if np.any(zero):
                    m = self.message(k, j) if msgs is None else msgs[k]
                    upd = np.where(zero, -m, upd)
                new[(j, k)] = upd
        else:
            # q_j^{t+1} = geometric mean of q_(j,k); u <- u * (q_j / |q_j|_1) ./ q_(j,k)
            log_qj = np.mean(np.stack([logqs[k] for k in self.nbrs[j]]), axis=0)
            log_qj_hat = log_qj - logsumexp(log_qj, axis=0)
            for k in self.nbrs[j]:
                new[(j, k)] = self.Lam[(j, k)] + log_qj_hat - logqs[k]
        return new

    def update_node_theorem(self, j: int, msgs: Dict[int, np.ndarray]) -> Dict[Tuple[int, int], np.ndarray]:
        """New Lam_(j,k) by the closed form of Theorem tree_dual_var, from the
        messages m_{k->j} = log K_(j,k)(u_(k,j) * gamma_k) only."""
        new = {}
        if self.prob.is_fixed[j]:
            for k in self.nbrs[j]:
                new[(j, k)] = -msgs[k]                       # u = 1 ./ (K u')
        else:
            N = len(self.nbrs[j])
            log_v = np.mean(np.stack([msgs[k] for k in self.nbrs[j]]), axis=0)   # v_j
            rho = -N * logsumexp(log_v, axis=0)                                 # rho_j
            for k in self.nbrs[j]:
                new[(j, k)] = rho / N + log_v - msgs[k]
        return new

    # ----------------------------------------------------------------- loop
    def current_side(self) -> List[int]:
        return self.S1 if (self.t % 2 == 1) else self.S2

    def tstep(self, check_equivalence: bool = False, stop_tol: Optional[float] = None):
        """One half-sweep: error of the side about to be updated, then the update.

        Returns (E_S, E_S_max, stopped) for the state *before* the update.  When
        ``stop_tol`` is given, t >= 2 and E_S <= stop_tol, the update is skipped
        (check-then-update) and ``stopped`` is True."""
        S = self.current_side()
        msgs = {j: {k: self.message(k, j) for k in self.nbrs[j]} for j in S}
        logqs = {j: {k: self.log_q(j, k, msgs[j][k]) for k in self.nbrs[j]} for j in S}
        e_sum, e_max = 0.0, 0.0
        for j in S:
            s, m = self.node_error(j, logqs[j])
            e_sum += s
            e_max = max(e_max, m)
        if stop_tol is not None and self.t >= 2 and e_sum <= stop_tol:
            return e_sum, e_max, True
        updates = {}
        for j in S:
            upd = self.update_node_algorithm(j, logqs[j], msgs[j])
            if check_equivalence:
                alt = self.update_node_theorem(j, msgs[j])
                for key in upd:
                    a, b = upd[key], alt[key]
                    scale = max(1.0, float(np.max(np.abs(b))))
                    if not np.allclose(a, b, rtol=0, atol=1e-12 * scale):
                        raise AssertionError(f"algorithm and theorem forms differ at {key}")
            updates.update(upd)
        self.Lam.update(updates)
        self.t += 1
        return e_sum, e_max, False

    def solve(self, tol: float = 1e-6, max_steps: int = 100000, check_equivalence: bool = False,
              history: Optional[list] = None) -> dict:
        """Run until the stopping sum of the current state is <= tol.

        The sum at half-sweep t >= 2 equals the error of the side about to be
        updated (the other side was scaled exactly one half-sweep before); the
        first half-sweep is never a stopping point."""
        status = "not_converged"
        e_last = (float("inf"), float("inf"))
        steps_done = 0
        while True:
            if steps_done >= max_steps:
                if self.t >= 2:
                    e_last = self.side_error(self.current_side())
                break
            e_sum, e_max, stopped = self.tstep(check_equivalence=check_equivalence, stop_tol=tol)
            if self.t >= 2 or stopped:
                if history is not None and (stopped or self.t > 2):
                    history.append(e_sum)
            if stopped:
                e_last = (e_sum, e_max)
                status = "converged"
                break
            if self.t > 2:
                e_last = (e_sum, e_max)
            steps_done += 1
        return {"status": status, "t": self.t, "updates": steps_done, "err_sum": e_last[0], "err_max": e_last[1]}

    # ------------------------------------------------- Gauss-Seidel schedule
    def gs_order(self) -> List[int]:
        """The nodes with neighbours in breadth-first order from node 0 (each
        node's neighbours ascending): the order of one Gauss-Seidel sweep."""
        seen = [False] * self.prob.n_nodes
        seen[0] = True
        order, dq = [], deque([0])
        while dq:
            v = dq.popleft()
            if self.nbrs[v]:
                order.append(v)
            for w in self.nbrs[v]:
                if not seen[w]:
                    seen[w] = True
                    dq.append(w)
        return order

    def gs_update(self, j: int) -> None:
        """Node j takes the update of eq. bipartite_tree_updates1/2 from the
        current potentials of its neighbours, and keeps it at once."""
        msgs = {k: self.message(k, j) for k in self.nbrs[j]}
        logqs = {k: self.log_q(j, k, msgs[k]) for k in self.nbrs[j]}
        self.Lam.update(self.update_node_algorithm(j, logqs, msgs))

    def gs_sweep(self) -> None:
        """One node-sequential sweep: every node in gs_order() updated in turn,
        each from its neighbours' latest potentials (the same per-node rule as
        Algorithm tree_local_reg, with the bipartite classes replaced by single
        nodes)."""
        for j in self.gs_order():
            self.gs_update(j)

    def solve_gauss_seidel(self, tol: float = 1e-6, max_sweeps: int = 100000, check_every: int = 1,
                           history: Optional[list] = None) -> dict:
        """Sweeps until the stopping sum of the whole state (every node, both
        classes: no class is exact after a sweep) is <= tol, tested before
        the first sweep and after every check_every sweeps."""
        sweeps = 0
        while True:
            if sweeps % check_every == 0 or sweeps >= max_sweeps:
                e_sum, e_max = self.full_error()
                if history is not None:
                    history.append(e_sum)
                if e_sum <= tol:
                    return {"status": "converged", "sweeps": sweeps, "err_sum": e_sum, "err_max": e_max}
                if sweeps >= max_sweeps:
                    return {"status": "not_converged", "sweeps": sweeps, "err_sum": e_sum, "err_max": e_max}
            self.gs_sweep()
            sweeps += 1

    def run_fixed(self, steps: int, check_equivalence: bool = False) -> List[Tuple[float, float]]:
        """Exactly ``steps`` half-sweeps; returns the per-step (E_S, E_S_max)."""
        return [self.tstep(check_equivalence=check_equivalence)[:2] for _ in range(steps)]

    # ------------------------------------------------------------ outputs
    def potentials(self, Lam=None) -> np.ndarray:
        """Concatenated log-scalings: for edge e=(a,b), Lam_(a,b) then Lam_(b,a)."""
        Lam = self.Lam if Lam is None else Lam
        out = []
        for a, b in self.prob.edges:
            out.append(Lam[(int(a), int(b))])
            out.append(Lam[(int(b), int(a))])
        return np.concatenate(out) if out else np.zeros(0)

    def set_potentials(self, flat: np.ndarray) -> Dict[Tuple[int, int], np.ndarray]:
        Lam = {}
        o = 0
        for a, b in self.prob.edges:
            a, b = int(a), int(b)
            na, nb = int(self.prob.sizes[a]), int(self.prob.sizes[b])
            Lam[(a, b)] = np.asarray(flat[o:o + na], dtype=np.float64).copy(); o += na
            Lam[(b, a)] = np.asarray(flat[o:o + nb], dtype=np.float64).copy(); o += nb
        if o != flat.shape[0]:
            raise ValueError("potential vector has the wrong length")
        return Lam

    def log_coupling(self, e: int, Lam=None) -> np.ndarray:
        """log B_e for edge e=(a,b), an n_a x n_b matrix (eq. bi-marginal_B_sol)."""
        Lam = self.Lam if Lam is None else Lam
        a, b = int(self.prob.edges[e][0]), int(self.prob.edges[e][1])
        return ((Lam[(a, b)] + self.log_gamma[a])[:, None] + (Lam[(b, a)] + self.log_gamma[b])[None, :]
                - self.cost(a, b) / self.eps)

    def coupling(self, e: int, Lam=None) -> np.ndarray:
        return np.exp(self.log_coupling(e, Lam))

    def evaluate(self, Lam=None) -> dict:
        """Objective values of the state, computed from the explicit plans.

        dual      D = -eps * f(u, rho)  (eq. tree_dual_mass_consv), with
                  rho_j = sum_k Lam_(j,k)(x) (read at every x; its spread is
                  returned as ``rho_spread``)
        primal    P = sum_e <C_e, B_e> + eps * H(B_e | M_e)   (eq. ot_graph_pairwise_mass,
                  entropy with the -1 term of eq. entropy_term)
        transport T = sum_e <C_e, B_e>
        masses    ||B_e||_1 per edge
        error     stopping sum over every node and its largest term
        scale     s = sum |eps <Lam, mu>| + sum |eps rho| + eps |E|, used for
                  relative comparisons of D"""
        Lam = self.Lam if Lam is None else Lam
        p = self.prob
        eps = self.eps
        T = 0.0
        H = 0.0
        masses = []
        for e in range(p.n_edges):
            a, b = int(p.edges[e][0]), int(p.edges[e][1])
            lB = self.log_coupling(e, Lam)
            B = np.exp(lB)
            lM = self.log_gamma[a][:, None] + self.log_gamma[b][None, :]
            with np.errstate(invalid="ignore"):
                ent = np.where(B > 0, B * (lB - lM - 1.0), 0.0)
            H += float(np.sum(ent))
            T += float(np.sum(self.cost(a, b) * B))
            masses.append(float(np.sum(B)))
        lin = 0.0
        scale = eps * p.n_edges
        rho_sum = 0.0
        rho_spread = 0.0
        for j in range(p.n_nodes):
            if p.is_fixed[j]:
                for k in self.nbrs[j]:
                    fin = np.isfinite(Lam[(j, k)]) & (self.mu[j] > 0)
                    v = float(np.dot(Lam[(j, k)][fin], self.mu[j][fin]))
                    lin += v
                    scale += eps * abs(v)
            else:
                tot = np.sum(np.stack([Lam[(j, k)] for k in self.nbrs[j]]), axis=0)
                rho = float(np.mean(tot))
                rho_spread = max(rho_spread, float(np.max(tot) - np.min(tot)))
                rho_sum += rho
                scale += eps * abs(rho)
        D = eps * (lin + rho_sum - sum(masses))
        P = T + eps * H
        err_sum, err_max = self.full_error(Lam)
        return {"dual": D, "primal": P, "transport": T, "gap": P - D, "masses": masses,
                "err_sum": err_sum, "err_max": err_max, "rho_spread": rho_spread, "scale": scale}

    def node_marginal(self, j: int, Lam=None) -> np.ndarray:
        """q_bar_j: the arithmetic mean over k of the plan marginals B_(j,k) 1."""
        Lam = self.Lam if Lam is None else Lam
        qs = [np.exp(self.log_q(j, k, self.message(k, j, Lam), Lam)) for k in self.nbrs[j]]
        return np.mean(np.stack(qs), axis=0)
