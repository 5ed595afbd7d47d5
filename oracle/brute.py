"""Independent brute-force and textbook solvers used to pin the oracle (test infrastructure).

None of these follows the paper's bipartite update; each reaches the same
answer by a different published route, so agreement pins the oracle:

* ``sinkhorn_textbook``  — plain multiplicative Sinkhorn scaling for one
  two-marginal entropic OT problem (Cuturi 2013; the background of Section 2.1).
* ``ibp_barycenter``     — iterative Bregman projections for the entropic
  barycenter with equal weights (Benamou, Carlier, Cuturi, Nenna, Peyre 2015).
* ``full_tensor_mot``    — the full-tensor iterative scaling of Algorithm
  "sinkhorn" (globally regularised MOT, eq. omt_multi_regularized) on tiny trees.
* ``dual_lbfgs``         — a generic quasi-Newton maximisation of the dual of the
  locally regularised problem (eq. tree_dual_mass_consv) with the free-node
  constraint eliminated.
* ``lp_coupled`` / ``lp_full_tensor`` — the unregularised problems
  (eq. ot_graph_pairwise and eq. omt_multi_discrete) solved by HiGHS.
* ``plans_from_scalings`` / ``stopping_sum_from_plans`` — the plans of
  eq. bi-marginal_B_sol formed as explicit matrices from the scalings
  ``u = exp(Lam)`` (no log-sum-exp, no message), and the stopping sum of
  Algorithm tree_local_reg read off their row and column sums.
* ``sinkhorn_violation_history`` — the marginal violation of textbook Sinkhorn
  iterates, the stopping sum's value on a single edge with both ends given.
"""
from __future__ import annotations

import itertools
from typing import List, Tuple

import numpy as np
from scipy.optimize import linprog, minimize
from scipy.sparse import coo_matrix

from workloads.problem import TreeProblem, COST_SQEUCLID


def _edge_cost(prob: TreeProblem, e: int) -> np.ndarray:
    a, b = int(prob.edges[e][0]), int(prob.edges[e][1])
    if prob.cost_kind == COST_SQEUCLID:
        X, Y = prob.node_support(a), prob.node_support(b)
        return np.sum((X[:, None, :] - Y[None, :, :]) ** 2, axis=2)
    return np.asarray(prob.cost[e], dtype=np.float64)


# ----------------------------------------------------------------------------
def sinkhorn_textbook(mu: np.ndarray, nu: np.ndarray, C: np.ndarray, eps: float, iters: int = 5000) -> np.ndarray:
    """Plan diag(a) K diag(b) with K = exp(-C/eps) after alternating a = mu/(K b), b = nu/(K^T a)."""
    K = np.exp(-C / eps)
    b = np.ones_like(nu)
    for _ in range(iters):
        a = mu / (K @ b)
        b = nu / (K.T @ a)
    return a[:, None] * K * b[None, :]


def ibp_barycenter(mus: List[np.ndarray], Cs: List[np.ndarray], eps: float, rounds: int) -> List[List[np.ndarray]]:
    """Equal-weight IBP for the barycenter: plans pi_l = diag(a_l) K_l diag(b_l)
    with rows on the barycenter grid and columns on leaf l.

    Each round projects onto the leaf constraints (b_l = mu_l / K_l^T a_l) and
    then onto the common-barycenter constraint (p = prod_l (a_l * K_l b_l)^(1/L),
    a_l = p / K_l b_l).  Returns the list of plans after each leaf projection."""
    L = len(mus)
    Ks = [np.exp(-C / eps) for C in Cs]
    a = [np.ones(C.shape[0]) for C in Cs]
    out = []
    for _ in range(rounds):
        b = [mus[l] / (Ks[l].T @ a[l]) for l in range(L)]
        out.append([a[l][:, None] * Ks[l] * b[l][None, :] for l in range(L)])
        Kb = [Ks[l] @ b[l] for l in range(L)]
        logp = np.mean([np.log(a[l] * Kb[l]) for l in range(L)], axis=0)
        p = np.exp(logp)
        a = [p / Kb[l] for l in range(L)]
    return out


# ----------------------------------------------------------------------------
def full_cost_tensor(prob: TreeProblem) -> np.ndarray:
    """C(x_1, ..., x_J) = sum_e C_e(x_a, x_b) (the tree-structured cost, eq. cost_structure)."""
    shape = tuple(int(s) for s in prob.sizes)
    C = np.zeros(shape)
    for e in range(prob.n_edges):
        a, b = int(prob.edges[e][0]), int(prob.edges[e][1])
        Ce = _edge_cost(prob, e)
        lo, hi = min(a, b), max(a, b)
        M = Ce if a < b else Ce.T          # rows on node lo, columns on node hi
        sh = [1] * prob.n_nodes
        sh[lo] = M.shape[0]
        sh[hi] = M.shape[1]
        C = C + M.reshape(sh)
    return C


def _proj(B: np.ndarray, j: int) -> np.ndarray:
    axes = tuple(i for i in range(B.ndim) if i != j)
    return B.sum(axis=axes)


def full_tensor_mot(prob: TreeProblem, iters: int = 3000) -> np.ndarray:
    """Algorithm "sinkhorn": B = K * U * M with u_j scaled on the constrained nodes."""
    C = full_cost_tensor(prob)
    K = np.exp(-C / prob.eps)
    Mt = np.ones_like(K)
    for j in range(prob.n_nodes):
        if prob.is_fixed[j]:
            sh = [1] * prob.n_nodes
            sh[j] = int(prob.sizes[j])
            Mt = Mt * prob.node_marginal(j).reshape(sh)
    u = [np.ones(int(s)) for s in prob.sizes]
    fixed = [j for j in range(prob.n_nodes) if prob.is_fixed[j]]

    def tensor_u():
        U = np.ones_like(K)
        for j in range(prob.n_nodes):
            sh = [1] * prob.n_nodes
            sh[j] = int(prob.sizes[j])
            U = U * u[j].reshape(sh)
        return U

    KM = K * Mt
    for _ in range(iters):
        for j in fixed:
            Pj = _proj(KM * tensor_u(), j)
            u[j] = u[j] * prob.node_marginal(j) / Pj
    return KM * tensor_u()


def pairwise_marginal(B: np.ndarray, a: int, b: int) -> np.ndarray:
    axes = tuple(i for i in range(B.ndim) if i not in (a, b))
    P = B.sum(axis=axes)
    return P if a < b else P.T


def glue(plans: List[np.ndarray], prob: TreeProblem) -> np.ndarray:
    """Tree-Markov joint B(x) = prod_e B_e(x_a, x_b) / prod_j q_j(x_j)^(deg_j - 1)."""
    shape = tuple(int(s) for s in prob.sizes)
    n = prob.n_nodes
    logB = np.zeros(shape)
    deg = np.zeros(n, dtype=int)
    q = [None] * n
    for e in range(prob.n_edges):
        a, b = int(prob.edges[e][0]), int(prob.edges[e][1])
        deg[a] += 1
        deg[b] += 1
        Be = plans[e]
        q[a] = Be.sum(axis=1) if q[a] is None else q[a]
        q[b] = Be.sum(axis=0) if q[b] is None else q[b]
        lo, hi = min(a, b), max(a, b)
        M = Be if a < b else Be.T
        sh = [1] * n
        sh[lo] = M.shape[0]
        sh[hi] = M.shape[1]
        logB = logB + np.log(M).reshape(sh)
    for j in range(n):
        sh = [1] * n
        sh[j] = int(prob.sizes[j])
        logB = logB - (deg[j] - 1) * np.log(q[j]).reshape(sh)
    return np.exp(logB)


def global_objective(B: np.ndarray, prob: TreeProblem) -> float:
    """<C, B> + eps * H(B | prod_{j in Gamma} mu_j) with the -1 term (eq. entropy_term)."""
    C = full_cost_tensor(prob)
    logM = np.zeros_like(B)
    for j in range(prob.n_nodes):
        if prob.is_fixed[j]:
            sh = [1] * prob.n_nodes
            sh[j] = int(prob.sizes[j])
            logM = logM + np.log(prob.node_marginal(j)).reshape(sh)
    with np.errstate(divide="ignore", invalid="ignore"):
        H = np.where(B > 0, B * (np.log(B) - logM - 1.0), 0.0)
    return float(np.sum(C * B) + prob.eps * np.sum(H))


def local_objective(plans: List[np.ndarray], prob: TreeProblem) -> float:
    """sum_e <C_e, B_e> + eps * H(B_e | gamma_a (x) gamma_b) (eq. ot_graph_pairwise_mass)."""
    tot = 0.0
    for e in range(prob.n_edges):
        a, b = int(prob.edges[e][0]), int(prob.edges[e][1])
        Be = plans[e]
        lg = []
        for j in (a, b):
            lg.append(np.log(prob.node_marginal(j)) if prob.is_fixed[j] else np.zeros(int(prob.sizes[j])))
        logM = lg[0][:, None] + lg[1][None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            H = np.where(Be > 0, Be * (np.log(Be) - logM - 1.0), 0.0)
        tot += float(np.sum(_edge_cost(prob, e) * Be) + prob.eps * np.sum(H))
    return tot


# ----------------------------------------------------------------------------
def dual_lbfgs(prob: TreeProblem, gtol: float = 1e-13, maxiter: int = 200000) -> Tuple[float, np.ndarray]:
    """Maximise D(lambda) = sum_{j in Gamma, k} <lambda_(j,k), mu_j> + sum_{j free} tau_j
    - eps * sum_e ||B_e(lambda)||_1 over lambda, with lambda_(j,k_last) = tau_j - sum of
    the other lambda_(j,k) at each free node j.  Returns (D*, potentials as
    Lam = lambda/eps in edge order (a,b) then (b,a))."""
    n = prob.n_nodes
    eps = prob.eps
    nbrs = [[] for _ in range(n)]
    for a, b in prob.edges:
        nbrs[int(a)].append(int(b))
        nbrs[int(b)].append(int(a))
    for j in range(n):
        nbrs[j].sort()
    # variable layout
    slots = {}
    o = 0
    for j in range(n):
        nj = int(prob.sizes[j])
        ks = nbrs[j] if prob.is_fixed[j] else nbrs[j][:-1]
        for k in ks:
            slots[(j, k)] = (o, o + nj)
            o += nj
        if not prob.is_fixed[j]:
            slots[("tau", j)] = (o, o + 1)
            o += 1
    nvar = o
    Cs = [_edge_cost(prob, e) for e in range(prob.n_edges)]
    lg = [np.log(prob.node_marginal(j)) if prob.is_fixed[j] else np.zeros(int(prob.sizes[j])) for j in range(n)]

    def unpack(z):
        lam = {}
        for j in range(n):
            if prob.is_fixed[j]:
                for k in nbrs[j]:
                    s = slots[(j, k)]
                    lam[(j, k)] = z[s[0]:s[1]]
            else:
                tau = z[slots[("tau", j)][0]]
                acc = np.full(int(prob.sizes[j]), tau)
                for k in nbrs[j][:-1]:
                    s = slots[(j, k)]
                    lam[(j, k)] = z[s[0]:s[1]]
                    acc = acc - lam[(j, k)]
                lam[(j, nbrs[j][-1])] = acc
        return lam

    def negD(z):
        lam = unpack(z)
        val = 0.0
        grad_lam = {key: np.zeros_like(v) for key, v in lam.items()}
        for j in range(n):
            if prob.is_fixed[j]:
                mu = prob.node_marginal(j)
                for k in nbrs[j]:
                    val += float(lam[(j, k)] @ mu)
                    grad_lam[(j, k)] += mu
        gz = np.zeros(nvar)
        for j in range(n):
            if not prob.is_fixed[j]:
                val += float(z[slots[("tau", j)][0]])
                gz[slots[("tau", j)][0]] += 1.0
        for e in range(prob.n_edges):
            a, b = int(prob.edges[e][0]), int(prob.edges[e][1])
            Bm = np.exp((lam[(a, b)][:, None] + lam[(b, a)][None, :] - Cs[e]) / eps + lg[a][:, None] + lg[b][None, :])
            val -= eps * float(Bm.sum())
            grad_lam[(a, b)] -= Bm.sum(axis=1)
            grad_lam[(b, a)] -= Bm.sum(axis=0)
        # chain rule through the parametrisation
        for j in range(n):
            if prob.is_fixed[j]:
                for k in nbrs[j]:
                    s = slots[(j, k)]
                    gz[s[0]:s[1]] += grad_lam[(j, k)]
            else:
                last = grad_lam[(j, nbrs[j][-1])]
                gz[slots[("tau", j)][0]] += float(last.sum())
                for k in nbrs[j][:-1]:
                    s = slots[(j, k)]
                    gz[s[0]:s[1]] += grad_lam[(j, k)] - last
        return -val, -gz

    res = minimize(negD, np.zeros(nvar), jac=True, method="L-BFGS-B",
                   options={"maxiter": maxiter, "gtol": gtol, "ftol": 1e-16, "maxcor": 50})
    lam = unpack(res.x)
    flat = []
    for a, b in prob.edges:
        flat.append(lam[(int(a), int(b))] / eps)
        flat.append(lam[(int(b), int(a))] / eps)
    return -float(res.fun), np.concatenate(flat)


# ----------------------------------------------------------------------------
def lp_coupled(prob: TreeProblem) -> float:
    """Unregularised coupled problem (eq. ot_graph_pairwise): variables are the
    edge plans and the marginals of free nodes."""
    n = prob.n_nodes
    sizes = [int(s) for s in prob.sizes]
    var_off = []
    o = 0
    for e in range(prob.n_edges):
        a, b = int(prob.edges[e][0]), int(prob.edges[e][1])
        var_off.append(o)
        o += sizes[a] * sizes[b]
    nu_off = {}
    for j in range(n):
        if not prob.is_fixed[j]:
            nu_off[j] = o
            o += sizes[j]
    nvar = o
    c = np.zeros(nvar)
    rows, cols, vals, rhs = [], [], [], []
    r = 0

    def add_marg(e, j, axis):
        nonlocal r
        a, b = int(prob.edges[e][0]), int(prob.edges[e][1])
        na, nb = sizes[a], sizes[b]
        for x in range(sizes[j]):
            if axis == 0:
                idx = [var_off[e] + x * nb + y for y in range(nb)]
            else:
                idx = [var_off[e] + y * nb + x for y in range(na)]
            rows.extend([r] * len(idx)); cols.extend(idx); vals.extend([1.0] * len(idx))
            if prob.is_fixed[j]:
                rhs.append(float(prob.node_marginal(j)[x]))
            else:
                rows.append(r); cols.append(nu_off[j] + x); vals.append(-1.0)
                rhs.append(0.0)
            r += 1

    for e in range(prob.n_edges):
        a, b = int(prob.edges[e][0]), int(prob.edges[e][1])
        c[var_off[e]:var_off[e] + sizes[a] * sizes[b]] = _edge_cost(prob, e).ravel()
        add_marg(e, a, 0)
        add_marg(e, b, 1)
    for j in nu_off:
        idx = list(range(nu_off[j], nu_off[j] + sizes[j]))
        rows.extend([r] * len(idx)); cols.extend(idx); vals.extend([1.0] * len(idx)); rhs.append(1.0); r += 1
    A = coo_matrix((vals, (rows, cols)), shape=(r, nvar)).tocsr()
    res = linprog(c, A_eq=A, b_eq=np.array(rhs), bounds=(0, None), method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    return float(res.fun)


def lp_full_tensor(prob: TreeProblem) -> float:
    """Unregularised MOT on the full tensor (eq. omt_multi_discrete)."""
    C = full_cost_tensor(prob)
    shape = C.shape
    nvar = C.size
    rows, cols, vals, rhs = [], [], [], []
    r = 0
    flat_idx = np.arange(nvar).reshape(shape)
    for j in range(prob.n_nodes):
        if not prob.is_fixed[j]:
            continue
        mu = prob.node_marginal(j)
        for x in range(shape[j]):
            idx = np.take(flat_idx, x, axis=j).ravel()
            rows.extend([r] * idx.size); cols.extend(idx.tolist()); vals.extend([1.0] * idx.size)
            rhs.append(float(mu[x]))
            r += 1
    A = coo_matrix((vals, (rows, cols)), shape=(r, nvar)).tocsr()
    res = linprog(C.ravel(), A_eq=A, b_eq=np.array(rhs), bounds=(0, None), method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    return float(res.fun)


# ----------------------------------------------------------------------------
def plans_from_scalings(prob: TreeProblem, lam_flat: np.ndarray) -> List[np.ndarray]:
    """B_e = diag(u_(a,b) * gamma_a) K_e diag(u_(b,a) * gamma_b) with u = exp(Lam)
    and K_e = exp(-C_e / eps) (eq. bi-marginal_B_sol), as dense matrices.
    ``lam_flat`` is in edge order: Lam_(a,b) (n_a values) then Lam_(b,a)."""
    plans = []
    o = 0
    for e in range(prob.n_edges):
        a, b = int(prob.edges[e][0]), int(prob.edges[e][1])
        na, nb = int(prob.sizes[a]), int(prob.sizes[b])
        ua = np.exp(np.asarray(lam_flat[o:o + na], dtype=np.float64)); o += na
        ub = np.exp(np.asarray(lam_flat[o:o + nb], dtype=np.float64)); o += nb
        ga = prob.node_marginal(a) if prob.is_fixed[a] else np.ones(na)
        gb = prob.node_marginal(b) if prob.is_fixed[b] else np.ones(nb)
        K = np.exp(-_edge_cost(prob, e) / prob.eps)
        plans.append((ua * ga)[:, None] * K * (ub * gb)[None, :])
    return plans


def plan_marginals(prob: TreeProblem, plans: List[np.ndarray]) -> List[dict]:
    """For every node j, {k: B_(j,k) 1} (row sums seen from j's side)."""
    out = [dict() for _ in range(prob.n_nodes)]
    for e in range(prob.n_edges):
        a, b = int(prob.edges[e][0]), int(prob.edges[e][1])
        out[a][b] = plans[e].sum(axis=1)
        out[b][a] = plans[e].sum(axis=0)
    return out


def stopping_sum_from_plans(prob: TreeProblem, plans: List[np.ndarray], nodes=None) -> Tuple[float, float]:
    """Stopping sum of Algorithm tree_local_reg over ``nodes`` (default: all):
    a constrained node adds ||B_(j,k) 1 - mu_j||_1 for each incident edge, a
    free node adds sum_k ||B_(j,k) 1 - q_bar_j||_1 with q_bar_j the arithmetic
    mean of its plan marginals (Lemma f_upper_bound_tree).  Returns the sum
    and its largest single term."""
    marg = plan_marginals(prob, plans)
    nodes = range(prob.n_nodes) if nodes is None else nodes
    terms = []
    for j in nodes:
        qs = [marg[j][k] for k in sorted(marg[j])]
        if prob.is_fixed[j]:
            mu = prob.node_marginal(j)
            terms += [float(np.abs(q - mu).sum()) for q in qs]
        else:
            qbar = sum(qs) / len(qs)
            terms += [float(np.abs(q - qbar).sum()) for q in qs]
    return float(sum(terms)), float(max(terms) if terms else 0.0)


def sinkhorn_violation_history(mu: np.ndarray, nu: np.ndarray, C: np.ndarray, eps: float,
                               steps: int) -> List[float]:
    """Textbook Sinkhorn on K = exp(-C/eps) started from the column scaling
    b = nu: after each half-step (rows first) the L1 violation of the marginal
    that the half-step did not fit, i.e. ||B^T 1 - nu||_1 after a row scaling
    and ||B 1 - mu||_1 after a column scaling."""
    K = np.exp(-C / eps)
    a = np.ones_like(mu)
    b = nu.copy()
    out = []
    for s in range(steps):
        if s % 2 == 0:
            with np.errstate(divide="ignore", invalid="ignore"):
                a = np.where(mu > 0, mu / (K @ b), 0.0)
            B = a[:, None] * K * b[None, :]
            out.append(float(np.abs(B.sum(axis=0) - nu).sum()))
        else:
            with np.errstate(divide="ignore", invalid="ignore"):
                b = np.where(nu > 0, nu / (K.T @ a), 0.0)
            B = a[:, None] * K * b[None, :]
            out.append(float(np.abs(B.sum(axis=1) - mu).sum()))
    return out
