"""Problem descriptions on modified junction trees (Section 4 of the paper).

A modified junction tree (Definition jt_general) alternates separators and
cost cliques: every cost clique has exactly two neighbouring separators, and
the separator--clique graph is a tree.  The descriptions here cover the case
in which every cost clique's variables are the disjoint union of its two
separators' variables and a constraint, when present, fixes the joint
marginal of all of a separator's variables.  The Wasserstein least-squares
problem of Section 2 (cliques {0, j, J+1} hanging off the separator {0, J+1},
constrained separators {j}) is of this kind.

Only problem data lives here (supports, marginals, cost tensors); no method
arithmetic.  Every random draw comes from
``numpy.random.Generator(PCG64(SeedSequence([cfg_id, instance_id])))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from .gen import rng_for, grid_1d, gaussian_mixture


@dataclass
class JunctionProblem:
    var_sizes: List[int]                         # support size n_v of every variable
    var_support: List[np.ndarray]                # [n_v, dim] points of every variable
    separators: List[Tuple[int, ...]]            # the variables of each separator, in tensor-axis order
    sep_fixed: List[bool]                        # separator in Q_Gamma (its joint marginal is given)
    sep_marginal: List[Optional[np.ndarray]]     # given marginal, a tensor over the separator's variables
    cliques: List[Tuple[int, int]]               # the two neighbouring separators (a, b) of each cost clique
    clique_cost: List[np.ndarray]                # C_c over (variables of a) then (variables of b)
    eps: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    def sep_shape(self, s: int) -> Tuple[int, ...]:
        return tuple(int(self.var_sizes[v]) for v in self.separators[s])

    def sep_size(self, s: int) -> int:
        return int(np.prod(self.sep_shape(s))) if self.separators[s] else 1

    @property
    def n_separators(self) -> int:
        return len(self.separators)

    @property
    def n_cliques(self) -> int:
        return len(self.cliques)


def log_normal_marginal(rng: np.random.Generator, pts: np.ndarray) -> np.ndarray:
    """A seeded log-normal density on [0, 1] points (the paper's experiments draw
    the constrained marginals from log-normal distributions): location
    U(-1.5, -0.5), shape U(0.3, 0.7), evaluated at the points shifted into
    (0, 1], floored at 300 nats below its maximum and normalised."""
    x = pts[:, 0] + 1.0 / max(pts.shape[0], 2)
    mu = rng.uniform(-1.5, -0.5)
    sig = rng.uniform(0.3, 0.7)
    ld = -np.log(x) - 0.5 * ((np.log(x) - mu) / sig) ** 2
    ld = np.maximum(ld, ld.max() - 300.0)
    p = np.exp(ld - ld.max())
    return p / p.sum()


def make_wls(J: int = 3, n: int = 10, alpha: float = 10.0, eps: float = 0.05, cfg_id: int = 6,
             instance: int = 0, marginals: str = "lognormal") -> JunctionProblem:
    """Wasserstein least squares (Section 2, eq. wls_cost) on its modified
    junction tree (Figure wls_modified_jt).  Variables 0 and J+1 are the two
    unknown end distributions, variables 1..J the observed ones at times
    t_j = (j - 1) / (J - 1) (t_1 = 0 when J = 1); all on a uniform grid of n
    points in [0, 1].  Separator 0 = {0, J+1} (free); separator j = {j}
    (constrained, marginal rho_{t_j}).  Clique j joins separators 0 and j with
    cost  |x_j - (1 - t_j) x_0 - t_j x_{J+1}|^2 + (alpha / J) |x_0 - x_{J+1}|^2
    over axes (x_0, x_{J+1}, x_j) (the alpha term split evenly over the cliques
    that contain both end variables)."""
    rng = rng_for(cfg_id, instance)
    pts = grid_1d(n)
    sizes = [n] * (J + 2)
    support = [pts.copy() for _ in range(J + 2)]
    seps: List[Tuple[int, ...]] = [(0, J + 1)] + [(j,) for j in range(1, J + 1)]
    fixed = [False] + [True] * J
    marg: List[Optional[np.ndarray]] = [None]
    for _ in range(J):
        marg.append(log_normal_marginal(rng, pts) if marginals == "lognormal" else gaussian_mixture(rng, pts, 2))
    x = pts[:, 0]
    cliques, costs = [], []
    for j in range(1, J + 1):
        t = (j - 1) / (J - 1) if J > 1 else 0.0
        C = ((x[None, None, :] - (1.0 - t) * x[:, None, None] - t * x[None, :, None]) ** 2
             + (alpha / J) * (x[:, None, None] - x[None, :, None]) ** 2)
        cliques.append((0, j))
        costs.append(C)
    return JunctionProblem(sizes, support, seps, fixed, marg, cliques, costs, float(eps),
                           name=f"wls-J{J}-n{n}", meta={"cfg": cfg_id, "instance": instance, "alpha": alpha})


def make_random_junction(n_seps: int = 5, max_vars: int = 2, n_lo: int = 2, n_hi: int = 4, eps: float = 0.3,
                         cfg_id: int = 7, instance: int = 0) -> JunctionProblem:
    """A random modified junction tree for tests: a random tree over n_seps
    separators, each holding 1..max_vars fresh variables with random support
    sizes in [n_lo, n_hi]; each tree edge is a cost clique with a seeded
    uniform cost tensor in [0, 1]; a random half of the separators (at least
    one) are constrained with Dirichlet(1) joint marginals."""
    rng = rng_for(cfg_id, instance)
    sizes, support, seps = [], [], []
    for _ in range(n_seps):
        k = int(rng.integers(1, max_vars + 1))
        vs = []
        for _ in range(k):
            n = int(rng.integers(n_lo, n_hi + 1))
            vs.append(len(sizes))
            sizes.append(n)
            support.append(rng.uniform(0.0, 1.0, size=(n, 1)))
        seps.append(tuple(vs))
    cliques = [(int(rng.integers(0, s)), s) for s in range(1, n_seps)]
    fixed = [bool(b) for b in rng.integers(0, 2, size=n_seps)]
    if not any(fixed):
        fixed[0] = True
    marg: List[Optional[np.ndarray]] = []
    for s in range(n_seps):
        if fixed[s]:
            shape = tuple(sizes[v] for v in seps[s])
            g = rng.exponential(1.0, size=shape)
            marg.append(g / g.sum())
        else:
            marg.append(None)
    costs = []
    for a, b in cliques:
        shape = tuple(sizes[v] for v in seps[a]) + tuple(sizes[v] for v in seps[b])
        costs.append(rng.uniform(0.0, 1.0, size=shape))
    return JunctionProblem(sizes, support, seps, fixed, marg, cliques, costs, float(eps),
                           name=f"rjt-{n_seps}", meta={"cfg": cfg_id, "instance": instance})


def as_tree_problem(jp: JunctionProblem):
    """The same problem written as a tree over separators (plain re-indexing):
    node s = separator s with one support point per joint state (C order over
    its variables), edge c = clique c with its cost tensor read as an
    (states of a) x (states of b) matrix, explicit cost.  The supports are
    placeholders (the state index), as explicit costs do not read them."""
    from .problem import TreeProblem, COST_EXPLICIT
    sizes = np.array([jp.sep_size(s) for s in range(jp.n_separators)], dtype=np.int32)
    support = np.concatenate([np.arange(n, dtype=np.float64).reshape(-1, 1) for n in sizes])
    fixed = np.array([1 if f else 0 for f in jp.sep_fixed], dtype=np.uint8)
    marg = [np.asarray(jp.sep_marginal[s], dtype=np.float64).reshape(-1) for s in range(jp.n_separators)
            if jp.sep_fixed[s]]
    edges = np.array(jp.cliques, dtype=np.int32).reshape(-1, 2)
    cost = [np.asarray(jp.clique_cost[c], dtype=np.float64).reshape(sizes[a], sizes[b])
            for c, (a, b) in enumerate(jp.cliques)]
    return TreeProblem(n_nodes=jp.n_separators, edges=edges, sizes=sizes, dim=1, support=support, is_fixed=fixed,
                       marginal=np.concatenate(marg) if marg else np.zeros(0), eps=jp.eps,
                       cost_kind=COST_EXPLICIT, cost=cost, name=jp.name + "-as-tree", meta=dict(jp.meta))


def from_tree_problem(tp) -> JunctionProblem:
    """A tree problem written as a modified junction tree: one single-variable
    separator per node, one clique per edge whose cost tensor is the edge's
    squared-Euclidean cost matrix (plain re-indexing)."""
    off = tp.offsets()
    supp = [tp.support[off[j]:off[j + 1]].copy() for j in range(tp.n_nodes)]
    costs = []
    for a, b in tp.edges:
        X, Y = supp[int(a)], supp[int(b)]
        costs.append(np.sum((X[:, None, :] - Y[None, :, :]) ** 2, axis=2))
    marg = [tp.node_marginal(j).copy() if tp.is_fixed[j] else None for j in range(tp.n_nodes)]
    return JunctionProblem([int(s) for s in tp.sizes], supp, [(j,) for j in range(tp.n_nodes)],
                           [bool(f) for f in tp.is_fixed], marg, [(int(a), int(b)) for a, b in tp.edges], costs,
                           float(tp.eps), name=tp.name + "-as-junction", meta=dict(tp.meta))
