"""Seeded generators for the five workload shapes.

The paper's experiments (Section 5) use marginals on a uniform grid of d points
in [0, 1] with squared-Euclidean cost; no dataset is involved.  The shapes here
stand in for the paper's barycenter (star) problem and for the HMM-like chain
and random-tree structures named in its introduction.  Every random draw comes
from ``numpy.random.Generator(PCG64(SeedSequence([cfg_id, instance_id])))``.

Recipes
-------
* 1D grid of n points: ``x_i = i / (n - 1)`` (a single point sits at 0).
* 2D grid of n points: ``a = floor(sqrt(n))``, ``b = ceil(n / a)``, points
  ``(i / (a - 1), j / (b - 1))`` row-major, first n kept.
* Gaussian mixture with c components: weights Dirichlet(1), means
  U(0.15, 0.85)^D, isotropic standard deviations U(0.03, 0.10); the
  log-density is evaluated at the support points in float64, floored at 300
  below its maximum (so every entry is strictly positive) and normalised to
  unit mass.
* Dirichlet(1) weights: normalised Exp(1) draws.
* Random trees: a Pruefer sequence of n - 2 uniform draws decoded with the
  textbook smallest-leaf rule.
"""
from __future__ import annotations

import heapq
from typing import List, Optional

import numpy as np

from .problem import TreeProblem, COST_SQEUCLID

CONFIG_NAMES = {
    1: "star-barycenter-3leaf-n64",
    2: "chain-hmm-32node-n1024",
    3: "random-tree-256node-2d",
    4: "batched-stars-512",
    5: "warmstart-star-8leaf-n1024",
}


def rng_for(cfg_id: int, instance_id: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(cfg_id), int(instance_id)])))


def grid_1d(n: int) -> np.ndarray:
    if n == 1:
        return np.zeros((1, 1))
    return (np.arange(n, dtype=np.float64) / (n - 1)).reshape(n, 1)


def grid_2d(n: int) -> np.ndarray:
    a = int(np.floor(np.sqrt(n)))
    b = int(np.ceil(n / a))
    ia = np.arange(a, dtype=np.float64) / max(a - 1, 1)
    ib = np.arange(b, dtype=np.float64) / max(b - 1, 1)
    pts = np.stack(np.meshgrid(ia, ib, indexing="ij"), axis=-1).reshape(-1, 2)
    return np.ascontiguousarray(pts[:n])


def gaussian_mixture(rng: np.random.Generator, pts: np.ndarray, c: int) -> np.ndarray:
    d = pts.shape[1]
    w = rng.exponential(1.0, size=c)
    w = w / w.sum()
    means = rng.uniform(0.15, 0.85, size=(c, d))
    sds = rng.uniform(0.03, 0.10, size=c)
    comp = np.empty((c, pts.shape[0]))
    for i in range(c):
        r2 = np.sum((pts - means[i]) ** 2, axis=1)
        comp[i] = np.log(w[i]) - 0.5 * r2 / sds[i] ** 2 - d * np.log(sds[i]) - 0.5 * d * np.log(2 * np.pi)
    top = comp.max(axis=0)
    ld = top + np.log(np.sum(np.exp(comp - top), axis=0))
    ld = np.maximum(ld, ld.max() - 300.0)
    p = np.exp(ld - ld.max())
    return p / p.sum()


def dirichlet1(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.exponential(1.0, size=n)
    return g / g.sum()


def prufer_decode(seq) -> np.ndarray:
    """Textbook decoding of a Pruefer sequence into n - 1 edges (a < b)."""
    seq = [int(s) for s in seq]
    n = len(seq) + 2
    degree = [1] * n
    for s in seq:
        degree[s] += 1
    leaves = [i for i in range(n) if degree[i] == 1]
    heapq.heapify(leaves)
    edges = []
    for s in seq:
        leaf = heapq.heappop(leaves)
        edges.append((min(leaf, s), max(leaf, s)))
        degree[leaf] -= 1
        degree[s] -= 1
        if degree[s] == 1:
            heapq.heappush(leaves, s)
    u = heapq.heappop(leaves)
    v = heapq.heappop(leaves)
    edges.append((min(u, v), max(u, v)))
    return np.array(edges, dtype=np.int32)


def _assemble(n_nodes, edges, sizes, dim, pts_list, fixed, marg_list, eps, name, meta=None) -> TreeProblem:
    sizes = np.asarray(sizes, dtype=np.int32)
    support = np.ascontiguousarray(np.concatenate(pts_list, axis=0).astype(np.float64))
    is_fixed = np.asarray(fixed, dtype=np.uint8)
    marg = [m for j, m in enumerate(marg_list) if is_fixed[j]]
    marginal = np.ascontiguousarray(np.concatenate(marg) if marg else np.zeros(0))
    return TreeProblem(n_nodes=int(n_nodes), edges=np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2)),
                       sizes=sizes, dim=int(dim), support=support, is_fixed=is_fixed, marginal=marginal,
                       eps=float(eps), cost_kind=COST_SQEUCLID, name=name, meta=dict(meta or {}))


def make_star(n: int = 64, leaves: int = 3, eps: float = 0.01, comps: int = 2, dim: int = 1,
              cfg_id: int = 1, instance: int = 0, sizes: Optional[List[int]] = None) -> TreeProblem:
    """Barycenter star: free center 0, fixed leaves 1..L; all nodes share one grid
    unless ``sizes`` gives per-node support sizes (each on its own grid)."""
    rng = rng_for(cfg_id, instance)
    n_nodes = leaves + 1
    sizes = list(sizes) if sizes is not None else [n] * n_nodes
    grid = grid_1d if dim == 1 else grid_2d
    pts = [grid(s) for s in sizes]
    fixed = [0] + [1] * leaves
    marg = [None] + [gaussian_mixture(rng, pts[j], comps) for j in range(1, n_nodes)]
    edges = [(0, j) for j in range(1, n_nodes)]
    return _assemble(n_nodes, edges, sizes, dim, pts, fixed, marg, eps,
                     f"star-L{leaves}-n{n}-d{dim}", {"cfg": cfg_id, "instance": instance})


def make_chain(n_nodes: int = 32, n: int = 1024, eps: float = 1e-3, every: int = 4, comps: int = 3,
               cfg_id: int = 2, instance: int = 0) -> TreeProblem:
    """HMM-like chain 0-1-...-(N-1); nodes 0, every, 2*every, ... are observed."""
    rng = rng_for(cfg_id, instance)
    pts = [grid_1d(n) for _ in range(n_nodes)]
    fixed = [1 if j % every == 0 else 0 for j in range(n_nodes)]
    marg = [gaussian_mixture(rng, pts[j], comps) if fixed[j] else None for j in range(n_nodes)]
    edges = [(j, j + 1) for j in range(n_nodes - 1)]
    return _assemble(n_nodes, edges, [n] * n_nodes, 1, pts, fixed, marg, eps,
                     f"chain-{n_nodes}-n{n}", {"cfg": cfg_id, "instance": instance})


def make_random_tree(n_nodes: int = 256, n_lo: int = 256, n_hi: int = 4096, eps: float = 5e-3, dim: int = 2,
                     cfg_id: int = 3, instance: int = 0) -> TreeProblem:
    """Random Pruefer tree; leaves are observed with Dirichlet(1) marginals."""
    rng = rng_for(cfg_id, instance)
    seq = rng.integers(0, n_nodes, size=n_nodes - 2)
    edges = prufer_decode(seq)
    sizes = rng.integers(n_lo, n_hi + 1, size=n_nodes)
    grid = grid_1d if dim == 1 else grid_2d
    pts = [grid(int(s)) for s in sizes]
    deg = np.zeros(n_nodes, dtype=np.int64)
    for a, b in edges:
        deg[a] += 1
        deg[b] += 1
    fixed = [1 if deg[j] == 1 else 0 for j in range(n_nodes)]
    marg = [dirichlet1(rng, int(sizes[j])) if fixed[j] else None for j in range(n_nodes)]
    return _assemble(n_nodes, edges, sizes, dim, pts, fixed, marg, eps,
                     f"prufer-{n_nodes}", {"cfg": cfg_id, "instance": instance})


def make_batched_stars(count: int = 512, l_lo: int = 4, l_hi: int = 16, n_lo: int = 128, n_hi: int = 2048,
                       eps: float = 1e-2, comps: int = 2, cfg_id: int = 4, first_instance: int = 0) -> List[TreeProblem]:
    """Independent barycenter stars of uneven size; each instance draws its leaf
    count L, support size n and dimension D, and all its nodes share one grid."""
    out = []
    for i in range(first_instance, first_instance + count):
        rng = rng_for(cfg_id, i)
        L = int(rng.integers(l_lo, l_hi + 1))
        n = int(rng.integers(n_lo, n_hi + 1))
        dim = int(rng.integers(1, 3))
        grid = grid_1d if dim == 1 else grid_2d
        pts = [grid(n) for _ in range(L + 1)]
        fixed = [0] + [1] * L
        marg = [None] + [gaussian_mixture(rng, pts[j], comps) for j in range(1, L + 1)]
        edges = [(0, j) for j in range(1, L + 1)]
        out.append(_assemble(L + 1, edges, [n] * (L + 1), dim, pts, fixed, marg, eps,
                             f"bstar-{i}-L{L}-n{n}-d{dim}", {"cfg": cfg_id, "instance": i}))
    return out


def make_warmstart_star(instance: int, n: int = 1024, leaves: int = 8, eps: float = 1e-2,
                        cfg_id: int = 5) -> TreeProblem:
    """Star with 8 observed leaves; each leaf is a mixture of 1..3 components."""
    rng = rng_for(cfg_id, instance)
    pts = [grid_1d(n) for _ in range(leaves + 1)]
    marg = [None]
    for j in range(1, leaves + 1):
        c = int(rng.integers(1, 4))
        marg.append(gaussian_mixture(rng, pts[j], c))
    edges = [(0, j) for j in range(1, leaves + 1)]
    return _assemble(leaves + 1, edges, [n] * (leaves + 1), 1, pts, [0] + [1] * leaves, marg, eps,
                     f"wstar-{instance}-n{n}", {"cfg": cfg_id, "instance": instance})


def make_lognormal_star(leaves: int, d: int, eps: float, instance: int = 0, cfg_id: int = 8) -> TreeProblem:
    """The barycenter problem of the paper's experiments (Section 5): a free
    center and `leaves` constrained leaves, all on a uniform grid of d points in
    [0, 1], squared-Euclidean cost, leaf marginals drawn from seeded log-normal
    densities (the recipe of workloads.junction.log_normal_marginal)."""
    from .junction import log_normal_marginal
    rng = rng_for(cfg_id, instance)
    pts = [grid_1d(d) for _ in range(leaves + 1)]
    marg = [None] + [log_normal_marginal(rng, pts[j]) for j in range(1, leaves + 1)]
    edges = [(0, j) for j in range(1, leaves + 1)]
    return _assemble(leaves + 1, edges, [d] * (leaves + 1), 1, pts, [0] + [1] * leaves, marg, eps,
                     f"lnstar-L{leaves}-d{d}", {"cfg": cfg_id, "instance": instance})


def make_config(cfg_id: int, scale: str = "full"):
    """Problem(s) for one workload.  ``scale='small'`` keeps the structure but
    shrinks sizes so the FP64 oracle finishes in seconds."""
    small = scale == "small"
    if cfg_id == 1:
        return make_star(n=64, leaves=3, eps=0.01)
    if cfg_id == 2:
        return make_chain(n_nodes=12 if small else 32, n=200 if small else 1024, eps=1e-3)
    if cfg_id == 3:
        if small:
            return make_random_tree(n_nodes=24, n_lo=40, n_hi=300, eps=5e-3)
        return make_random_tree()
    if cfg_id == 4:
        if small:
            return make_batched_stars(count=6, l_lo=2, l_hi=5, n_lo=20, n_hi=300)
        return make_batched_stars()
    if cfg_id == 5:
        return make_warmstart_star(instance=0, n=128 if small else 1024)
    raise ValueError(cfg_id)


def make_tree(edges, sizes, fixed, dim: int = 1, eps: float = 0.3, cfg_id: int = 99, instance: int = 0,
              support: str = "random", marginals: str = "dirichlet") -> TreeProblem:
    """Arbitrary small tree for tests: supports are seeded uniform points in
    [0, 1]^dim (``support='random'``) or grids (``'grid'``); constrained nodes
    get Dirichlet(1) marginals (``'dirichlet'``) or 2-component mixtures (``'gm'``)."""
    rng = rng_for(cfg_id, instance)
    edges = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    n_nodes = len(sizes)
    pts = []
    for s in sizes:
        if support == "random":
            pts.append(rng.uniform(0.0, 1.0, size=(int(s), dim)))
        else:
            pts.append(grid_1d(int(s)) if dim == 1 else grid_2d(int(s)))
    marg = []
    for j in range(n_nodes):
        if not fixed[j]:
            marg.append(None)
        elif marginals == "dirichlet":
            marg.append(dirichlet1(rng, int(sizes[j])))
        else:
            marg.append(gaussian_mixture(rng, pts[j], 2))
    return _assemble(n_nodes, edges, sizes, dim, pts, fixed, marg, eps, f"tree-{n_nodes}",
                     {"cfg": cfg_id, "instance": instance})
