"""Seeded synthetic inputs for tree-structured coupled bi-marginal OT.

This package builds problem descriptions only: tree topology, per-node support
points, the given marginals of the constrained nodes and the regularisation
parameter. It holds none of the solver's arithmetic, so both the FP64 CPU
oracle and the HIP path can consume it without sharing any method code.
"""
from .problem import TreeProblem, COST_SQEUCLID, COST_EXPLICIT
from .gen import (
    rng_for,
    grid_1d,
    grid_2d,
    gaussian_mixture,
    dirichlet1,
    prufer_decode,
    make_star,
    make_chain,
    make_random_tree,
    make_batched_stars,
    make_warmstart_star,
    make_lognormal_star,
    make_config,
    make_tree,
    CONFIG_NAMES,
)
from .junction import JunctionProblem, make_wls, make_random_junction, as_tree_problem, from_tree_problem

__all__ = [
    "TreeProblem", "COST_SQEUCLID", "COST_EXPLICIT", "rng_for", "grid_1d",
    "grid_2d", "gaussian_mixture", "dirichlet1", "prufer_decode", "make_star",
    "make_chain", "make_random_tree", "make_batched_stars",
    "make_warmstart_star", "make_lognormal_star", "make_config", "make_tree", "CONFIG_NAMES", "JunctionProblem", "make_wls",
    "make_random_junction", "as_tree_problem", "from_tree_problem",
]
