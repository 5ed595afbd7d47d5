"""FP64 reference of the rounding step (test infrastructure only).

Algorithm "round" of the paper: after a half-sweep that updated the colour
class opposite to S, the plans B_(j,k) with j in S miss their marginal on j's
side.  Every such plan is rounded onto the transport polytope whose row
marginal is the target on j's side -- mu_j for a constrained node, the
arithmetic mean q_bar_j = mean_k B_(j,k) 1 for a free node -- and whose
column marginal is the plan's current column marginal B_(j,k)^T 1, with the
rounding of Altschuler, Weed and Rigollet (NeurIPS 2017, their Algorithm 2):

    X = diag(min(r / (F 1), 1)),      F' = X F
    Y = diag(min(c / (F'^T 1), 1)),   F'' = F' Y
    e_r = r - F'' 1,  e_c = c - F''^T 1,
    G = F'' + e_r e_c^T / ||e_r||_1   (G = F'' when e_r = 0).

The result has exactly the marginals (r, c), and Lemma "round" bounds the
change of the transport cost by 2 C_inf times the stopping sum.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np


def awr_round(F: np.ndarray, r: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Altschuler-Weed-Rigollet rounding of F onto the polytope U(r, c)."""
    rf = F.sum(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        x = np.where(rf > 0, np.minimum(r / rf, 1.0), 1.0)
    F1 = x[:, None] * F
    cf = F1.sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        y = np.where(cf > 0, np.minimum(c / cf, 1.0), 1.0)
    F2 = F1 * y[None, :]
    er = r - F2.sum(axis=1)
    ec = c - F2.sum(axis=0)
    s = er.sum()
    if s <= 0:
        return F2
    return F2 + np.outer(er, ec) / s


def round_plans(oracle, side: List[int]) -> Dict[int, np.ndarray]:
    """Rounded plans of every edge, as n_a x n_b matrices keyed by edge id.

    ``side`` is the class S whose marginals mismatch (the one not updated
    last); edges are rounded on their S end, the other end's marginal kept."""
    p = oracle.prob
    out = {}
    S = set(side)
    for e in range(p.n_edges):
        a, b = int(p.edges[e][0]), int(p.edges[e][1])
        B = oracle.coupling(e)
        j = a if a in S else b
        k = b if j == a else a
        Bjk = B if j == a else B.T                 # rows on j
        if p.is_fixed[j]:
            r = oracle.mu[j]
        else:
            qs = []
            for kk in oracle.nbrs[j]:
                ee = oracle.edge_of[(j, kk)]
                Be = oracle.coupling(ee)
                qs.append(Be.sum(axis=1) if int(p.edges[ee][0]) == j else Be.sum(axis=0))
            r = np.mean(np.stack(qs), axis=0)
        G = awr_round(Bjk, r, Bjk.sum(axis=0))
        out[e] = G if j == a else G.T
    return out


def rounded_transport(oracle, side: List[int]) -> Tuple[float, Dict[int, np.ndarray]]:
    plans = round_plans(oracle, side)
    T = sum(float(np.sum(oracle.cost(int(oracle.prob.edges[e][0]), int(oracle.prob.edges[e][1])) * G))
            for e, G in plans.items())
    return T, plans
