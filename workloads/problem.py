"""Plain container for one tree-structured coupled OT instance.

Fields follow the problem statement of Section 3 (coupled bi-marginal OT on a
tree, with the given marginals on the node set Gamma):

* ``edges[e] = (a, b)``: the coupling of edge ``e`` is an ``n_a x n_b`` matrix
  whose rows index the support of ``a``.
* ``support``: per-node point clouds, concatenated in node order, shape
  ``[sum_j n_j, dim]``, float64.  Used when ``cost_kind == COST_SQEUCLID``
  (cost ``|x - y|^2``).
* ``is_fixed[j]``: 1 when node ``j`` is in Gamma (its marginal is given).
* ``marginal``: concatenated given marginals of the fixed nodes, in node
  order, float64; each block is non-negative and sums to one.
* ``cost``: for ``COST_EXPLICIT``, a list of per-edge ``n_a x n_b`` float32
  matrices in edge order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

COST_SQEUCLID = 0
COST_EXPLICIT = 1


@dataclass
class TreeProblem:
    n_nodes: int
    edges: np.ndarray            # int32 [n_edges, 2]
    sizes: np.ndarray            # int32 [n_nodes]
    dim: int
    support: np.ndarray          # float64 [sum n, dim]
    is_fixed: np.ndarray         # uint8 [n_nodes]
    marginal: np.ndarray         # float64 [sum_{fixed} n]
    eps: float
    cost_kind: int = COST_SQEUCLID
    cost: Optional[List[np.ndarray]] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    # ---- plain indexing helpers (no solver arithmetic) ----
    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    def offsets(self) -> np.ndarray:
        off = np.zeros(self.n_nodes + 1, dtype=np.int64)
        off[1:] = np.cumsum(self.sizes)
        return off

    def node_support(self, j: int) -> np.ndarray:
        off = self.offsets()
        return self.support[off[j]:off[j + 1]]

    def marginal_offsets(self) -> np.ndarray:
        """Offset of node j's block inside ``marginal`` (-1 for free nodes)."""
        out = np.full(self.n_nodes, -1, dtype=np.int64)
        o = 0
        for j in range(self.n_nodes):
            if self.is_fixed[j]:
                out[j] = o
                o += int(self.sizes[j])
        return out

    def node_marginal(self, j: int) -> np.ndarray:
        mo = self.marginal_offsets()
        if mo[j] < 0:
            raise ValueError(f"node {j} is not constrained")
        return self.marginal[mo[j]:mo[j] + int(self.sizes[j])]

    def pairs_per_tstep(self) -> int:
        """Number of (x, y) pairs one half-sweep touches: every edge carries
        exactly one message per half-sweep, of size n_a * n_b."""
        return int(sum(int(self.sizes[a]) * int(self.sizes[b]) for a, b in self.edges))
