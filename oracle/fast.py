"""The FP64 oracle with its message log-sum-exp in plain C (test infrastructure).

``FastTreeOracle`` is ``TreeOracle`` with one step, the message
``m_{k->j} = log K_(j,k)(u_(k,j) * gamma_k)`` (Theorem tree_dual_var, eq. q),
computed by ``oracle/lse.c`` instead of numpy: the same two-pass stabilised sum
per row in FP64, rows spread over host threads.  Everything else (update,
stopping sum, objectives) is the numpy oracle's.  It exists for workloads the
numpy oracle is too slow for (the 256-node tree, converged references) and for
timing the oracle on every host core.  The test suite runs every oracle pin
against it as well.

Only the test suite, the smoke entry point and the benchmark's CPU-baseline
leg may import this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from workloads.problem import COST_SQEUCLID, COST_EXPLICIT

from .tree_ot import TreeOracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lse.c")
LIB = os.path.join(HERE, "liboracle_lse.so")

_lib = None


def build() -> str:
    """Compile oracle/lse.c with gcc (plain -O2, no fast-math: libm exp/log)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", SRC, "-o", tmp, "-lm"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle build failed: {' '.join(cmd)}\n{r.stdout}")
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_message_sqeuclid.argtypes = [dp, dp, dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                                ctypes.c_double, dp, ctypes.c_int]
        lib.oracle_message_sqeuclid.restype = None
        lib.oracle_message_explicit.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int, dp, ctypes.c_int64,
                                                ctypes.c_int64, ctypes.c_double, dp, ctypes.c_int]
        lib.oracle_message_explicit.restype = None
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(load().oracle_max_threads())


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class FastTreeOracle(TreeOracle):
    """TreeOracle whose messages are summed in C; ``threads`` host threads
    (0: all the OpenMP runtime offers)."""

    threads = 0

    def __init__(self, prob, first_color=None, threads=None):
        super().__init__(prob, first_color)
        if threads is not None:
            self.threads = int(threads)
        self._lib = load()
        self._sup = [np.ascontiguousarray(prob.node_support(j), dtype=np.float64) for j in range(prob.n_nodes)] \
            if prob.cost_kind == COST_SQEUCLID else None
        self._cost32 = None
        if prob.cost_kind == COST_EXPLICIT:
            self._cost32 = [np.ascontiguousarray(c, dtype=np.float32) for c in prob.cost]

    def message(self, k: int, j: int, Lam=None) -> np.ndarray:
        Lam = self.Lam if Lam is None else Lam
        w = np.ascontiguousarray(Lam[(k, j)] + self.log_gamma[k], dtype=np.float64)
        n_dst, n_src = int(self.prob.sizes[j]), int(self.prob.sizes[k])
        out = np.empty(n_dst)
        if self.prob.cost_kind == COST_SQEUCLID:
            self._lib.oracle_message_sqeuclid(_dp(self._sup[j]), _dp(self._sup[k]), _dp(w), n_dst, n_src,
                                              int(self.prob.dim), self.eps, _dp(out), int(self.threads))
        else:
            e = self.edge_of[(j, k)]
            a = int(self.prob.edges[e][0])
            C = self._cost32[e]
            self._lib.oracle_message_explicit(C.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), 0 if a == j else 1,
                                              _dp(w), n_dst, n_src, self.eps, _dp(out), int(self.threads))
        return out
