"""Python binding of libgmot (gfx950 solver for tree-structured coupled OT).

Every step of the solver runs in the HIP library; this module only converts
arguments.  Problems are described by any object with the fields of
``workloads.TreeProblem`` (n_nodes, edges, sizes, dim, support, is_fixed,
marginal, eps, cost_kind, cost).  PyTorch is optional: pass a torch CUDA
stream (or its integer handle) to order the library's work on it, and torch
tensors to the ``*_dev`` methods for device-to-device transfers.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (GMOT_OK, GMOT_EINVAL, GMOT_EMARGINAL, GMOT_ENOMEM, GMOT_EDEVICE, GMOT_ENOTSUP, GMOT_ESTATE,
                   GMOT_CONVERGED, GMOT_NOT_CONVERGED, GMOT_NONFINITE, GMOT_COST_SQEUCLID, GMOT_COST_EXPLICIT,
                   GMOT_PREC_FP32CORE, GMOT_PREC_FP64)

STATUS_NAMES = {GMOT_CONVERGED: "converged", GMOT_NOT_CONVERGED: "not_converged", GMOT_NONFINITE: "nonfinite"}
PRECISIONS = {"fp32core": GMOT_PREC_FP32CORE, "fp64": GMOT_PREC_FP64}
SCHEDULES = {"layer": 0, "per_node": 1, "gauss_seidel": 2}
PASSES = {"auto": 0, "one": 1, "two": 2}


class GmotError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = _lib.load()
        msg = lib.gmot_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib.gmot_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def _check(code: int, where: str) -> None:
    if code != GMOT_OK:
        raise GmotError(code, where)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(getattr(stream, "cuda_stream"))


class Context:
    """A device and the stream all library work is ordered on.

    The library counts the problems, batches and networks created on a
    context as references to it, so closing the context (or the garbage
    collector finalising objects of one reference cycle in any order) never
    leaves a live handle on a freed context."""

    def __init__(self, device: int = 0, stream=None):
        self._lib = _lib.load()
        h = C.c_void_p()
        _check(self._lib.gmot_ctx_create(C.byref(h), int(device), _stream_handle(stream)), "gmot_ctx_create")
        self._h = h
        self.device = int(device)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.gmot_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _as(arr, dtype):
    return np.ascontiguousarray(np.asarray(arr, dtype=dtype))


class Problem:
    """One tree instance resident in device memory."""

    def __init__(self, ctx: Context, prob, first_color: int = -1):
        self._lib = ctx._lib
        self.ctx = ctx
        self.n_nodes = int(prob.n_nodes)
        self.edges = _as(prob.edges, np.int32).reshape(-1, 2)
        self.sizes = _as(prob.sizes, np.int32)
        keep = []
        d = _lib.TreeDesc()
        d.n_nodes = self.n_nodes
        d.n_edges = int(self.edges.shape[0])
        e = self.edges.reshape(-1)
        keep.append(e)
        d.edges = e.ctypes.data_as(_lib.I32P)
        keep.append(self.sizes)
        d.sizes = self.sizes.ctypes.data_as(_lib.I32P)
        d.dim = int(prob.dim)
        sup = _as(prob.support, np.float64).reshape(-1)
        keep.append(sup)
        d.support = sup.ctypes.data_as(_lib.DP)
        fx = _as(prob.is_fixed, np.uint8)
        keep.append(fx)
        d.is_fixed = fx.ctypes.data_as(C.POINTER(C.c_uint8))
        mg = _as(prob.marginal, np.float64).reshape(-1)
        keep.append(mg)
        d.marginal = mg.ctypes.data_as(_lib.DP)
        d.cost_kind = int(getattr(prob, "cost_kind", GMOT_COST_SQEUCLID))
        if d.cost_kind == GMOT_COST_EXPLICIT:
            cst = np.ascontiguousarray(np.concatenate([np.asarray(c, dtype=np.float32).reshape(-1) for c in prob.cost]))
            keep.append(cst)
            d.cost = cst.ctypes.data_as(C.POINTER(C.c_float))
        d.eps = float(prob.eps)
        h = C.c_void_p()
        _check(self._lib.gmot_problem_create(ctx._h, C.byref(d), int(first_color), C.byref(h)), "gmot_problem_create")
        self._h = h
        self.n_pot = int(self._lib.gmot_potentials_size(h))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.gmot_problem_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _opts(tol, max_steps, check_every, precision, restart, timing=False, verify=True,
              schedule="layer", passes="auto") -> _lib.Opts:
        o = _lib.Opts()
        o.tol = float(tol)
        o.max_steps = int(max_steps)
        o.check_every = int(check_every)
        o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        o.restart = 1 if restart else 0
        o.timing = 1 if timing else 0
        o.skip_verify = 0 if verify else 1
        o.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
        o.msg_passes = PASSES[passes] if isinstance(passes, str) else int(passes)
        return o

    @staticmethod
    def _stats(fn, h, reset) -> dict:
        st = _lib.Stats()
        _check(fn(h, C.byref(st), 1 if reset else 0), "gmot_*_stats")
        out = {}
        for name, _ in _lib.Stats._fields_:
            v = getattr(st, name)
            if name.startswith("group_"):
                out[name] = [float(x) for x in v]
            else:
                out[name] = float(v) if "ms" in name or "pairs" in name else int(v)
        return out

    def stats(self, reset: bool = False) -> dict:
        """Kernel timing accumulated by solves run with timing=True."""
        return self._stats(self._lib.gmot_problem_stats, self._h, reset)

    @staticmethod
    def _autotune(fn, h) -> dict:
        w, r, g, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        _check(fn(h, C.byref(w), C.byref(r), C.byref(g), C.byref(ms)), "gmot_*_autotune")
        return {"waves_per_block": w.value, "rows_per_lane": r.value, "lane_groups": g.value,
                "ms_per_half_sweep": ms.value}

    def autotune(self) -> dict:
        """Pick the fastest node-kernel block shape for this problem (state untouched)."""
        return self._autotune(self._lib.gmot_problem_autotune, self._h)

    @staticmethod
    def _res(r: _lib.Result) -> dict:
        return {"status": STATUS_NAMES.get(r.status, str(r.status)), "steps": int(r.steps), "t": int(r.t),
                "err_sum": float(r.err_sum), "err_max": float(r.err_max), "seconds": float(r.seconds)}

    def solve(self, tol: float = 1e-6, max_steps: int = 100000, check_every: int = 0, precision="fp32core",
              restart: bool = True, timing: bool = False, verify: bool = True, schedule="layer",
              passes="auto") -> dict:
        o = self._opts(tol, max_steps, check_every, precision, restart, timing, verify, schedule, passes)
        r = _lib.Result()
        _check(self._lib.gmot_solve(self._h, C.byref(o), C.byref(r)), "gmot_solve")
        return self._res(r)

    def evaluate(self) -> dict:
        ev = _lib.Eval()
        _check(self._lib.gmot_evaluate(self._h, C.byref(ev)), "gmot_evaluate")
        return {name: float(getattr(ev, name)) for name, _ in _lib.Eval._fields_}

    def potentials(self) -> np.ndarray:
        out = np.empty(self.n_pot, dtype=np.float64)
        _check(self._lib.gmot_get_potentials(self._h, out.ctypes.data_as(_lib.DP)), "gmot_get_potentials")
        return out

    def set_potentials(self, lam) -> None:
        a = _as(lam, np.float64).reshape(-1)
        if a.shape[0] != self.n_pot:
            raise ValueError(f"expected {self.n_pot} potentials, got {a.shape[0]}")
        _check(self._lib.gmot_set_potentials(self._h, a.ctypes.data_as(_lib.DP)), "gmot_set_potentials")

    def potentials_dev(self, out_tensor) -> None:
        """Copy the potentials into a float64 device tensor (stream-ordered)."""
        if out_tensor.numel() != self.n_pot or str(out_tensor.dtype) != "torch.float64":
            raise ValueError("need a float64 device tensor of potentials_size elements")
        _check(self._lib.gmot_get_potentials_dev(self._h, C.c_void_p(out_tensor.data_ptr())), "gmot_get_potentials_dev")

    def set_potentials_dev(self, in_tensor) -> None:
        if in_tensor.numel() != self.n_pot or str(in_tensor.dtype) != "torch.float64":
            raise ValueError("need a float64 device tensor of potentials_size elements")
        _check(self._lib.gmot_set_potentials_dev(self._h, C.c_void_p(in_tensor.data_ptr())), "gmot_set_potentials_dev")

    def coupling(self, edge: int) -> np.ndarray:
        a, b = self.edges[edge]
        out = np.empty((int(self.sizes[a]), int(self.sizes[b])), dtype=np.float64)
        _check(self._lib.gmot_get_coupling(self._h, int(edge), out.ctypes.data_as(_lib.DP)), "gmot_get_coupling")
        return out

    def node_marginal(self, node: int) -> np.ndarray:
        out = np.empty(int(self.sizes[node]), dtype=np.float64)
        _check(self._lib.gmot_get_node_marginal(self._h, int(node), out.ctypes.data_as(_lib.DP)),
               "gmot_get_node_marginal")
        return out

    def round(self) -> dict:
        """gmot_round: rounded transport, per-edge transport, err_side, c_inf, side."""
        r = _lib.RoundResult()
        per_edge = np.zeros(max(len(self.edges), 1), dtype=np.float64)
        _check(self._lib.gmot_round(self._h, C.byref(r), per_edge.ctypes.data_as(_lib.DP)), "gmot_round")
        return {"transport": r.transport, "edge_transport": per_edge[:len(self.edges)].copy(),
                "err_side": r.err_side, "c_inf": r.c_inf, "side": r.side}

    def rounded_coupling(self, edge: int) -> np.ndarray:
        a, b = self.edges[edge]
        out = np.empty((int(self.sizes[a]), int(self.sizes[b])), dtype=np.float64)
        _check(self._lib.gmot_get_rounded_coupling(self._h, int(edge), out.ctypes.data_as(_lib.DP)),
               "gmot_get_rounded_coupling")
        return out


class JunctionTree(Problem):
    """A coupled MOT problem on a modified junction tree (gmot_junction_create),
    from any object with the fields of ``workloads.JunctionProblem``.  It is a
    Problem over separators: potentials in clique order, couplings are clique
    plans as (states of a) x (states of b) matrices, node marginals are
    separator marginals (flattened in C order)."""

    def __init__(self, ctx: Context, jp, first_color: int = -1):
        self._lib = ctx._lib
        self.ctx = ctx
        keep = []
        d = _lib.JunctionDesc()
        vs = _as(jp.var_sizes, np.int32)
        keep.append(vs)
        d.n_vars = int(vs.shape[0])
        d.var_sizes = vs.ctypes.data_as(_lib.I32P)
        seps = [tuple(int(v) for v in sv) for sv in jp.separators]
        nv = _as([len(sv) for sv in seps], np.int32)
        sv = _as([v for t in seps for v in t], np.int32)
        keep += [nv, sv]
        d.n_seps = len(seps)
        d.sep_nvars = nv.ctypes.data_as(_lib.I32P)
        d.sep_vars = sv.ctypes.data_as(_lib.I32P)
        fx = _as([1 if f else 0 for f in jp.sep_fixed], np.uint8)
        keep.append(fx)
        d.sep_fixed = fx.ctypes.data_as(C.POINTER(C.c_uint8))
        mg = [np.asarray(jp.sep_marginal[s], dtype=np.float64).reshape(-1) for s in range(len(seps)) if jp.sep_fixed[s]]
        mg = _as(np.concatenate(mg) if mg else np.zeros(1), np.float64)
        keep.append(mg)
        d.sep_marginal = mg.ctypes.data_as(_lib.DP)
        cl = _as(jp.cliques, np.int32).reshape(-1)
        keep.append(cl)
        d.n_cliques = len(jp.cliques)
        d.cliques = cl.ctypes.data_as(_lib.I32P)
        cost = [np.asarray(c, dtype=np.float32).reshape(-1) for c in jp.clique_cost]
        cst = _as(np.concatenate(cost) if cost else np.zeros(1), np.float32)
        keep.append(cst)
        d.clique_cost = cst.ctypes.data_as(C.POINTER(C.c_float))
        d.eps = float(jp.eps)
        h = C.c_void_p()
        _check(self._lib.gmot_junction_create(ctx._h, C.byref(d), int(first_color), C.byref(h)),
               "gmot_junction_create")
        self._h = h
        self.n_nodes = len(seps)
        self.edges = _as(jp.cliques, np.int32).reshape(-1, 2)
        self.sizes = _as([int(np.prod([jp.var_sizes[v] for v in t])) for t in seps], np.int32)
        self.n_pot = int(self._lib.gmot_potentials_size(h))


class Batch:
    """Many problems advanced by the same launches."""

    def __init__(self, ctx: Context, problems: Sequence[Problem]):
        self._lib = ctx._lib
        self.ctx = ctx
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[p._h.value for p in self.problems])
        h = C.c_void_p()
        _check(self._lib.gmot_batch_create(ctx._h, arr, len(self.problems), C.byref(h)), "gmot_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.gmot_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, tol: float = 1e-6, max_steps: int = 100000, check_every: int = 0, precision="fp32core",
              restart: bool = True, timing: bool = False, verify: bool = True, schedule="layer",
              passes="auto") -> List[dict]:
        o = Problem._opts(tol, max_steps, check_every, precision, restart, timing, verify, schedule, passes)
        rs = (_lib.Result * len(self.problems))()
        _check(self._lib.gmot_batch_solve(self._h, C.byref(o), rs), "gmot_batch_solve")
        return [Problem._res(r) for r in rs]

    def evaluate(self) -> List[dict]:
        """gmot_batch_evaluate: every instance's FP64 objective values in shared launches."""
        evs = (_lib.Eval * len(self.problems))()
        _check(self._lib.gmot_batch_evaluate(self._h, evs), "gmot_batch_evaluate")
        return [{name: float(getattr(ev, name)) for name, _ in _lib.Eval._fields_} for ev in evs]

    def stats(self, reset: bool = False) -> dict:
        return Problem._stats(self._lib.gmot_batch_stats, self._h, reset)

    def autotune(self) -> dict:
        return Problem._autotune(self._lib.gmot_batch_autotune, self._h)


def _handles(problems) -> "C.Array":
    return (C.c_void_p * len(problems))(*[p._h.value for p in problems])


def _dptr(t) -> C.c_void_p:
    """Device pointer of a contiguous float32 torch tensor."""
    if str(t.dtype) != "torch.float32" or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("need a contiguous float32 device tensor")
    return C.c_void_p(t.data_ptr())


class MLP:
    """Warm-start network trained and run by the library's HIP kernels."""

    def __init__(self, ctx: Context, widths: Sequence[int], seed: int = 0):
        self._lib = ctx._lib
        self.ctx = ctx
        self.widths = [int(w) for w in widths]
        arr = (C.c_int32 * len(self.widths))(*self.widths)
        h = C.c_void_p()
        _check(self._lib.gmot_mlp_create(ctx._h, len(self.widths) - 1, arr, int(seed), C.byref(h)), "gmot_mlp_create")
        self._h = h
        self.n_params = int(self._lib.gmot_mlp_num_params(h))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.gmot_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        _check(self._lib.gmot_mlp_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float))), "gmot_mlp_get_params")
        return out

    def set_params(self, p) -> None:
        a = _as(p, np.float32).reshape(-1)
        if a.shape[0] != self.n_params:
            raise ValueError("wrong parameter count")
        _check(self._lib.gmot_mlp_set_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float))), "gmot_mlp_set_params")

    def forward(self, x, y) -> None:
        _check(self._lib.gmot_mlp_forward_dev(self._h, _dptr(x), int(x.shape[0]), _dptr(y)), "gmot_mlp_forward_dev")

    def forward_static(self, x, y) -> None:
        """gmot_mlp_forward_static: the forward pass with no allocation (static workspace)."""
        _check(self._lib.gmot_mlp_forward_static(self._h, _dptr(x), int(x.shape[0]), _dptr(y)),
               "gmot_mlp_forward_static")

    def loss_grad(self, x, t, grad=None) -> float:
        loss = C.c_double()
        g = _dptr(grad) if grad is not None else None
        _check(self._lib.gmot_mlp_loss_grad_dev(self._h, _dptr(x), _dptr(t), int(x.shape[0]), C.byref(loss), g),
               "gmot_mlp_loss_grad_dev")
        return loss.value

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        _check(self._lib.gmot_mlp_adam_step(self._h, lr, beta1, beta2, eps), "gmot_mlp_adam_step")

    def train_step(self, x, t, lr: float) -> float:
        loss = C.c_double()
        _check(self._lib.gmot_mlp_train_step_dev(self._h, _dptr(x), _dptr(t), int(x.shape[0]), lr, C.byref(loss)),
               "gmot_mlp_train_step_dev")
        return loss.value

    def warm_start(self, problems: Sequence[Problem], shift: float, scale: float, out_scale: float) -> int:
        rej = C.c_int32()
        _check(self._lib.gmot_mlp_warm_start(self._h, _handles(problems), len(problems), shift, scale, out_scale,
                                             C.byref(rej)), "gmot_mlp_warm_start")
        return rej.value


def star_features(problems: Sequence[Problem], x, shift: float, scale: float) -> None:
    lib = _lib.load()
    _check(lib.gmot_star_features_dev(_handles(problems), len(problems), shift, scale, _dptr(x)), "gmot_star_features_dev")


def star_targets(problems: Sequence[Problem], t, out_scale: float) -> None:
    lib = _lib.load()
    _check(lib.gmot_star_targets_dev(_handles(problems), len(problems), out_scale, _dptr(t)), "gmot_star_targets_dev")


def star_apply(problems: Sequence[Problem], y, out_scale: float) -> int:
    lib = _lib.load()
    rej = C.c_int32()
    _check(lib.gmot_star_apply_dev(_handles(problems), len(problems), _dptr(y), out_scale, C.byref(rej)),
           "gmot_star_apply_dev")
    return rej.value


def last_tiles() -> dict:
    lib = _lib.load()
    v = [C.c_int32() for _ in range(4)]
    lib.gmot_last_tiles(*[C.byref(x) for x in v])
    return {"rows_per_block": v[0].value, "waves_per_block": v[1].value, "blocks_c0": v[2].value,
            "blocks_c1": v[3].value}


__all__ = ["Context", "Problem", "JunctionTree", "Batch", "MLP", "GmotError", "last_tiles", "star_features", "star_targets",
           "star_apply", "STATUS_NAMES"]
