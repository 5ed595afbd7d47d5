"""ctypes declarations of libgmot's C ABI (include/gmot.h); marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmot.so")

GMOT_OK = 0
GMOT_EINVAL = -1
GMOT_EMARGINAL = -2
GMOT_ENOMEM = -3
GMOT_EDEVICE = -4
GMOT_ENOTSUP = -5
GMOT_ESTATE = -6

GMOT_CONVERGED = 0
GMOT_NOT_CONVERGED = 1
GMOT_NONFINITE = 2

GMOT_COST_SQEUCLID = 0
GMOT_COST_EXPLICIT = 1

GMOT_PREC_FP32CORE = 0
GMOT_PREC_FP64 = 1


class TreeDesc(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32),
        ("n_edges", C.c_int32),
        ("edges", C.POINTER(C.c_int32)),
        ("sizes", C.POINTER(C.c_int32)),
        ("dim", C.c_int32),
        ("support", C.POINTER(C.c_double)),
        ("is_fixed", C.POINTER(C.c_uint8)),
        ("marginal", C.POINTER(C.c_double)),
        ("cost_kind", C.c_int32),
        ("cost", C.POINTER(C.c_float)),
        ("eps", C.c_double),
    ]


class JunctionDesc(C.Structure):
    _fields_ = [
        ("n_vars", C.c_int32),
        ("var_sizes", C.POINTER(C.c_int32)),
        ("n_seps", C.c_int32),
        ("sep_nvars", C.POINTER(C.c_int32)),
        ("sep_vars", C.POINTER(C.c_int32)),
        ("sep_fixed", C.POINTER(C.c_uint8)),
        ("sep_marginal", C.POINTER(C.c_double)),
        ("n_cliques", C.c_int32),
        ("cliques", C.POINTER(C.c_int32)),
        ("clique_cost", C.POINTER(C.c_float)),
        ("eps", C.c_double),
    ]


class Opts(C.Structure):
    _fields_ = [
        ("tol", C.c_double),
        ("max_steps", C.c_int64),
        ("check_every", C.c_int32),
        ("precision", C.c_int32),
        ("restart", C.c_int32),
        ("timing", C.c_int32),
        ("skip_verify", C.c_int32),
        ("schedule", C.c_int32),
        ("msg_passes", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("msg_ms", C.c_double),
        ("sweep_ms", C.c_double),
        ("msg_launches", C.c_int64),
        ("msg_pairs", C.c_double),
        ("graph_launches", C.c_int64),
        ("group_ms", C.c_double * 7),
        ("group_pairs", C.c_double * 7),
    ]


class Result(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("reserved", C.c_int32),
        ("steps", C.c_int64),
        ("t", C.c_int64),
        ("err_sum", C.c_double),
        ("err_max", C.c_double),
        ("seconds", C.c_double),
    ]


class Eval(C.Structure):
    _fields_ = [
        ("dual", C.c_double), ("primal", C.c_double), ("transport", C.c_double), ("gap", C.c_double),
        ("err_sum", C.c_double), ("err_max", C.c_double), ("mass_min", C.c_double), ("mass_max", C.c_double),
        ("rho_spread", C.c_double), ("scale", C.c_double),
    ]


class RoundResult(C.Structure):
    _fields_ = [
        ("transport", C.c_double), ("err_side", C.c_double), ("c_inf", C.c_double),
        ("side", C.c_int32), ("reserved", C.c_int32),
    ]


VP = C.c_void_p
I32P = C.POINTER(C.c_int32)
DP = C.POINTER(C.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "gmot_ctx_create": (C.c_int, [C.POINTER(VP), C.c_int, VP]),
    "gmot_ctx_destroy": (None, [VP]),
    "gmot_problem_create": (C.c_int, [VP, C.POINTER(TreeDesc), C.c_int32, C.POINTER(VP)]),
    "gmot_junction_create": (C.c_int, [VP, C.POINTER(JunctionDesc), C.c_int32, C.POINTER(VP)]),
    "gmot_problem_destroy": (None, [VP]),
    "gmot_solve": (C.c_int, [VP, C.POINTER(Opts), C.POINTER(Result)]),
    "gmot_evaluate": (C.c_int, [VP, C.POINTER(Eval)]),
    "gmot_potentials_size": (C.c_int64, [VP]),
    "gmot_get_potentials": (C.c_int, [VP, DP]),
    "gmot_set_potentials": (C.c_int, [VP, DP]),
    "gmot_get_potentials_dev": (C.c_int, [VP, VP]),
    "gmot_set_potentials_dev": (C.c_int, [VP, VP]),
    "gmot_get_coupling": (C.c_int, [VP, C.c_int32, DP]),
    "gmot_get_node_marginal": (C.c_int, [VP, C.c_int32, DP]),
    "gmot_round": (C.c_int, [VP, C.POINTER(RoundResult), DP]),
    "gmot_get_rounded_coupling": (C.c_int, [VP, C.c_int32, DP]),
    "gmot_batch_create": (C.c_int, [VP, C.POINTER(VP), C.c_int32, C.POINTER(VP)]),
    "gmot_batch_destroy": (None, [VP]),
    "gmot_batch_solve": (C.c_int, [VP, C.POINTER(Opts), C.POINTER(Result)]),
    "gmot_batch_evaluate": (C.c_int, [VP, C.POINTER(Eval)]),
    "gmot_strerror": (C.c_char_p, [C.c_int]),
    "gmot_last_error": (C.c_char_p, []),
    "gmot_last_tiles": (C.c_int, [I32P, I32P, I32P, I32P]),
    "gmot_mlp_create": (C.c_int, [VP, C.c_int32, I32P, C.c_uint64, C.POINTER(VP)]),
    "gmot_mlp_destroy": (None, [VP]),
    "gmot_mlp_num_params": (C.c_int64, [VP]),
    "gmot_mlp_get_params": (C.c_int, [VP, C.POINTER(C.c_float)]),
    "gmot_mlp_set_params": (C.c_int, [VP, C.POINTER(C.c_float)]),
    "gmot_mlp_forward_dev": (C.c_int, [VP, VP, C.c_int32, VP]),
    "gmot_mlp_forward_static": (C.c_int, [VP, VP, C.c_int32, VP]),
    "gmot_mlp_loss_grad_dev": (C.c_int, [VP, VP, VP, C.c_int32, DP, VP]),
    "gmot_mlp_adam_step": (C.c_int, [VP, C.c_float, C.c_float, C.c_float, C.c_float]),
    "gmot_mlp_train_step_dev": (C.c_int, [VP, VP, VP, C.c_int32, C.c_float, DP]),
    "gmot_mlp_last_error": (C.c_char_p, []),
    "gmot_star_features_dev": (C.c_int, [C.POINTER(VP), C.c_int32, C.c_float, C.c_float, VP]),
    "gmot_star_targets_dev": (C.c_int, [C.POINTER(VP), C.c_int32, C.c_float, VP]),
    "gmot_star_apply_dev": (C.c_int, [C.POINTER(VP), C.c_int32, VP, C.c_float, I32P]),
    "gmot_mlp_warm_start": (C.c_int, [VP, C.POINTER(VP), C.c_int32, C.c_float, C.c_float, C.c_float, I32P]),
    "gmot_problem_autotune": (C.c_int, [VP, I32P, I32P, I32P, DP]),
    "gmot_batch_autotune": (C.c_int, [VP, I32P, I32P, I32P, DP]),
    "gmot_problem_stats": (C.c_int, [VP, C.POINTER(Stats), C.c_int32]),
    "gmot_batch_stats": (C.c_int, [VP, C.POINTER(Stats), C.c_int32]),
}

_LIB = None


def load() -> C.CDLL:
    """Load the in-tree libgmot.so; raise if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libgmot.so is not built ({LIB_PATH}); run `python -m paper_2406_10849_amd.build`")
    # PyTorch wheels carry their own HIP runtime with the same soname.  Loading
    # torch first makes libgmot bind to that runtime, so the process holds one
    # HIP runtime and torch streams and device pointers can be passed in; the
    # other order would load a second runtime next to torch's.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
