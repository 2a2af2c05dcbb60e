"""ctypes binding of libnmpc.so (argument marshalling only).

Every function keeps the C name and signature of include/nmpc.h.  Loading
fails loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmpc.so")

NMPC_OK = 0
NMPC_MAX_ITER, NMPC_LINESEARCH_FAIL, NMPC_REG_FAIL, NMPC_NONFINITE = 1, 2, 3, 4
NMPC_ERR_INVALID_ARG, NMPC_ERR_BAD_ORDER, NMPC_ERR_STRUCT_MISMATCH = -1, -2, -3
NMPC_ERR_NO_DEVICE, NMPC_ERR_HIP, NMPC_ERR_OOM, NMPC_ERR_UNSUPPORTED = -4, -5, -6, -7
NMPC_FAMILY_DISTILLATION, NMPC_FAMILY_HEATED_PLATE, NMPC_FAMILY_REFLUX_COLUMN, NMPC_FAMILY_STAGE_MODEL = 1, 2, 3, 4
NMPC_ORDER_NESTED_DISSECTION, NMPC_ORDER_MIN_DEGREE, NMPC_ORDER_FAMILY_DISSECTION = 0, 1, 2
NMPC_KKT_LIFTED, NMPC_KKT_HYKKT = 0, 1


class nmpc_stage_model(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nu", C.c_int32), ("na", C.c_int32), ("n_alg_rows", C.c_int32),
                ("n_setpoint", C.c_int32), ("uses_traj", C.c_int32),
                ("row_ptr", C.POINTER(C.c_int32)), ("row_cols", C.POINTER(C.c_int32)),
                ("prev_ptr", C.POINTER(C.c_int32)), ("prev_cols", C.POINTER(C.c_int32)),
                ("prev_coef", C.POINTER(C.c_double)), ("n_ineq_rows", C.c_int32),
                ("ineq_ptr", C.POINTER(C.c_int32)), ("ineq_cols", C.POINTER(C.c_int32)), ("nw", C.c_int32),
                ("w_rows", C.POINTER(C.c_int32)), ("w_cols", C.POINTER(C.c_int32)), ("nw_cross", C.c_int32),
                ("wx_rows", C.POINTER(C.c_int32)), ("wx_cols", C.POINTER(C.c_int32)),
                ("lb", C.POINTER(C.c_double)), ("ub", C.POINTER(C.c_double)),
                ("code_object", C.c_void_p), ("code_object_size", C.c_uint64), ("tag", C.c_uint64),
                ("scratch_per_stage", C.c_int64)]


class nmpc_structure(C.Structure):
    _fields_ = [("family", C.c_int32), ("horizon", C.c_int32), ("dt", C.c_double),
                ("n_trays", C.c_int32), ("alpha", C.c_double), ("feed_flow", C.c_double),
                ("move_penalty", C.c_double), ("x_lo", C.c_double), ("x_hi", C.c_double),
                ("u_lo", C.c_double), ("u_hi", C.c_double),
                ("grid", C.c_int32), ("t_hi", C.c_double), ("c_lo", C.c_double), ("c_hi", C.c_double),
                ("cond_slope", C.c_double), ("ordering", C.c_int32), ("control_horizon", C.c_int32),
                ("feed_tray", C.c_int32), ("distillate", C.c_double), ("feed_comp", C.c_double),
                ("hold_cond", C.c_double), ("hold_tray", C.c_double), ("hold_reb", C.c_double),
                ("u_weight", C.c_double), ("flow_hi", C.c_double),
                ("stage_model", C.POINTER(nmpc_stage_model))]


class nmpc_options(C.Structure):
    _fields_ = [("tol", C.c_double), ("gamma", C.c_double), ("mu0_cold", C.c_double),
                ("mu0_warm", C.c_double), ("mu_min", C.c_double), ("kappa_eps", C.c_double),
                ("kappa_mu", C.c_double), ("theta_mu", C.c_double), ("tau_min", C.c_double),
                ("armijo", C.c_double), ("ls_max", C.c_int32), ("max_iter", C.c_int32),
                ("kappa_sigma", C.c_double), ("eta_first", C.c_double), ("eta_min", C.c_double),
                ("eta_max", C.c_double), ("kp_first", C.c_double), ("kp", C.c_double), ("km", C.c_double),
                ("bound_push", C.c_double), ("slack_push", C.c_double),
                ("filter_gamma_theta", C.c_double), ("filter_gamma_phi", C.c_double),
                ("filter_s_theta", C.c_double), ("filter_s_phi", C.c_double), ("filter_delta", C.c_double),
                ("alpha_min_frac", C.c_double), ("theta_max_fact", C.c_double), ("theta_min_fact", C.c_double),
                ("filter_cap", C.c_int32), ("soc_max", C.c_int32), ("soc_kappa", C.c_double),
                ("merit_fallback", C.c_int32), ("timing", C.c_int32), ("graph", C.c_int32),
                ("fixed_mu", C.c_int32), ("kkt", C.c_int32), ("hykkt_gamma", C.c_double),
                ("hykkt_cg_tol", C.c_double), ("hykkt_cg_max", C.c_int32)]


class nmpc_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("factorizations", C.c_int32),
                ("ls_trials", C.c_int32), ("mu", C.c_double), ("eta", C.c_double), ("E0", C.c_double),
                ("objective", C.c_double), ("ms_total", C.c_double), ("ms_eval", C.c_double),
                ("ms_assemble", C.c_double), ("ms_factor", C.c_double), ("ms_solve", C.c_double),
                ("ms_linesearch", C.c_double), ("factor_launches", C.c_int32), ("passes", C.c_int32),
                ("timing_lost", C.c_int32), ("cg_iters", C.c_int32)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)
_L = C.POINTER(C.c_int64)

SIGNATURES = {
    "nmpc_default_options": (None, [C.POINTER(nmpc_options)]),
    "nmpc_create_problem": (C.c_int32, [C.POINTER(nmpc_structure), C.POINTER(_P)]),
    "nmpc_destroy": (None, [_P]),
    "nmpc_sizes": (C.c_int32, [_P, _I, _I, _I, _I, _I, _L]),
    "nmpc_analyze": (C.c_int32, [_P]),
    "nmpc_symbolic_sizes": (C.c_int32, [_P, _I, _L, _L, _L, _L, _I]),
    "nmpc_export_symbolic": (C.c_int32, [_P, _I, _I, _I, _I, _L, _I]),
    "nmpc_pattern_sizes": (C.c_int32, [_P, _L, _L, _L]),
    "nmpc_export_patterns": (C.c_int32, [_P, _I, _I, _I, _I, _I, _I]),
    "nmpc_set_parameters": (C.c_int32, [_P, _D, _D, _D, _D]),
    "nmpc_solve": (C.c_int32, [_P, C.c_int32, C.POINTER(nmpc_options), C.POINTER(nmpc_result)]),
    "nmpc_get_solution": (C.c_int32, [_P, _D, _D, _D, _D, _D, _D, _D]),
    "nmpc_get_iterate": (C.c_int32, [_P, _D, _D, _D, _D, _D, _D]),
    "nmpc_set_iterate": (C.c_int32, [_P, _D, _D, _D, _D, _D, _D]),
    "nmpc_eval": (C.c_int32, [_P, _D, _D, _D, _D, _D, _D, _D, _D, _D]),
    "nmpc_factor": (C.c_int32, [_P, _D, C.c_double, _I, _D]),
    "nmpc_linear_solve": (C.c_int32, [_P, _D, _D]),
    "nmpc_assemble": (C.c_int32, [_P, C.c_double, _D, _D]),
    "nmpc_adjoint": (C.c_int32, [_P, _D, C.c_double, _D, _D, _D, _D]),
    # device pointers and the caller's stream as plain addresses (0 = NULL)
    "nmpc_set_parameters_dev": (C.c_int32, [_P] + [C.c_void_p] * 5),
    "nmpc_get_solution_dev": (C.c_int32, [_P] + [C.c_void_p] * 8),
    "nmpc_adjoint_dev": (C.c_int32, [_P] + [C.c_void_p] * 7),
    "nmpc_jacobian_u1_x0": (C.c_int32, [_P, _D]),
    "nmpc_jacobian_u1_x0_noalloc": (C.c_int32, [_P, C.c_void_p, C.c_void_p]),
    "nmpc_closed_loop_dev": (C.c_int32, [_P, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                         C.POINTER(nmpc_options), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.c_void_p]),
    "nmpc_solution_id": (C.c_int32, [_P, _L, _I]),
    "nmpc_autotune": (C.c_int32, [_P, C.c_int32, _I]),
    "nmpc_batch_create": (C.c_int32, [C.POINTER(_P), C.c_int32, C.POINTER(_P)]),
    "nmpc_batch_solve": (C.c_int32, [_P, C.c_int32, C.POINTER(nmpc_options), C.POINTER(nmpc_result)]),
    "nmpc_batch_destroy": (None, [_P]),
    "nmpc_last_error": (C.c_char_p, []),
    "nmpc_device_available": (C.c_int32, []),
}

_lib = None


def lib():
    """Load libnmpc.so once; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2606_04725_amd.build` (needs hipcc)")
        # One HIP runtime per process: torch ships its own libamdhip64 (same
        # SONAME, found through its own directory).  Loaded first, it also
        # serves this library; loaded after this library it would come up as a
        # second runtime that sees no device, so torch goes first.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def declared_symbols(header=None):
    """Names of the functions the public header declares."""
    import re
    header = header or os.path.join(os.path.dirname(HERE), "include", "nmpc.h")
    txt = open(header).read()
    return sorted(set(re.findall(r"\b(nmpc_[a-z_0-9]+)\s*\(", txt)))
