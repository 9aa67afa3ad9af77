"""ctypes declarations of the C ABI in include/kchol.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkchol.so")

KC_OK, KC_EINVAL, KC_ENOMEM, KC_EWORKSPACE, KC_EHIP, KC_ESTATE, KC_ERANGE = range(7)
KC_RULE_MAX, KC_RULE_MIN = 0, 1
KC_FP64, KC_MIXED = 0, 1
KC_PIVOT_ZERO, KC_PIVOT_SHIFT = 0, 1
KC_ORDER_SPATIAL, KC_ORDER_LONGEST = 0, 1


class kc_kernel(C.Structure):
    _fields_ = [("nu", C.c_double), ("lengthscale", C.c_double)]


class kc_plan_info_t(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("rule", C.c_int32), ("rho", C.c_double),
                ("nnz", C.c_int64), ("max_col", C.c_int64), ("max_row", C.c_int64),
                ("nlevels", C.c_int32), ("nrlevels", C.c_int32), ("nunits", C.c_int64),
                ("t_order_s", C.c_double), ("t_pattern_s", C.c_double), ("t_schedule_s", C.c_double),
                ("ninst", C.c_int32)]


class kc_pcg_info_t(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("max_rel_residual", C.c_double),
                ("t_matvec_ms", C.c_double), ("t_precond_ms", C.c_double), ("true_rel_residual", C.c_double),
                ("restarts", C.c_int32), ("pad", C.c_int32)]


class kc_factor_stats_t(C.Structure):
    _fields_ = [("nonpositive", C.c_int64), ("shifted", C.c_int64), ("rank", C.c_int64),
                ("updates", C.c_int64), ("exp_hard", C.c_int64), ("nonfinite", C.c_int64),
                ("match_errors", C.c_int64)]


EXPORTED = ("kc_status_string", "kc_last_error", "kc_analyze", "kc_plan_info", "kc_plan_export", "kc_plan_levels", "kc_plan_set_delta_limit",
            "kc_plan_destroy", "kc_factor_bytes", "kc_factor_create", "kc_factorize", "kc_theta", "kc_solve_bytes",
            "kc_solve", "kc_factorize_solve", "kc_factor_stats", "kc_factor_export_L", "kc_factor_destroy", "kc_device_count",
            "kc_dense_matvec", "kc_pcg_bytes", "kc_pcg", "kc_analyze_batched", "kc_factorize_batched",
            "kc_factor_tune", "kc_factor_set_schedule", "kc_factor_schedule", "kc_graph_create", "kc_graph_info", "kc_graph_launch", "kc_graph_destroy", "kc_analyze_supernodal",
            "kc_plan_supernodes", "kc_solve_noalloc", "kc_factor_match_bytes", "kc_factor_match_build",
            "kc_factor_use_groups", "kc_factor_set_stage_limit")

_LIB = None


class KCholError(RuntimeError):
    pass


def load():
    """Load the HIP library; raise if it has not been built (there is no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise KCholError(f"{LIB_PATH} is missing: build it with `python -m paper_1706_02205_amd.build`")
    # torch ships its own HIP runtime (soname libamdhip64.so.7).  Loading torch
    # first makes the library bind to that same runtime instead of mapping a
    # second one, so device memory and streams from torch are valid here.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    P = C.POINTER
    sig = {
        "kc_status_string": (C.c_char_p, [C.c_int]),
        "kc_last_error": (C.c_char_p, []),
        "kc_analyze": (C.c_int, [vp, i64, i32, f64, C.c_int, i32, P(vp)]),
        "kc_plan_info": (C.c_int, [vp, P(kc_plan_info_t)]),
        "kc_plan_export": (C.c_int, [vp, vp, vp, vp, vp]),
        "kc_plan_levels": (C.c_int, [vp, vp]),
        "kc_plan_set_delta_limit": (C.c_int, [vp, C.c_uint32, vp]),
        "kc_plan_destroy": (None, [vp]),
        "kc_factor_bytes": (C.c_int, [vp, C.c_int, P(sz)]),
        "kc_factor_create": (C.c_int, [vp, C.c_int, vp, sz, vp, P(vp)]),
        "kc_factorize": (C.c_int, [vp, vp, kc_kernel, C.c_int, f64, i32, vp]),
        "kc_theta": (C.c_int, [vp, vp, kc_kernel, vp, vp]),
        "kc_solve_bytes": (C.c_int, [vp, i32, P(sz)]),
        "kc_solve": (C.c_int, [vp, vp, vp, i32, vp, sz, vp]),
        "kc_factorize_solve": (C.c_int, [vp, vp, kc_kernel, vp, C.c_int, f64, vp, vp, i32, vp, sz, vp]),
        "kc_factor_stats": (C.c_int, [vp, P(kc_factor_stats_t)]),
        "kc_factor_export_L": (C.c_int, [vp, vp]),
        "kc_factor_destroy": (None, [vp]),
        "kc_device_count": (i32, []),
        "kc_dense_matvec": (C.c_int, [vp, i64, i32, kc_kernel, vp, vp, i32, vp]),
        "kc_pcg_bytes": (C.c_int, [vp, i32, P(sz)]),
        "kc_pcg": (C.c_int, [vp, vp, kc_kernel, vp, vp, i32, f64, i32, vp, sz, vp, P(kc_pcg_info_t)]),
        "kc_analyze_batched": (C.c_int, [vp, vp, i32, i32, f64, C.c_int, i32, P(vp)]),
        "kc_factorize_batched": (C.c_int, [vp, vp, f64, vp, C.c_int, f64, i32, vp]),
        "kc_factor_tune": (C.c_int, [vp, vp, f64, f64, vp, C.c_int, f64, i32, vp, P(i32)]),
        "kc_graph_create": (C.c_int, [vp, vp, f64, f64, vp, C.c_int, f64, vp, vp, i32, vp, sz, P(vp)]),
        "kc_graph_launch": (C.c_int, [vp, vp]),
        "kc_factor_set_schedule": (C.c_int, [vp, i32, C.c_int64, C.c_int]),
        "kc_factor_schedule": (C.c_int, [vp, P(i32), P(C.c_int64), P(C.c_int)]),
        "kc_graph_info": (C.c_int, [vp, P(C.c_int64), P(i32)]),
        "kc_graph_destroy": (None, [vp]),
        "kc_analyze_supernodal": (C.c_int, [vp, i64, i32, f64, i32, P(vp)]),
        "kc_plan_supernodes": (C.c_int, [vp, vp, P(i64)]),
        "kc_solve_noalloc": (C.c_int, [vp, vp, vp, i32, vp]),
        "kc_factor_match_bytes": (C.c_int, [vp, vp, P(sz)]),
        "kc_factor_match_build": (C.c_int, [vp, vp, sz, vp]),
        "kc_factor_use_groups": (C.c_int, [vp, i32]),
        "kc_factor_set_stage_limit": (C.c_int, [vp, i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = L
    return L


def check(rc: int, what: str) -> None:
    if rc != KC_OK:
        L = load()
        raise KCholError(f"{what}: {L.kc_status_string(rc).decode()} ({L.kc_last_error().decode()})")
