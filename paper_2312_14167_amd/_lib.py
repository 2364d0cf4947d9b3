"""ctypes declarations of include/fr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfrmi.so")

FR_OK, FR_ERR_ARG, FR_ERR_MESH, FR_ERR_UNSUPPORTED, FR_ERR_HIP, FR_ERR_NONFINITE, FR_ERR_OOM = 0, -1, -2, -3, -4, -5, -6
FR_NOALLOC_SCRATCH_BYTES = 32 << 20   # include/fr.h
FR_TUNE_MAX = 8                       # include/fr.h
FR_EULER, FR_NAVIER_STOKES = 0, 1
FR_FP64, FR_FP32 = 0, 1

STATUS_NAMES = {0: "FR_OK", -1: "FR_ERR_ARG", -2: "FR_ERR_MESH", -3: "FR_ERR_UNSUPPORTED", -4: "FR_ERR_HIP",
                -5: "FR_ERR_NONFINITE", -6: "FR_ERR_OOM"}


class fr_mesh_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("p", C.c_int32), ("geom_q", C.c_int32), ("n_periodic", C.c_int32),
                ("n_elem", C.c_int64), ("n_node", C.c_int64),
                ("node_xyz", C.c_void_p), ("elem_nodes", C.c_void_p), ("face_bc", C.c_void_p),
                ("periodic_vec", C.c_void_p), ("n_mesh", C.c_int32), ("reserved0", C.c_int32),
                ("mesh_elem_begin", C.c_void_p)]


class fr_params(C.Structure):
    _fields_ = [("equations", C.c_int32), ("precision", C.c_int32),
                ("gamma", C.c_double), ("prandtl", C.c_double), ("ldg_beta", C.c_double), ("ldg_tau", C.c_double),
                ("rho_inf", C.c_void_p), ("vel_inf", C.c_void_p), ("p_inf", C.c_void_p), ("mu", C.c_void_p),
                ("n_probe", C.c_int32), ("max_samples", C.c_int32),
                ("probe_xyz", C.c_void_p), ("probe_mesh", C.c_void_p),
                ("forces", C.c_int32), ("reserved0", C.c_int32)]


class FrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    """Load libfrmi.so; raises if the HIP library has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_14167_amd.build` "
                          "(the FR path has no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.fr_build_operators.argtypes = [C.POINTER(fr_mesh_desc), C.POINTER(fr_params), C.POINTER(vp)]
    L.fr_state_shape.argtypes = [vp, C.POINTER(i64)]
    L.fr_solpt_coords.argtypes = [vp, vp]
    L.fr_rhs.argtypes = [vp, vp, vp, vp]
    L.fr_rk_step.argtypes = [vp, vp, vp, i32, i32, vp]
    L.fr_probe_oaspl.argtypes = [vp, dbl, vp, vp, vp, C.POINTER(i64), vp]
    L.fr_probe_series.argtypes = [vp, vp, i64, C.POINTER(i64), vp]
    L.fr_force_coefficients.argtypes = [vp, i32, vp, vp, vp, vp]
    L.fr_reset_accumulators.argtypes = [vp, vp]
    L.fr_rhs_vjp.argtypes = [vp, vp, vp, vp, vp, vp]
    L.fr_rhs_vjp_noalloc.argtypes = [vp, vp, vp, vp, vp]
    L.fr_solver_info.argtypes = [vp, vp]
    L.fr_profile_enable.argtypes = [vp, i32]
    L.fr_profile_read.argtypes = [vp, vp, vp, vp]
    L.fr_probe_vjp.argtypes = [vp, vp, vp, vp, vp, vp]
    L.fr_rk_step_stages.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp]
    L.fr_rk_step_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.fr_rk_segment_vjp.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, vp, vp]
    L.fr_autotune.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp]
    L.fr_tune_candidates.argtypes = [vp, i32, vp, C.POINTER(i32)]
    L.fr_tune_select.argtypes = [vp, i32, i32]
    L.fr_tune_cache_clear.argtypes = []
    L.fr_tune_cache_clear.restype = None
    L.fr_geo_adjoint_begin.argtypes = [vp, vp]
    L.fr_geo_adjoint_end.argtypes = [vp, vp, vp]
    L.fr_stats_prms_cumulative.argtypes = [vp, i64, vp]
    L.fr_stats_observer_oaspl.argtypes = [vp, i32, i64, vp, i32, dbl, vp, vp]
    L.fr_stats_psd_welch.argtypes = [vp, i64, i32, dbl, vp, vp, i64, C.POINTER(i64)]
    L.fr_destroy.argtypes = [vp]
    L.fr_destroy.restype = None
    L.fr_vdeg_build.argtypes = [C.POINTER(fr_mesh_desc), vp, C.POINTER(fr_params), C.POINTER(vp)]
    L.fr_vdeg_groups.argtypes = [vp, C.POINTER(i32), vp, vp, vp, C.POINTER(i64)]
    L.fr_vdeg_group_elems.argtypes = [vp, i32, vp]
    L.fr_vdeg_solpt_coords.argtypes = [vp, i32, vp]
    L.fr_vdeg_rhs.argtypes = [vp, vp, vp, vp]
    L.fr_vdeg_rk_step.argtypes = [vp, vp, vp, i32, i32, vp]
    L.fr_vdeg_reset_accumulators.argtypes = [vp, vp]
    L.fr_vdeg_probe_series.argtypes = [vp, vp, i64, C.POINTER(i64), vp]
    L.fr_vdeg_mean_force.argtypes = [vp, vp, C.POINTER(i64), vp]
    L.fr_vdeg_destroy.argtypes = [vp]
    L.fr_vdeg_destroy.restype = None
    L.fr_last_error.argtypes = []
    L.fr_last_error.restype = C.c_char_p
    for name in ("fr_build_operators", "fr_state_shape", "fr_solpt_coords", "fr_rhs", "fr_rk_step",
                 "fr_probe_oaspl", "fr_probe_series", "fr_force_coefficients", "fr_reset_accumulators", "fr_rhs_vjp", "fr_rhs_vjp_noalloc",
                 "fr_solver_info",
                 "fr_profile_enable", "fr_profile_read", "fr_probe_vjp", "fr_rk_step_stages", "fr_rk_step_vjp", "fr_rk_segment_vjp",
                 "fr_autotune", "fr_tune_candidates", "fr_tune_select", "fr_geo_adjoint_begin", "fr_geo_adjoint_end", "fr_stats_prms_cumulative",
                 "fr_stats_observer_oaspl", "fr_stats_psd_welch", "fr_vdeg_build", "fr_vdeg_groups",
                 "fr_vdeg_group_elems", "fr_vdeg_solpt_coords", "fr_vdeg_rhs", "fr_vdeg_rk_step",
                 "fr_vdeg_reset_accumulators", "fr_vdeg_probe_series", "fr_vdeg_mean_force"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def check(status: int):
    if status != FR_OK:
        raise FrError(status, lib().fr_last_error().decode())
