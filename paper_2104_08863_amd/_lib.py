"""ctypes binding of the chanflow C ABI (include/chanflow.h).

Argument marshalling only: every step of every call runs in the HIP library.
There is no fallback: if libchanflow.so is missing the import of the binding
raises.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# CHANFLOW_LIB may point at another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("CHANFLOW_LIB") or os.path.join(PKG, "libchanflow.so")
HOSTLIB_PATH = os.path.join(PKG, "libchanflow_host.so")

CF_OK, CF_ERR_ARG, CF_ERR_UNSUPPORTED, CF_ERR_NOMEM, CF_ERR_DEVICE, CF_ERR_NUMERIC = range(6)
CF_FP64, CF_MIXED = 0, 1
KERNELS = ["r2c_x", "fft_z_fwd", "ysolve", "special_lines", "fft_z_inv", "c2r_x", "divergence",
           "rk_stage1", "rk_stage2", "correct", "rhs_adjoint", "correct_weighted", "rk2_fused",
           "slab_local", "slab_finish"]
CF_PLAN_STEP, CF_PLAN_ADJOINT, CF_PLAN_Y_DCT, CF_PLAN_TUNE_PARTS = 1, 2, 4, 8


class cf_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("n_parts", C.c_int), ("drop_tol", C.c_double),
                ("fp64_kx", C.c_int), ("fp64_kz", C.c_int), ("refine_passes", C.c_int),
                ("flags", C.c_int), ("lines_per_block", C.c_int), ("drop_parts", C.c_int)]


class cf_plan_info(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("precision", C.c_int),
                ("n_parts", C.c_int), ("rows_per_part", C.c_int), ("n_lines", C.c_longlong),
                ("n_drop_lines", C.c_longlong), ("n_special", C.c_longlong),
                ("k2_threshold", C.c_double), ("workspace_bytes", C.c_size_t), ("lines_per_block", C.c_int),
                ("slab_iface_bytes", C.c_size_t), ("drop_parts", C.c_int), ("n_dropped_lines", C.c_longlong)]


_P = C.c_void_p
_D = C.c_double
_I = C.c_int

# name -> (restype, argtypes); one entry per declaration of include/chanflow.h
SIGNATURES = {
    "cf_options_default": (None, [C.POINTER(cf_options)]),
    "cf_plan_create": (_I, [C.POINTER(_P), _I, _I, _I, _D, _D, C.POINTER(_D), C.POINTER(cf_options)]),
    "cf_plan_destroy": (None, [_P]),
    "cf_plan_query": (_I, [_P, C.POINTER(cf_plan_info)]),
    "cf_plan_tuning": (_I, [_P, _I, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I), C.POINTER(_D)]),
    "cf_poisson_solve": (_I, [_P, _P, _P, _P]),
    "cf_divergence": (_I, [_P, _P, _P, _P, _P, _D, _P]),
    "cf_projection_step": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _D, _D, _D, _P]),
    "cf_rk2_predictor": (_I, [_P, _P, _P, _P, _P, _P, _P, _D, _D, _D, _P]),
    "cf_plane_stats": (_I, [_P, _P, _P, _P, _P, _P]),
    "cf_run_steps": (_I, [_P, _P, _P, _P, _P, _P, _P, C.c_int, _D, _D, _D, C.c_int, _P, _P, C.c_int, _P]),
    "cf_projection_step_adjoint": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _D, _D, _D, _P]),
    "cf_rhs_adjoint": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _D, _P]),
    "cf_forward_spectral": (_I, [_P, _P, _P, _P]),
    "cf_inverse_spectral": (_I, [_P, _P, _P, _P]),
    "cf_solve_spectral": (_I, [_P, _P, _P, _P]),
    "cf_solve_spectral_slabs": (_I, [_P, _I, _P, _P, _P, _P]),
    "cf_solve_spectral_slabs_noalloc": (_I, [_P, _I, _P, _P, _P]),
    "cf_plan_numeric_status": (_I, [_P, _P]),
    "cf_plan_set_timing": (_I, [_P, _I]),
    "cf_plan_reset_timing": (_I, [_P]),
    "cf_plan_get_timing": (_I, [_P, _I, C.POINTER(_D), C.POINTER(C.c_longlong)]),
    "cf_kernel_name": (C.c_char_p, [_I]),
    "cf_status_string": (C.c_char_p, [_I]),
    "cf_last_error": (C.c_char_p, []),
}

HOST_SIGNATURES = {
    "cfh_fft_c2c": (_I, [_I, _I, _I, _P, _P]),
    "cfh_rfft": (_I, [_I, _I, _P, _P]),
    "cfh_irfft": (_I, [_I, _I, _P, _P]),
    "cfh_pdd_line": (_I, [_I, _I, _P, _P, _D, _I, _I, _P, _P]),
    "cfh_pdd_line_grouped": (_I, [_I, _I, _I, _P, _P, _D, _I, _P, _P]),
    "cfh_xcd_slab_block": (_I, [_I, _I]),
}

_lib = None
_hostlib = None


def _bind(lib, sigs):
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def lib():
    """The HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2104_08863_amd.build`")
        _lib = _bind(C.CDLL(LIB_PATH), SIGNATURES)
    return _lib


def hostlib():
    global _hostlib
    if _hostlib is None:
        if not os.path.exists(HOSTLIB_PATH):
            raise ImportError(f"{HOSTLIB_PATH} is missing: run the build")
        _hostlib = _bind(C.CDLL(HOSTLIB_PATH), HOST_SIGNATURES)
    return _hostlib


class ChanflowError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.cf_last_error().decode()
        super().__init__(f"{where}: {L.cf_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def check(status: int, where: str):
    if status != CF_OK:
        raise ChanflowError(status, where)
