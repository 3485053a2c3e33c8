"""ctypes binding of the HIP library's C ABI (include/ibm.h): argument marshalling
only. Every step of the method runs in the library's kernels; there is no
fallback -- loading fails loudly when the built library is missing."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; IBM_HIP_LIB names another build of the same sources
LIB_PATH = os.environ.get("IBM_HIP_LIB") or os.path.join(PKG, "libibm_hip.so")

IBM_OK, IBM_E_ARG, IBM_E_SIZE, IBM_E_HIP, IBM_E_NOT_CONVERGED, IBM_E_NONFINITE, IBM_E_STATE = range(7)
STATUS_NAMES = {0: "IBM_OK", 1: "IBM_E_ARG", 2: "IBM_E_SIZE", 3: "IBM_E_HIP",
                4: "IBM_E_NOT_CONVERGED", 5: "IBM_E_NONFINITE", 6: "IBM_E_STATE"}
IBM_PERIODIC, IBM_INFLOW, IBM_OUTFLOW, IBM_SLIP = 0, 1, 2, 3
IBM_SUPERSONIC_INFLOW, IBM_SUPERSONIC_OUTFLOW = 4, 5
IBM_FP64, IBM_FP32 = 0, 1
IBM_CONV_VANLEER, IBM_CONV_LINEAR = 0, 1
IBM_MU_SUTHERLAND, IBM_MU_CONSTANT = 0, 1
IBM_DIFF_EXPLICIT, IBM_DIFF_IMPLICIT = 0, 1
IBM_SCHEME_PRESSURE, IBM_SCHEME_DENSITY = 0, 1
IBM_DEDUPE = 1
IBM_NO_HEAT = 2
IBM_RECORD = 1

# every function the header declares, with (restype, argtypes)
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


class ibm_grid_desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("precision", ctypes.c_int32),
        ("convection", ctypes.c_int32),
        ("viscosity_law", ctypes.c_int32),
        ("diffusion", ctypes.c_int32),
        ("Re", ctypes.c_double),
        ("Ma", ctypes.c_double),
        ("Pr", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("sutherland_S", ctypes.c_double),
        ("U_inf", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("dt_theta_max", ctypes.c_double),
        ("dt_u_max", ctypes.c_double),
        ("cg_rtol", ctypes.c_double),
        ("cg_maxit", ctypes.c_int32),
        ("max_markers", ctypes.c_int32),
        ("n_outer", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
    ]


class ibm_step_info(ctypes.Structure):
    _fields_ = [
        ("steps_done", ctypes.c_int64),
        ("step", ctypes.c_int64),
        ("cg_iters_last", ctypes.c_int32),
        ("cg_iters_total", ctypes.c_int32),
        ("cg_residual", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("time", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("diff_iters_total", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


SIGNATURES = {
    "ibm_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(ibm_grid_desc), ctypes.c_int32,
                                              ctypes.c_int32]),
    "ibm_create_grid": (ctypes.c_int, [ctypes.POINTER(ibm_grid_desc), _P, ctypes.c_size_t,
                                       ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "ibm_create_grid_noalloc": (ctypes.c_int, [ctypes.POINTER(ibm_grid_desc), ctypes.c_int32, _P,
                                               ctypes.POINTER(_P)]),
    "ibm_destroy": (None, [_P]),
    "ibm_last_error": (ctypes.c_char_p, [_P]),
    "ibm_dt": (ctypes.c_double, [_P]),
    "ibm_init_primitive": (ctypes.c_int, [_P, _P, _P, _P]),
    "ibm_set_state": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int64]),
    "ibm_get_state": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "ibm_set_markers": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, ctypes.c_uint32]),
    "ibm_set_motion": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double]),
    "ibm_set_wall_temperature": (ctypes.c_int, [_P, _P]),
    "ibm_step": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_uint32, _P,
                                ctypes.POINTER(ibm_step_info)]),
    "ibm_wall_fluxes": (ctypes.c_int, [_P, _P, _P, _D]),
    "ibm_wall_heat_flux": (ctypes.c_int, [_P, _P]),
    "ibm_markers_in_use": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), _P, _P]),
    "ibm_get_field": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "ibm_adjoint_step": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _D, _P]),
    "ibm_tape_length": (ctypes.c_int32, [_P]),
    "ibm_shape_gradient": (ctypes.c_int, [_P, _P]),
    "ibm_profile": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ibm_profile_read": (ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int64)]),
}

PROF_CLASSES = ["predictor", "markers", "setup", "cg", "diffusion", "correct", "rebuild"]

_lib = None


def load():
    """Loads libibm_hip.so (built by ``__graft_entry__.build()``); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                              "(run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class IBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, ctx=None, what=""):
    if status != IBM_OK:
        msg = ""
        if ctx:
            raw = load().ibm_last_error(ctx)
            msg = raw.decode() if raw else ""
        raise IBMError(status, f"{what} {msg}".strip())
