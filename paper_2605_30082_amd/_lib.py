"""ctypes binding of libmgp.so (the C ABI declared in include/mgp.h).

Argument marshalling only: every step of the solve runs in the HIP kernels of
the library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmgp.so")

# status codes, enums and flags (values as in include/mgp.h)
MG_OK, MG_EINVAL, MG_ENOMEM, MG_EHIP, MG_ENOCONV, MG_ENONFINITE = 0, -1, -2, -3, -4, -5
MG_BC_NEUMANN = 0
MG_PREC_FP64, MG_PREC_MIXED = 0, 1
MG_FLAG_ZERO_GUESS, MG_FLAG_TIMING, MG_FLAG_FCG, MG_FLAG_LEVEL_LAUNCHES = 1, 2, 4, 8
MG_HIST_MAX = 256
MG_MAX_LEVELS = 16
MG_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024
MG_K_SWEEP, MG_K_RESTRICT, MG_K_PROLONG, MG_K_OUTER, MG_K_NORM, MG_K_SWEEP2, MG_K_SWEEP2R, MG_K_COUNT = range(8)

STATUS_NAMES = {
    MG_OK: "MG_OK", MG_EINVAL: "MG_EINVAL", MG_ENOMEM: "MG_ENOMEM", MG_EHIP: "MG_EHIP",
    MG_ENOCONV: "MG_ENOCONV", MG_ENONFINITE: "MG_ENONFINITE",
}


class MgOpts(ctypes.Structure):
    _fields_ = [("pre", ctypes.c_int), ("post", ctypes.c_int), ("max_cycles", ctypes.c_int),
                ("coarse_max", ctypes.c_int), ("precision", ctypes.c_int), ("flags", ctypes.c_int)]


class MgStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("status", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("rhs_mean_removed", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("hist", ctypes.c_double * MG_HIST_MAX),
                ("kernel_ms", ctypes.c_double * MG_K_COUNT),
                ("kernel_launches", ctypes.c_longlong * MG_K_COUNT),
                ("kernel_bytes", ctypes.c_double * MG_K_COUNT),
                ("kernel_ms_finest", ctypes.c_double * MG_K_COUNT),
                ("kernel_launches_finest", ctypes.c_longlong * MG_K_COUNT),
                ("kernel_bytes_finest", ctypes.c_double * MG_K_COUNT)]


_D = ctypes.c_void_p       # device pointer
_I = ctypes.c_int
_F = ctypes.c_double
_CTX = ctypes.c_void_p
_DIMS = ctypes.POINTER(ctypes.c_int)

SIGNATURES = {
    "mg_setup": (_I, [ctypes.POINTER(_CTX), _D, _D, _D, _DIMS, _F, _I, ctypes.POINTER(MgOpts), ctypes.c_void_p]),
    "mg_update": (_I, [_CTX, _D, _D, _D]),
    "mg_setup_density": (_I, [ctypes.POINTER(_CTX), _D, _DIMS, _F, _I, ctypes.POINTER(MgOpts), ctypes.c_void_p]),
    "mg_update_density": (_I, [_CTX, _D]),
    "mg_set_timing_classes": (_I, [_CTX, ctypes.c_uint]),
    "mg_solve": (_I, [_CTX, _D, _D, _F, ctypes.POINTER(MgStats)]),
    "mg_solve_adjoint": (_I, [_CTX, _D, _D, _F, ctypes.POINTER(MgStats)]),
    "mg_face_grad": (_I, [_CTX, _D, _D, _D, _D, _D]),
    "mg_apply": (_I, [_CTX, _D, _D]),
    "mg_destroy": (None, [_CTX]),
    "mg_last_error": (ctypes.c_char_p, [_CTX]),
    "mg_faces_from_vof": (_I, [_D, _D, _DIMS, _F, _F, _F, _D, _D, _D, ctypes.c_void_p]),
    "mg_divergence": (_I, [_D, _D, _D, _DIMS, _F, _F, _D, ctypes.c_void_p]),
    "mg_density_from_vof": (_I, [_D, _D, _DIMS, _F, _F, _F, _D, ctypes.c_void_p]),
    "mg_faces_from_density": (_I, [_D, _DIMS, _D, _D, _D, ctypes.c_void_p]),
    "mg_density_grad": (_I, [_D, _DIMS, _D, _D, _D, _D, ctypes.c_void_p]),
    "mg_vof_grad": (_I, [_D, _D, _DIMS, _F, _F, _F, _D, _D, _D, _D, _D, ctypes.c_void_p]),
    "mg_velocity_correct": (_I, [_D, _D, _D, _D, _DIMS, _F, _F, _D, _D, _D, ctypes.c_void_p]),
    "mg_plan_levels": (_I, [_DIMS, _I]),
    "mg_level_info": (_I, [_CTX, _I, _DIMS, ctypes.POINTER(ctypes.c_double)]),
    "mg_level_faces": (_I, [_CTX, _I, _D, _D, _D]),
    "mg_smooth": (_I, [_CTX, _I, _I, _D, _D, _I, _I]),
    "mg_residual_restrict": (_I, [_CTX, _I, _I, _D, _D, _D]),
    "mg_presmooth_restrict": (_I, [_CTX, _I, _I, _D, _D, _D]),
    "mg_prolong_correct": (_I, [_CTX, _I, _I, _D, _D]),
    "mg_coarse_solve": (_I, [_CTX, _D, _D]),
    "mg_residual_norm2": (_I, [_CTX, _D, _D, ctypes.POINTER(ctypes.c_double)]),
    "mg_solve_noalloc": (_I, [_D, _D, _D, _DIMS, _F, _I, ctypes.POINTER(MgOpts), _D, _D, _F,
                              ctypes.POINTER(MgStats), ctypes.c_void_p]),
}

_lib = None


class MgError(RuntimeError):
    def __init__(self, status: int, text: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {text}")


def load() -> ctypes.CDLL:
    """Load libmgp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2605_30082_amd.build` (hipcc, gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def dims_arg(dims) -> ctypes.Array:
    return (ctypes.c_int * 3)(*[int(d) for d in dims])


def last_error(ctx=None) -> str:
    s = load().mg_last_error(ctx)
    return s.decode(errors="replace") if s else ""


def check(status: int, ctx=None) -> None:
    if status != MG_OK:
        raise MgError(status, last_error(ctx))
