"""ctypes loader for libfcmdp.so (the HIP library declared in include/fcmdp.h).

Loading fails loudly if the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# FCMDP_LIBRARY selects another build of the same library (e.g. a tuning
# variant); by default the in-tree build is used.
LIB_PATH = os.environ.get("FCMDP_LIBRARY") or os.path.join(_HERE, "libfcmdp.so")

OK, EINVAL, EDOMAIN, ENOMEM, EHIP, ECAPACITY = 0, -1, -2, -3, -4, -5
TORQUE_CURL, TORQUE_DERIVATIVE = 0, 1
BOTTOM_WALL, SLIT_CHANNEL = 0, 1
FP64, MIXED = 0, 1


class Params(ctypes.Structure):
    _fields_ = [
        ("geometry", ctypes.c_int),
        ("Lx", ctypes.c_double),
        ("Ly", ctypes.c_double),
        ("H", ctypes.c_double),
        ("Nx", ctypes.c_int),
        ("Ny", ctypes.c_int),
        ("Nz", ctypes.c_int),
        ("w", ctypes.c_int),
        ("beta_m", ctypes.c_double),
        ("beta_d", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("max_particles", ctypes.c_int64),
        ("slip0", ctypes.c_double),
        ("slipH", ctypes.c_double),
        ("wall0", ctypes.c_double * 2),
        ("wallH", ctypes.c_double * 2),
        ("torque_route", ctypes.c_int),
    ]


class FcmdpError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2210_01837_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.fcmdp_create_solver.argtypes = [ctypes.POINTER(Params), vp,
                                          ctypes.POINTER(vp)]
        L.fcmdp_create_solver.restype = ci
        L.fcmdp_workspace_bytes.argtypes = [ctypes.POINTER(Params), i64,
                                            ctypes.POINTER(ctypes.c_size_t)]
        L.fcmdp_workspace_bytes.restype = ci
        L.fcmdp_apply_mobility.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
        L.fcmdp_apply_mobility.restype = ci
        L.fcmdp_lanczos_sqrt.argtypes = [vp, i64, vp, vp, vp, ci,
                                         ctypes.c_double, ctypes.POINTER(ci),
                                         ctypes.POINTER(ctypes.c_double), vp]
        L.fcmdp_lanczos_sqrt.restype = ci
        L.fcmdp_lanczos_sqrt_noalloc.argtypes = L.fcmdp_lanczos_sqrt.argtypes
        L.fcmdp_lanczos_sqrt_noalloc.restype = ci
        L.fcmdp_status.argtypes = [vp, ctypes.POINTER(i64)]
        L.fcmdp_status.restype = ci
        L.fcmdp_destroy_solver.argtypes = [vp, vp]
        L.fcmdp_destroy_solver.restype = None
        L.fcmdp_strerror.argtypes = [ci]
        L.fcmdp_strerror.restype = ctypes.c_char_p
        L.fcmdp_solver_info.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.fcmdp_solver_info.restype = ci
        L.fcmdp_stage_spread.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.fcmdp_stage_spread.restype = ci
        L.fcmdp_stage_fft_forward.argtypes = [vp, vp, vp, ci, ci, vp]
        L.fcmdp_stage_fft_forward.restype = ci
        L.fcmdp_stage_solve.argtypes = [vp, vp, vp, ci, ci, vp]
        L.fcmdp_stage_solve.restype = ci
        L.fcmdp_stage_fft_inverse.argtypes = [vp, vp, vp, ci, ci, vp]
        L.fcmdp_stage_fft_inverse.restype = ci
        L.fcmdp_stage_interp.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.fcmdp_stage_interp.restype = ci
        L.fcmdp_set_profiling.argtypes = [vp, ci]
        L.fcmdp_set_profiling.restype = ci
        L.fcmdp_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(i64)]
        L.fcmdp_stage_times.restype = ci
        L.fcmdp_set_variant.argtypes = [vp, ci, ci]
        L.fcmdp_set_variant.restype = ci
        L.fcmdp_set_wall_velocity.argtypes = [vp, vp, vp]
        L.fcmdp_set_wall_velocity.restype = ci
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().fcmdp_strerror(code).decode()


def check(code: int, what: str) -> None:
    if code != OK:
        raise FcmdpError(code, what)
