"""ctypes declarations of the C ABI in include/kct.h (argument marshalling only).

The library is loaded from this package directory (``libkct.so``, built by
``paper_2110_13526_amd.build``).  A missing library is an error: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkct.so")

KCT_OK, KCT_ERR_INVALID_ARG, KCT_ERR_UNSUPPORTED, KCT_ERR_HIP, KCT_ERR_WORKSPACE, KCT_ERR_NUMERIC = range(6)
KCT_F32, KCT_BF16, KCT_F16, KCT_F64 = 0, 1, 2, 3
KCT_SOLVER_CGLS, KCT_SOLVER_LSQR, KCT_SOLVER_WITH_JACOBI = 0, 1, 0x100
STOP_MAXITER, STOP_TOL, STOP_BREAKDOWN, STOP_NUMERIC = 0, 1, 2, 3

# Every symbol include/kct.h declares.
EXPORTS = (
    "kct_geometry_create", "kct_geometry_destroy", "kct_geometry_dims", "kct_project_workspace_size",
    "kct_project", "kct_backproject", "kct_solver_workspace_size", "kct_cgls_solve", "kct_lsqr_solve",
    "kct_diag_normal", "kct_batch_create", "kct_batch_destroy", "kct_batch_workspace_size", "kct_batch_tune",
    "kct_batch_cgls_solve", "kct_geometry_set_projector", "kct_last_error", "kct_project_noalloc",
    "kct_batch_latencies", "kct_timing_enable", "kct_timing_get",
)
NOALLOC_SCRATCH_BYTES = 64 << 20

PROJECTOR_SIDDON, PROJECTOR_TT = 0, 1


class VolumeDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("vz", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("cz", ctypes.c_double)]


class ConeDesc(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("angle0", ctypes.c_double), ("arc", ctypes.c_double),
                ("angles", ctypes.POINTER(ctypes.c_double)),
                ("sid", ctypes.c_double), ("sdd", ctypes.c_double),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
                ("du", ctypes.c_double), ("dv", ctypes.c_double),
                ("off_u", ctypes.c_double), ("off_v", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("err_tol", ctypes.c_double), ("x0_is_zero", ctypes.c_int32),
                ("history", ctypes.c_void_p), ("tikhonov", ctypes.c_double), ("jacobi", ctypes.c_int32),
                ("recompute_every", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("nb0", ctypes.c_double), ("nb", ctypes.c_double),
                ("nr2", ctypes.c_double), ("stop_reason", ctypes.c_int32)]


class KctError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"kct status {status}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libkct.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2110_13526_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    st = ctypes.c_int
    L.kct_geometry_create.argtypes = [ctypes.POINTER(VolumeDesc), ctypes.POINTER(ConeDesc), ctypes.POINTER(vp)]
    L.kct_geometry_create.restype = st
    L.kct_geometry_destroy.argtypes = [vp]
    L.kct_geometry_destroy.restype = None
    L.kct_geometry_dims.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.kct_geometry_dims.restype = st
    L.kct_project_workspace_size.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.kct_project_workspace_size.restype = st
    L.kct_project.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    L.kct_project.restype = st
    L.kct_project_noalloc.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.kct_project_noalloc.restype = st
    L.kct_batch_latencies.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.kct_batch_latencies.restype = st
    L.kct_timing_enable.argtypes = [ctypes.c_int32]
    L.kct_timing_enable.restype = st
    dptr = ctypes.POINTER(ctypes.c_double)
    L.kct_timing_get.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), dptr, dptr, dptr]
    L.kct_timing_get.restype = st
    L.kct_backproject.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.kct_backproject.restype = st
    L.kct_solver_workspace_size.argtypes = [vp, ctypes.c_int, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    L.kct_solver_workspace_size.restype = st
    for name in ("kct_cgls_solve", "kct_lsqr_solve"):
        f = getattr(L, name)
        f.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.POINTER(SolveOpts), vp, ctypes.c_size_t,
                      ctypes.POINTER(SolveInfo), vp]
        f.restype = st
    L.kct_diag_normal.argtypes = [vp, vp, vp]
    L.kct_diag_normal.restype = st
    L.kct_geometry_set_projector.argtypes = [vp, ctypes.c_int32]
    L.kct_geometry_set_projector.restype = st
    L.kct_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(vp)]
    L.kct_batch_create.restype = st
    L.kct_batch_destroy.argtypes = [vp]
    L.kct_batch_destroy.restype = None
    L.kct_batch_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.kct_batch_workspace_size.restype = st
    L.kct_batch_tune.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_char_p, vp]
    L.kct_batch_tune.restype = st
    L.kct_batch_cgls_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(SolveOpts),
                                       ctypes.c_int32, vp, ctypes.c_size_t, ctypes.POINTER(SolveInfo), vp]
    L.kct_batch_cgls_solve.restype = st
    L.kct_last_error.argtypes = []
    L.kct_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status):
    if status != KCT_OK:
        msg = load().kct_last_error().decode(errors="replace")
        raise KctError(status, msg)
