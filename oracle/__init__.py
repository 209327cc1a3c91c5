"""FP64 CPU oracle for the cone-beam projector pair, CGLS and LSQR.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark use it; the HIP library never does, and this package imports
nothing from it.  The arithmetic lives in ``kct_oracle.c`` (plain C, double
precision, OpenMP); this module only marshals numpy arrays through ctypes.

Geometry is passed as the plain description used everywhere in the tests (see
``kct_inputs.ConeGeometry``): any object with the attributes
``nx, ny, nz, vx, vy, vz, cx, cy, cz, n_views, nu, nv, sid, sdd, du, dv, off_u,
off_v`` and an ``angles()`` method returning the view angles in radians.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kct_oracle.c")
_LIB = os.path.join(_HERE, "libkct_oracle.so")

STOP_MAXITER, STOP_TOL, STOP_BREAKDOWN, STOP_NUMERIC = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        geo = [i32p, dp, dp]
        L.oracle_project.argtypes = geo + [dp, dp]
        L.oracle_project.restype = None
        L.oracle_project_rays.argtypes = geo + [dp, i64p, ctypes.c_int64, dp]
        L.oracle_project_rays.restype = None
        L.oracle_backproject.argtypes = geo + [dp, dp]
        L.oracle_backproject.restype = None
        L.oracle_project32.argtypes = geo + [dp, dp]
        L.oracle_project32.restype = None
        L.oracle_backproject32.argtypes = geo + [dp, dp]
        L.oracle_backproject32.restype = None
        L.oracle_backproject_voxels.argtypes = geo + [dp, i64p, ctypes.c_int64, dp]
        L.oracle_backproject_voxels.restype = None
        L.oracle_count_nnz.argtypes = geo
        L.oracle_count_nnz.restype = ctypes.c_int64
        L.oracle_assemble.argtypes = geo + [ctypes.c_int64, i64p, i64p, dp]
        L.oracle_assemble.restype = ctypes.c_int64
        L.oracle_cgls.argtypes = geo + [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_int, dp, dp, dp, ip]
        L.oracle_cgls.restype = ctypes.c_int
        L.oracle_lsqr.argtypes = geo + [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                        dp, dp, dp, ip]
        L.oracle_lsqr.restype = ctypes.c_int
        L.oracle_cgls_ex.argtypes = geo + [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           dp, dp, dp, ip]
        L.oracle_cgls_ex.restype = ctypes.c_int
        L.oracle_lsqr_ex.argtypes = geo + [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp, dp, ip]
        L.oracle_lsqr_ex.restype = ctypes.c_int
        L.oracle_diag_normal.argtypes = geo + [dp]
        L.oracle_diag_normal.restype = None
        L.oracle_cgls_jacobi.argtypes = geo + [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp, dp, ip]
        L.oracle_cgls_jacobi.restype = ctypes.c_int
        L.oracle_cgls_jacobi_ex.argtypes = geo + [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                                  dp, dp, dp, ip]
        L.oracle_cgls_jacobi_ex.restype = ctypes.c_int
        L.oracle_tt_project.argtypes = geo + [dp, dp]
        L.oracle_tt_project.restype = None
        L.oracle_tt_backproject.argtypes = geo + [dp, dp]
        L.oracle_tt_backproject.restype = None
        L.oracle_tt_diag_normal.argtypes = geo + [dp]
        L.oracle_tt_diag_normal.restype = None
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _ptr(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _geo(g):
    dims = np.array([g.nx, g.ny, g.nz, g.n_views, g.nu, g.nv], dtype=np.int32)
    par = np.array([g.vx, g.vy, g.vz, g.cx, g.cy, g.cz, g.sid, g.sdd, g.du, g.dv,
                    g.off_u, g.off_v], dtype=np.float64)
    ang = np.ascontiguousarray(g.angles(), dtype=np.float64)
    return dims, par, ang


def _gargs(gt):
    dims, par, ang = gt
    return [_ptr(dims, ctypes.c_int32), _ptr(par), _ptr(ang)]


def _vol(g, x):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    assert x.size == g.nx * g.ny * g.nz, "volume size does not match the geometry"
    return x


def _proj(g, b):
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    assert b.size == g.n_views * g.nv * g.nu, "projection size does not match the geometry"
    return b


def project(g, x):
    """b = A x, shape (n_views, nv, nu)."""
    gt = _geo(g)
    x = _vol(g, x)
    b = np.empty(g.n_views * g.nv * g.nu, dtype=np.float64)
    lib().oracle_project(*_gargs(gt), _ptr(x), _ptr(b))
    return b.reshape(g.n_views, g.nv, g.nu)


def project32(g, x):
    """b = A x in single-precision arithmetic (weights and x rounded to float,
    float fused multiply-adds along each ray), shape (n_views, nv, nu)."""
    gt = _geo(g)
    x = _vol(g, x)
    b = np.empty(g.n_views * g.nv * g.nu, dtype=np.float64)
    lib().oracle_project32(*_gargs(gt), _ptr(x), _ptr(b))
    return b.reshape(g.n_views, g.nv, g.nu)


def backproject32(g, y):
    """r = A^T y in single-precision arithmetic (per voxel, float fused
    multiply-adds in ray order), shape (nz, ny, nx)."""
    gt = _geo(g)
    y = _proj(g, y)
    r = np.empty(g.nx * g.ny * g.nz, dtype=np.float64)
    lib().oracle_backproject32(*_gargs(gt), _ptr(y), _ptr(r))
    return r.reshape(g.nz, g.ny, g.nx)


def project_rays(g, x, rays):
    """(A x)_i for the flat ray indices ``rays``."""
    gt = _geo(g)
    x = _vol(g, x)
    rays = np.ascontiguousarray(rays, dtype=np.int64)
    out = np.empty(rays.size, dtype=np.float64)
    lib().oracle_project_rays(*_gargs(gt), _ptr(x), _ptr(rays, ctypes.c_int64), rays.size, _ptr(out))
    return out


def backproject(g, y):
    """r = A^T y, shape (nz, ny, nx)."""
    gt = _geo(g)
    y = _proj(g, y)
    r = np.empty(g.nx * g.ny * g.nz, dtype=np.float64)
    lib().oracle_backproject(*_gargs(gt), _ptr(y), _ptr(r))
    return r.reshape(g.nz, g.ny, g.nx)


def backproject_voxels(g, y, voxels):
    """(A^T y)_j for the flat voxel indices ``voxels`` (direct segment-box weights)."""
    gt = _geo(g)
    y = _proj(g, y)
    voxels = np.ascontiguousarray(voxels, dtype=np.int64)
    out = np.empty(voxels.size, dtype=np.float64)
    lib().oracle_backproject_voxels(*_gargs(gt), _ptr(y), _ptr(voxels, ctypes.c_int64), voxels.size,
                                    _ptr(out))
    return out


def count_nnz(g):
    gt = _geo(g)
    return int(lib().oracle_count_nnz(*_gargs(gt)))


def assemble(g):
    """A as a scipy CSR matrix (m x n).  Tiny grids only."""
    import scipy.sparse as sp
    gt = _geo(g)
    nnz = count_nnz(g)
    rows = np.empty(nnz, dtype=np.int64)
    cols = np.empty(nnz, dtype=np.int64)
    vals = np.empty(nnz, dtype=np.float64)
    got = lib().oracle_assemble(*_gargs(gt), nnz, _ptr(rows, ctypes.c_int64), _ptr(cols, ctypes.c_int64),
                                _ptr(vals))
    assert got == nnz
    m = g.n_views * g.nv * g.nu
    n = g.nx * g.ny * g.nz
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, n))


class SolveResult:
    def __init__(self, x, iters, nb, nb0, stop, history):
        self.x, self.iterations, self.nb, self.nb0, self.stop_reason = x, iters, nb, nb0, stop
        self.history = history

    def __repr__(self):
        return f"SolveResult(iterations={self.iterations}, nb={self.nb:.6g}, stop={self.stop_reason})"


# "siddon32": the Siddon pair in single-precision arithmetic (project32 /
# backproject32), for solves in the precision structure of a single-precision
# GPU path (with store32: vectors and projector in float, scalars in double).
PROJECTORS = {"siddon": 0, "tt": 1, "siddon32": 2}


def cgls(g, b, K, x0=None, err=0.0, literal_update=False, tikhonov=0.0, recompute_every=0, projector="siddon",
         store32=False):
    """Algorithm 1 (CGLS with delayed residual) in FP64.

    tikhonov = lambda adds lambda^2 |x|^2 to the objective (CGLS on [A; lambda I]);
    recompute_every = k > 0 recomputes e = b - A x after every k-th iteration;
    projector "siddon", "tt" or "siddon32" selects the operator;
    store32 rounds the vectors x, r, d, e, p to single precision after every
    update (scalars and norms stay double): the single-precision storage form
    of Section 5, used to measure how far that rounding alone moves the iterates."""
    gt = _geo(g)
    b = _proj(g, b)
    x = np.zeros(g.nx * g.ny * g.nz) if x0 is None else _vol(g, x0).copy()
    hist = np.zeros(max(K, 1), dtype=np.float64)
    nb, nb0 = ctypes.c_double(0), ctypes.c_double(0)
    it = ctypes.c_int(0)
    stop = lib().oracle_cgls_ex(*_gargs(gt), _ptr(b), _ptr(x), int(K), float(err), int(x0 is None),
                                int(bool(literal_update)), float(tikhonov), int(recompute_every),
                                PROJECTORS[projector], int(bool(store32)), _ptr(hist),
                                ctypes.byref(nb), ctypes.byref(nb0), ctypes.byref(it))
    return SolveResult(x.reshape(g.nz, g.ny, g.nx), it.value, nb.value, nb0.value, stop,
                       hist[: it.value].copy())


def lsqr(g, b, K, x0=None, err=0.0, damp=0.0, projector="siddon", store32=False):
    """LSQR (Paige & Saunders) in FP64, iterations aligned with CGLS.

    damp = lambda > 0 solves min |b - A x|^2 + lambda^2 |x - x0|^2;
    store32 rounds u, v, w and x to single precision after every update."""
    gt = _geo(g)
    b = _proj(g, b)
    x = np.zeros(g.nx * g.ny * g.nz) if x0 is None else _vol(g, x0).copy()
    hist = np.zeros(max(K, 1), dtype=np.float64)
    nb, nb0 = ctypes.c_double(0), ctypes.c_double(0)
    it = ctypes.c_int(0)
    stop = lib().oracle_lsqr_ex(*_gargs(gt), _ptr(b), _ptr(x), int(K), float(err), int(x0 is None),
                                float(damp), PROJECTORS[projector], int(bool(store32)), _ptr(hist), ctypes.byref(nb), ctypes.byref(nb0),
                                ctypes.byref(it))
    return SolveResult(x.reshape(g.nz, g.ny, g.nx), it.value, nb.value, nb0.value, stop,
                       hist[: it.value].copy())


def diag_normal(g):
    """diag(A^T A) = sum_i w_ij^2 per voxel, FP64."""
    gt = _geo(g)
    out = np.zeros(g.nx * g.ny * g.nz)
    lib().oracle_diag_normal(*_gargs(gt), _ptr(out))
    return out.reshape(g.nz, g.ny, g.nx)


def cgls_jacobi(g, b, K, x0=None, err=0.0, projector="siddon"):
    """Jacobi-preconditioned CGLS (Algorithm 1 on A diag(A^T A)^(-1/2)) in FP64,
    with the Siddon or the TT operator and that operator's diagonal."""
    if projector not in ("siddon", "tt"):
        raise ValueError("cgls_jacobi takes the siddon or the tt operator")
    gt = _geo(g)
    b = _proj(g, b)
    x = np.zeros(g.nx * g.ny * g.nz) if x0 is None else _vol(g, x0).copy()
    hist = np.zeros(max(K, 1), dtype=np.float64)
    nb, nb0 = ctypes.c_double(0), ctypes.c_double(0)
    it = ctypes.c_int(0)
    stop = lib().oracle_cgls_jacobi_ex(*_gargs(gt), _ptr(b), _ptr(x), int(K), float(err), int(x0 is None),
                                       PROJECTORS[projector], _ptr(hist), ctypes.byref(nb), ctypes.byref(nb0),
                                       ctypes.byref(it))
    return SolveResult(x.reshape(g.nz, g.ny, g.nx), it.value, nb.value, nb0.value, stop,
                       hist[: it.value].copy())


def tt_project(g, x):
    """b = A_TT x, the trapezoid-trapezoid footprint projector, FP64."""
    gt = _geo(g)
    x = _vol(g, x)
    b = np.zeros(g.n_views * g.nv * g.nu)
    lib().oracle_tt_project(*_gargs(gt), _ptr(x), _ptr(b))
    return b.reshape(g.n_views, g.nv, g.nu)


def tt_backproject(g, y):
    """r = A_TT^T y, FP64."""
    gt = _geo(g)
    y = _proj(g, y)
    r = np.zeros(g.nx * g.ny * g.nz)
    lib().oracle_tt_backproject(*_gargs(gt), _ptr(y), _ptr(r))
    return r.reshape(g.nz, g.ny, g.nx)


def tt_diag_normal(g):
    """diag(A_TT^T A_TT) = sum_i a_ij^2 per voxel, FP64."""
    gt = _geo(g)
    out = np.zeros(g.nx * g.ny * g.nz)
    lib().oracle_tt_diag_normal(*_gargs(gt), _ptr(out))
    return out.reshape(g.nz, g.ny, g.nx)


def num_threads():
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of the following oracle calls (results do not depend on it)."""
    lib().oracle_set_num_threads(int(n))
