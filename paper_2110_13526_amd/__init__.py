"""MI355X cone-beam projector pair and Krylov solvers (Kulvait & Rose, arXiv 2110.13526).

Thin Python binding over the C ABI of ``include/kct.h``: every step of the
projectors and of CGLS / LSQR runs in the HIP kernels of ``libkct.so``; this
module only checks tensors, allocates outputs and workspaces with torch, and
passes device pointers and the current HIP stream.

    g = Geometry(nx=..., ..., n_views=..., nu=..., nv=..., du=..., dv=...)
    b = project(g, x)            # b = A x           (Section 2, Eq. 1)
    r = backproject(g, b)        # r = A^T b         (Section 2, Eq. 2)
    x, info = cgls(g, b, K)      # Algorithm 1
    x, info = lsqr(g, b, K)

Volumes are torch tensors of shape (nz, ny, nx), projections (n_views, nv, nu),
on the GPU, contiguous, with dtype float32, bfloat16 or float16 (storage type;
accumulation is single precision and solver scalars double precision), or
float64 for the projector pair alone (double accumulation of the same
single-precision weights).  The solvers return the iterate x in float32
whatever the storage type of b.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Optional, Sequence

from . import _lib
from ._lib import KctError, STOP_BREAKDOWN, STOP_MAXITER, STOP_NUMERIC, STOP_TOL

__all__ = ["Geometry", "Batch", "project", "backproject", "diag_normal", "cgls", "lsqr", "SolveInfo", "KctError",
           "STOP_MAXITER", "STOP_TOL", "STOP_BREAKDOWN", "STOP_NUMERIC"]


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t == torch.float32:
        return _lib.KCT_F32
    if t == torch.bfloat16:
        return _lib.KCT_BF16
    if t == torch.float16:
        return _lib.KCT_F16
    if t == torch.float64:
        return _lib.KCT_F64
    raise TypeError(f"unsupported storage dtype {t} (float32, bfloat16, float16 or float64)")


def _stream_handle(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Geometry:
    """Cone-beam geometry handle (owns the device ray tables of one GPU).

    Lengths in mm; view angles t_k = angle0 + k * arc / n_views unless
    ``angles`` is given (radians).  See include/kct.h for the convention.
    ``projector`` is "siddon" (exact intersection lengths, the default) or
    "tt" (separable trapezoid footprints, Section 3).
    """

    PROJECTORS = {"siddon": _lib.PROJECTOR_SIDDON, "tt": _lib.PROJECTOR_TT}

    FIELDS = ("nx", "ny", "nz", "vx", "vy", "vz", "n_views", "nu", "nv", "du", "dv", "sid", "sdd", "cx", "cy",
              "cz", "off_u", "off_v", "angle0", "arc")

    def __init__(self, nx, ny, nz, vx, vy, vz, n_views, nu, nv, du, dv, sid=500.0, sdd=1000.0, cx=0.0, cy=0.0,
                 cz=0.0, off_u=0.0, off_v=0.0, angle0=0.0, arc=2.0 * math.pi,
                 angles: Optional[Sequence[float]] = None, device=None, projector: str = "siddon"):
        torch = _torch()
        L = _lib.load()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.vx, self.vy, self.vz = float(vx), float(vy), float(vz)
        self.n_views, self.nu, self.nv = int(n_views), int(nu), int(nv)
        self.du, self.dv, self.sid, self.sdd = float(du), float(dv), float(sid), float(sdd)
        self.cx, self.cy, self.cz = float(cx), float(cy), float(cz)
        self.off_u, self.off_v, self.angle0, self.arc = float(off_u), float(off_v), float(angle0), float(arc)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        vol = _lib.VolumeDesc(self.nx, self.ny, self.nz, self.vx, self.vy, self.vz, self.cx, self.cy, self.cz)
        self._angles = None
        ang_ptr = None
        if angles is not None:
            arr = (ctypes.c_double * self.n_views)(*[float(a) for a in angles])
            if len(angles) != self.n_views:
                raise ValueError("len(angles) must equal n_views")
            self._angles = arr
            ang_ptr = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
        cone = _lib.ConeDesc(self.n_views, self.angle0, self.arc, ang_ptr, self.sid, self.sdd, self.nu, self.nv,
                             self.du, self.dv, self.off_u, self.off_v)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(L.kct_geometry_create(ctypes.byref(vol), ctypes.byref(cone), ctypes.byref(h)))
        self._h = h
        self.projector = "siddon"
        if projector != "siddon":
            self.set_projector(projector)

    def set_projector(self, projector: str):
        """Switch the projector model of every later call with this geometry."""
        if projector not in self.PROJECTORS:
            raise ValueError(f"projector must be one of {sorted(self.PROJECTORS)}")
        _lib.check(_lib.load().kct_geometry_set_projector(self.handle, self.PROJECTORS[projector]))
        self.projector = projector

    @classmethod
    def from_desc(cls, d, device=None, projector: str = "siddon"):
        """Build from any object with the geometry attributes (e.g. kct_inputs.ConeGeometry)."""
        kw = {f: getattr(d, f) for f in cls.FIELDS}
        ang = getattr(d, "explicit_angles", None)
        return cls(**kw, angles=ang, device=device, projector=projector)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("geometry was closed")
        return self._h

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def proj_shape(self):
        return (self.n_views, self.nv, self.nu)

    @property
    def n_vox(self):
        return self.nx * self.ny * self.nz

    @property
    def n_rays(self):
        return self.n_views * self.nv * self.nu

    def project_workspace_bytes(self, dtype):
        n = ctypes.c_size_t()
        _lib.check(_lib.load().kct_project_workspace_size(self.handle, _dtype_code(dtype), ctypes.byref(n)))
        return n.value

    def solver_workspace_bytes(self, dtype, solver, jacobi: bool = False):
        n = ctypes.c_size_t()
        code = {"cgls": _lib.KCT_SOLVER_CGLS, "lsqr": _lib.KCT_SOLVER_LSQR}[solver]
        if jacobi:
            code |= _lib.KCT_SOLVER_WITH_JACOBI
        _lib.check(_lib.load().kct_solver_workspace_size(self.handle, _dtype_code(dtype), code, ctypes.byref(n)))
        return n.value

    def latencies(self):
        """Seconds from the set-up of the last batched solve to each instance's
        completion, on the device clock (see kct_batch_latencies)."""
        n = len(self.geometries)
        out = (ctypes.c_double * n)()
        _lib.check(_lib.load().kct_batch_latencies(self.handle, out))
        return list(out)

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.load().kct_geometry_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_tensor(t, shape, name, device):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, the geometry on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    _dtype_code(t.dtype)


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def project(g: Geometry, x, out=None, workspace=None, transposed_copy: bool = True):
    """b = A x (forward projection).  Returns a (n_views, nv, nu) tensor of x's dtype.

    With ``transposed_copy`` (default) the library first writes a copy of x with
    x and y swapped into ``workspace`` (allocated here if None) so that views
    whose rays run mostly along x read neighbouring addresses; without it every
    view reads x in place (same result bit for bit, slower)."""
    torch = _torch()
    _check_tensor(x, g.vol_shape, "x", g.device)
    if out is None:
        out = torch.empty(g.proj_shape, dtype=x.dtype, device=g.device)
    _check_tensor(out, g.proj_shape, "out", g.device)
    if out.dtype != x.dtype:
        raise TypeError("out must have x's dtype")
    ws_ptr, ws_bytes = None, 0
    if transposed_copy:
        if workspace is None:
            workspace = _workspace(g.project_workspace_bytes(x.dtype), g.device)
        ws_ptr, ws_bytes = ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
    with torch.cuda.device(g.device):
        _lib.check(_lib.load().kct_project(g.handle, _dtype_code(x.dtype), ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), ws_ptr, ws_bytes,
                                           _stream_handle(g.device)))
    return out


def backproject(g: Geometry, b, out=None):
    """r = A^T b (backprojection, exact transpose of project)."""
    torch = _torch()
    _check_tensor(b, g.proj_shape, "b", g.device)
    if out is None:
        out = torch.empty(g.vol_shape, dtype=b.dtype, device=g.device)
    _check_tensor(out, g.vol_shape, "out", g.device)
    if out.dtype != b.dtype:
        raise TypeError("out must have b's dtype")
    with torch.cuda.device(g.device):
        _lib.check(_lib.load().kct_backproject(g.handle, _dtype_code(b.dtype), ctypes.c_void_p(b.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()), _stream_handle(g.device)))
    return out


@dataclasses.dataclass
class SolveInfo:
    iterations: int
    nb0: float
    nb: float
    nr2: float
    stop_reason: int
    history: Optional[object] = None


def diag_normal(g: Geometry, out=None):
    """diag(A^T A) = sum_i w_ij^2 per voxel (float32 volume), the diagonal that
    Jacobi preconditioning inverts."""
    torch = _torch()
    if out is None:
        out = torch.empty(g.vol_shape, dtype=torch.float32, device=g.device)
    _check_tensor(out, g.vol_shape, "out", g.device)
    if out.dtype != torch.float32:
        raise TypeError("out must be float32")
    with torch.cuda.device(g.device):
        _lib.check(_lib.load().kct_diag_normal(g.handle, ctypes.c_void_p(out.data_ptr()), _stream_handle(g.device)))
    return out


def _solve(which, g, b, K, x0, err, history, workspace, out, tikhonov=0.0, jacobi=False, recompute_every=0):
    """b (and the workspace vectors) in b's storage dtype; the iterate x is float32."""
    torch = _torch()
    _check_tensor(b, g.proj_shape, "b", g.device)
    if out is None:
        out = torch.empty(g.vol_shape, dtype=torch.float32, device=g.device)
    _check_tensor(out, g.vol_shape, "out", g.device)
    if out.dtype != torch.float32:
        raise TypeError("the solution x is float32 (16-bit iterates stagnate)")
    if x0 is not None:
        _check_tensor(x0, g.vol_shape, "x0", g.device)
        if x0.data_ptr() != out.data_ptr():
            out.copy_(x0)
    hist = torch.zeros(max(int(K), 1), dtype=torch.float64, device=g.device) if history else None
    opts = _lib.SolveOpts(int(K), float(err), int(x0 is None), ctypes.c_void_p(hist.data_ptr()) if hist is not None
                          else None, float(tikhonov), int(bool(jacobi)), int(recompute_every))
    if workspace is None:
        workspace = _workspace(g.solver_workspace_bytes(b.dtype, which, jacobi=bool(jacobi)), g.device)
    ws_bytes = workspace.numel() * workspace.element_size()
    info = _lib.SolveInfo()
    fn = _lib.load().kct_cgls_solve if which == "cgls" else _lib.load().kct_lsqr_solve
    with torch.cuda.device(g.device):
        st = fn(g.handle, _dtype_code(b.dtype), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                ctypes.byref(opts), ctypes.c_void_p(workspace.data_ptr()), ws_bytes, ctypes.byref(info),
                _stream_handle(g.device))
    if st not in (_lib.KCT_OK, _lib.KCT_ERR_NUMERIC):
        _lib.check(st)
    res = SolveInfo(info.iterations, info.nb0, info.nb, info.nr2, info.stop_reason,
                    hist[: info.iterations].clone() if hist is not None else None)
    if st == _lib.KCT_ERR_NUMERIC:
        raise KctError(st, _lib.load().kct_last_error().decode(errors="replace"))
    return out, res


def cgls(g: Geometry, b, K: int, x0=None, err: float = 0.0, history: bool = False, workspace=None, out=None,
         tikhonov: float = 0.0, jacobi: bool = False, recompute_every: int = 0):
    """CGLS with delayed residual computation (Algorithm 1): returns (x_K, SolveInfo).

    tikhonov = lambda adds lambda^2 |x|^2 to the objective; jacobi preconditions
    with diag(A^T A)^(-1/2); recompute_every = k recomputes e = b - A x after
    every k-th iteration (see kct_solve_opts in include/kct.h)."""
    return _solve("cgls", g, b, K, x0, err, history, workspace, out, tikhonov, jacobi, recompute_every)


def lsqr(g: Geometry, b, K: int, x0=None, err: float = 0.0, history: bool = False, workspace=None, out=None,
         tikhonov: float = 0.0):
    """LSQR (Paige & Saunders), iterations aligned with CGLS: returns (x_K, SolveInfo).

    tikhonov = lambda > 0 (damping, x0 = 0 only) minimises |b - A x|^2 + lambda^2 |x|^2;
    info.nb is then the norm of the stacked residual [b - A x; -lambda x]."""
    return _solve("lsqr", g, b, K, x0, err, history, workspace, out, tikhonov)


def timing_enable(on: bool = True):
    """Start (clearing the record) or stop recording the duration of every
    projector launch of the solvers' iterations (kct_timing_enable)."""
    _lib.check(_lib.load().kct_timing_enable(1 if on else 0))


def timing_get(kind: str):
    """(count, average ms, min ms, max ms) of the recorded "forward" or
    "backward" launches (kct_timing_get)."""
    n = ctypes.c_int32(0)
    avg, lo, hi = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    _lib.check(_lib.load().kct_timing_get({"forward": 0, "backward": 1}[kind], ctypes.byref(n), ctypes.byref(avg),
                                          ctypes.byref(lo), ctypes.byref(hi)))
    return n.value, avg.value, lo.value, hi.value


class Batch:
    """Batched CGLS over independent reconstructions with their own geometries
    (kct_batch_* in include/kct.h): every step of Algorithm 1 is one launch for
    all instances (persistent work-queue launches for the projector steps), one
    iteration is replayed as a HIP graph.  FP32 storage.

        batch = Batch([g1, g2, ...])
        batch.tune(cache="tune.txt")            # optional: forward and backprojection variants
        xs, infos = batch.cgls([b1, b2, ...], K)
        seconds = batch.latencies()             # per-instance completion times of that solve
    """

    def __init__(self, geometries: Sequence[Geometry]):
        torch = _torch()
        if not geometries:
            raise ValueError("a batch needs at least one geometry")
        self.geometries = list(geometries)
        self.device = self.geometries[0].device
        for g in self.geometries:
            if g.device != self.device:
                raise ValueError("all geometries of a batch must be on one device")
        arr = (ctypes.c_void_p * len(self.geometries))(*[g.handle.value for g in self.geometries])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().kct_batch_create(arr, len(self.geometries), ctypes.byref(h)))
        self._h = h
        self._ws = None

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("batch was closed")
        return self._h

    def workspace_bytes(self):
        n = ctypes.c_size_t()
        _lib.check(_lib.load().kct_batch_workspace_size(self.handle, ctypes.byref(n)))
        return n.value

    def _workspace(self, workspace):
        if workspace is not None:
            return workspace
        if self._ws is None:
            self._ws = _workspace(self.workspace_bytes(), self.device)
        return self._ws

    def tune(self, cache: Optional[str] = None, workspace=None):
        """Choose each instance's forward and backprojection variants by timing (see kct_batch_tune)."""
        torch = _torch()
        ws = self._workspace(workspace)
        with torch.cuda.device(self.device):
            _lib.check(_lib.load().kct_batch_tune(self.handle, ctypes.c_void_p(ws.data_ptr()),
                                                  ws.numel() * ws.element_size(),
                                                  cache.encode() if cache else None, _stream_handle(self.device)))

    def cgls(self, bs, K: int, err: float = 0.0, graph: bool = True, workspace=None, outs=None):
        """x_i = CGLS_K(b_i) from x0 = 0 for every instance: returns (list of x, list of SolveInfo)."""
        torch = _torch()
        n = len(self.geometries)
        if len(bs) != n:
            raise ValueError(f"expected {n} projection tensors")
        if outs is None:
            outs = [torch.empty(g.vol_shape, dtype=torch.float32, device=self.device) for g in self.geometries]
        for g, b, x in zip(self.geometries, bs, outs):
            _check_tensor(b, g.proj_shape, "b", self.device)
            _check_tensor(x, g.vol_shape, "x", self.device)
            if b.dtype != torch.float32 or x.dtype != torch.float32:
                raise TypeError("batched CGLS uses float32 storage")
        ws = self._workspace(workspace)
        bp = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
        xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in outs])
        opts = _lib.SolveOpts(int(K), float(err), 1, None, 0.0, 0, 0)
        infos = (_lib.SolveInfo * n)()
        with torch.cuda.device(self.device):
            st = _lib.load().kct_batch_cgls_solve(self.handle, bp, xp, ctypes.byref(opts), int(bool(graph)),
                                                   ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                                   infos, _stream_handle(self.device))
        if st != _lib.KCT_OK:
            _lib.check(st)
        res = [SolveInfo(i.iterations, i.nb0, i.nb, i.nr2, i.stop_reason) for i in infos]
        return outs, res

    def latencies(self):
        """Seconds from the set-up of the last batched solve to each instance's
        completion, on the device clock (see kct_batch_latencies)."""
        n = len(self.geometries)
        out = (ctypes.c_double * n)()
        _lib.check(_lib.load().kct_batch_latencies(self.handle, out))
        return list(out)

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.load().kct_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
