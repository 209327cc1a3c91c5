"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds geometry descriptions (plain numbers), the seeded ellipsoid
phantom and the noise models.  It contains none of the projector or solver
arithmetic: both the FP64 oracle and the HIP library receive what is made here
and compute on their own.

Geometry convention (also stated in the oracle and the library): world frame in
mm, rotation axis +z, source at (SID cos t, SID sin t, 0), flat detector at
distance SDD from the source, detector u axis (-sin t, cos t, 0), v axis +z,
pixel centres at (i - (n-1)/2) * pitch + offset, volume centred at (cx, cy, cz).
Views are t_k = angle0 + k * arc / n_views (a full 360 degree orbit without the
duplicated end point unless stated otherwise).

Phantom recipe (stands in for the paper's 3D Shepp-Logan phantom, Section 4,
whose parameter table is not reproduced here): N ellipsoids with additive
densities.  Ellipsoid 0 is the base: centred, axis aligned, semi-axes
(0.45, 0.40, 0.42) L with L the volume side in mm, density 1.  Each further
ellipsoid draws, in this order from numpy's PCG64 ``default_rng(seed)``: centre
~ U[-0.35 L, 0.35 L]^3 about the volume centre, three semi-axes ~ U[4, 28] L/64
mm, a rotation from a normalised 4-vector of N(0, 1) (a uniform random
quaternion) and a density ~ U[-0.8, 1.0].  A voxel's value is the sum of the
densities of the ellipsoids that contain its centre (or the mean over s^3
sub-samples when ``supersample = s``).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class ConeGeometry:
    """Circular cone-beam geometry and voxel grid (all lengths in mm)."""

    nx: int
    ny: int
    nz: int
    vx: float
    vy: float
    vz: float
    n_views: int
    nu: int
    nv: int
    du: float
    dv: float
    sid: float = 500.0
    sdd: float = 1000.0
    cx: float = 0.0
    cy: float = 0.0
    cz: float = 0.0
    off_u: float = 0.0
    off_v: float = 0.0
    angle0: float = 0.0
    arc: float = 2.0 * math.pi
    explicit_angles: Optional[Sequence[float]] = None

    def angles(self) -> np.ndarray:
        if self.explicit_angles is not None:
            a = np.asarray(self.explicit_angles, dtype=np.float64)
            assert a.size == self.n_views
            return a
        k = np.arange(self.n_views, dtype=np.float64)
        return self.angle0 + k * (self.arc / self.n_views)

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_rays(self) -> int:
        return self.n_views * self.nv * self.nu

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def proj_shape(self):
        return (self.n_views, self.nv, self.nu)

    def side_mm(self) -> float:
        return max(self.nx * self.vx, self.ny * self.vy, self.nz * self.vz)

    def replace(self, **kw) -> "ConeGeometry":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------- configs

def t16(variant: str = "base") -> ConeGeometry:
    """Tiny test grid: 16^3 @ 1 mm, 12 views, 48 x 48 detector @ 1 mm, SID 500, SDD 1000.

    Variants: ``offcenter`` (volume centre +3.1, -2.3, +1.7 mm), ``aniso``
    (1 x 1 x 2.5 mm voxels), ``odd`` (47 x 45 detector, so central rays lie in
    voxel planes).
    """
    g = ConeGeometry(nx=16, ny=16, nz=16, vx=1.0, vy=1.0, vz=1.0, n_views=12, nu=48, nv=48,
                     du=1.0, dv=1.0)
    if variant == "base":
        return g
    if variant == "offcenter":
        return g.replace(cx=3.1, cy=-2.3, cz=1.7)
    if variant == "aniso":
        return g.replace(vz=2.5)
    if variant == "odd":
        return g.replace(nu=47, nv=45)
    raise ValueError(variant)


def config(name: str) -> ConeGeometry:
    """Named workloads.

    c1     64^3 @ 1.0 mm, 90 views, 96 x 96 @ 1.0 mm (truncated detector)
    c2     256^3 @ 0.5 mm, 360 views, 384 x 384 @ 0.8 mm
    c3     512^3 @ 0.25 mm, 720 views, 616 x 480 @ 0.6 mm
    c3down 128^3 @ 1.0 mm, 720 views, 154 x 120 @ 2.4 mm (c3 re-discretised)
    c5     192^3 @ 0.5 mm, 180 views, 256 x 256 @ 0.8 mm
    fd24   24^3 @ 2.0 mm, 24 views, 48 x 48 @ 2.0 mm
    All: SID 500 mm, SDD 1000 mm, views uniform over 360 degrees.
    """
    if name == "c1":
        return ConeGeometry(64, 64, 64, 1.0, 1.0, 1.0, 90, 96, 96, 1.0, 1.0)
    if name == "c2":
        return ConeGeometry(256, 256, 256, 0.5, 0.5, 0.5, 360, 384, 384, 0.8, 0.8)
    if name == "c3":
        return ConeGeometry(512, 512, 512, 0.25, 0.25, 0.25, 720, 616, 480, 0.6, 0.6)
    if name == "c3down":
        return ConeGeometry(128, 128, 128, 1.0, 1.0, 1.0, 720, 154, 120, 2.4, 2.4)
    if name == "c5":
        return ConeGeometry(192, 192, 192, 0.5, 0.5, 0.5, 180, 256, 256, 0.8, 0.8)
    if name == "fd24":
        return ConeGeometry(24, 24, 24, 2.0, 2.0, 2.0, 24, 48, 48, 2.0, 2.0)
    raise ValueError(name)


def batch_instance(i: int, scale: float = 1.0) -> ConeGeometry:
    """Instance i of the batched workload (48 uneven reconstructions), drawn
    from default_rng(4000 + i) in this order: volume side n in {64, 96, 128, 192},
    views in 60..360, square detector side in 96..288 pixels of 1 mm, SID in
    [400, 700] mm, SDD in [800, 1400] mm (at least SID + 100).  The voxel size
    makes the volume fill 95 % of the cylinder the detector sees:
    v = 0.95 * 2 * SID * sin(atan(side / (2 SDD))) / n.  ``scale`` shrinks n,
    views and side for small test batches (geometry ratios kept)."""
    rng = np.random.default_rng(4000 + i)
    n = int(rng.choice([64, 96, 128, 192]))
    views = int(rng.integers(60, 361))
    side = int(rng.integers(96, 289))
    sid = float(rng.uniform(400.0, 700.0))
    sdd = float(rng.uniform(800.0, 1400.0))
    sdd = max(sdd, sid + 100.0)
    if scale != 1.0:
        n = max(8, int(round(n * scale)))
        views = max(4, int(round(views * scale)))
        side = max(8, int(round(side * scale)))
    du = 1.0 / scale
    vox = 0.95 * 2.0 * sid * math.sin(math.atan(side * du / (2.0 * sdd))) / n
    return ConeGeometry(n, n, n, vox, vox, vox, views, side, side, du, du, sid=sid, sdd=sdd)


SEEDS = {"c1": 101, "c2": 202, "c3": 303, "c3down": 303, "c5": 5000, "fd24": 5000}
N_ELLIPSOIDS = {"c1": 10, "c2": 20, "c3": 20, "c3down": 20, "c5": 10, "fd24": 10}


# ----------------------------------------------------------------- phantom

@dataclasses.dataclass
class Ellipsoid:
    centre: np.ndarray  # (3,) mm, world frame
    semi: np.ndarray  # (3,) mm
    rot: np.ndarray  # (3, 3), columns are the ellipsoid axes in world frame
    density: float


def _quat_to_rot(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def draw_ellipsoids(g: ConeGeometry, n: int, seed: int) -> List[Ellipsoid]:
    """The phantom's ellipsoids, drawn in the documented order."""
    rng = np.random.default_rng(seed)
    L = g.side_mm()
    c0 = np.array([g.cx, g.cy, g.cz], dtype=np.float64)
    out = [Ellipsoid(c0.copy(), np.array([0.45, 0.40, 0.42]) * L, np.eye(3), 1.0)]
    for _ in range(n - 1):
        centre = c0 + rng.uniform(-0.35 * L, 0.35 * L, size=3)
        semi = rng.uniform(4.0, 28.0, size=3) * (L / 64.0)
        q = rng.standard_normal(4)
        q = q / np.linalg.norm(q)
        dens = rng.uniform(-0.8, 1.0)
        out.append(Ellipsoid(centre, semi, _quat_to_rot(q), float(dens)))
    return out


def voxelize(g: ConeGeometry, ells: Sequence[Ellipsoid], supersample: int = 1,
             dtype=np.float32) -> np.ndarray:
    """Sum of ellipsoid densities at voxel centres (or the mean over s^3 sub-samples)."""
    x = np.zeros(g.vol_shape, dtype=np.float64)
    s = int(supersample)
    sub = (np.arange(s) + 0.5) / s  # sub-sample offsets inside a voxel, in voxel units
    X0 = g.cx - 0.5 * g.nx * g.vx
    Y0 = g.cy - 0.5 * g.ny * g.vy
    Z0 = g.cz - 0.5 * g.nz * g.vz
    for e in ells:
        ext = np.sqrt(((e.rot * e.semi[None, :]) ** 2).sum(axis=1))  # half extent per world axis
        lo = e.centre - ext
        hi = e.centre + ext
        ix0 = max(int(math.floor((lo[0] - X0) / g.vx)), 0)
        ix1 = min(int(math.ceil((hi[0] - X0) / g.vx)), g.nx)
        iy0 = max(int(math.floor((lo[1] - Y0) / g.vy)), 0)
        iy1 = min(int(math.ceil((hi[1] - Y0) / g.vy)), g.ny)
        iz0 = max(int(math.floor((lo[2] - Z0) / g.vz)), 0)
        iz1 = min(int(math.ceil((hi[2] - Z0) / g.vz)), g.nz)
        if ix0 >= ix1 or iy0 >= iy1 or iz0 >= iz1:
            continue
        M = (e.rot / e.semi[None, :]).T  # maps world offsets to unit-sphere coordinates
        xs = X0 + (np.arange(ix0, ix1)[:, None] + sub[None, :]) * g.vx  # (nx', s)
        ys = Y0 + (np.arange(iy0, iy1)[:, None] + sub[None, :]) * g.vy
        xs = (xs - e.centre[0]).reshape(-1)
        ys = (ys - e.centre[1]).reshape(-1)
        for iz in range(iz0, iz1):
            zs = Z0 + (iz + sub) * g.vz - e.centre[2]  # (s,)
            # unit coords: u = M @ [dx, dy, dz]
            acc = np.zeros((iy1 - iy0, ix1 - ix0), dtype=np.float64)
            for dz in zs:
                u = (M[:, 0][:, None, None] * xs[None, None, :] + M[:, 1][:, None, None] * ys[None, :, None]
                     + M[:, 2][:, None, None] * dz)
                inside = (u * u).sum(axis=0) <= 1.0  # (ny'*s, nx'*s)
                acc += inside.reshape(iy1 - iy0, s, ix1 - ix0, s).sum(axis=(1, 3))
            x[iz, iy0:iy1, ix0:ix1] += e.density * acc / float(s ** 3)
    return x.astype(dtype)


def phantom(g: ConeGeometry, n_ellipsoids: int, seed: int, supersample: int = 1,
            dtype=np.float32) -> np.ndarray:
    return voxelize(g, draw_ellipsoids(g, n_ellipsoids, seed), supersample, dtype)


# ----------------------------------------------------------------- noise

def gaussian_noise(b: np.ndarray, rel_sigma: float, seed: int) -> np.ndarray:
    """b + N(0, (rel_sigma * max(b))^2), seeded."""
    rng = np.random.default_rng(seed)
    sigma = rel_sigma * float(np.max(b))
    return (b + sigma * rng.standard_normal(b.shape)).astype(b.dtype)


def poisson_log_noise(b: np.ndarray, photons: float, seed: int) -> np.ndarray:
    """Transmission noise: scale c = 4 / max(b), I ~ Poisson(photons * exp(-c b)),
    returned as -ln(max(I, 1) / photons) / c (the log-transformed line integral)."""
    rng = np.random.default_rng(seed)
    c = 4.0 / float(np.max(b))
    lam = photons * np.exp(-c * b.astype(np.float64))
    counts = rng.poisson(lam)
    return (-np.log(np.maximum(counts, 1) / photons) / c).astype(b.dtype)


def random_volume(g: ConeGeometry, seed: int, dtype=np.float64) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=g.vol_shape).astype(dtype)


def random_projections(g: ConeGeometry, seed: int, dtype=np.float64) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=g.proj_shape).astype(dtype)
