"""Independent brute-force cone-beam system matrix for tiny grids (test pin).

For every (ray, voxel) pair the weight is the length of the source -> pixel-centre
segment inside the voxel box, found with the slab method (intersect the three
parameter intervals of the box's face pairs).  A direction component that is
exactly zero uses the half-open rule lo <= s < hi.  Written from the definition
of the Siddon model (the chord length of a ray through each voxel, Section 3 of
the paper) with its own geometry code; it shares nothing with the oracle's
traversal.
"""
import numpy as np
import scipy.sparse as sp


def rays(g):
    """Source (n_views, 3) and pixel centres (n_views, nv, nu, 3) under the convention."""
    th = g.angles()
    c, s = np.cos(th), np.sin(th)
    src = np.stack([g.sid * c, g.sid * s, np.zeros_like(c)], axis=-1)
    cen = src - g.sdd * np.stack([c, s, np.zeros_like(c)], axis=-1)
    eu = np.stack([-s, c, np.zeros_like(c)], axis=-1)
    u = (np.arange(g.nu) - 0.5 * (g.nu - 1)) * g.du + g.off_u
    v = (np.arange(g.nv) - 0.5 * (g.nv - 1)) * g.dv + g.off_v
    q = (cen[:, None, None, :] + u[None, None, :, None] * eu[:, None, None, :]
         + v[None, :, None, None] * np.array([0.0, 0.0, 1.0])[None, None, None, :])
    return src, q


def _axis_intervals(s, d, lo, vox, n):
    """Per ray and per cell along one axis: the segment-parameter interval inside the cell."""
    edges = lo + np.arange(n + 1) * vox  # (n+1,)
    a_lo = np.empty((s.size, n))
    a_hi = np.empty((s.size, n))
    nz = d != 0
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (edges[None, :] - s[:, None]) / d[:, None]
    t0, t1 = t[:, :-1], t[:, 1:]
    a_lo[nz] = np.minimum(t0, t1)[nz]
    a_hi[nz] = np.maximum(t0, t1)[nz]
    z = ~nz
    if z.any():
        inside = (s[z][:, None] >= edges[None, :-1]) & (s[z][:, None] < edges[None, 1:])
        a_lo[z] = np.where(inside, -np.inf, np.inf)
        a_hi[z] = np.where(inside, np.inf, -np.inf)
    return a_lo, a_hi


def matrix(g, chunk=512):
    """Assemble A (m x n, CSR) pair by pair.  Tiny grids only."""
    src, q = rays(g)
    X0 = g.cx - 0.5 * g.nx * g.vx
    Y0 = g.cy - 0.5 * g.ny * g.vy
    Z0 = g.cz - 0.5 * g.nz * g.vz
    rows, cols, vals = [], [], []
    nray_view = g.nv * g.nu
    for k in range(g.n_views):
        qk = q[k].reshape(-1, 3)
        sk = np.broadcast_to(src[k], qk.shape)
        d = qk - sk
        length = np.sqrt((d * d).sum(axis=1))
        for c0 in range(0, nray_view, chunk):
            sl = slice(c0, min(c0 + chunk, nray_view))
            xl, xh = _axis_intervals(sk[sl, 0], d[sl, 0], X0, g.vx, g.nx)
            yl, yh = _axis_intervals(sk[sl, 1], d[sl, 1], Y0, g.vy, g.ny)
            zl, zh = _axis_intervals(sk[sl, 2], d[sl, 2], Z0, g.vz, g.nz)
            lo = np.maximum(np.maximum(zl[:, :, None, None], yl[:, None, :, None]), xl[:, None, None, :])
            hi = np.minimum(np.minimum(zh[:, :, None, None], yh[:, None, :, None]), xh[:, None, None, :])
            lo = np.maximum(lo, 0.0)
            hi = np.minimum(hi, 1.0)
            w = np.maximum(hi - lo, 0.0) * length[sl][:, None, None, None]
            r, j = np.nonzero(w.reshape(w.shape[0], -1) > 0)
            rows.append(k * nray_view + c0 + r)
            cols.append(j)
            vals.append(w.reshape(w.shape[0], -1)[r, j])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(g.n_rays, g.n_vox))


def box_chord(g, box_lo, box_hi):
    """Chord length of every ray through one axis-aligned box (closed form)."""
    src, q = rays(g)
    s = np.broadcast_to(src[:, None, None, :], q.shape).reshape(-1, 3)
    qq = q.reshape(-1, 3)
    d = qq - s
    amin = np.zeros(s.shape[0])
    amax = np.ones(s.shape[0])
    for a in range(3):
        with np.errstate(divide="ignore", invalid="ignore"):
            t0 = (box_lo[a] - s[:, a]) / d[:, a]
            t1 = (box_hi[a] - s[:, a]) / d[:, a]
        par = d[:, a] == 0
        lo = np.where(par, np.where((s[:, a] >= box_lo[a]) & (s[:, a] < box_hi[a]), -np.inf, np.inf),
                      np.minimum(t0, t1))
        hi = np.where(par, np.where((s[:, a] >= box_lo[a]) & (s[:, a] < box_hi[a]), np.inf, -np.inf),
                      np.maximum(t0, t1))
        amin = np.maximum(amin, lo)
        amax = np.minimum(amax, hi)
    return (np.maximum(amax - amin, 0.0) * np.sqrt((d * d).sum(axis=1))).reshape(g.proj_shape)


def ellipsoid_chords(g, e):
    """Analytic line integral of a uniform ellipsoid (density e.density) along every ray.

    Solves |M (s + t d - c)| = 1 for t (M maps world offsets to unit-sphere
    coordinates) and returns density * |t2 - t1| * |d| clipped to the segment.
    """
    src, q = rays(g)
    s = np.broadcast_to(src[:, None, None, :], q.shape).reshape(-1, 3)
    d = q.reshape(-1, 3) - s
    M = (e.rot / e.semi[None, :]).T
    p = (s - e.centre[None, :]) @ M.T
    m = d @ M.T
    A = (m * m).sum(1)
    B = 2 * (p * m).sum(1)
    C = (p * p).sum(1) - 1.0
    disc = B * B - 4 * A * C
    ok = disc > 0
    sq = np.sqrt(np.where(ok, disc, 0.0))
    t1 = np.clip((-B - sq) / (2 * A), 0.0, 1.0)
    t2 = np.clip((-B + sq) / (2 * A), 0.0, 1.0)
    chord = np.where(ok, (t2 - t1) * np.sqrt((d * d).sum(1)), 0.0)
    return (e.density * chord).reshape(g.proj_shape)
