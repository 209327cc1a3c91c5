/*
 * kct_oracle.c -- plain, slow FP64 CPU oracle for the cone-beam projector pair
 * and the two Krylov solvers of Kulvait & Rose, "Software Implementation of the
 * Krylov Methods Based Reconstruction for the 3D Cone Beam CT Operator"
 * (Fully3D 2021, arXiv 2110.13526).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or table with the HIP library.
 *
 * What it computes (all in double precision):
 *
 *   A      -- Section 2, Eq. (1): b = A x.  A is the cone-beam operator with the
 *             Siddon ray model named in Section 3: ray i runs from the source to
 *             the centre of detector pixel i, and w_ij is the length (mm) of the
 *             part of that segment lying inside voxel j.  Implemented by the
 *             classic Siddon traversal: intersect the segment with the volume
 *             box, merge the sorted parameters at which it crosses the x, y and z
 *             voxel planes, and give every piece between consecutive crossings
 *             to the voxel it lies in (the entry cell of each axis is found by
 *             counting that axis' planes crossed before the entry point, then
 *             every crossing moves one cell; this stays exact for rays running
 *             within rounding distance of a voxel plane).
 *   A^T    -- Section 2, Eq. (2): the same traversal, scattering w_ij * y_i into
 *             r_j.  Parallel over disjoint z-slabs of the output (each ray is
 *             clipped to the slab), so it is deterministic without atomics.
 *   CGLS   -- Section 2, Algorithm 1 (CGLS with delayed residual computation),
 *             step for step.  The direction update is read as d = r + beta d
 *             (the printed "d = d + beta r" is not conjugate gradients); the
 *             printed form is kept behind a flag so tests can show it fails.
 *   LSQR   -- named in Section 2 (Paige & Saunders 1982); not printed in the
 *             paper, so the published Golub-Kahan bidiagonalisation + Givens
 *             form is followed, with x0 entering through u = b - A x0.
 *   Variants named in Sections 3, 5 and 7: the Tikhonov (L2) term
 *             lambda^2 |x|^2 (CGLS on the stacked system [A; lambda I]; LSQR
 *             with Paige & Saunders' damping), the diagonal of A^T A and
 *             Jacobi-preconditioned CGLS (Algorithm 1 on A diag(A^T A)^(-1/2)),
 *             and CGLS with the discrepancy recomputed every k iterations.
 *   A_TT   -- the separable trapezoid-footprint model named in Section 3 (the
 *             projector of the experiments in Section 4), with its adjoint and
 *             squared-weight sums; CGLS and LSQR run on either operator.
 *
 * Geometry convention (the paper gives only SID, SDD, pixel size and the number
 * of angles, Section 4): right-handed world frame in mm, rotation axis +z,
 * source s_k = (SID cos t, SID sin t, 0), detector centre c_k = s_k - SDD
 * (cos t, sin t, 0), detector axes e_u = (-sin t, cos t, 0), e_v = (0, 0, 1),
 * pixel centre q = c_k + u e_u + v e_v with u = (iu - (nu-1)/2) du + off_u,
 * v = (iv - (nv-1)/2) dv + off_v.  Voxel (ix,iy,iz) spans
 * [X0 + ix vx, X0 + (ix+1) vx] x ... with X0 = cx - nx vx / 2 (same for y, z).
 * Memory order: x[iz][iy][ix] (ix fastest), b[k][iv][iu] (iu fastest).
 * A ray that lies exactly in a voxel plane is given to the cell above the plane
 * (cells are half-open [lo, hi)); this only matters for measure-zero ties.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Geometry passed as two plain arrays:
 *   dims[6] = { nx, ny, nz, n_views, nu, nv }
 *   par[12] = { vx, vy, vz, cx, cy, cz, sid, sdd, du, dv, off_u, off_v }
 *   angles[n_views] in radians.                                           */
typedef struct {
    int nx, ny, nz, nviews, nu, nv;
    double vx, vy, vz, cx, cy, cz, sid, sdd, du, dv, off_u, off_v;
    const double *ang;
} og_t;

static og_t og_make(const int32_t *dims, const double *par, const double *angles)
{
    og_t g;
    g.nx = dims[0]; g.ny = dims[1]; g.nz = dims[2];
    g.nviews = dims[3]; g.nu = dims[4]; g.nv = dims[5];
    g.vx = par[0]; g.vy = par[1]; g.vz = par[2];
    g.cx = par[3]; g.cy = par[4]; g.cz = par[5];
    g.sid = par[6]; g.sdd = par[7]; g.du = par[8]; g.dv = par[9];
    g.off_u = par[10]; g.off_v = par[11];
    g.ang = angles;
    return g;
}

/* Source and pixel centre of ray (k, iv, iu) under the convention above. */
static void og_ray(const og_t *g, int k, int iv, int iu, double s[3], double q[3])
{
    double c = cos(g->ang[k]), sn = sin(g->ang[k]);
    double u = ((double)iu - 0.5 * (double)(g->nu - 1)) * g->du + g->off_u;
    double v = ((double)iv - 0.5 * (double)(g->nv - 1)) * g->dv + g->off_v;
    s[0] = g->sid * c;
    s[1] = g->sid * sn;
    s[2] = 0.0;
    double cen0 = s[0] - g->sdd * c, cen1 = s[1] - g->sdd * sn;
    q[0] = cen0 + u * (-sn);
    q[1] = cen1 + u * c;
    q[2] = v;
}

/* Position of voxel plane m (0..n) along one axis. */
static double og_plane(double lo, double vox, int m) { return lo + (double)m * vox; }

/* Per-thread scratch for one traversal: the merged list and one list per axis. */
typedef struct {
    double *al, *ax[3];
} og_scratch;

static og_scratch og_scratch_new(const og_t *g)
{
    og_scratch sc;
    sc.al = (double *)malloc(sizeof(double) * (size_t)(g->nx + g->ny + g->nz + 8));
    sc.ax[0] = (double *)malloc(sizeof(double) * (size_t)(g->nx + 2));
    sc.ax[1] = (double *)malloc(sizeof(double) * (size_t)(g->ny + 2));
    sc.ax[2] = (double *)malloc(sizeof(double) * (size_t)(g->nz + 2));
    return sc;
}

static void og_scratch_free(og_scratch *sc)
{
    free(sc->al);
    for (int a = 0; a < 3; ++a) free(sc->ax[a]);
}

/*
 * Siddon traversal of the segment s -> q, restricted to z-cells [zlo, zhi).
 * Writes the (voxel index, weight) pairs of every piece with positive length
 * and returns their count.  idx/w must hold nx + ny + (zhi - zlo) + 4 entries.
 */
static int og_trace(const og_t *g, og_scratch *sc, const double s[3], const double q[3],
                    int zlo, int zhi, int64_t *idx, double *w)
{
    const int n[3] = { g->nx, g->ny, g->nz };
    const double vox[3] = { g->vx, g->vy, g->vz };
    double lo[3], d[3];
    lo[0] = g->cx - 0.5 * g->nx * g->vx;
    lo[1] = g->cy - 0.5 * g->ny * g->vy;
    lo[2] = g->cz - 0.5 * g->nz * g->vz;
    for (int a = 0; a < 3; ++a) d[a] = q[a] - s[a];
    const int mlo[3] = { 0, 0, zlo }, mhi[3] = { n[0], n[1], zhi };

    /* 1. clip the segment (alpha in [0,1]) to the box of cells [mlo, mhi). */
    double amin = 0.0, amax = 1.0;
    for (int a = 0; a < 3; ++a) {
        double p0 = og_plane(lo[a], vox[a], mlo[a]);
        double p1 = og_plane(lo[a], vox[a], mhi[a]);
        if (d[a] != 0.0) {
            double a0 = (p0 - s[a]) / d[a], a1 = (p1 - s[a]) / d[a];
            double lo_a = a0 < a1 ? a0 : a1, hi_a = a0 < a1 ? a1 : a0;
            if (lo_a > amin) amin = lo_a;
            if (hi_a < amax) amax = hi_a;
        } else if (!(s[a] >= p0 && s[a] < p1)) {
            return 0; /* parallel to this axis and outside the half-open slab */
        }
    }
    if (!(amax > amin)) return 0;

    /* 2. the crossing parameters of each axis inside (amin, amax), ascending,
     *    and the cell each axis is in at amin: the number of that axis' planes
     *    crossed at or before amin fixes it (cells are counted along the ray). */
    double **ax = sc->ax;
    int cnt[3], cell[3], step[3];
    for (int a = 0; a < 3; ++a) {
        cnt[a] = 0;
        if (d[a] == 0.0) {
            cell[a] = (int)floor((s[a] - lo[a]) / vox[a]);
            step[a] = 0;
            continue;
        }
        int before = 0;
        if (d[a] > 0) {
            for (int m = mlo[a]; m <= mhi[a]; ++m) {
                double t = (og_plane(lo[a], vox[a], m) - s[a]) / d[a];
                if (t <= amin) ++before;
                else if (t < amax) ax[a][cnt[a]++] = t;
            }
            cell[a] = mlo[a] + before - 1;
            step[a] = 1;
        } else {
            for (int m = mhi[a]; m >= mlo[a]; --m) {
                double t = (og_plane(lo[a], vox[a], m) - s[a]) / d[a];
                if (t <= amin) ++before;
                else if (t < amax) ax[a][cnt[a]++] = t;
            }
            cell[a] = mhi[a] - before;
            step[a] = -1;
        }
    }
    /* 3. walk the three sorted lists in merged order; each piece between two
     *    consecutive parameters lies in the current cell, and passing a
     *    crossing moves that axis one cell along the ray. */
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    int i0 = 0, i1 = 0, i2 = 0, out = 0;
    double t_cur = amin;
    for (;;) {
        double t0 = i0 < cnt[0] ? ax[0][i0] : INFINITY;
        double t1 = i1 < cnt[1] ? ax[1][i1] : INFINITY;
        double t2 = i2 < cnt[2] ? ax[2][i2] : INFINITY;
        int which;
        double t_next;
        if (t0 <= t1 && t0 <= t2) { which = 0; t_next = t0; }
        else if (t1 <= t2) { which = 1; t_next = t1; }
        else { which = 2; t_next = t2; }
        int last = !(t_next < amax);
        if (last) t_next = amax;
        double dl = t_next - t_cur;
        if (dl > 0.0 && cell[0] >= mlo[0] && cell[0] < mhi[0] && cell[1] >= mlo[1] && cell[1] < mhi[1]
            && cell[2] >= mlo[2] && cell[2] < mhi[2]) {
            idx[out] = ((int64_t)cell[2] * g->ny + cell[1]) * g->nx + cell[0];
            w[out] = dl * len;
            ++out;
        }
        if (last) break;
        t_cur = t_next;
        cell[which] += step[which];
        if (which == 0) ++i0;
        else if (which == 1) ++i1;
        else ++i2;
    }
    (void)sc->al;
    return out;
}

static int og_cap(const og_t *g) { return g->nx + g->ny + g->nz + 4; }

/* ---------------------------------------------------------------- A, A^T */

/* b = A x (Eq. 1). */
void oracle_project(const int32_t *dims, const double *par, const double *angles,
                    const double *x, double *b)
{
    og_t g = og_make(dims, par, angles);
    int64_t nrays = (int64_t)g.nviews * g.nv * g.nu;
#pragma omp parallel
    {
        int cap = og_cap(&g);
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        double *w = (double *)malloc(sizeof(double) * (size_t)cap);
        og_scratch sc = og_scratch_new(&g);
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < nrays; ++r) {
            int k = (int)(r / ((int64_t)g.nv * g.nu));
            int iv = (int)((r / g.nu) % g.nv);
            int iu = (int)(r % g.nu);
            double s[3], q[3];
            og_ray(&g, k, iv, iu, s, q);
            int n = og_trace(&g, &sc, s, q, 0, g.nz, idx, w);
            double acc = 0.0;
            for (int j = 0; j < n; ++j) acc += w[j] * x[idx[j]];
            b[r] = acc;
        }
        free(idx);
        free(w);
        og_scratch_free(&sc);
    }
}

/* b_i = (A x)_i for a list of ray indices only (sampled checks at full size). */
void oracle_project_rays(const int32_t *dims, const double *par, const double *angles,
                         const double *x, const int64_t *rays, int64_t nsel, double *out)
{
    og_t g = og_make(dims, par, angles);
#pragma omp parallel
    {
        int cap = og_cap(&g);
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        double *w = (double *)malloc(sizeof(double) * (size_t)cap);
        og_scratch sc = og_scratch_new(&g);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nsel; ++t) {
            int64_t r = rays[t];
            int k = (int)(r / ((int64_t)g.nv * g.nu));
            int iv = (int)((r / g.nu) % g.nv);
            int iu = (int)(r % g.nu);
            double s[3], q[3];
            og_ray(&g, k, iv, iu, s, q);
            int n = og_trace(&g, &sc, s, q, 0, g.nz, idx, w);
            double acc = 0.0;
            for (int j = 0; j < n; ++j) acc += w[j] * x[idx[j]];
            out[t] = acc;
        }
        free(idx);
        free(w);
        og_scratch_free(&sc);
    }
}

/* r = A^T y (Eq. 2).  Parallel over z-slabs; every slab visits all rays.  The
 * partition does not change the result: a piece's weight does not depend on
 * the slab it is clipped to, and each voxel sums its pieces in ray order. */
void oracle_backproject(const int32_t *dims, const double *par, const double *angles,
                        const double *y, double *r)
{
    og_t g = og_make(dims, par, angles);
    int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
    memset(r, 0, sizeof(double) * (size_t)nvox);
    int64_t nrays = (int64_t)g.nviews * g.nv * g.nu;
    int nslab = 2 * omp_get_max_threads();
    if (nslab > g.nz) nslab = g.nz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int sl = 0; sl < nslab; ++sl) {
        int zlo = (int)((int64_t)g.nz * sl / nslab);
        int zhi = (int)((int64_t)g.nz * (sl + 1) / nslab);
        int cap = og_cap(&g);
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        double *w = (double *)malloc(sizeof(double) * (size_t)cap);
        og_scratch sc = og_scratch_new(&g);
        for (int64_t ri = 0; ri < nrays; ++ri) {
            if (y[ri] == 0.0) continue;
            int k = (int)(ri / ((int64_t)g.nv * g.nu));
            int iv = (int)((ri / g.nu) % g.nv);
            int iu = (int)(ri % g.nu);
            double s[3], q[3];
            og_ray(&g, k, iv, iu, s, q);
            int n = og_trace(&g, &sc, s, q, zlo, zhi, idx, w);
            for (int j = 0; j < n; ++j) r[idx[j]] += w[j] * y[ri];
        }
        free(idx);
        free(w);
        og_scratch_free(&sc);
    }
}

/* The same pair in single-precision arithmetic, the precision of the paper's
 * GPU projectors (Section 5): every weight and input element rounded to float,
 * each sum formed by float fused multiply-adds (fmaf: one rounding per term),
 * along the ray for A and per voxel in ray order for A^T.  The weights are the
 * double-precision ones of og_trace; only their use is single precision. */
void oracle_project32(const int32_t *dims, const double *par, const double *angles,
                      const double *x, double *b)
{
    og_t g = og_make(dims, par, angles);
    int64_t nrays = (int64_t)g.nviews * g.nv * g.nu;
#pragma omp parallel
    {
        int cap = og_cap(&g);
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        double *w = (double *)malloc(sizeof(double) * (size_t)cap);
        og_scratch sc = og_scratch_new(&g);
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < nrays; ++r) {
            int k = (int)(r / ((int64_t)g.nv * g.nu));
            int iv = (int)((r / g.nu) % g.nv);
            int iu = (int)(r % g.nu);
            double s[3], q[3];
            og_ray(&g, k, iv, iu, s, q);
            int n = og_trace(&g, &sc, s, q, 0, g.nz, idx, w);
            float acc = 0.0f;
            for (int j = 0; j < n; ++j) acc = fmaf((float)w[j], (float)x[idx[j]], acc);
            b[r] = (double)acc;
        }
        free(idx);
        free(w);
        og_scratch_free(&sc);
    }
}

void oracle_backproject32(const int32_t *dims, const double *par, const double *angles,
                          const double *y, double *r)
{
    og_t g = og_make(dims, par, angles);
    int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
    float *rf = (float *)calloc((size_t)nvox, sizeof(float));
    int64_t nrays = (int64_t)g.nviews * g.nv * g.nu;
    int nslab = 2 * omp_get_max_threads();
    if (nslab > g.nz) nslab = g.nz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int sl = 0; sl < nslab; ++sl) {
        int zlo = (int)((int64_t)g.nz * sl / nslab);
        int zhi = (int)((int64_t)g.nz * (sl + 1) / nslab);
        int cap = og_cap(&g);
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        double *w = (double *)malloc(sizeof(double) * (size_t)cap);
        og_scratch sc = og_scratch_new(&g);
        for (int64_t ri = 0; ri < nrays; ++ri) {
            if (y[ri] == 0.0) continue;
            int k = (int)(ri / ((int64_t)g.nv * g.nu));
            int iv = (int)((ri / g.nu) % g.nv);
            int iu = (int)(ri % g.nu);
            double s[3], q[3];
            og_ray(&g, k, iv, iu, s, q);
            int n = og_trace(&g, &sc, s, q, zlo, zhi, idx, w);
            const float yf = (float)y[ri];
            for (int j = 0; j < n; ++j) rf[idx[j]] = fmaf((float)w[j], yf, rf[idx[j]]);
        }
        free(idx);
        free(w);
        og_scratch_free(&sc);
    }
    for (int64_t i = 0; i < nvox; ++i) r[i] = (double)rf[i];
    free(rf);
}

/* diag(A^T A)_j = sum_i w_ij^2 (the squared column norms of A; the diagonal of
 * the normal equations that Jacobi preconditioning uses, Section 5).  Same
 * slab-parallel scatter as the backprojection, with squared weights. */
void oracle_diag_normal(const int32_t *dims, const double *par, const double *angles, double *out)
{
    og_t g = og_make(dims, par, angles);
    int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
    memset(out, 0, sizeof(double) * (size_t)nvox);
    int64_t nrays = (int64_t)g.nviews * g.nv * g.nu;
    int nslab = 2 * omp_get_max_threads();
    if (nslab > g.nz) nslab = g.nz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int sl = 0; sl < nslab; ++sl) {
        int zlo = (int)((int64_t)g.nz * sl / nslab);
        int zhi = (int)((int64_t)g.nz * (sl + 1) / nslab);
        int cap = og_cap(&g);
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        double *w = (double *)malloc(sizeof(double) * (size_t)cap);
        og_scratch sc = og_scratch_new(&g);
        for (int64_t ri = 0; ri < nrays; ++ri) {
            int k = (int)(ri / ((int64_t)g.nv * g.nu));
            int iv = (int)((ri / g.nu) % g.nv);
            int iu = (int)(ri % g.nu);
            double s[3], q[3];
            og_ray(&g, k, iv, iu, s, q);
            int n = og_trace(&g, &sc, s, q, zlo, zhi, idx, w);
            for (int j = 0; j < n; ++j) out[idx[j]] += w[j] * w[j];
        }
        free(idx);
        free(w);
        og_scratch_free(&sc);
    }
}

/* Length of the segment s->q inside the half-open box [b0, b1) (slab method). */
static double og_seg_box(const double s[3], const double q[3], const double b0[3], const double b1[3])
{
    double amin = 0.0, amax = 1.0;
    for (int a = 0; a < 3; ++a) {
        double d = q[a] - s[a];
        if (d != 0.0) {
            double a0 = (b0[a] - s[a]) / d, a1 = (b1[a] - s[a]) / d;
            double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0;
            if (lo > amin) amin = lo;
            if (hi < amax) amax = hi;
        } else if (!(s[a] >= b0[a] && s[a] < b1[a])) {
            return 0.0;
        }
    }
    if (!(amax > amin)) return 0.0;
    double dx = q[0] - s[0], dy = q[1] - s[1], dz = q[2] - s[2];
    return (amax - amin) * sqrt(dx * dx + dy * dy + dz * dz);
}

/*
 * r_j = (A^T y)_j for a list of voxel indices only.  Each weight is the plain
 * definition |segment_i ∩ box_j|; candidate pixels come from the bounding box of
 * the eight projected voxel corners, widened by two pixels.
 */
void oracle_backproject_voxels(const int32_t *dims, const double *par, const double *angles,
                               const double *y, const int64_t *vox, int64_t nsel, double *out)
{
    og_t g = og_make(dims, par, angles);
    double lo[3] = { g.cx - 0.5 * g.nx * g.vx, g.cy - 0.5 * g.ny * g.vy, g.cz - 0.5 * g.nz * g.vz };
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nsel; ++t) {
        int64_t j = vox[t];
        int ix = (int)(j % g.nx), iy = (int)((j / g.nx) % g.ny), iz = (int)(j / ((int64_t)g.nx * g.ny));
        double b0[3] = { lo[0] + ix * g.vx, lo[1] + iy * g.vy, lo[2] + iz * g.vz };
        double b1[3] = { lo[0] + (ix + 1) * g.vx, lo[1] + (iy + 1) * g.vy, lo[2] + (iz + 1) * g.vz };
        double acc = 0.0;
        for (int k = 0; k < g.nviews; ++k) {
            double c = cos(g.ang[k]), sn = sin(g.ang[k]);
            double s[3] = { g.sid * c, g.sid * sn, 0.0 };
            double cen[3] = { s[0] - g.sdd * c, s[1] - g.sdd * sn, 0.0 };
            double eu[3] = { -sn, c, 0.0 };
            double nrm[3] = { -c, -sn, 0.0 };
            double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
            for (int cc = 0; cc < 8; ++cc) {
                double p[3] = { (cc & 1) ? b1[0] : b0[0], (cc & 2) ? b1[1] : b0[1], (cc & 4) ? b1[2] : b0[2] };
                double rel[3] = { p[0] - s[0], p[1] - s[1], p[2] - s[2] };
                double depth = rel[0] * nrm[0] + rel[1] * nrm[1];
                double scale = g.sdd / depth;
                double pu = (rel[0] * eu[0] + rel[1] * eu[1]) * scale;
                double pv = rel[2] * scale;
                (void)cen;
                double fu = (pu - g.off_u) / g.du + 0.5 * (g.nu - 1);
                double fv = (pv - g.off_v) / g.dv + 0.5 * (g.nv - 1);
                if (fu < umin) umin = fu;
                if (fu > umax) umax = fu;
                if (fv < vmin) vmin = fv;
                if (fv > vmax) vmax = fv;
            }
            int u0 = (int)floor(umin) - 2, u1 = (int)ceil(umax) + 2;
            int v0 = (int)floor(vmin) - 2, v1 = (int)ceil(vmax) + 2;
            if (u0 < 0) u0 = 0;
            if (v0 < 0) v0 = 0;
            if (u1 > g.nu - 1) u1 = g.nu - 1;
            if (v1 > g.nv - 1) v1 = g.nv - 1;
            for (int iv = v0; iv <= v1; ++iv)
                for (int iu = u0; iu <= u1; ++iu) {
                    double sr[3], q[3];
                    og_ray(&g, k, iv, iu, sr, q);
                    double wl = og_seg_box(sr, q, b0, b1);
                    if (wl > 0.0) acc += wl * y[((int64_t)k * g.nv + iv) * g.nu + iu];
                }
        }
        out[t] = acc;
    }
}

/* Number of positive weights of A (structural nonzeros of the Siddon model). */
int64_t oracle_count_nnz(const int32_t *dims, const double *par, const double *angles)
{
    og_t g = og_make(dims, par, angles);
    int64_t nrays = (int64_t)g.nviews * g.nv * g.nu;
    int64_t total = 0;
#pragma omp parallel reduction(+ : total)
    {
        int cap = og_cap(&g);
        int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        double *w = (double *)malloc(sizeof(double) * (size_t)cap);
        og_scratch sc = og_scratch_new(&g);
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < nrays; ++r) {
            int k = (int)(r / ((int64_t)g.nv * g.nu));
            int iv = (int)((r / g.nu) % g.nv);
            int iu = (int)(r % g.nu);
            double s[3], q[3];
            og_ray(&g, k, iv, iu, s, q);
            total += og_trace(&g, &sc, s, q, 0, g.nz, idx, w);
        }
        free(idx);
        free(w);
        og_scratch_free(&sc);
    }
    return total;
}

/* All (ray, voxel, weight) triples of A in ray order; returns the count written
 * (at most cap).  For tiny grids only: lets tests assemble A as a sparse matrix. */
int64_t oracle_assemble(const int32_t *dims, const double *par, const double *angles,
                        int64_t cap, int64_t *rows, int64_t *cols, double *vals)
{
    og_t g = og_make(dims, par, angles);
    int64_t nrays = (int64_t)g.nviews * g.nv * g.nu;
    int tcap = og_cap(&g);
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)tcap);
    double *w = (double *)malloc(sizeof(double) * (size_t)tcap);
    og_scratch sc = og_scratch_new(&g);
    int64_t out = 0;
    for (int64_t r = 0; r < nrays; ++r) {
        int k = (int)(r / ((int64_t)g.nv * g.nu));
        int iv = (int)((r / g.nu) % g.nv);
        int iu = (int)(r % g.nu);
        double s[3], q[3];
        og_ray(&g, k, iv, iu, s, q);
        int n = og_trace(&g, &sc, s, q, 0, g.nz, idx, w);
        for (int j = 0; j < n && out < cap; ++j) {
            rows[out] = r;
            cols[out] = idx[j];
            vals[out] = w[j];
            ++out;
        }
    }
    free(idx);
    free(w);
    og_scratch_free(&sc);
    return out;
}

/* --------------------------------------------------------- vector helpers */

static double og_dot(const double *a, const double *b, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Single-precision storage of a solver vector (store32 = 1): every element
 * rounded to the nearest float.  This is the storage form of the solvers that
 * Section 5 allows (vectors in float, the scalars kept in double): the oracle
 * offers it to measure how far that rounding alone moves the iterates of an
 * otherwise double-precision solve.  store32 = 0 leaves the vector as it is. */
static void og_store(double *v, int64_t n, int store32)
{
    if (!store32) return;
    for (int64_t i = 0; i < n; ++i) v[i] = (double)(float)v[i];
}

/* Stop reasons shared by both solvers. */
enum { OG_STOP_MAXITER = 0, OG_STOP_TOL = 1, OG_STOP_BREAKDOWN = 2, OG_STOP_NUMERIC = 3 };

/*
 * CGLS with delayed residual computation -- Algorithm 1, in the paper's order.
 * Inputs b, x (= x0 on entry, x_K on return), ERR, K.  Outputs x, the number of
 * iterations i and the final discrepancy norm NB.  history[i-1] = NB_i / NB0.
 * The stop test is NB > ERR * NB0 (multiplication form, so NB0 = 0 is safe);
 * NR2 = 0 or NP2 = 0 is a breakdown that stops with the current x.
 * literal_update = 1 uses the printed direction update d = d + beta r.
 */
void oracle_tt_project(const int32_t *dims, const double *par, const double *angles, const double *x, double *b);
void oracle_tt_backproject(const int32_t *dims, const double *par, const double *angles, const double *y, double *r);

/* Long runs can report each CGLS iteration on stderr (environment variable
 * KCT_ORACLE_PROGRESS set); the arithmetic is not affected. */
static int og_progress_flag(void)
{
    const char *v = getenv("KCT_ORACLE_PROGRESS");
    return v && *v && *v != '0';
}
#define og_progress og_progress_flag()

/* The operator of a solve: the Siddon pair (projector 0), the TT pair (1), or
 * the Siddon pair in single-precision arithmetic (projector 2, see
 * oracle_project32). */
static void og_A(int projector, const int32_t *dims, const double *par, const double *angles, const double *x,
                 double *b)
{
    if (projector == 1) oracle_tt_project(dims, par, angles, x, b);
    else if (projector == 2) oracle_project32(dims, par, angles, x, b);
    else oracle_project(dims, par, angles, x, b);
}

static void og_AT(int projector, const int32_t *dims, const double *par, const double *angles, const double *y,
                  double *r)
{
    if (projector == 1) oracle_tt_backproject(dims, par, angles, y, r);
    else if (projector == 2) oracle_backproject32(dims, par, angles, y, r);
    else oracle_backproject(dims, par, angles, y, r);
}

/* e = e - alpha p (the update of Algorithm 1), or e = b - A x when recompute. */
static void og_cgls_discrepancy(int projector, const int32_t *dims, const double *par, const double *angles,
                                const double *b, const double *x, double *e, double *p, double alpha, int64_t m,
                                int recompute)
{
    if (recompute) {
        og_A(projector, dims, par, angles, x, p);
        for (int64_t t = 0; t < m; ++t) e[t] = b[t] - p[t];
    } else {
        for (int64_t t = 0; t < m; ++t) e[t] -= alpha * p[t];
    }
}

/*
 * CGLS with the Tikhonov term of the paper's conclusions, lambda^2 |x|^2 (CGLS
 * on the stacked system [A; lambda I] x = [b; 0]): the residual of the lower
 * block is -lambda x, so r = A^T e - lambda^2 x and |[A; lambda I] d|^2 =
 * |A d|^2 + lambda^2 |d|^2; e = b - A x stays the data discrepancy whose norm
 * is NB.  recompute_every = k > 0 replaces the update e -= alpha p by
 * e = b - A x after every k-th iteration (the periodic recomputation of the
 * discrepancy that Section 5 discusses).  lambda = 0, k = 0 is Algorithm 1.
 * store32 = 1 rounds x, r, d, e and p to single precision after every update
 * (og_store); the norms and scalars stay double.
 */
int oracle_cgls_ex(const int32_t *dims, const double *par, const double *angles,
                   const double *b, double *x, int K, double err, int x0_is_zero,
                   int literal_update, double lambda, int recompute_every, int projector, int store32,
                   double *history, double *out_nb, double *out_nb0, int *out_iters)
{
    const double l2 = lambda * lambda;
    og_t g = og_make(dims, par, angles);
    int64_t n = (int64_t)g.nx * g.ny * g.nz;
    int64_t m = (int64_t)g.nviews * g.nv * g.nu;
    double *d = (double *)calloc((size_t)n, sizeof(double));
    double *r = (double *)calloc((size_t)n, sizeof(double));
    double *e = (double *)calloc((size_t)m, sizeof(double));
    double *p = (double *)calloc((size_t)m, sizeof(double));
    int stop = OG_STOP_MAXITER, i = 0;

    double NB0 = sqrt(og_dot(b, b, m));
    double NB = NB0;
    if (K <= 0) goto done;
    if (x0_is_zero) memset(x, 0, sizeof(double) * (size_t)n);
    /* p = A x ; e = b - p */
    if (x0_is_zero) memset(p, 0, sizeof(double) * (size_t)m);
    else og_A(projector, dims, par, angles, x, p);
    og_store(p, m, store32);
    for (int64_t t = 0; t < m; ++t) e[t] = b[t] - p[t];
    og_store(e, m, store32);
    NB = sqrt(og_dot(e, e, m));
    /* r = A^T e - lambda^2 x ; d = r ; NR2_old = |r|^2 */
    og_AT(projector, dims, par, angles, e, r);
    if (l2 != 0.0)
        for (int64_t t = 0; t < n; ++t) r[t] -= l2 * x[t];
    og_store(r, n, store32);
    memcpy(d, r, sizeof(double) * (size_t)n);
    double NR2_old = og_dot(r, r, n);
    if (NR2_old == 0.0) { stop = OG_STOP_BREAKDOWN; goto done; }
    /* p = A d ; NP2 = |p|^2 + lambda^2 |d|^2 ; alpha ; x += alpha d ; e -= alpha p ; NB */
    og_A(projector, dims, par, angles, d, p);
    og_store(p, m, store32);
    double NP2 = og_dot(p, p, m) + l2 * og_dot(d, d, n);
    if (NP2 == 0.0) { stop = OG_STOP_BREAKDOWN; goto done; }
    double alpha = NR2_old / NP2;
    for (int64_t t = 0; t < n; ++t) x[t] += alpha * d[t];
    og_store(x, n, store32);
    i = 1;
    og_cgls_discrepancy(projector, dims, par, angles, b, x, e, p, alpha, m, recompute_every > 0 && i % recompute_every == 0);
    og_store(e, m, store32);
    NB = sqrt(og_dot(e, e, m));
    if (history) history[0] = NB0 > 0 ? NB / NB0 : 0.0;
    if (!isfinite(NB)) { stop = OG_STOP_NUMERIC; goto done; }
    while (NB > err * NB0 && i < K) {
        og_AT(projector, dims, par, angles, e, r);
        if (l2 != 0.0)
            for (int64_t t = 0; t < n; ++t) r[t] -= l2 * x[t];
        og_store(r, n, store32);
        double NR2_now = og_dot(r, r, n);
        if (NR2_now == 0.0) { stop = OG_STOP_BREAKDOWN; goto done; }
        double beta = NR2_now / NR2_old;
        if (literal_update)
            for (int64_t t = 0; t < n; ++t) d[t] = d[t] + beta * r[t];
        else
            for (int64_t t = 0; t < n; ++t) d[t] = r[t] + beta * d[t];
        og_store(d, n, store32);
        NR2_old = NR2_now;
        og_A(projector, dims, par, angles, d, p);
        og_store(p, m, store32);
        NP2 = og_dot(p, p, m) + l2 * og_dot(d, d, n);
        if (NP2 == 0.0) { stop = OG_STOP_BREAKDOWN; goto done; }
        alpha = NR2_old / NP2;
        for (int64_t t = 0; t < n; ++t) x[t] += alpha * d[t];
        og_store(x, n, store32);
        i = i + 1;
        og_cgls_discrepancy(projector, dims, par, angles, b, x, e, p, alpha, m, recompute_every > 0 && i % recompute_every == 0);
        og_store(e, m, store32);
        NB = sqrt(og_dot(e, e, m));
        if (og_progress) fprintf(stderr, "oracle cgls: iteration %d of %d\n", i, K);
        if (history) history[i - 1] = NB0 > 0 ? NB / NB0 : 0.0;
        if (!isfinite(NB)) { stop = OG_STOP_NUMERIC; goto done; }
    }
    if (i >= K) stop = OG_STOP_MAXITER;
    else stop = OG_STOP_TOL;
done:
    if (out_nb) *out_nb = NB;
    if (out_nb0) *out_nb0 = NB0;
    if (out_iters) *out_iters = i;
    free(d); free(r); free(e); free(p);
    return stop;
}

void oracle_tt_diag_normal(const int32_t *dims, const double *par, const double *angles, double *out);

/*
 * Jacobi-preconditioned CGLS (Section 5): Algorithm 1 applied to the operator
 * A M, M = diag(A^T A)^(-1/2) (0 where the diagonal is 0), for the correction
 * z of x = x0 + M z, starting from z = 0.  Products: (A M) d = A (M d),
 * (A M)^T e = M (A^T e).  NB = |b - A x| as in Algorithm 1.  projector 0 is the
 * Siddon pair, 1 the TT pair (Sections 3, 4) with its own diagonal.
 */
int oracle_cgls_jacobi_ex(const int32_t *dims, const double *par, const double *angles,
                          const double *b, double *x, int K, double err, int x0_is_zero, int projector,
                          double *history, double *out_nb, double *out_nb0, int *out_iters)
{
    og_t g = og_make(dims, par, angles);
    int64_t n = (int64_t)g.nx * g.ny * g.nz;
    int64_t m = (int64_t)g.nviews * g.nv * g.nu;
    double *M = (double *)calloc((size_t)n, sizeof(double));
    double *d = (double *)calloc((size_t)n, sizeof(double));
    double *r = (double *)calloc((size_t)n, sizeof(double));
    double *md = (double *)calloc((size_t)n, sizeof(double));
    double *e = (double *)calloc((size_t)m, sizeof(double));
    double *p = (double *)calloc((size_t)m, sizeof(double));
    int stop = OG_STOP_MAXITER, i = 0;
    double NB0 = sqrt(og_dot(b, b, m)), NB = NB0;
    if (K <= 0) goto done;
    if (projector == 1) oracle_tt_diag_normal(dims, par, angles, M);
    else oracle_diag_normal(dims, par, angles, M);
    for (int64_t t = 0; t < n; ++t) M[t] = M[t] > 0.0 ? 1.0 / sqrt(M[t]) : 0.0;
    if (x0_is_zero) memset(x, 0, sizeof(double) * (size_t)n);
    /* e = b - A x0 */
    if (x0_is_zero) memset(p, 0, sizeof(double) * (size_t)m);
    else og_A(projector, dims, par, angles, x, p);
    for (int64_t t = 0; t < m; ++t) e[t] = b[t] - p[t];
    NB = sqrt(og_dot(e, e, m));
    double NR2_old = 0.0;
    while (i < K) {
        /* r = (A M)^T e */
        og_AT(projector, dims, par, angles, e, r);
        for (int64_t t = 0; t < n; ++t) r[t] *= M[t];
        double NR2 = og_dot(r, r, n);
        if (NR2 == 0.0) { stop = OG_STOP_BREAKDOWN; goto done; }
        if (i == 0) memcpy(d, r, sizeof(double) * (size_t)n);
        else {
            double beta = NR2 / NR2_old;
            for (int64_t t = 0; t < n; ++t) d[t] = r[t] + beta * d[t];
        }
        NR2_old = NR2;
        /* p = (A M) d; alpha = NR2 / |p|^2; z += alpha d, i.e. x += alpha M d; e -= alpha p */
        for (int64_t t = 0; t < n; ++t) md[t] = M[t] * d[t];
        og_A(projector, dims, par, angles, md, p);
        double NP2 = og_dot(p, p, m);
        if (NP2 == 0.0) { stop = OG_STOP_BREAKDOWN; goto done; }
        double alpha = NR2 / NP2;
        for (int64_t t = 0; t < n; ++t) x[t] += alpha * md[t];
        for (int64_t t = 0; t < m; ++t) e[t] -= alpha * p[t];
        NB = sqrt(og_dot(e, e, m));
        i = i + 1;
        if (history) history[i - 1] = NB0 > 0 ? NB / NB0 : 0.0;
        if (!isfinite(NB)) { stop = OG_STOP_NUMERIC; goto done; }
        if (!(NB > err * NB0)) { stop = i >= K ? OG_STOP_MAXITER : OG_STOP_TOL; goto done; }
    }
    stop = OG_STOP_MAXITER;
done:
    if (out_nb) *out_nb = NB;
    if (out_nb0) *out_nb0 = NB0;
    if (out_iters) *out_iters = i;
    free(M); free(d); free(r); free(md); free(e); free(p);
    return stop;
}

int oracle_cgls_jacobi(const int32_t *dims, const double *par, const double *angles,
                       const double *b, double *x, int K, double err, int x0_is_zero, double *history,
                       double *out_nb, double *out_nb0, int *out_iters)
{
    return oracle_cgls_jacobi_ex(dims, par, angles, b, x, K, err, x0_is_zero, 0, history, out_nb, out_nb0,
                                 out_iters);
}

int oracle_cgls(const int32_t *dims, const double *par, const double *angles,
                const double *b, double *x, int K, double err, int x0_is_zero,
                int literal_update, double *history, double *out_nb, double *out_nb0,
                int *out_iters)
{
    return oracle_cgls_ex(dims, par, angles, b, x, K, err, x0_is_zero, literal_update, 0.0, 0, 0, 0, history, out_nb,
                          out_nb0, out_iters);
}

/*
 * LSQR (Paige & Saunders 1982), the method the paper pairs with CGLS.
 *   beta u = b - A x0, alpha v = A^T u, w = v, phibar = beta, rhobar = alpha;
 *   per iteration: beta u = A v - alpha u; alpha v = A^T u - beta v;
 *   rho = hypot(rhobar, beta); c = rhobar/rho; s = beta/rho; theta = s alpha;
 *   rhobar = -c alpha; phi = c phibar; phibar = s phibar;
 *   x += (phi/rho) w; w = v - (theta/rho) w.
 * |phibar| estimates |b - A x_i|; history[i-1] = |phibar| / |b|.  The A^T of
 * the last iteration is not needed for x_K and is skipped, so K iterations cost
 * K products with A and K with A^T (one more A when x0 != 0), as for CGLS.
 */
/*
 * With damp = lambda > 0 the method solves min |b - A x|^2 + lambda^2 |x - x0|^2
 * (Paige & Saunders' damped least squares): before each rotation rhobar is
 * rotated against lambda, rhobar1 = hypot(rhobar, lambda), c1 = rhobar/rhobar1,
 * s1 = lambda/rhobar1, psi = s1 phibar, phibar = c1 phibar, and rhobar1 takes
 * rhobar's place; sqrt(phibar^2 + sum psi^2) then estimates the norm of the
 * stacked residual [b - A x; -lambda (x - x0)] (|phibar| when lambda = 0).
 * store32 = 1 rounds u, v, w and x to single precision after every update
 * (og_store); the norms and the rotation scalars stay double.
 */
int oracle_lsqr_ex(const int32_t *dims, const double *par, const double *angles,
                   const double *b, double *x, int K, double err, int x0_is_zero, double damp, int projector,
                   int store32, double *history, double *out_nb, double *out_nb0, int *out_iters)
{
    og_t g = og_make(dims, par, angles);
    int64_t n = (int64_t)g.nx * g.ny * g.nz;
    int64_t m = (int64_t)g.nviews * g.nv * g.nu;
    double *u = (double *)calloc((size_t)m, sizeof(double));
    double *tmpm = (double *)calloc((size_t)m, sizeof(double));
    double *v = (double *)calloc((size_t)n, sizeof(double));
    double *w = (double *)calloc((size_t)n, sizeof(double));
    double *tmpn = (double *)calloc((size_t)n, sizeof(double));
    int stop = OG_STOP_MAXITER, i = 0;
    double NB0 = sqrt(og_dot(b, b, m));
    double phibar = NB0, res2 = 0.0;
    if (K <= 0) goto done;
    if (x0_is_zero) memset(x, 0, sizeof(double) * (size_t)n);
    if (x0_is_zero) memcpy(u, b, sizeof(double) * (size_t)m);
    else {
        og_A(projector, dims, par, angles, x, tmpm);
        for (int64_t t = 0; t < m; ++t) u[t] = b[t] - tmpm[t];
    }
    double beta = sqrt(og_dot(u, u, m));
    phibar = beta;
    if (beta == 0.0) { stop = OG_STOP_BREAKDOWN; goto done; }
    for (int64_t t = 0; t < m; ++t) u[t] /= beta;
    og_store(u, m, store32);
    og_AT(projector, dims, par, angles, u, v);
    double alpha = sqrt(og_dot(v, v, n));
    if (alpha == 0.0) { stop = OG_STOP_BREAKDOWN; goto done; }
    for (int64_t t = 0; t < n; ++t) v[t] /= alpha;
    og_store(v, n, store32);
    memcpy(w, v, sizeof(double) * (size_t)n);
    double rhobar = alpha;
    while (i < K) {
        /* bidiagonalisation: beta u = A v - alpha u */
        og_A(projector, dims, par, angles, v, tmpm);
        for (int64_t t = 0; t < m; ++t) u[t] = tmpm[t] - alpha * u[t];
        og_store(u, m, store32);
        beta = sqrt(og_dot(u, u, m));
        int last = (i + 1 == K);
        double alpha_next = 0.0;
        if (beta != 0.0) {
            for (int64_t t = 0; t < m; ++t) u[t] /= beta;
            og_store(u, m, store32);
            if (!last) {
                /* alpha v = A^T u - beta v */
                og_AT(projector, dims, par, angles, u, tmpn);
                for (int64_t t = 0; t < n; ++t) v[t] = tmpn[t] - beta * v[t];
                og_store(v, n, store32);
                alpha_next = sqrt(og_dot(v, v, n));
                if (alpha_next != 0.0)
                    for (int64_t t = 0; t < n; ++t) v[t] /= alpha_next;
                og_store(v, n, store32);
            }
        }
        /* damping rotation, then the Givens rotation */
        if (damp != 0.0) {
            double rhobar1 = sqrt(rhobar * rhobar + damp * damp);
            double psi = (damp / rhobar1) * phibar;
            res2 += psi * psi;
            phibar = (rhobar / rhobar1) * phibar;
            rhobar = rhobar1;
        }
        double rho = sqrt(rhobar * rhobar + beta * beta);
        double c = rhobar / rho, s = beta / rho;
        double theta = s * alpha_next;
        rhobar = -c * alpha_next;
        double phi = c * phibar;
        phibar = s * phibar;
        for (int64_t t = 0; t < n; ++t) x[t] += (phi / rho) * w[t];
        og_store(x, n, store32);
        for (int64_t t = 0; t < n; ++t) w[t] = v[t] - (theta / rho) * w[t];
        og_store(w, n, store32);
        alpha = alpha_next;
        i = i + 1;
        double nb = sqrt(phibar * phibar + res2);
        if (history) history[i - 1] = NB0 > 0 ? nb / NB0 : 0.0;
        if (!isfinite(phibar)) { stop = OG_STOP_NUMERIC; goto done; }
        if (beta == 0.0 || (!last && alpha_next == 0.0)) { stop = OG_STOP_BREAKDOWN; goto done; }
        if (!(nb > err * NB0)) { stop = OG_STOP_TOL; goto done; }
    }
    stop = OG_STOP_MAXITER;
done:
    if (out_nb) *out_nb = sqrt(phibar * phibar + res2);
    if (out_nb0) *out_nb0 = NB0;
    if (out_iters) *out_iters = i;
    free(u); free(tmpm); free(v); free(w); free(tmpn);
    return stop;
}

int oracle_lsqr(const int32_t *dims, const double *par, const double *angles,
                const double *b, double *x, int K, double err, int x0_is_zero,
                double *history, double *out_nb, double *out_nb0, int *out_iters)
{
    return oracle_lsqr_ex(dims, par, angles, b, x, K, err, x0_is_zero, 0.0, 0, 0, history, out_nb, out_nb0,
                          out_iters);
}

/* ---------------------------------------------------------------- TT footprint projector
 *
 * The separable-footprint projector with trapezoid transaxial and trapezoid
 * axial footprints (Section 3 names footprint methods after Long et al. 2010;
 * the experiments of Section 4 use the TT variant).  The paper gives no
 * formulas; the reading implemented here:
 *   a_ij = L_i * F_u(i, j) * F_v(i, j), where
 *   F_u  is the mean, over the extent of ray i's detector column, of the
 *        unit-height trapezoid whose breakpoints are the detector u-coordinates
 *        of the four in-plane corners of voxel j (its exact transaxial shadow,
 *        with linear ramps);
 *   F_v  is the same along v, with breakpoints v(z_lo, D_min), v(z_lo, D_max),
 *        v(z_hi, D_min), v(z_hi, D_max): the voxel's z extent seen from the
 *        nearest and the farthest of its in-plane corners (depths D along the
 *        central ray);
 *   L_i  is the length of the longest chord of a voxel parallel to ray i,
 *        min(vx / |d_x|, vy / |d_y|, vz / |d_z|) for the unit direction d of ray i
 *        (source -> pixel centre).
 * The trapezoids of neighbouring voxels share breakpoints and have
 * complementary ramps, so they sum to one across a row of voxels.
 */

/* Integral of the unit trapezoid t[0] <= t[1] <= t[2] <= t[3] from -inf to u. */
static double tt_cum(const double t[4], double u)
{
    if (u <= t[0]) return 0.0;
    double g = 0.0;
    if (u < t[1]) return (u - t[0]) * (u - t[0]) / (2.0 * (t[1] - t[0]));
    g += 0.5 * (t[1] - t[0]);
    if (u < t[2]) return g + (u - t[1]);
    g += t[2] - t[1];
    if (u < t[3]) return g + 0.5 * (t[3] - t[2]) - (t[3] - u) * (t[3] - u) / (2.0 * (t[3] - t[2]));
    return g + 0.5 * (t[3] - t[2]);
}

static void tt_sort4(double t[4])
{
    for (int i = 1; i < 4; ++i)
        for (int j = i; j > 0 && t[j] < t[j - 1]; --j) {
            double h = t[j]; t[j] = t[j - 1]; t[j - 1] = h;
        }
}

/* Transaxial breakpoints (mm on the detector u axis, sorted) of voxel column
 * (ix, iy) in view k, and the smallest / largest depth of its corners. */
static void tt_transaxial(const og_t *g, int k, int ix, int iy, double tu[4], double *dmin, double *dmax)
{
    double c = cos(g->ang[k]), sn = sin(g->ang[k]);
    double sx = g->sid * c, sy = g->sid * sn;
    double x0 = g->cx - 0.5 * g->nx * g->vx + ix * g->vx, y0 = g->cy - 0.5 * g->ny * g->vy + iy * g->vy;
    *dmin = INFINITY;
    *dmax = -INFINITY;
    for (int q = 0; q < 4; ++q) {
        double px = x0 + ((q & 1) ? g->vx : 0.0), py = y0 + ((q & 2) ? g->vy : 0.0);
        double dx = px - sx, dy = py - sy;
        double depth = -(c * dx + sn * dy);
        tu[q] = g->sdd * (-sn * dx + c * dy) / depth;
        if (depth < *dmin) *dmin = depth;
        if (depth > *dmax) *dmax = depth;
    }
    tt_sort4(tu);
}

/* Axial breakpoints (mm on the detector v axis, sorted) of voxel layer iz. */
static void tt_axial(const og_t *g, int iz, double dmin, double dmax, double tv[4])
{
    double zlo = g->cz - 0.5 * g->nz * g->vz + iz * g->vz, zhi = zlo + g->vz;
    tv[0] = g->sdd * zlo / dmin;
    tv[1] = g->sdd * zlo / dmax;
    tv[2] = g->sdd * zhi / dmin;
    tv[3] = g->sdd * zhi / dmax;
    tt_sort4(tv);
}

/* L_i of every ray of view k, [iv][iu]. */
static void tt_amplitudes(const og_t *g, int k, double *L)
{
    for (int iv = 0; iv < g->nv; ++iv)
        for (int iu = 0; iu < g->nu; ++iu) {
            double s[3], q[3];
            og_ray(g, k, iv, iu, s, q);
            double d[3] = { q[0] - s[0], q[1] - s[1], q[2] - s[2] };
            double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double l = INFINITY;
            double vox[3] = { g->vx, g->vy, g->vz };
            for (int a = 0; a < 3; ++a)
                if (d[a] != 0.0) {
                    double la = vox[a] * n / fabs(d[a]);
                    if (la < l) l = la;
                }
            L[(int64_t)iv * g->nu + iu] = l;
        }
}

/* Detector index range [*a, *b] (clamped) whose pixels meet the open interval
 * (t0, t3) of a detector axis with n pixels of pitch p and offset off. */
static void tt_range(double t0, double t3, int n, double p, double off, int *a, int *b)
{
    double h = 0.5 * (double)(n - 1);
    int lo = (int)ceil((t0 - off) / p + h - 0.5), hi = (int)floor((t3 - off) / p + h + 0.5);
    *a = lo < 0 ? 0 : lo;
    *b = hi > n - 1 ? n - 1 : hi;
}

static double tt_pixel_mean(const double t[4], int i, int n, double p, double off)
{
    double c = ((double)i - 0.5 * (double)(n - 1)) * p + off;
    return (tt_cum(t, c + 0.5 * p) - tt_cum(t, c - 0.5 * p)) / p;
}

/* b = A_TT x.  Parallel over views; within a view voxels are visited in index
 * order, so the sums are deterministic. */
void oracle_tt_project(const int32_t *dims, const double *par, const double *angles, const double *x, double *b)
{
    og_t g = og_make(dims, par, angles);
    int64_t per_view = (int64_t)g.nv * g.nu;
    memset(b, 0, sizeof(double) * (size_t)(per_view * g.nviews));
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < g.nviews; ++k) {
        double *bk = b + (int64_t)k * per_view;
        double *L = (double *)malloc(sizeof(double) * (size_t)per_view);
        tt_amplitudes(&g, k, L);
        for (int iy = 0; iy < g.ny; ++iy)
            for (int ix = 0; ix < g.nx; ++ix) {
                double tu[4], dmin, dmax;
                tt_transaxial(&g, k, ix, iy, tu, &dmin, &dmax);
                int ua, ub;
                tt_range(tu[0], tu[3], g.nu, g.du, g.off_u, &ua, &ub);
                for (int iz = 0; iz < g.nz; ++iz) {
                    double xv = x[((int64_t)iz * g.ny + iy) * g.nx + ix];
                    if (xv == 0.0) continue;
                    double tv[4];
                    tt_axial(&g, iz, dmin, dmax, tv);
                    int va, vb;
                    tt_range(tv[0], tv[3], g.nv, g.dv, g.off_v, &va, &vb);
                    for (int iu = ua; iu <= ub; ++iu) {
                        double fu = tt_pixel_mean(tu, iu, g.nu, g.du, g.off_u);
                        if (fu == 0.0) continue;
                        for (int iv = va; iv <= vb; ++iv) {
                            double fv = tt_pixel_mean(tv, iv, g.nv, g.dv, g.off_v);
                            int64_t i = (int64_t)iv * g.nu + iu;
                            bk[i] += L[i] * fu * fv * xv;
                        }
                    }
                }
            }
        free(L);
    }
}

/* r = A_TT^T y (square = 0), or r_j = sum_i a_ij^2 (square = 1, y unused).
 * Each voxel gathers over its footprint in every view. */
static void og_tt_gather(const int32_t *dims, const double *par, const double *angles, const double *y, double *r,
                         int square)
{
    og_t g = og_make(dims, par, angles);
    int64_t per_view = (int64_t)g.nv * g.nu;
    int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
    memset(r, 0, sizeof(double) * (size_t)nvox);
    double *L = (double *)malloc(sizeof(double) * (size_t)(per_view * g.nviews));
    for (int k = 0; k < g.nviews; ++k) tt_amplitudes(&g, k, L + (int64_t)k * per_view);
#pragma omp parallel for schedule(dynamic, 1)
    for (int iy = 0; iy < g.ny; ++iy)
        for (int ix = 0; ix < g.nx; ++ix)
            for (int k = 0; k < g.nviews; ++k) {
                const double *yk = square ? y : y + (int64_t)k * per_view, *Lk = L + (int64_t)k * per_view;
                double tu[4], dmin, dmax;
                tt_transaxial(&g, k, ix, iy, tu, &dmin, &dmax);
                int ua, ub;
                tt_range(tu[0], tu[3], g.nu, g.du, g.off_u, &ua, &ub);
                for (int iz = 0; iz < g.nz; ++iz) {
                    double tv[4];
                    tt_axial(&g, iz, dmin, dmax, tv);
                    int va, vb;
                    tt_range(tv[0], tv[3], g.nv, g.dv, g.off_v, &va, &vb);
                    double acc = 0.0;
                    for (int iu = ua; iu <= ub; ++iu) {
                        double fu = tt_pixel_mean(tu, iu, g.nu, g.du, g.off_u);
                        if (fu == 0.0) continue;
                        for (int iv = va; iv <= vb; ++iv) {
                            int64_t i = (int64_t)iv * g.nu + iu;
                            double a = Lk[i] * fu * tt_pixel_mean(tv, iv, g.nv, g.dv, g.off_v);
                            acc += square ? a * a : a * yk[i];
                        }
                    }
                    r[((int64_t)iz * g.ny + iy) * g.nx + ix] += acc;
                }
            }
    free(L);
}

void oracle_tt_backproject(const int32_t *dims, const double *par, const double *angles, const double *y, double *r)
{
    og_tt_gather(dims, par, angles, y, r, 0);
}

/* diag(A_TT^T A_TT)_j = sum_i a_ij^2. */
void oracle_tt_diag_normal(const int32_t *dims, const double *par, const double *angles, double *out)
{
    og_tt_gather(dims, par, angles, NULL, out, 1);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following calls (timing runs on one core); the results do
 * not depend on it: rays are independent, and each voxel of the slab scatter
 * sums its rays in ray order whatever the slab partition. */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
