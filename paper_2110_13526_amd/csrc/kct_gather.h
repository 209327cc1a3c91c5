// kct_gather.h -- the pieces of the brick-gather backprojector (A^T, Section 2,
// Eq. 2), written as plain functions so the kernel is a short sequence of
// calls between barriers.
//
// A workgroup owns a brick of BX x BY x TZ voxels; each of its 256 lanes owns
// one (x, y) position and the TZ voxels above it.  For every view the
// workgroup
//   1. bounds the brick's shadow on the detector (the eight projected corners),
//   2. stages the shadow's pixels into LDS, already multiplied by the ray
//      length factor L of their ray, together with the per-column and per-row
//      ray parameters,
//   3. lets each lane gather: candidate columns from a bound on its voxel
//      column's projection, the in-plane xi-interval of each column's rays in
//      the voxel column (shared by the TZ voxels), candidate rows from the
//      z-range of those rays, and for every candidate the exact weight of
//      kct_weights.h.
// The shadow is staged in chunks of at most CH_COLS x CH_ROWS pixels, so any
// geometry works; typical bricks need one chunk.
#pragma once

#pragma clang fp contract(off)

#include "kct_internal.h"
#include "kct_weights.h"

namespace kct {

constexpr int BX = 16, BY = 16, TZ = 16;  // brick; BX * BY = 256 lanes
constexpr int CH_COLS = 48, CH_ROWS = 40;  // staged shadow chunk

struct ColStage {   // per staged detector column
    float eta_c, inv_a, tcv, kz;
    float gz;       // d T / d xi with T = (segment fraction) / vz
    float pad[3];
};

struct RowStage {   // per staged detector row
    float qz, inv_qz;
};

// Detector coordinates (column, row; fractional pixel indices) of the ray
// through world point (px, py, pz) in view vp.
__host__ __device__ __forceinline__ void project_point(const GeoDev &g, const ViewParam &vp, float px, float py,
                                                       float pz, float &fu, float &fv)
{
    const float dx = px - vp.sx, dy = py - vp.sy;
    const float num = -vp.s * dx + vp.c * dy;
    const float den = -vp.c * dx - vp.s * dy;  // depth along the central ray (> 0)
    const float sc = g.sdd / den;
    fu = (num * sc - g.off_u) / g.du + g.cu;
    fv = (pz * sc - g.off_v) / g.dv + g.cv;
}

// Candidate detector columns [ua, ub] of the voxel column whose in-plane centre
// is (xc, yc): the projective image of its square, bounded around the image of
// the centre (a bound with margin; the weight function decides).
__host__ __device__ __forceinline__ void voxel_columns(const GeoDev &g, const ViewParam &vp, float xc, float yc,
                                                       int &ua, int &ub)
{
    const float dx = xc - vp.sx, dy = yc - vp.sy;
    const float num = -vp.s * dx + vp.c * dy;
    const float den = -vp.c * dx - vp.s * dy;
    const float dn = 0.5f * (g.vx * fabsf(vp.s) + g.vy * fabsf(vp.c));  // half extent along e_u
    const float dd = 0.5f * (g.vx * fabsf(vp.c) + g.vy * fabsf(vp.s));  // half extent along depth
    const float inv = 1.0f / den;
    const float inv2 = 1.0f / (den - dd);
    const float uc = g.sdd * num * inv;
    const float hw = g.sdd * (dn + dd * fabsf(num) * inv) * inv2;
    const float fc = (uc - g.off_u) / g.du + g.cu;
    const float hc = hw / g.du + 1e-3f;
    ua = (int)ceilf(fc - hc);
    ub = (int)floorf(fc + hc);
}

// One lane's share of one staged chunk of one view: add w_ij * (L_i e_i) to the
// accumulators of its voxels (ix, iy, iz0 + j), j < nzb, for every staged ray
// i = (column cu0 + c, row cv0 + r).  s_e[r * CH_COLS + c] holds L_i e_i.
__host__ __device__ __forceinline__ void gather_chunk(const GeoDev &g, const ViewParam &vp, int ix, int iy, int iz0,
                                                      int nzb, const float *s_e, const ColStage *s_col,
                                                      const RowStage *s_row, int cu0, int ncol, int cv0, int nrow,
                                                      float (&acc)[TZ])
{
    int ixi, ieta;
    float hxi, heta;
    if (vp.dom == 0) { ixi = ix; ieta = iy; hxi = g.hx; heta = g.hy; }
    else { ixi = iy; ieta = ix; hxi = g.hy; heta = g.hx; }
    const float lo_xi = (float)ixi - hxi;
    const float hi_xi = lo_xi + 1.0f;
    int ua, ub;
    voxel_columns(g, vp, g.x0 + ((float)ix + 0.5f) * g.vx, g.y0 + ((float)iy + 0.5f) * g.vy, ua, ub);
    ua = ua < cu0 ? cu0 : ua;
    ub = ub > cu0 + ncol - 1 ? cu0 + ncol - 1 : ub;
    const float mbz0 = (float)iz0 - g.hz;  // lower plane of the first voxel (centred index)
    const float zz0 = mbz0 + g.zc;         // the same plane as a height above the source plane
    const float vofs = -g.off_v / g.dv + g.cv;
    const int vmax = cv0 + nrow - 1;
    for (int iu = ua; iu <= ub; ++iu) {
        const ColStage cs = s_col[iu - cu0];
        float lo_e, hi_e;
        cell_range(ieta, heta, cs.eta_c, cs.inv_a, lo_e, hi_e);
        const float lo = fmaxf(lo_xi, lo_e), hi = fminf(hi_xi, hi_e);
        if (!(hi > lo)) continue;
        // Rows: a ray of height qz is at zeta = qz * T - zc, T = tcv + xi * gz > 0;
        // inside [lo, hi] it meets the z-cell [zz, zz + 1] (heights) only if
        // qz lies in [zz, zz + 1] / [Tmin, Tmax].
        const float T1 = cs.tcv + lo * cs.gz, T2 = cs.tcv + hi * cs.gz;
        const float ra = 1.0f / (fmaxf(T1, T2) * g.dv), rb = 1.0f / (fminf(T1, T2) * g.dv);
        float pa = zz0 * ra, pb = zz0 * rb;
        const float *e_col = s_e + (iu - cu0);
#pragma unroll
        for (int j = 0; j < TZ; ++j) {
            if (j < nzb) {
            const float zz1 = zz0 + (float)(j + 1);
            const float na = zz1 * ra, nb = zz1 * rb;
            const float vlo = fminf(pa, pb) + vofs, vhi = fmaxf(na, nb) + vofs;
            pa = na;
            pb = nb;
            int va = (int)ceilf(vlo - 0.01f), vb = (int)floorf(vhi + 0.01f);
            va = va < cv0 ? cv0 : va;
            vb = vb > vmax ? vmax : vb;
            const float mb = mbz0 + (float)j;
            for (int v = va; v <= vb; ++v) {
                const RowStage rs = s_row[v - cv0];
                const float zeta_c = zeta_centre(rs.qz, cs.tcv, g.zc);
                const float czr = zeta_inv_slope(rs.inv_qz, cs.kz);
                float lo_z, hi_z;
                cell_range_mb(iz0 + j, mb, g.hz, zeta_c, czr, lo_z, hi_z);
                const float w = fminf(hi, hi_z) - fmaxf(lo, lo_z);
                if (w > 0.0f) acc[j] = __builtin_fmaf(w, e_col[(v - cv0) * CH_COLS], acc[j]);
            }
            }
        }
    }
}

}  // namespace kct
