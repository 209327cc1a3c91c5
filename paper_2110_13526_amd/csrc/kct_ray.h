// kct_ray.h -- the two traversals of the weight function: along a ray (the
// forward projector's Siddon walk) and around a voxel (the backprojector's
// gather over views and candidate pixels).  Both call the functions of
// kct_weights.h on the same table entries, so they see identical weights.
// Host-callable as well, so the exact kernel arithmetic can be run on a CPU.
#pragma once

#pragma clang fp contract(off)

#include "kct_internal.h"
#include "kct_weights.h"

namespace kct {

// Walk one ray through the volume and return sum_j (xi-length in voxel j) * x_j.
// base/sxi/seta/szeta address the volume as [zeta][xi][eta].
template <typename T>
__host__ __device__ __forceinline__ float trace_ray(const T *__restrict__ base, int sxi, int seta, int szeta, int nxi,
                                           int neta, int nz, float hxi, float heta, float hz, float eta_c,
                                           float inv_a, float a, float zeta_c, float czr)
{
    // Parameter interval of the ray inside the volume box.
    float lo_e, hi_e, lo_z, hi_z;
    if (inv_a == 0.0f) {
        int m = parallel_cell(eta_c, heta);
        bool in = m >= 0 && m < neta;
        lo_e = in ? -INFINITY : INFINITY;
        hi_e = in ? INFINITY : -INFINITY;
    } else {
        float b0 = cross_at(-heta, eta_c, inv_a), b1 = cross_at(heta, eta_c, inv_a);
        lo_e = fminf(b0, b1);
        hi_e = fmaxf(b0, b1);
    }
    if (czr == 0.0f) {
        int m = parallel_cell(zeta_c, hz);
        bool in = m >= 0 && m < nz;
        lo_z = in ? -INFINITY : INFINITY;
        hi_z = in ? INFINITY : -INFINITY;
    } else {
        float b0 = cross_at(-hz, zeta_c, czr), b1 = cross_at(hz, zeta_c, czr);
        lo_z = fminf(b0, b1);
        hi_z = fmaxf(b0, b1);
    }
    const float entry = fmaxf(-hxi, fmaxf(lo_e, lo_z));
    const float exit_ = fminf(hxi, fminf(hi_e, hi_z));
    if (!(exit_ > entry)) return 0.0f;

    // Start every axis at its entry cell or one cell earlier along the ray
    // (clamped into the volume).  An earlier cell ends at or before the entry
    // point, so it receives a zero length and the walk moves on.
    int mx = (int)floorf(entry + hxi) - 1;
    mx = mx < 0 ? 0 : (mx > nxi - 1 ? nxi - 1 : mx);
    float lx = (float)mx - hxi;
    float hx = lx + 1.0f;

    int me, ste;
    float le, he, mbe;
    if (inv_a == 0.0f) {
        me = parallel_cell(eta_c, heta);
        ste = 0;
        le = -INFINITY;
        he = INFINITY;
        mbe = 0.0f;
    } else {
        ste = inv_a > 0.0f ? 1 : -1;
        int m = (int)floorf(eta_c + a * entry + heta) - ste;
        me = m < 0 ? 0 : (m > neta - 1 ? neta - 1 : m);
        float mb_lo = (float)(ste > 0 ? me : me + 1) - heta;
        mbe = (float)(ste > 0 ? me + 1 : me) - heta;
        le = cross_at(mb_lo, eta_c, inv_a);
        he = cross_at(mbe, eta_c, inv_a);
    }
    int mz, stz;
    float lz, hzv, mbz;
    if (czr == 0.0f) {
        mz = parallel_cell(zeta_c, hz);
        stz = 0;
        lz = -INFINITY;
        hzv = INFINITY;
        mbz = 0.0f;
    } else {
        stz = czr > 0.0f ? 1 : -1;
        int m = (int)floorf(zeta_c + entry / czr + hz) - stz;
        mz = m < 0 ? 0 : (m > nz - 1 ? nz - 1 : m);
        float mb_lo = (float)(stz > 0 ? mz : mz + 1) - hz;
        mbz = (float)(stz > 0 ? mz + 1 : mz) - hz;
        lz = cross_at(mb_lo, zeta_c, czr);
        hzv = cross_at(mbz, zeta_c, czr);
    }

    int idx = mz * szeta + mx * sxi + me * seta;
    const int de = ste * seta, dz = stz * szeta;
    const float fste = (float)ste, fstz = (float)stz;
    float acc = 0.0f;
    const int maxit = nxi + neta + nz + 8;
    for (int it = 0; it < maxit; ++it) {
        const float lmax = fmaxf(lx, fmaxf(le, lz));
        if (!(lmax < exit_)) break;
        const float hmin = fminf(hx, fminf(he, hzv));
        const float w = fmaxf(hmin - lmax, 0.0f);
        acc = __builtin_fmaf(w, to_f32(base[idx]), acc);
        const bool ax = hx == hmin, ae = he == hmin, az = hzv == hmin;
        lx = ax ? hx : lx;
        hx = ax ? hx + 1.0f : hx;
        idx += ax ? sxi : 0;
        const float mbe_n = mbe + fste;
        const float he_n = cross_at(mbe_n, eta_c, inv_a);
        le = ae ? he : le;
        mbe = ae ? mbe_n : mbe;
        he = ae ? he_n : he;
        idx += ae ? de : 0;
        const float mbz_n = mbz + fstz;
        const float hz_n = cross_at(mbz_n, zeta_c, czr);
        lz = az ? hzv : lz;
        mbz = az ? mbz_n : mbz;
        hzv = az ? hz_n : hzv;
        idx += az ? dz : 0;
    }
    return acc;
}

// Sum over all views of w_ij * L_i * e_i for voxel (ix, iy, iz): the
// backprojection of one voxel.  Candidate detector columns come from projecting
// the voxel's in-plane square, candidate rows from the z-range of each
// column's rays inside the voxel's column; both are bounds with a margin, the
// weight function decides.
template <typename T>
__host__ __device__ __forceinline__ float gather_voxel(const GeoDev &g, const T *__restrict__ proj, int ix, int iy,
                                                       int iz)
{
    float acc = 0.0f;
    const float wx0 = g.x0 + (float)ix * g.vx, wx1 = wx0 + g.vx;
    const float wy0 = g.y0 + (float)iy * g.vy, wy1 = wy0 + g.vy;
    const float zA = (float)iz - g.hz + g.zc;  // z-cell bounds as qz * T ranges
    const float zB = zA + 1.0f;
    for (int k = 0; k < g.nviews; ++k) {
        const ViewParam vp = g.views[k];
        // Detector columns whose in-plane rays can meet the voxel square:
        // project its four corners (a bound only; the weight decides).
        float fmin = INFINITY, fmax = -INFINITY;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const float dx = ((cc & 1) ? wx1 : wx0) - vp.sx;
            const float dy = ((cc & 2) ? wy1 : wy0) - vp.sy;
            const float num = -vp.s * dx + vp.c * dy;
            const float den = -vp.c * dx - vp.s * dy;
            const float f = (g.sdd * num / den - g.off_u) / g.du + g.cu;
            fmin = fminf(fmin, f);
            fmax = fmaxf(fmax, f);
        }
        int u0 = (int)ceilf(fmin - 0.01f), u1 = (int)floorf(fmax + 0.01f);
        u0 = u0 < 0 ? 0 : u0;
        u1 = u1 > g.nu - 1 ? g.nu - 1 : u1;
        int ixi, ieta;
        float hxi, heta;
        if (vp.dom == 0) { ixi = ix; ieta = iy; hxi = g.hx; heta = g.hy; }
        else { ixi = iy; ieta = ix; hxi = g.hy; heta = g.hx; }
        const float lo_xi = (float)ixi - hxi;
        const float hi_xi = (float)(ixi + 1) - hxi;
        for (int iu = u0; iu <= u1; ++iu) {
            const ColParam cp = g.cols[(size_t)k * g.nu + iu];
            float lo_e, hi_e;
            cell_range(ieta, heta, cp.eta_c, cp.inv_a, lo_e, hi_e);
            const float lo = fmaxf(lo_xi, lo_e), hi = fminf(hi_xi, hi_e);
            if (!(hi > lo)) continue;
            // Detector rows whose rays meet the z-cell within [lo, hi] (a bound).
            const float gz = cp.gp * g.inv_vz;
            const float T1 = cp.tcv + lo * gz, T2 = cp.tcv + hi * gz;
            const float qlo = fminf(zA / T1, zA / T2), qhi = fmaxf(zB / T1, zB / T2);
            int v0 = (int)ceilf((qlo - g.off_v) / g.dv + g.cv - 0.01f);
            int v1 = (int)floorf((qhi - g.off_v) / g.dv + g.cv + 0.01f);
            v0 = v0 < 0 ? 0 : v0;
            v1 = v1 > g.nv - 1 ? g.nv - 1 : v1;
            for (int iv = v0; iv <= v1; ++iv) {
                const RowParam rp = g.rows[iv];
                const float zeta_c = zeta_centre(rp.qz, cp.tcv, g.zc);
                const float czr = zeta_inv_slope(rp.inv_qz, cp.kz);
                float lo_z, hi_z;
                cell_range(iz, g.hz, zeta_c, czr, lo_z, hi_z);
                const float w = fminf(hi, hi_z) - fmaxf(lo, lo_z);
                if (w > 0.0f) {
                    const float L = ray_length_per_xi(cp.lxy2, rp.qz, cp.gp);
                    const float e = to_f32(proj[((size_t)k * g.nv + iv) * g.nu + iu]);
                    acc = __builtin_fmaf(w, L * e, acc);
                }
            }
        }
    }
    return acc;
}

}  // namespace kct
