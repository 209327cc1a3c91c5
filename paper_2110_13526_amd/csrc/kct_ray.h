// kct_ray.h -- the forward projector's walk along one ray (Siddon's merge of
// the three families of voxel-plane crossings).  It evaluates the weight
// function of kct_weights.h, as the backprojector's gather (kct_gather.h) does,
// on the same table entries, so both see identical weights.  Host-callable as
// well, so the kernel arithmetic can be run on a CPU.
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

}  // namespace kct
