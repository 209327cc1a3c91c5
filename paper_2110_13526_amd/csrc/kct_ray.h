// kct_ray.h -- the forward projector's walk along one ray (Siddon's merge of
// the three families of voxel-plane crossings, in increasing xi).  It evaluates the weight
// function of kct_weights.h, as the backprojector's gather (kct_gather.h) does,
// on the same table entries, so both see identical weights.  Host-callable as
// well, so the kernel arithmetic can be run on a CPU.
#pragma once

#pragma clang fp contract(off)

#include "kct_internal.h"
#include "kct_weights.h"

namespace kct {

// Walk one ray through the volume and return sum_j (xi-length in voxel j) * x_j.
//
// The walk is split so that a wavefront whose lanes are rays of one detector
// column (different rows) does identical in-plane work in every lane:
//   * the in-plane walk (xi and eta planes) depends on the column only; it
//     enumerates the pieces [t0, t1] of the ray's shadow in the (x, y) plane,
//     one per in-plane cell, in increasing xi;
//   * the zeta walk is per lane: inside each in-plane piece the lane adds the
//     piece's part in its current z-cell and steps to the next z-cell when the
//     ray crosses a z-plane before t1 (rare: z-slopes are small).
// Every weight is min(the three highs) - max(the three lows) of kct_weights.h:
// t0 equals the larger in-plane low (the walk starts at an exact cell and t0 is
// always the crossing at which the current in-plane cell was entered).
// Volume addressing: element (zeta cell m, xi cell i, eta cell e) is at
// vol[m * sz + i * sxi + e * seta].  With the z-fastest copy of the volume
// (sz = 1) the 64 lanes of a wavefront read neighbouring addresses.
// z-cells -1 and nz stand for "below" and "above" the volume: nothing is read
// there, and the crossing out of the volume is never followed back.
template <typename T>
__host__ __device__ __forceinline__ float trace_ray(const T *__restrict__ vol, int sxi, int seta, int sz, int nxi,
                                                    int neta, int nz, float hxi, float heta, float hz, float eta_c,
                                                    float inv_a, float a, float zeta_c, float czr)
{
    // In-plane extent [t_start, t_end] of the ray inside the volume's (x, y) box.
    float lo_e, hi_e;
    if (inv_a == 0.0f) {
        const int m = parallel_cell(eta_c, heta);
        const bool in = m >= 0 && m < neta;
        lo_e = in ? -INFINITY : INFINITY;
        hi_e = in ? INFINITY : -INFINITY;
    } else {
        const float b0 = cross_at(-heta, eta_c, inv_a), b1 = cross_at(heta, eta_c, inv_a);
        lo_e = fminf(b0, b1);
        hi_e = fmaxf(b0, b1);
    }
    const float t_start = fmaxf(-hxi, lo_e);
    const float t_end = fminf(hxi, hi_e);
    if (!(t_end > t_start)) return 0.0f;
    // This lane's extent in z; a ray that never meets the volume does nothing.
    if (czr == 0.0f) {
        const int m = parallel_cell(zeta_c, hz);
        if (m < 0 || m >= nz) return 0.0f;
    } else {
        const float b0 = cross_at(-hz, zeta_c, czr), b1 = cross_at(hz, zeta_c, czr);
        if (!(fminf(t_end, fmaxf(b0, b1)) > fmaxf(t_start, fminf(b0, b1)))) return 0.0f;
    }

    // Exact in-plane cells at t_start: lo <= t_start < hi on both axes.
    int mx = (int)floorf(t_start + hxi);
    mx = mx < 0 ? 0 : (mx > nxi - 1 ? nxi - 1 : mx);
    float hx = (float)(mx + 1) - hxi;
    while (hx <= t_start && mx < nxi - 1) { ++mx; hx += 1.0f; }
    while (hx - 1.0f > t_start && mx > 0) { --mx; hx -= 1.0f; }
    int me, ste;
    float he, mbe;
    if (inv_a == 0.0f) {
        me = parallel_cell(eta_c, heta);
        ste = 0;
        he = INFINITY;
        mbe = 0.0f;
    } else {
        ste = inv_a > 0.0f ? 1 : -1;
        int m = (int)floorf(eta_c + a * t_start + heta);
        me = m < 0 ? 0 : (m > neta - 1 ? neta - 1 : m);
        mbe = (float)(ste > 0 ? me + 1 : me) - heta;  // plane of the cell's exit crossing
        he = cross_at(mbe, eta_c, inv_a);
        float le = cross_at(mbe - (float)ste, eta_c, inv_a);
        while (he <= t_start && me + ste >= 0 && me + ste < neta) {
            me += ste;
            mbe += (float)ste;
            le = he;
            he = cross_at(mbe, eta_c, inv_a);
        }
        while (le > t_start && me - ste >= 0 && me - ste < neta) {
            me -= ste;
            mbe -= (float)ste;
            he = le;
            le = cross_at(mbe - (float)ste, eta_c, inv_a);
        }
    }

    // z state: start at the cell of t_start or one before it along the ray
    // (clamped to the sentinels -1 / nz); the first piece then moves on.
    int mz, stz, hb;
    float lz, hzv;
    if (czr == 0.0f) {
        mz = parallel_cell(zeta_c, hz);
        stz = 0;
        hb = 0;
        lz = -INFINITY;
        hzv = INFINITY;
    } else {
        stz = czr > 0.0f ? 1 : -1;
        int m = (int)floorf(zeta_c + t_start / czr + hz) - stz;
        mz = m < -1 ? -1 : (m > nz ? nz : m);
        hb = stz > 0 ? mz + 1 : mz;
        const int lb = hb - stz;
        lz = (lb >= 0 && lb <= nz) ? cross_at((float)lb - hz, zeta_c, czr) : -INFINITY;
        hzv = (hb >= 0 && hb <= nz) ? cross_at((float)hb - hz, zeta_c, czr) : INFINITY;
    }

    int base = mx * sxi + me * seta;
    const int de = ste * seta;
    const float fste = (float)ste;
    float acc = 0.0f;
    float t0 = t_start;
    for (int guard = nxi + neta + 4; t0 < t_end && guard > 0; --guard) {
        const float t1 = fminf(hx, he);
        for (int zg = nz + 2; zg > 0; --zg) {
            const float w = fminf(t1, hzv) - fmaxf(t0, lz);
            if (w > 0.0f && (unsigned)mz < (unsigned)nz) acc = __builtin_fmaf(w, to_f32(vol[base + mz * sz]), acc);
            if (!(hzv < t1)) break;
            lz = hzv;
            mz += stz;
            hb += stz;
            hzv = (hb >= 0 && hb <= nz) ? cross_at((float)hb - hz, zeta_c, czr) : INFINITY;
        }
        if (hx == t1) {
            hx += 1.0f;
            base += sxi;
        }
        if (he == t1) {
            mbe += fste;
            he = cross_at(mbe, eta_c, inv_a);
            base += de;
        }
        t0 = t1;
    }
    return acc;
}

}  // namespace kct
