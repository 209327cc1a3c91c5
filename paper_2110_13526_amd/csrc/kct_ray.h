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

// v for a value equal in every lane of the wavefront, made visibly uniform on
// the GPU (a scalar copy), so that addresses built from it stay scalar.
__host__ __device__ __forceinline__ int uniform_int(int v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_readfirstlane(v);
#else
    return v;
#endif
}

// x unchanged, as a value the compiler has to hold in a register where this
// stands: a computation on it cannot move above that point (on the host: x).
__host__ __device__ __forceinline__ unsigned settle(unsigned x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+v"(x));
#endif
    return x;
}

// Element m of a z-column as an accumulator value, 0 for m outside [0, nz)
// (cells outside the volume).  ZCol<T, 1> is a column of the z-fastest copy:
// on the GPU a buffer resource over the column's nz elements (built in scalar
// registers from the column's base, which is equal in every lane of the
// wavefront), so each load takes a 32-bit per-lane byte offset, no 64-bit
// address arithmetic, and the hardware's range check supplies the 0 outside
// the column.  ZCol<T, 0> is a column of the z-slowest layout (stride sz), read
// through its pointer.
template <typename T, int SZ> struct ZCol {
    const T *col;
    int nz, sz;
    __host__ __device__ __forceinline__ ZCol(const T *c, int n, int s) : col(c), nz(n), sz(s) {}
    __host__ __device__ __forceinline__ T raw(int m) const
    {
        const bool in = (unsigned)m < (unsigned)nz;
        const T v = col[in ? (unsigned)m * (unsigned)(SZ == 1 ? 1 : sz) : 0u];
        return in ? v : T{};
    }
    __host__ __device__ __forceinline__ acc_t<T> at(int m) const { return to_acc(raw(m)); }
    // the bits of a 2-byte element, zero-extended
    __host__ __device__ __forceinline__ unsigned bits16(int m) const
    {
        return (unsigned)__builtin_bit_cast(unsigned short, raw(m));
    }
};

#if defined(__HIP_DEVICE_COMPILE__)
template <typename T> struct ZCol<T, 1> {
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ __forceinline__ ZCol(const T *c, int nz, int)
        : rsrc(__builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(c), (short)0, nz * (int)sizeof(T), 0x00020000))
    {
    }
    __device__ __forceinline__ T raw(int m) const
    {
        const int boff = m * (int)sizeof(T);  // m outside [0, nz): beyond the resource, read as 0
        if constexpr (sizeof(T) == 4) {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rsrc, boff, 0, 0));
        } else if constexpr (sizeof(T) == 2) {
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(rsrc, boff, 0, 0));
        } else {
            static_assert(sizeof(T) == 8, "4-, 2- or 8-byte storage");
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rsrc, boff, 0, 0));
        }
    }
    __device__ __forceinline__ acc_t<T> at(int m) const { return to_acc(raw(m)); }
    __device__ __forceinline__ unsigned bits16(int m) const
    {
        return (unsigned)__builtin_amdgcn_raw_buffer_load_b16(rsrc, m * 2, 0, 0);
    }
};
#endif

// z-walk state of one ray: current z-cell mz, walking direction stz (and as a
// float, fstz), the index-frame coordinate hbf of the plane where the walk
// leaves mz (an exact small integer or half-integer, so stepping it by +-1 is
// exact), and the crossings lz (entry into mz) and hzv (exit from mz).  Cells
// outside [0, nz) hold no voxel and read as 0: the walk starts at most one
// cell outside the volume (-1 / nz, entry or exit at +-inf when the ray meets
// no plane on that side), and once it has crossed the last plane it steps on
// through such cells, whose crossings are those of the continued plane grid.
// Between pieces lz <= t0 <= hzv holds for the piece [t0, t1] about to be
// walked, so the part of the ray in mz inside the piece is min(t1, hzv) - t0,
// and that of a cell entered inside it (at its lz >= t0) is min(t1, hzv) - lz:
// the min-of-highs minus max-of-lows of kct_weights.h, whose other terms are
// then known, and never negative.
struct ZWalk {
    int mz, stz;
    float hbf, fstz;
    float lz, hzv, nzc, czr;  // nzc = zeta_offset(zeta_c, czr)
};

// Move the walk into the next z-cell along the ray.
__host__ __device__ __forceinline__ void zwalk_step(ZWalk &s)
{
    s.lz = s.hzv;
    s.mz += s.stz;
    s.hbf += s.fstz;
    s.hzv = zeta_cross(s.hbf, s.nzc, s.czr);
}

// Start the z-walk of a ray at the in-plane entry t_start: in the cell of
// t_start (estimated one cell early, clamped to the sentinels, then stepped
// on until its exit lies at or after t_start).  A ray that never meets the
// volume in [t_start, t_end] gets an inert state in cell -1 (read as 0, no
// crossing).
__host__ __device__ __forceinline__ void zwalk_init(ZWalk &s, float zeta_c, float czr, int nz, float hz,
                                                    float t_start, float t_end)
{
    s.nzc = zeta_offset(zeta_c, czr);
    s.czr = czr;
    s.hbf = 0.0f;
    s.fstz = 0.0f;
    if (czr == 0.0f) {
        s.mz = parallel_cell(zeta_c, hz);
        s.stz = 0;
        s.lz = -INFINITY;
        s.hzv = INFINITY;
        if (s.mz < 0 || s.mz >= nz) { s.mz = -1; s.lz = INFINITY; }
        return;
    }
    const float b0 = zeta_cross(-hz, s.nzc, czr), b1 = zeta_cross((float)nz - hz, s.nzc, czr);
    if (!(fminf(t_end, fmaxf(b0, b1)) > fmaxf(t_start, fminf(b0, b1)))) {
        s.mz = -1;
        s.stz = 0;
        s.lz = INFINITY;
        s.hzv = INFINITY;
        return;
    }
    s.stz = czr > 0.0f ? 1 : -1;
    s.fstz = (float)s.stz;
    const int m = (int)floorf(zeta_c + t_start / czr + hz) - s.stz;
    s.mz = m < -1 ? -1 : (m > nz ? nz : m);
    const int hb = s.stz > 0 ? s.mz + 1 : s.mz;
    const int lb = hb - s.stz;
    s.hbf = (float)hb - hz;
    s.lz = (lb >= 0 && lb <= nz) ? zeta_cross((float)lb - hz, s.nzc, czr) : -INFINITY;
    s.hzv = (hb >= 0 && hb <= nz) ? zeta_cross(s.hbf, s.nzc, czr) : INFINITY;
    for (int guard = nz + 2; s.hzv < t_start && guard > 0; --guard) zwalk_step(s);
}

// The rest of the ray's part inside the in-plane piece [t0, t1] (in-plane cell
// whose z-column starts at col; element m of it at col[m * SZ]) after the
// z-cells already added: one more z-cell per z-plane crossed before t1 (the
// piece loop takes the first crossing; z-slopes are small, so more are rare).
// The guard only ends walks through cells outside the volume.
template <typename T, int SZ>
__host__ __device__ __forceinline__ void zwalk_steps(ZWalk &s, const T *__restrict__ col, int sz, int nz,
                                                     float t1, acc_t<T> &acc)
{
    for (int guard = nz + 1; s.hzv < t1 && guard > 0; --guard) {
        zwalk_step(s);
        const float w = fminf(t1, s.hzv) - s.lz;
        if ((unsigned)s.mz < (unsigned)nz) {
            const unsigned off = SZ == 1 ? (unsigned)s.mz : (unsigned)s.mz * (unsigned)sz;
            acc = fma_acc(w, to_acc(col[off]), acc);
        }
    }
}

// Walk R rays of one detector column (rows differ, so zeta_c and czr differ)
// through the volume and return sum_j (xi-length in voxel j) * x_j per ray, in
// the accumulator precision of the storage type.
//
// The walk is split so that rays of one detector column do identical in-plane
// work and share it:
//   * the in-plane walk (xi and eta planes) depends on the column only; it
//     enumerates the pieces [t0, t1] of the rays' shadow in the (x, y) plane,
//     one per in-plane cell, in increasing xi;
//   * the zeta walk is per ray: inside each in-plane piece the ray adds the
//     piece's part in its current z-cell and steps to the next z-cell when it
//     crosses a z-plane before t1 (rare: z-slopes are small).
// Every weight is min(the three highs) - max(the three lows) of kct_weights.h:
// t0 equals the larger in-plane low (the walk starts at an exact cell and t0 is
// always the crossing at which the current in-plane cell was entered).
// Volume addressing: element (zeta cell m, xi cell i, eta cell e) is at
// vol[m * sz + i * sxi + e * seta].  With the z-fastest copy of the volume
// (sz = 1, which SZ = 1 fixes at compile time), lanes that hold neighbouring
// rows read neighbouring addresses.  The in-plane walk depends on the column
// only: with uniform column parameters it runs on scalar branches.
template <typename T, int R, int SZ = 0>
__host__ __device__ __forceinline__ void trace_rays(const T *__restrict__ vol, int sxi, int seta, int sz, int nxi,
                                                    int neta, int nz, float hxi, float heta, float hz, float eta_c,
                                                    float inv_a, float a, const float (&zeta_c)[R],
                                                    const float (&czr)[R], acc_t<T> (&acc)[R])
{
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0;
    // In-plane extent [t_start, t_end] of the rays inside the volume's (x, y) box.
    float lo_e, hi_e;
    if (inv_a == 0.0f) {
        const int m = parallel_cell(eta_c, heta);
        const bool in = m >= 0 && m < neta;
        lo_e = in ? -INFINITY : INFINITY;
        hi_e = in ? INFINITY : -INFINITY;
    } else {
        const float b0 = cross_at(-heta, eta_c, inv_a), b1 = cross_at((float)neta - heta, eta_c, inv_a);
        lo_e = fminf(b0, b1);
        hi_e = fmaxf(b0, b1);
    }
    const float t_start = fmaxf(-hxi, lo_e);
    const float t_end = fminf((float)nxi - hxi, hi_e);
    if (!(t_end > t_start)) return;
    ZWalk zs[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        zwalk_init(zs[r], zeta_c[r], czr[r], nz, hz, t_start, t_end);
        any = any || zs[r].hzv != INFINITY || zs[r].lz != INFINITY;
    }
    if (!any) return;

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

    // The z-walk over one in-plane piece [t0, t1] for every row, as far as its
    // first crossed z-plane: the weight w and cell m of the current z-cell, and
    // w2 and m2 of the cell entered at that plane (w2 = 0 and m2 = m when the
    // ray crosses none).
    auto first_cells = [&](float t0, float t1, float (&w)[R], int (&m)[R], float (&w2)[R], int (&m2)[R]) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            ZWalk &z = zs[r];
            w[r] = fminf(t1, z.hzv) - t0;
            m[r] = z.mz;
            const bool c = z.hzv < t1;
            const float nhbf = z.hbf + z.fstz;
            const float nhzv = zeta_cross(nhbf, z.nzc, z.czr);
            if (c) {
                z.lz = z.hzv;
                z.mz += z.stz;
                z.hbf = nhbf;
                z.hzv = nhzv;
            }
            w2[r] = c ? fminf(t1, z.hzv) - z.lz : 0.0f;
            m2[r] = z.mz;
        }
    };
    // One in-plane piece [t0, t1] inside the in-plane cell whose z-column
    // starts at vol + base: the current z-cell of every row, then the z-cells
    // entered inside the piece, the same additions in the same order as a walk
    // that handles one z-cell at a time.  A cell outside the volume reads as 0
    // and leaves the sum as it is.
    auto piece = [&](float t0, float t1, int base) {
        float w[R], w2[R];
        int m[R], m2[R];
        first_cells(t0, t1, w, m, w2, m2);
        const T *col = vol + uniform_int(base);
        const ZCol<T, SZ> zc(col, nz, sz);
        // the current cells' loads go out together; a crossed cell is read only
        // in the lanes whose ray enters it (the loads' cost grows with the lanes
        // that take part, and most pieces cross no z-plane).  2-byte values are
        // widened after the lanes rejoin, so that no lane waits for its load
        // inside the masked region
        acc_t<T> v[R], v2[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = zc.at(m[r]);
        if constexpr (sizeof(T) >= 4) {
#pragma unroll
            for (int r = 0; r < R; ++r) v2[r] = m2[r] != m[r] ? zc.at(m2[r]) : acc_t<T>(0);
        } else {
            unsigned x2[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                x2[r] = 0u;
                if (m2[r] != m[r]) x2[r] = zc.bits16(m2[r]);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) v2[r] = to_acc(__builtin_bit_cast(T, (unsigned short)settle(x2[r])));
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            acc[r] = fma_acc(w[r], v[r], acc[r]);
            acc[r] = fma_acc(w2[r], v2[r], acc[r]);
        }
        // further crossings inside the piece (steep rays only)
#pragma unroll
        for (int r = 0; r < R; ++r) zwalk_steps<T, SZ>(zs[r], col, sz, nz, t1, acc[r]);
    };
    int base = mx * sxi + me * seta;
    const int de = ste * seta;
    const float fste = (float)ste;
    // the in-plane walk past the end t1 of the current piece
    auto advance = [&](float t1) {
        if (hx == t1) {
            hx += 1.0f;
            base += sxi;
        }
        if (he == t1) {
            mbe += fste;
            he = cross_at(mbe, eta_c, inv_a);
            base += de;
        }
    };
    float t0 = t_start;
    for (int guard = nxi + neta + 4; t0 < t_end && guard > 0; --guard) {
        const float t1 = fminf(hx, he);
        piece(t0, t1, base);
        advance(t1);
        t0 = t1;
    }
}

}  // namespace kct
