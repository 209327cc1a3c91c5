// kct_tt.h -- the weight of the TT footprint projector (separable footprints,
// trapezoid transaxial x trapezoid axial; Section 3 names footprint methods,
// the experiments of Section 4 use this variant), shared by its forward and
// backward kernel so that both evaluate identical weights.
//
// Model: a_ij = L_i * F_u(i, j) * F_v(i, j).  F_u is the mean over ray i's
// detector column of the unit trapezoid whose breakpoints are the detector
// column coordinates of voxel j's four in-plane corners; F_v the mean over its
// detector row of the unit trapezoid with breakpoints v(z_lo, D_min),
// v(z_lo, D_max), v(z_hi, D_min), v(z_hi, D_max) (the voxel's z extent seen
// from its nearest and farthest in-plane corner, depths D along the central
// ray); L_i = min(vx / |d_x|, vy / |d_y|, vz / |d_z|) for ray i's unit direction
// d (the path of the ray through one cell of each axis, the shortest of the three).  Coordinates are detector pixel indices, pixel i
// spanning [i - 1/2, i + 1/2].  Corner and plane coordinates are computed from
// their integer plane indices, so neighbouring voxels share breakpoints
// bit for bit (their trapezoids then sum to one across a row of voxels).
#pragma once

#pragma clang fp contract(off)

#include "kct_internal.h"
#include "kct_weights.h"

namespace kct {

__host__ __device__ __forceinline__ void tt_sort4(float (&t)[4])
{
    float a = fminf(t[0], t[1]), b = fmaxf(t[0], t[1]);
    float c = fminf(t[2], t[3]), d = fmaxf(t[2], t[3]);
    const float lo = fminf(a, c), m1 = fmaxf(a, c);
    const float hi = fmaxf(b, d), m2 = fminf(b, d);
    t[0] = lo;
    t[1] = fminf(m1, m2);
    t[2] = fmaxf(m1, m2);
    t[3] = hi;
}

// Reciprocal (one hardware reciprocal on the GPU; both kernels of the pair use
// this same function, so their weights stay bitwise identical).
__host__ __device__ __forceinline__ float tt_rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// A unit trapezoid t[0] <= t[1] <= t[2] <= t[3] with the reciprocals of twice
// its ramp widths (used only where the ramp is wider than zero).
struct TTTrap {
    float t[4];
    float r1, r2;  // 1 / (2 (t1 - t0)), 1 / (2 (t3 - t2))
};

__host__ __device__ __forceinline__ void tt_ramps(TTTrap &p)
{
    p.r1 = 0.5f * tt_rcp(p.t[1] - p.t[0]);
    p.r2 = 0.5f * tt_rcp(p.t[3] - p.t[2]);
}

// Integral of the trapezoid from -inf to u.
__host__ __device__ __forceinline__ float tt_cum(const TTTrap &p, float u)
{
    const float(&t)[4] = p.t;
    if (u <= t[0]) return 0.0f;
    if (u < t[1]) {
        const float a = u - t[0];
        return a * a * p.r1;
    }
    const float g = 0.5f * (t[1] - t[0]);
    if (u < t[2]) return g + (u - t[1]);
    const float g2 = g + (t[2] - t[1]);
    if (u < t[3]) {
        const float b = t[3] - u;
        return g2 + 0.5f * (t[3] - t[2]) - b * b * p.r2;
    }
    return g2 + 0.5f * (t[3] - t[2]);
}

// Mean of the trapezoid over detector pixel i.
__host__ __device__ __forceinline__ float tt_mean(const TTTrap &p, int i)
{
    return tt_cum(p, (float)i + 0.5f) - tt_cum(p, (float)i - 0.5f);
}

// Transaxial trapezoid (detector column coordinates) of voxel column (ix, iy)
// in view vp, the smallest and largest depth of its corners and their
// reciprocals.
__host__ __device__ __forceinline__ void tt_transaxial(const GeoDev &g, const ViewParam &vp, int ix, int iy,
                                                       TTTrap &tu, float &dmin, float &dmax, float &rdmin,
                                                       float &rdmax)
{
    dmin = INFINITY;
    dmax = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float px = g.x0 + (float)(ix + (q & 1)) * g.vx;
        const float py = g.y0 + (float)(iy + (q >> 1)) * g.vy;
        // lateral coordinate (the source's is zero) and depth from the source,
        // both from the corner's own coordinates: no cancellation against the
        // source position
        const float num = -vp.s * px + vp.c * py;
        const float den = g.sid - (vp.c * px + vp.s * py);
        tu.t[q] = (g.sdd * num * tt_rcp(den) - g.off_u) * g.inv_du + g.cu;
        dmin = fminf(dmin, den);
        dmax = fmaxf(dmax, den);
    }
    tt_sort4(tu.t);
    tt_ramps(tu);
    rdmin = tt_rcp(dmin);
    rdmax = tt_rcp(dmax);
}

// Row scales of a voxel column: the detector row coordinate of height z seen
// at depth D is z * (SDD / (D dv)) + row_offset, with ka for the nearest and kb
// for the farthest corner depth (ka >= kb > 0).
__host__ __device__ __forceinline__ void tt_row_scales(const GeoDev &g, float rdmin, float rdmax, float &ka, float &kb)
{
    const float s = g.sdd * g.inv_dv;
    ka = s * rdmin;
    kb = s * rdmax;
}
__host__ __device__ __forceinline__ float tt_row_offset(const GeoDev &g) { return g.cv - g.off_v * g.inv_dv; }

// Axial trapezoid of voxel layer iz of a column with row scales ka, kb.  The
// row coordinate grows with z at either scale, so the two images of the lower
// plane lie below those of the upper plane and sorting needs only their
// inner pair.
__host__ __device__ __forceinline__ void tt_axial(const GeoDev &g, int iz, float ka, float kb, float off, TTTrap &tv)
{
    const float zl = g.z0 + (float)iz * g.vz, zh = g.z0 + (float)(iz + 1) * g.vz;
    const float la = __builtin_fmaf(zl, ka, off), lb = __builtin_fmaf(zl, kb, off);
    const float ha = __builtin_fmaf(zh, ka, off), hb = __builtin_fmaf(zh, kb, off);
    const float l1 = fmaxf(la, lb), h0 = fminf(ha, hb);
    tv.t[0] = fminf(la, lb);
    tv.t[1] = fminf(l1, h0);
    tv.t[2] = fmaxf(l1, h0);
    tv.t[3] = fmaxf(ha, hb);
    tt_ramps(tv);
}

// L_i from the Siddon length factor L per unit xi (the path through one xi
// cell) and the ray's d xi / d eta (inv_a) and d xi / d zeta (czr): the path
// through one cell of each axis is L, L |inv_a| and L |czr|; a zero inverse
// slope marks a ray parallel to that axis' planes.
__host__ __device__ __forceinline__ float tt_amplitude(float L, float inv_a, float czr)
{
    float m = 1.0f;
    if (inv_a != 0.0f) m = fminf(m, fabsf(inv_a));
    if (czr != 0.0f) m = fminf(m, fabsf(czr));
    return L * m;
}

// Pixels [a, b] of an axis whose extent meets the open interval (t0, t3).
__host__ __device__ __forceinline__ void tt_pixels(float t0, float t3, int &a, int &b)
{
    a = (int)ceilf(t0 - 0.5f);
    b = (int)floorf(t3 + 0.5f);
}

// In-plane line through the source and the detector point at column coordinate
// uc, in the view's dominant frame of voxel indices (kct_internal.h): eta = e0 + e1 xi.
__host__ __device__ __forceinline__ void tt_edge_line(const GeoDev &g, const ViewParam &vp, float uc, float &e0, float &e1)
{
    const float umm = (uc - g.cu) * g.du + g.off_u;
    const float px = vp.sx - g.sdd * vp.c - umm * vp.s;
    const float py = vp.sy - g.sdd * vp.s + umm * vp.c;
    const float sX = (vp.sx - g.x0) / g.vx - g.hx, sY = (vp.sy - g.y0) / g.vy - g.hy;
    const float pX = (px - g.x0) / g.vx - g.hx, pY = (py - g.y0) / g.vy - g.hy;
    const float sxi = vp.dom == 0 ? sX : sY, seta = vp.dom == 0 ? sY : sX;
    const float pxi = vp.dom == 0 ? pX : pY, peta = vp.dom == 0 ? pY : pX;
    e1 = (peta - seta) / (pxi - sxi);
    e0 = seta - e1 * sxi;
}


// Sums over the voxels j of rays (iu, iv[r]), r < R, of fl(F_u F_v) x_j,
// without L_i.  Walking the view's dominant axis slab by slab, the voxel
// columns inside the wedge between the rays through the column's two edges are
// visited (widened by 0.01 cell against rounding; columns outside get F_u = 0);
// a column's transaxial footprint is shared by the R rows, and for each row the
// z-cells whose axial footprint can meet it are visited.  active[r] = false: the
// lane takes part in the column's work but adds nothing for row r (a row past
// the detector).  Every row's sum takes its terms in the same order as with
// R = 1.  Volume element (iz, iy, ix) is vol_z[(iy nx + ix) nz + iz] (z-fastest
// copy) or vol[(iz ny + iy) nx + ix].
template <typename TV, int R>
__host__ __device__ __forceinline__ void tt_ray_sums(const GeoDev &g, const ViewParam &vp, int iu,
                                                     const int (&iv)[R], const bool (&active)[R],
                                                     const TV *__restrict__ vol, const TV *__restrict__ vol_z,
                                                     acc_t<TV> (&acc)[R])
{
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0;
    const bool dom0 = vp.dom == 0;
    const int nxi = dom0 ? g.nx : g.ny, neta = dom0 ? g.ny : g.nx;
    const float hxi = dom0 ? g.hx : g.hy, heta = dom0 ? g.hy : g.hx;
    float a0, a1, b0, b1;
    tt_edge_line(g, vp, (float)iu - 0.5f, a0, a1);
    tt_edge_line(g, vp, (float)iu + 0.5f, b0, b1);
    // each row's extent on the detector [mm]; at depth D a ray to height v is at z = v D / SDD
    float vlo[R], vhi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        vlo[r] = ((float)iv[r] - 0.5f - g.cv) * g.dv + g.off_v;
        vhi[r] = ((float)iv[r] + 0.5f - g.cv) * g.dv + g.off_v;
    }
    const float rsdd = 1.0f / g.sdd;
    const float roff = tt_row_offset(g);
    for (int m = 0; m < nxi; ++m) {
        const float xl = (float)m - hxi, xh = xl + 1.0f;
        const float ea = a0 + a1 * xl, eb = a0 + a1 * xh, ec = b0 + b1 * xl, ed = b0 + b1 * xh;
        const float emin = fminf(fminf(ea, eb), fminf(ec, ed)), emax = fmaxf(fmaxf(ea, eb), fmaxf(ec, ed));
        // the eta-cells meeting [emin, emax], widened by 0.01 cell against the rounding
        // differences to tt_transaxial's breakpoints
        int e_lo = (int)floorf(emin + heta - 0.01f), e_hi = (int)floorf(emax + heta + 0.01f);
        e_lo = e_lo < 0 ? 0 : e_lo;
        e_hi = e_hi > neta - 1 ? neta - 1 : e_hi;
        for (int e = e_lo; e <= e_hi; ++e) {
            const int ix = dom0 ? m : e, iy = dom0 ? e : m;
            TTTrap tu;
            float dmin, dmax, rdmin, rdmax;
            tt_transaxial(g, vp, ix, iy, tu, dmin, dmax, rdmin, rdmax);
            const float fu = tt_mean(tu, iu);
            if (!(fu > 0.0f)) continue;
            float ka, kb;
            tt_row_scales(g, rdmin, rdmax, ka, kb);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (!active[r]) continue;
                const float z1 = vlo[r] * dmin * rsdd, z2 = vlo[r] * dmax * rsdd;
                const float z3 = vhi[r] * dmin * rsdd, z4 = vhi[r] * dmax * rsdd;
                const float zmn = fminf(fminf(z1, z2), fminf(z3, z4)), zmx = fmaxf(fmaxf(z1, z2), fmaxf(z3, z4));
                // the z-cells meeting [zmn, zmx], widened by 0.01 cell against the rounding
                // differences to tt_axial's breakpoints (relative ~1e-6 of z)
                int za = (int)floorf((zmn - g.z0) * g.inv_vz - 0.01f), zb = (int)floorf((zmx - g.z0) * g.inv_vz + 0.01f);
                za = za < 0 ? 0 : za;
                zb = zb > g.nz - 1 ? g.nz - 1 : zb;
                for (int iz = za; iz <= zb; ++iz) {
                    TTTrap tv;
                    tt_axial(g, iz, ka, kb, roff, tv);
                    const float fv = tt_mean(tv, iv[r]);
                    if (fv > 0.0f) {
                        const TV xv = vol_z ? vol_z[((size_t)iy * g.nx + ix) * g.nz + iz]
                                            : vol[((size_t)iz * g.ny + iy) * g.nx + ix];
                        acc[r] = fma_acc(fu * fv, to_acc(xv), acc[r]);
                    }
                }
            }
        }
    }
}

// One lane's share of one staged chunk: add fl(F_u F_v) * s_le[pixel] to acc[j]
// for the voxels (ix, iy, iz0 + j), j < nzb, of a column with transaxial
// breakpoints tu and depth reciprocals rdmin, rdmax, over the staged pixels
// (column cu0 + c, row cv0 + r) at s_le[r * stride + c].  SQ: add
// fl(F_u F_v)^2 * s_le instead (with s_le = L^2 this sums the squared weights).
template <typename A, bool SQ, int NC = 4, int TZN = 16>
__host__ __device__ __forceinline__ void tt_gather_chunk(const GeoDev &g, int iz0, int nzb, const TTTrap &tu,
                                                         float rdmin, float rdmax, const A *s_le, int stride, int cu0,
                                                         int ncol, int cv0, int nrow, A (&acc)[TZN])
{
    int ua, ub;
    tt_pixels(tu.t[0], tu.t[3], ua, ub);
    ua = ua < cu0 ? cu0 : ua;
    ub = ub > cu0 + ncol - 1 ? cu0 + ncol - 1 : ub;
    const int vmax = cv0 + nrow - 1;
    float ka, kb;
    tt_row_scales(g, rdmin, rdmax, ka, kb);
    const float roff = tt_row_offset(g);
    for (int c0 = ua; c0 <= ub; c0 += NC) {
        // The axial trapezoids below do not depend on c0; computed inside the
        // loop they stay short-lived (hoisted out, all TZN of them would be
        // live at once and spill).  The empty asm keeps the compiler from
        // hoisting them.
        float kai = ka, kbi = kb;
#if defined(__HIP_DEVICE_COMPILE__)
        asm volatile("" : "+v"(kai), "+v"(kbi));
#endif
        float fu[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) fu[c] = c0 + c <= ub ? tt_mean(tu, c0 + c) : 0.0f;
#pragma unroll
        for (int j = 0; j < TZN; ++j) {
            if (j < nzb) {
                TTTrap tv;
                tt_axial(g, iz0 + j, kai, kbi, roff, tv);
                int va, vb;
                tt_pixels(tv.t[0], tv.t[3], va, vb);
                va = va < cv0 ? cv0 : va;
                vb = vb > vmax ? vmax : vb;
                for (int v = va; v <= vb; ++v) {
                    const float fv = tt_mean(tv, v);
                    const A *lrow = s_le + (v - cv0) * stride + (c0 - cu0);
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        if (c0 + c <= ub) {
                            const float wgt = fu[c] * fv;
                            if (wgt > 0.0f) acc[j] = fma_acc(SQ ? wgt * wgt : wgt, lrow[c], acc[j]);
                        }
                    }
                }
            }
        }
    }
}

}  // namespace kct
