// kct_gather.h -- the pieces of the brick-gather backprojector (A^T, Section 2,
// Eq. 2), written as plain functions so the kernel is a short sequence of
// calls between barriers.
//
// A workgroup owns a brick of BX x BY x TZ voxels; each of its 256 lanes owns
// one (x, y) position and the TZ voxels above it.  For every view the
// workgroup
//   1. bounds the brick's shadow on the detector (the eight projected corners),
//   2. stages, for every pixel of the shadow, the ray's z-parameters and its
//      value multiplied by the ray length factor L in LDS (one 16-byte record
//      per pixel), and the per-column in-plane ray parameters,
//   3. lets each lane gather: the exact interval of detector columns whose
//      rays cross its voxel column, the in-plane xi-interval of each of those
//      columns (shared by the TZ voxels), per voxel the candidate rows from
//      the z-range of those rays, and for every candidate the exact weight of
//      kct_weights.h.
// The shadow is staged in chunks of at most ch_cols(TZB) x ch_rows(TZB) pixels, so any
// geometry works; typical bricks need one chunk.
#pragma once

#pragma clang fp contract(off)

#include "kct_internal.h"
#include "kct_weights.h"

namespace kct {

constexpr int BX = 16, BY = 16, TZ = 16;   // brick; BX * BY = 256 lanes
constexpr int TZ_DEEP = 32;                // deeper bricks for large volumes (more voxels share a lane's setup)
constexpr int CH_ROWS_MAX = 36;            // staged shadow chunk: rows and columns by brick depth
// Columns of the staged chunk: 32 for the deep bricks of large volumes (whose
// shadows are at most about 28 x 28 pixels at typical magnifications; the
// smaller chunk measured faster there), 48 for the shallow bricks, whose
// volumes tend to have coarse voxels and wide shadows.
__host__ __device__ constexpr int ch_cols(int tzb) { return tzb == TZ_DEEP ? 32 : 48; }
__host__ __device__ constexpr int ch_rows(int tzb) { return tzb == TZ_DEEP ? 36 : 32; }
constexpr int NH = 2;                      // detector columns held in registers at once

struct ColStage {  // per staged detector column: in-plane ray parameters
    float eta_c, inv_a, tcv;  // ColParam's; columns parallel to the eta planes staged as below (PAR_INV)
    float gz;      // d T / d xi with T = (segment fraction) / vz
};

// Rays parallel to a family of planes are staged as if they crossed them at a
// slope of PAR_INV, with their coordinate on that axis moved to the middle of
// the cell they lie in: every plane is then crossed at least PAR_INV / 2 from
// the origin, far outside any xi-interval (finite, so the two crossings of a
// cell never give inf - inf), and the general crossing formula gives exactly
// the parallel-ray intervals of kct_weights.h: everything inside the ray's
// cell, nothing elsewhere.  Staged records and columns therefore need no
// parallel case.
constexpr float PAR_INV = 1.0e30f;

// Per staged pixel.  czr is d xi / d zeta of the pixel's ray and nzc its
// zeta_offset (from zeta at xi = 0: zeta_centre and zeta_inv_slope of its row
// and column); rows whose rays are parallel to the z-planes (qz == 0) staged
// as above.
template <typename A> struct PixStage {
    float nzc, czr;
    A le;          // L * e, in the accumulator precision
    float pad;
};
template <> struct PixStage<double> {  // the same 16 bytes with a double L * e
    float nzc, czr;
    double le;
};

// 1 / x to within a few ulp (bounds only).
__host__ __device__ __forceinline__ float rcp_approx(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// Detector coordinates (column, row; fractional pixel indices) of the ray
// through world point (px, py, pz) in view vp.  Used for bounds only.
__host__ __device__ __forceinline__ void project_point(const GeoDev &g, const ViewParam &vp, float px, float py,
                                                       float pz, float &fu, float &fv)
{
    const float dx = px - vp.sx, dy = py - vp.sy;
    const float num = -vp.s * dx + vp.c * dy;
    const float den = -vp.c * dx - vp.s * dy;  // depth along the central ray (> 0)
    const float inv = rcp_approx(den);
    fu = __builtin_fmaf(num * inv, g.ku, g.fu0);
    fv = __builtin_fmaf(pz * inv, g.kv, g.fv0);
}

// Median of x, a and b: x clamped to the interval between a and b.
__host__ __device__ __forceinline__ float med3f(float x, float a, float b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_fmed3f(x, a, b);
#else
    return fmaxf(fminf(x, a), fminf(fmaxf(x, a), b));
#endif
}

// Candidate detector columns [ua, ub] of the voxel column whose in-plane centre
// is (xc, yc): the projective image of its square, bounded around the image of
// the centre (a bound with margin; the weight function decides).
__host__ __device__ __forceinline__ void voxel_columns(const GeoDev &g, const ViewParam &vp, float xc, float yc,
                                                       int &ua, int &ub)
{
    // bounds only: fused multiply-adds round differently from the separate
    // operations by ~1e-7 relative, far inside the 0.01-column margin
    const float dx = xc - vp.sx, dy = yc - vp.sy;
    const float num = __builtin_fmaf(vp.c, dy, -vp.s * dx);
    const float den = __builtin_fmaf(-vp.c, dx, -vp.s * dy);
    const float inv = rcp_approx(den);
    const float inv2 = rcp_approx(den - vp.dd);  // dd: half extent along depth, dn: along e_u
    const float fc = __builtin_fmaf(num * inv, g.ku, g.fu0);
    const float hc = __builtin_fmaf(__builtin_fmaf(vp.dd * fabsf(num), inv, vp.dn) * inv2, g.ku, 0.01f);
    ua = (int)ceilf(fc - hc);
    ub = (int)floorf(fc + hc);
}

// xi-interval [lo, hi] in which the rays of a staged detector column cross the
// voxel column whose xi-cell starts at lo_xi and whose eta-cell is ieta (empty
// when hi <= lo): cell_range of kct_weights.h without its parallel case, which
// the staging removed (PAR_INV).
__host__ __device__ __forceinline__ void column_interval(const ColStage &cs, float lo_xi, int ieta, float heta,
                                                         float &lo, float &hi)
{
    const float mb = (float)ieta - heta;
    const float b0 = cross_at(mb, cs.eta_c, cs.inv_a), b1 = cross_at(mb + 1.0f, cs.eta_c, cs.inv_a);
    lo = fmaxf(lo_xi, fminf(b0, b1));
    hi = fminf(lo_xi + 1.0f, fmaxf(b0, b1));
}

// The staged form of a detector column (view with in-plane domain dom).
__host__ __device__ __forceinline__ ColStage stage_column(const GeoDev &g, int dom, const ColParam &cp)
{
    ColStage cs;
    const bool par = cp.inv_a == 0.0f;
    const float heta = dom == 0 ? g.hy : g.hx;
    cs.eta_c = par ? ((float)parallel_cell(cp.eta_c, heta) - heta) + 0.5f : cp.eta_c;
    cs.inv_a = par ? PAR_INV : cp.inv_a;
    cs.tcv = cp.tcv;
    cs.gz = cp.gp * g.inv_vz;
    return cs;
}

// One staged record, read as a whole (one 128-bit LDS read).
template <typename A> __host__ __device__ __forceinline__ PixStage<A> load_pix(const PixStage<A> *p) { return *p; }
template <> __host__ __device__ __forceinline__ PixStage<float> load_pix<float>(const PixStage<float> *p)
{
    const float4 v = *reinterpret_cast<const float4 *>(p);
    PixStage<float> r;
    r.nzc = v.x;
    r.czr = v.y;
    r.le = v.z;
    r.pad = v.w;
    return r;
}

// The candidates of one detector row for one voxel: the rays of the row in the
// nh (<= NH) staged hit columns starting at prow, whose in-plane xi-intervals
// are [lo[h], hi[h]] with lo[h] <= hi[h], against the voxel's z-planes mb and
// mb1.  Returns a + sum of w * (L e) (w^2 * le when SQ).  All NH records are
// read before the first is used; the staging buffer holds a spare record past
// its last, so prow + NH - 1 is always inside it.
template <typename A, bool SQ>
__host__ __device__ __forceinline__ A add_row(const PixStage<A> *prow, int nh, const float (&lo)[NH],
                                              const float (&hi)[NH], float mb, float mb1, A a)
{
    PixStage<A> p[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) p[h] = load_pix(prow + h);
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        if (h == 0 || h < nh) {
            const float b0 = zeta_cross(mb, p[h].nzc, p[h].czr), b1 = zeta_cross(mb1, p[h].nzc, p[h].czr);
            // With lo <= hi, med3(hi, b0, b1) - med3(lo, b0, b1) is the overlap
            // min(hi, max(b0, b1)) - max(lo, min(b0, b1)) wherever that is positive
            // (both medians then pick those operands) and exactly 0 elsewhere (both
            // medians clamp to the same end of [min, max], or hi = lo): a candidate
            // that misses adds 0 * le = 0 (le is finite) and leaves the sum as it is.
            const float w = med3f(hi[h], b0, b1) - med3f(lo[h], b0, b1);
            a = fma_acc(SQ ? w * w : w, p[h].le, a);
        }
    }
    return a;
}

// pg + r * CHC for a pointer pg into the LDS staging buffer: on the GPU one
// shift-and-add of the 32-bit LDS address when a row of records spans a power
// of two bytes.
template <typename A, int CHC>
__host__ __device__ __forceinline__ const PixStage<A> *row_record(const PixStage<A> *pg, int r)
{
#if defined(__HIP_DEVICE_COMPILE__)
    constexpr unsigned row_bytes = CHC * sizeof(PixStage<A>);
    if constexpr ((row_bytes & (row_bytes - 1)) == 0) {
        typedef const __attribute__((address_space(3))) PixStage<A> *lds_rec;
        const unsigned base = (unsigned)(size_t)(lds_rec)pg;
        unsigned addr;
        asm("v_lshl_add_u32 %0, %1, %3, %2" : "=v"(addr) : "v"(r), "v"(base), "i"(__builtin_ctz(row_bytes)));
        return (const PixStage<A> *)(lds_rec)(size_t)addr;
    }
#endif
    return pg + r * CHC;
}

// The voxels of one lane for one group of hit columns: voxel j (j < nzb) has
// the planes mbz0 + j and mbz0 + j + 1 and the candidate rows va1 + 1 .. vb with
// va1 = floor(l0 + j sl) and vb = floor(h0 + (j + 1) sh).  The first candidate
// row is evaluated for every voxel, without a branch: va1 is clamped to
// [vlow, vmax + 1] (vlow = first staged row - 1, vmax = last), so row va1 + 1 is
// a staged row or one of the two zero rows staged after them, and a row that
// is not a candidate has weight exactly 0 (the weights are exact).  Further
// rows, up to vb clamped to vmax, follow in a loop.  pg + va1 * CHC is the
// record of row va1 + 1 in the group's first column.
template <typename A, bool SQ, int CHC, int TZN>
__host__ __device__ __forceinline__ void voxel_rows(const PixStage<A> *pg, int nh, const float (&lo)[NH],
                                                    const float (&hi)[NH], float mbz0, int nzb, float l0, float sl,
                                                    float h0, float sh, int vlow, int vmax, A (&acc)[TZN])
{
    // The per-voxel plane values do not depend on the column group; computed
    // here they stay short-lived (hoisted out of the group loop, all TZ of them
    // would stay live through it).  The empty asm keeps the compiler from
    // hoisting them.
    float mbb = mbz0;
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+v"(mbb));
#endif
    float mb = mbb;  // lower plane of voxel j (exact: an integer or half-integer)
#pragma unroll
    for (int j = 0; j < TZN; ++j) {
        const float mb1 = mb + 1.0f;
        if (j < nzb) {
            // candidate rows va1 + 1 .. vb: floor(lo) + 1 is ceil(lo) except at an
            // integer lo, whose row lies 0.01 below the true bound and is rightly left out
            const float vlo = __builtin_fmaf((float)j, sl, l0), vhi = __builtin_fmaf((float)(j + 1), sh, h0);
            int va1 = (int)floorf(vlo), vb = (int)floorf(vhi);
            va1 = va1 < vlow ? vlow : (va1 > vmax + 1 ? vmax + 1 : va1);
            vb = vb > vmax ? vmax : vb;
            const PixStage<A> *prow = row_record<A, CHC>(pg, va1);
            A a = add_row<A, SQ>(prow, nh, lo, hi, mb, mb1, acc[j]);
            for (int v = va1 + 2; v <= vb; ++v) {
                prow += CHC;
                a = add_row<A, SQ>(prow, nh, lo, hi, mb, mb1, a);
            }
            acc[j] = a;
        }
        mb = mb1;
    }
}

// One lane's share of one staged chunk of one view: add w_ij * (L_i e_i) to the
// accumulators of its voxels (ix, iy, iz0 + j), j < nzb, for every staged ray
// i = (column cu0 + c, row cv0 + r); s_pix[r * CHC + c] describes ray i, and
// rows nrow and nrow + 1 of s_pix hold zero records (weight 0 for any voxel).
// SQ: accumulate w_ij^2 * le instead of w_ij * le (with le = L^2 this sums the
// squared weights, the diagonal of A^T A).
template <typename A, bool SQ, int CHC, int TZN>
__host__ __device__ __forceinline__ void gather_chunk(const GeoDev &g, const ViewParam &vp, int ix, int iy, int iz0,
                                                      int nzb, const PixStage<A> *s_pix, const ColStage *s_col,
                                                      int cu0, int ncol, int cv0, int nrow, A (&acc)[TZN])
{
    int ixi, ieta;
    float hxi, heta;
    if (vp.dom == 0) { ixi = ix; ieta = iy; hxi = g.hx; heta = g.hy; }
    else { ixi = iy; ieta = ix; hxi = g.hy; heta = g.hx; }
    const float lo_xi = (float)ixi - hxi;
    int ua, ub;
    voxel_columns(g, vp, g.x0 + ((float)ix + 0.5f) * g.vx, g.y0 + ((float)iy + 0.5f) * g.vy, ua, ub);
    ua = ua < cu0 ? cu0 : ua;
    ub = ub > cu0 + ncol - 1 ? cu0 + ncol - 1 : ub;
    // The columns whose rays cross the voxel column form an interval (the
    // rays of consecutive columns fan out monotonically from the source):
    // narrow the bound to its first and last hit.
    int ha = ub + 1, hb = ub;  // empty unless a column is hit
    for (int iu = ua; iu <= ub; ++iu) {
        float lo, hi;
        column_interval(s_col[iu - cu0], lo_xi, ieta, heta, lo, hi);
        if (hi > lo) {
            ha = iu < ha ? iu : ha;
            hb = iu;
        }
    }
    const float mbz0 = (float)iz0 - g.hz;  // lower plane of the first voxel (index frame)
    const float zz0 = mbz0 + g.zc;         // the same plane as a height above the source plane
    const float inv_nzb = rcp_approx((float)nzb);
    const float vofs_lo = g.fv0 - 0.01f, vofs_hi = g.fv0 + 0.01f;
    const int vmax = cv0 + nrow - 1;
    for (int c0 = ha; c0 <= hb; c0 += NH) {
        // xi-intervals of up to NH hit columns, and the range of T = tcv + xi gz
        // over them (a ray of height qz is at height qz T above the source plane)
        const int nh = hb - c0 + 1 < NH ? hb - c0 + 1 : NH;
        float lo[NH], hi[NH];
        float tmin = INFINITY, tmax = 0.0f;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int c = h < nh ? c0 + h : c0;
            const ColStage cs = s_col[c - cu0];
            column_interval(cs, lo_xi, ieta, heta, lo[h], hi[h]);
            if (h < nh && hi[h] > lo[h]) {
                const float T1 = cs.tcv + lo[h] * cs.gz, T2 = cs.tcv + hi[h] * cs.gz;
                tmin = fminf(tmin, fminf(T1, T2));
                tmax = fmaxf(tmax, fmaxf(T1, T2));
            }
            hi[h] = fmaxf(hi[h], lo[h]);  // an empty interval becomes [lo, lo]: its weights are 0 (add_row)
        }
        if (!(tmax > 0.0f)) continue;  // no column of this group is hit
        // Rows: inside these columns a ray of row height qz meets the z-cell with
        // planes at heights [zz, zz + 1] only if qz lies in [zz, zz + 1] / [Tmin, Tmax].
        // In row units a plane at height z bounds the rows from below by
        // f_lo(z) = min(z ra, z rb) and from above by f_hi(z) = max(z ra, z rb).
        // f_lo is concave and f_hi convex in z, so over the brick's planes the
        // chords between its lowest and highest plane bound them from the safe
        // side (exactly equal to them unless the brick straddles the source
        // plane z = 0): plane p gives lo_p = l0 + p sl and hi_p = h0 + p sh, one
        // fused multiply-add each.  Their rounding (~1e-5 row) is far inside the
        // 0.01-row margins.
        const float ra = __builtin_amdgcn_rcpf(tmax) * g.inv_dv, rb = __builtin_amdgcn_rcpf(tmin) * g.inv_dv;
        const float za = zz0, zb = zz0 + (float)nzb;  // lowest and highest plane of the brick
        const float a1 = za * ra, a2 = za * rb, b1 = zb * ra, b2 = zb * rb;
        const float sl = (fminf(b1, b2) - fminf(a1, a2)) * inv_nzb;
        const float sh = (fmaxf(b1, b2) - fmaxf(a1, a2)) * inv_nzb;
        const float l0 = fminf(a1, a2) + vofs_lo, h0 = fmaxf(a1, a2) + vofs_hi;
        const PixStage<A> *pg = s_pix + ((c0 - cu0) + (1 - cv0) * CHC);  // row va1 + 1 at pg + va1 * CHC
        voxel_rows<A, SQ, CHC, TZN>(pg, nh, lo, hi, mbz0, nzb, l0, sl, h0, sh, cv0 - 1, vmax, acc);
    }
}

}  // namespace kct
