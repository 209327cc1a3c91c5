// tt.hip -- the TT footprint projector pair (kct_tt.h) on gfx950, selected per
// geometry with kct_geometry_set_projector.  Both kernels evaluate the weight
// fl(F_u * F_v) of kct_tt.h on the same single-precision inputs, so, as for the
// Siddon pair, the backprojector is the exact transpose of the projector up to
// accumulation rounding; both write every output once (no atomics) and take
// every epilogue of the solvers (kct_epilogue.h).
//
//   forward   ray-driven: a wavefront holds 64 detector rows of one column.
//             Walking the view's dominant axis slab by slab, the wavefront
//             takes the voxel columns inside the wedge between the rays through
//             its column's two edges (identical work in every lane: transaxial
//             footprint F_u); each lane then visits the z-cells whose axial
//             footprint meets its row and accumulates F_u F_v x_j.
//   backward  voxel-driven gather over 16 x 16 x 16 bricks: per view the
//             brick's detector shadow is staged in LDS as L_i e_i; each lane
//             takes the detector columns of its voxel column's transaxial
//             footprint and, per voxel, the rows of its axial footprint.
#include <type_traits>

#include "kct_epilogue.h"
#include "kct_gather.h"
#include "kct_internal.h"
#include "kct_tt.h"
#include "kct_weights.h"

namespace kct {

constexpr int TT_COLS = 4;                           // forward: detector columns per workgroup
constexpr int TT_R = 2;                              // forward: detector rows per lane (share a column's footprints)
constexpr int TT_CH_COLS = 48, TT_CH_ROWS = 40;      // backward: staged shadow chunk
constexpr int TT_NXCD = 8;
constexpr int TT_TZ = TZ;                            // backward: voxels per lane along z

struct TTFwdGrid {
    int ncg, nbands, nviews;
    int64_t nblocks;
};

__host__ __device__ __forceinline__ TTFwdGrid tt_fwd_grid(const GeoDev &g)
{
    TTFwdGrid f;
    f.ncg = (g.nu + TT_COLS - 1) / TT_COLS;
    f.nbands = (g.nv + 64 * TT_R - 1) / (64 * TT_R);
    f.nviews = g.nviews;
    f.nblocks = (int64_t)f.ncg * f.nbands * f.nviews;
    return f;
}

int64_t tt_forward_num_blocks(const GeoDev &g) { return tt_fwd_grid(g).nblocks; }

// Backward grid: bricks of BX x BY x TT_TZ voxels.
int64_t tt_backward_grid_dims(const GeoDev &g, int &nbx, int &nby, int &nbz)
{
    nbx = (g.nx + BX - 1) / BX;
    nby = (g.ny + BY - 1) / BY;
    nbz = (g.nz + TT_TZ - 1) / TT_TZ;
    return (int64_t)nbx * nby * nbz;
}

__device__ __forceinline__ double tt_block_sum(double v)
{
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((__builtin_amdgcn_workitem_id_x() & 63) == 0) red[__builtin_amdgcn_workitem_id_x() >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (__builtin_amdgcn_workitem_id_x() == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
    return r;
}

template <typename TV, typename TP, int EPI>
__global__ __launch_bounds__(256) void k_forward_tt(GeoDev g, const TV *__restrict__ vol,
                                                    const TV *__restrict__ vol_z, TP *__restrict__ out,
                                                    const TP *__restrict__ aux, const Scalars *__restrict__ sc,
                                                    double *__restrict__ partials, const int *__restrict__ skip)
{
    if (skip && *skip) return;
    using A = acc_t<TV>;
    const TTFwdGrid fg = tt_fwd_grid(g);
    const int64_t w = __builtin_amdgcn_workgroup_id_x();
    const int64_t full = fg.nblocks & ~(int64_t)63;
    const int64_t L = w < full ? (w & ~(int64_t)63) + (w % TT_NXCD) * 8 + (w / TT_NXCD) % 8 : w;
    const int cg = (int)(L % fg.ncg);
    const int64_t rest = L / fg.ncg;
    const int k = (int)(rest % fg.nviews);
    const int band = (int)(rest / fg.nviews);
    const int iu = cg * TT_COLS + (int)(__builtin_amdgcn_workitem_id_x() >> 6);
    const bool col_ok = iu < g.nu;
    // lane rows: band * 64 TT_R + lane + 64 r
    int iv[TT_R];
    bool ok[TT_R];
#pragma unroll
    for (int r = 0; r < TT_R; ++r) {
        iv[r] = band * 64 * TT_R + (int)(__builtin_amdgcn_workitem_id_x() & 63) + 64 * r;
        ok[r] = col_ok && iv[r] < g.nv;
    }
    A acc[TT_R] = {};
    if (col_ok) tt_ray_sums<TV, TT_R>(g, g.views[k], iu, iv, ok, vol, vol_z, acc);
    double sq = 0.0;
#pragma unroll
    for (int r = 0; r < TT_R; ++r) {
        if (ok[r]) {
            const ColParam cp = g.cols[(size_t)k * g.nu + iu];
            const RowParam rp = g.rows[iv[r]];
            const float amp = tt_amplitude(ray_length_per_xi(cp.lxy2, rp.qz, cp.gp), cp.inv_a,
                                           zeta_inv_slope(rp.inv_qz, cp.kz));
            const size_t ray = ((size_t)k * g.nv + iv[r]) * g.nu + iu;
            sq += fwd_store<TP, EPI, A>(out, aux, sc, ray, (A)amp * acc[r]);
        }
    }
    if (EPI != FWD_PLAIN) {
        const double bs = tt_block_sum(sq);
        if (__builtin_amdgcn_workitem_id_x() == 0) partials[__builtin_amdgcn_workgroup_id_x()] = bs;
    }
}

template <typename T, int EPI>
__global__ __launch_bounds__(256, sizeof(acc_t<T>) == 4 ? 5 : 2) void k_backward_tt(GeoDev g, const T *__restrict__ proj, T *__restrict__ out,
                                                        T *__restrict__ out_z, const Scalars *__restrict__ sc,
                                                        double *__restrict__ partials, const int *__restrict__ skip,
                                                        int nbx, int nby, int nbz, const float *__restrict__ aux)
{
    if (skip && *skip) return;
    using A = acc_t<T>;
    constexpr bool SQ = EPI == BWD_DIAG || EPI == BWD_DIAG_INV;  // squared weights, e not read
    __shared__ A s_le[TT_CH_ROWS * TT_CH_COLS];

    const int nb = nbx * nby * nbz;
    const int w = __builtin_amdgcn_workgroup_id_x();
    const int b = (nb % TT_NXCD == 0) ? (w % TT_NXCD) * (nb / TT_NXCD) + w / TT_NXCD : w;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int ix = bx * BX + (int)(__builtin_amdgcn_workitem_id_x() % BX);
    const int iy = by * BY + (int)(__builtin_amdgcn_workitem_id_x() / BX);
    const int iz0 = bz * TT_TZ;
    const int nzb = g.nz - iz0 < TT_TZ ? g.nz - iz0 : TT_TZ;
    const bool valid = ix < g.nx && iy < g.ny;

    const int ex = (bx + 1) * BX < g.nx ? (bx + 1) * BX : g.nx;
    const int ey = (by + 1) * BY < g.ny ? (by + 1) * BY : g.ny;
    const float wx0 = g.x0 + (float)(bx * BX) * g.vx, wx1 = g.x0 + (float)ex * g.vx;
    const float wy0 = g.y0 + (float)(by * BY) * g.vy, wy1 = g.y0 + (float)ey * g.vy;
    const float wz0 = g.z0 + (float)iz0 * g.vz, wz1 = g.z0 + (float)(iz0 + nzb) * g.vz;

    A acc[TT_TZ];
#pragma unroll
    for (int j = 0; j < TT_TZ; ++j) acc[j] = 0;

    for (int k = 0; k < g.nviews; ++k) {
        const ViewParam vp = g.views[k];
        // shadow of the brick (the footprint never leaves the projected corners'
        // range): in every wavefront lanes 0..7 project one corner each and the
        // bounds are combined across those lanes, so each wavefront holds them
        // without a barrier (the same numbers in all)
        int u0, u1, v0, v1;
        {
            const int c = __builtin_amdgcn_workitem_id_x() & 7;
            float fu, fv;
            project_point(g, vp, (c & 1) ? wx1 : wx0, (c & 2) ? wy1 : wy0, (c & 4) ? wz1 : wz0, fu, fv);
            float umin = fu, umax = fu, vmin = fv, vmax = fv;
            for (int off = 1; off < 8; off <<= 1) {
                umin = fminf(umin, __shfl_xor(umin, off, 8));
                umax = fmaxf(umax, __shfl_xor(umax, off, 8));
                vmin = fminf(vmin, __shfl_xor(vmin, off, 8));
                vmax = fmaxf(vmax, __shfl_xor(vmax, off, 8));
            }
            // a pixel meets a footprint inside the projected corners' hull when its
            // extent (centre +- 0.5) overlaps the hull; 0.01 pixel more against rounding
            const int a0 = (int)ceilf(umin - 0.51f), a1 = (int)floorf(umax + 0.51f);
            const int b0 = (int)ceilf(vmin - 0.51f), b1 = (int)floorf(vmax + 0.51f);
            u0 = __builtin_amdgcn_readfirstlane(a0 < 0 ? 0 : a0);
            u1 = __builtin_amdgcn_readfirstlane(a1 > g.nu - 1 ? g.nu - 1 : a1);
            v0 = __builtin_amdgcn_readfirstlane(b0 < 0 ? 0 : b0);
            v1 = __builtin_amdgcn_readfirstlane(b1 > g.nv - 1 ? g.nv - 1 : b1);
        }
        const T *pk = SQ ? proj : proj + (size_t)k * g.nv * g.nu;  // not read when SQ
        const ColParam *ck = g.cols + (size_t)k * g.nu;
        TTTrap tu{};
        float dmin = 0.0f, dmax = 0.0f, rdmin = 0.0f, rdmax = 0.0f;
        if (valid) tt_transaxial(g, vp, ix, iy, tu, dmin, dmax, rdmin, rdmax);
        for (int cu0 = u0; cu0 <= u1; cu0 += TT_CH_COLS) {
            const int ncol = u1 - cu0 + 1 < TT_CH_COLS ? u1 - cu0 + 1 : TT_CH_COLS;
            for (int cv0 = v0; cv0 <= v1; cv0 += TT_CH_ROWS) {
                const int nrow = v1 - cv0 + 1 < TT_CH_ROWS ? v1 - cv0 + 1 : TT_CH_ROWS;
                // pixel t = r * ncol + c; t steps by 256: r by dr, c by dc, with carry
                {
                    int r = (int)__builtin_amdgcn_workitem_id_x() / ncol, c = (int)__builtin_amdgcn_workitem_id_x() - r * ncol;
                    const int dr = 256 / ncol, dc = 256 - dr * ncol;
                    for (int t = __builtin_amdgcn_workitem_id_x(); t < ncol * nrow; t += 256) {
                        // the projection value first: its load overlaps the parameter loads
                        // (offsets within one view fit in 32 bits: a projection has < 2^31 rays)
                        const A ev = SQ ? (A)0 : to_acc(pk[(unsigned)((cv0 + r) * g.nu + cu0 + c)]);
                        const ColParam cp = ck[cu0 + c];
                        const RowParam rp = g.rows[cv0 + r];
                        const A amp = (A)tt_amplitude(ray_length_per_xi(cp.lxy2, rp.qz, cp.gp), cp.inv_a,
                                                      zeta_inv_slope(rp.inv_qz, cp.kz));
                        s_le[r * TT_CH_COLS + c] = SQ ? amp * amp : amp * ev;
                        r += dr;
                        c += dc;
                        if (c >= ncol) {
                            c -= ncol;
                            ++r;
                        }
                    }
                }
                __syncthreads();
                if (valid)
                    tt_gather_chunk<A, SQ>(g, iz0, nzb, tu, rdmin, rdmax, s_le, TT_CH_COLS, cu0, ncol, cv0, nrow,
                                           acc);
                __syncthreads();
            }
        }
    }

    double sq = 0.0;
    if (valid) {
#pragma unroll
        for (int j = 0; j < TT_TZ; ++j) {
            if (j >= nzb) continue;
            const int iz = iz0 + j;
            const size_t vox = ((size_t)iz * g.ny + iy) * g.nx + ix;
            sq += bwd_store<T, EPI, A>(out, out_z, sc, aux, vox, ((size_t)iy * g.nx + ix) * g.nz + iz, acc[j]);
        }
    }
    if (bwd_has_partials<EPI>()) {
        const double bs = tt_block_sum(sq);
        if (__builtin_amdgcn_workitem_id_x() == 0) partials[w] = bs;
    }
}

template <typename TV, typename TP, int EPI>
static void launch_ftt(const GeoDev &g, const TV *vol, const TV *vol_z, TP *out, const TP *aux, const Scalars *sc,
                       double *partials, const int *skip, hipStream_t st)
{
    hipLaunchKernelGGL((k_forward_tt<TV, TP, EPI>), dim3((unsigned)tt_fwd_grid(g).nblocks), dim3(256), 0, st, g, vol,
                       vol_z, out, aux, sc, partials, skip);
}

template <typename TV, typename TP>
hipError_t launch_forward_tt(const GeoDev &g, const TV *vol, const TV *vol_z, TP *out, const TP *aux, int epi,
                             const Scalars *sc, double *partials, const int *skip, hipStream_t st)
{
    if constexpr (std::is_same<TV, double>::value) {
        if (epi != FWD_PLAIN) return hipErrorInvalidValue;
        launch_ftt<TV, TP, FWD_PLAIN>(g, vol, vol_z, out, aux, sc, partials, skip, st);
    } else {
        switch (epi) {
        case FWD_PLAIN: launch_ftt<TV, TP, FWD_PLAIN>(g, vol, vol_z, out, aux, sc, partials, skip, st); break;
        case FWD_NORM: launch_ftt<TV, TP, FWD_NORM>(g, vol, vol_z, out, aux, sc, partials, skip, st); break;
        case FWD_BMINUS: launch_ftt<TV, TP, FWD_BMINUS>(g, vol, vol_z, out, aux, sc, partials, skip, st); break;
        case FWD_LSQR: launch_ftt<TV, TP, FWD_LSQR>(g, vol, vol_z, out, aux, sc, partials, skip, st); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <typename T, int EPI>
static void launch_btt(const GeoDev &g, const T *proj, T *out, T *out_z, const Scalars *sc, double *partials,
                       const int *skip, const float *aux, hipStream_t st)
{
    int nbx, nby, nbz;
    const int64_t nb = tt_backward_grid_dims(g, nbx, nby, nbz);
    hipLaunchKernelGGL((k_backward_tt<T, EPI>), dim3((unsigned)nb), dim3(256), 0, st, g, proj, out, out_z, sc,
                       partials, skip, nbx, nby, nbz, aux);
}

template <typename T>
hipError_t launch_backward_tt(const GeoDev &g, const T *proj, T *out, T *out_z, int epi, const Scalars *sc,
                              double *partials, const int *skip, hipStream_t st, const float *aux)
{
    if constexpr (std::is_same<T, double>::value) {
        if (epi != BWD_PLAIN) return hipErrorInvalidValue;
        launch_btt<T, BWD_PLAIN>(g, proj, out, out_z, sc, partials, skip, aux, st);
    } else {
        switch (epi) {
        case BWD_PLAIN: launch_btt<T, BWD_PLAIN>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        case BWD_NORM: launch_btt<T, BWD_NORM>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        case BWD_LSQR0: launch_btt<T, BWD_LSQR0>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        case BWD_LSQR: launch_btt<T, BWD_LSQR>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        case BWD_TIK: launch_btt<T, BWD_TIK>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        case BWD_JACOBI: launch_btt<T, BWD_JACOBI>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        default:
            if constexpr (std::is_same<T, float>::value) {
                if (epi == BWD_DIAG) {
                    launch_btt<T, BWD_DIAG>(g, proj, out, out_z, sc, partials, skip, aux, st);
                    break;
                }
                if (epi == BWD_DIAG_INV) {
                    launch_btt<T, BWD_DIAG_INV>(g, proj, out, out_z, sc, partials, skip, aux, st);
                    break;
                }
            }
            return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

#define KCT_TTF(TV, TP)                                                                                         \
    template hipError_t launch_forward_tt<TV, TP>(const GeoDev &, const TV *, const TV *, TP *, const TP *, int, \
                                                  const Scalars *, double *, const int *, hipStream_t);
KCT_TTF(float, float)
KCT_TTF(bf16, bf16)
KCT_TTF(_Float16, _Float16)
KCT_TTF(float, bf16)
KCT_TTF(float, _Float16)
KCT_TTF(double, double)

#define KCT_TTB(T)                                                                                                \
    template hipError_t launch_backward_tt<T>(const GeoDev &, const T *, T *, T *, int, const Scalars *, double *, \
                                              const int *, hipStream_t, const float *);
KCT_TTB(float)
KCT_TTB(bf16)
KCT_TTB(_Float16)
KCT_TTB(double)

}  // namespace kct
