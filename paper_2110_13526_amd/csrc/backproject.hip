// backproject.hip -- r = A^T e (Section 2, Eq. 2) as a voxel-driven gather on
// gfx950: one workgroup per brick of BX x BY x TZ voxels, all views in one
// launch, the brick's detector shadow staged in LDS per view (see
// kct_gather.h).  Every voxel is written once by the lane that owns it; no
// atomics; bitwise reproducible.
//
// Workgroups are assigned to bricks so that each of the eight XCDs (which fill
// round-robin in dispatch order) owns a contiguous range of bricks: bricks that
// neighbour each other share most of their detector shadow, so the staged
// projection values are reused from the XCD's own L2.
#include <type_traits>

#include "kct_batch.h"
#include "kct_epilogue.h"
#include "kct_gather.h"
#include "kct_internal.h"
#include "kct_weights.h"

namespace kct {

constexpr int NXCD = 8;

__device__ __forceinline__ double bwd_block_sum(double v)
{
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
    return r;
}

// backward_block runs workgroup w (0 <= w < nbx * nby * nbz) of the
// backprojection into one volume; its partial sum goes to partials[w].
template <typename T, int EPI, int TZB>
__device__ __forceinline__ void backward_block(const GeoDev &g, int w, const T *__restrict__ proj,
                                               T *__restrict__ out, T *__restrict__ out_z,
                                               const Scalars *__restrict__ sc, double *__restrict__ partials,
                                               int nbx, int nby, int nbz, const float *__restrict__ aux)
{
    using A = acc_t<T>;
    constexpr bool SQ = EPI == BWD_DIAG || EPI == BWD_DIAG_INV;  // squared weights, e not read
    constexpr int CHC = ch_cols(TZB);
    __shared__ PixStage<A> s_pix[CH_ROWS * CHC];
    __shared__ ColStage s_col[CHC];

    // XCD-aware brick assignment
    const int nb = nbx * nby * nbz;
    const int b = (nb % NXCD == 0) ? (w % NXCD) * (nb / NXCD) + w / NXCD : w;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int ix = bx * BX + (int)(threadIdx.x % BX);
    const int iy = by * BY + (int)(threadIdx.x / BX);
    const int iz0 = bz * TZB;
    const int nzb = g.nz - iz0 < TZB ? g.nz - iz0 : TZB;
    const bool valid = ix < g.nx && iy < g.ny;

    // brick corners in world coordinates (clamped to the volume)
    const int ex = (bx + 1) * BX < g.nx ? (bx + 1) * BX : g.nx;
    const int ey = (by + 1) * BY < g.ny ? (by + 1) * BY : g.ny;
    const float wx0 = g.x0 + (float)(bx * BX) * g.vx, wx1 = g.x0 + (float)ex * g.vx;
    const float wy0 = g.y0 + (float)(by * BY) * g.vy, wy1 = g.y0 + (float)ey * g.vy;
    const float wz0 = g.z0 + (float)iz0 * g.vz, wz1 = g.z0 + (float)(iz0 + nzb) * g.vz;

    // rays parallel to the z-planes lie in z-cell pcell; their staged zc is
    // that cell's middle (see PixStage)
    const int pcell = parallel_cell(-g.zc, g.hz);
    const float pzadd = ((float)pcell - g.hz + 0.5f) + g.zc;

    A acc[TZB];
#pragma unroll
    for (int j = 0; j < TZB; ++j) acc[j] = 0;

    for (int k = 0; k < g.nviews; ++k) {
        const ViewParam vp = g.views[k];
        // 1. shadow of the brick: in every wavefront lanes 0..7 project one
        //    corner each and the bounds are combined across those lanes, so
        //    each wavefront holds them without a barrier (the same numbers in all)
        int u0, u1, v0, v1;
        {
            const int c = threadIdx.x & 7;
            float fu, fv;
            project_point(g, vp, (c & 1) ? wx1 : wx0, (c & 2) ? wy1 : wy0, (c & 4) ? wz1 : wz0, fu, fv);
            float umin = fu, umax = fu, vmin = fv, vmax = fv;
            for (int off = 1; off < 8; off <<= 1) {
                umin = fminf(umin, __shfl_xor(umin, off, 8));
                umax = fmaxf(umax, __shfl_xor(umax, off, 8));
                vmin = fminf(vmin, __shfl_xor(vmin, off, 8));
                vmax = fmaxf(vmax, __shfl_xor(vmax, off, 8));
            }
            // a ray through the brick meets the detector inside the convex hull of the
            // projected corners: the pixel centres in [min, max], widened by 0.01 pixel
            // against rounding (relative ~1e-7 of the coordinates)
            const int a0 = (int)ceilf(umin - 0.01f), a1 = (int)floorf(umax + 0.01f);
            const int b0 = (int)ceilf(vmin - 0.01f), b1 = (int)floorf(vmax + 0.01f);
            u0 = __builtin_amdgcn_readfirstlane(a0 < 0 ? 0 : a0);
            u1 = __builtin_amdgcn_readfirstlane(a1 > g.nu - 1 ? g.nu - 1 : a1);
            v0 = __builtin_amdgcn_readfirstlane(b0 < 0 ? 0 : b0);
            v1 = __builtin_amdgcn_readfirstlane(b1 > g.nv - 1 ? g.nv - 1 : b1);
        }
        const T *pk = SQ ? proj : proj + (size_t)k * g.nv * g.nu;  // not read when SQ
        const ColParam *ck = g.cols + (size_t)k * g.nu;
        for (int cu0 = u0; cu0 <= u1; cu0 += CHC) {
            const int ncol = u1 - cu0 + 1 < CHC ? u1 - cu0 + 1 : CHC;
            for (int cv0 = v0; cv0 <= v1; cv0 += CH_ROWS) {
                const int nrow = v1 - cv0 + 1 < CH_ROWS ? v1 - cv0 + 1 : CH_ROWS;
                // 2. stage the chunk: per pixel the z-parameters of its ray and L * e,
                //    per column the in-plane parameters
                //    (pixel t = r * ncol + c; t steps by 256: r by dr, c by dc, with carry)
                {
                    int r = (int)threadIdx.x / ncol, c = (int)threadIdx.x - r * ncol;
                    const int dr = 256 / ncol, dc = 256 - dr * ncol;
                    for (int t = threadIdx.x; t < ncol * nrow; t += 256) {
                        // the projection value first: its load overlaps the parameter loads
                        // (offsets within one view fit in 32 bits: a projection has < 2^31 rays)
                        const A ev = SQ ? (A)0 : to_acc(pk[(unsigned)((cv0 + r) * g.nu + cu0 + c)]);
                        const ColParam cp = ck[cu0 + c];
                        const RowParam rp = g.rows[cv0 + r];
                        const bool par = rp.inv_qz == 0.0f;
                        PixStage<A> ps;
                        ps.zc = zeta_centre(rp.qz, cp.tcv, g.zc) + (par ? pzadd : 0.0f);
                        ps.czr = zeta_inv_slope(par ? INFINITY : rp.inv_qz, cp.kz);
                        const A L = (A)ray_length_per_xi(cp.lxy2, rp.qz, cp.gp);
                        ps.le = SQ ? L * L : L * ev;
                        s_pix[r * CHC + c] = ps;
                        r += dr;
                        c += dc;
                        if (c >= ncol) {
                            c -= ncol;
                            ++r;
                        }
                    }
                }
                if (threadIdx.x < ncol) {
                    const ColParam cp = ck[cu0 + threadIdx.x];
                    ColStage cs;
                    cs.eta_c = cp.eta_c;
                    cs.inv_a = cp.inv_a;
                    cs.tcv = cp.tcv;
                    cs.gz = cp.gp * g.inv_vz;
                    s_col[threadIdx.x] = cs;
                }
                __syncthreads();
                // 3. gather
                if (valid) gather_chunk<A, SQ, CHC>(g, vp, ix, iy, iz0, nzb, s_pix, s_col, cu0, ncol, cv0, nrow, acc);
                __syncthreads();
            }
        }
    }

    double sq = 0.0;
    if (valid) {
#pragma unroll
        for (int j = 0; j < TZB; ++j) {
            if (j >= nzb) continue;
            const int iz = iz0 + j;
            const size_t vox = ((size_t)iz * g.ny + iy) * g.nx + ix;
            sq += bwd_store<T, EPI, A>(out, out_z, sc, aux, vox, ((size_t)iy * g.nx + ix) * g.nz + iz, acc[j]);
        }
    }
    if (bwd_has_partials<EPI>()) {
        const double bs = bwd_block_sum(sq);
        if (threadIdx.x == 0) partials[w] = bs;
    }
}

template <typename T, int EPI, int TZB>
__global__ __launch_bounds__(256, sizeof(acc_t<T>) != 4 ? 2 : 6) void k_backward(GeoDev g, const T *__restrict__ proj,
                                                                                T *__restrict__ out,
                                                                                T *__restrict__ out_z,
                                                                                const Scalars *__restrict__ sc,
                                                                                double *__restrict__ partials,
                                                                                const int *__restrict__ skip, int nbx,
                                                                                int nby, int nbz,
                                                                                const float *__restrict__ aux)
{
    if (skip && *skip) return;
    backward_block<T, EPI, TZB>(g, blockIdx.x, proj, out, out_z, sc, partials, nbx, nby, nbz, aux);
}

// Brick depth of a single backprojection: TZ_DEEP voxels per lane when the
// volume still gives at least 5120 such bricks (over three rounds of six workgroups
// per compute unit), else TZ (small volumes need the workgroups more than the
// shared setup).
static int bwd_depth(const GeoDev &g)
{
    const int64_t deep = (int64_t)((g.nx + BX - 1) / BX) * ((g.ny + BY - 1) / BY) * ((g.nz + TZ_DEEP - 1) / TZ_DEEP);
    return deep >= 5120 ? TZ_DEEP : TZ;
}

static void bwd_grid(const GeoDev &g, int tz, int &nbx, int &nby, int &nbz)
{
    nbx = (g.nx + BX - 1) / BX;
    nby = (g.ny + BY - 1) / BY;
    nbz = (g.nz + tz - 1) / tz;
}

// Grid of the batched backprojection (bricks of depth TZ for every instance).
int64_t backward_grid_dims(const GeoDev &g, int &nbx, int &nby, int &nbz)
{
    bwd_grid(g, TZ, nbx, nby, nbz);
    return (int64_t)nbx * nby * nbz;
}

// Batched r = A^T e with |r|^2 partials for every instance.
__global__ __launch_bounds__(256, 6) void kb_backward(const BatchInst *__restrict__ B,
                                                      const int64_t *__restrict__ off, int count)
{
    const int64_t w = blockIdx.x;
    const int i = batch_find(off, count, w);
    const BatchInst *bi = B + i;
    if (bi->sc->done) return;
    const int64_t lw = w - off[i];
    if (lw >= (int64_t)bi->nbx * bi->nby * bi->nbz) return;  // padding of the instance's grid
    backward_block<float, BWD_NORM, TZ>(bi->g, (int)lw, bi->e, bi->r, nullptr, bi->sc, bi->part, bi->nbx, bi->nby,
                                        bi->nbz, nullptr);
}

hipError_t launch_batch_backward(const BatchInst *B, const int64_t *off, int count, int64_t blocks, hipStream_t st)
{
    hipLaunchKernelGGL(kb_backward, dim3((unsigned)blocks), dim3(256), 0, st, B, off, count);
    return hipGetLastError();
}

// Workgroups (and partial sums) of a single backprojection with g: at most the
// count of TZ-deep bricks.
int64_t backward_num_blocks(const GeoDev &g)
{
    int nbx, nby, nbz;
    if (g.projector == KCT_PROJECTOR_TT) return tt_backward_grid_dims(g, nbx, nby, nbz);
    bwd_grid(g, bwd_depth(g), nbx, nby, nbz);
    return (int64_t)nbx * nby * nbz;
}

template <typename T, int EPI>
static void launch_bwd(const GeoDev &g, const T *proj, T *out, T *out_z, const Scalars *sc, double *partials,
                       const int *skip, const float *aux, hipStream_t st)
{
    const int tz = bwd_depth(g);
    int nbx, nby, nbz;
    bwd_grid(g, tz, nbx, nby, nbz);
    const dim3 grid((unsigned)(nbx * nby * nbz));
    if (tz == TZ_DEEP)
        hipLaunchKernelGGL((k_backward<T, EPI, TZ_DEEP>), grid, dim3(256), 0, st, g, proj, out, out_z, sc, partials,
                           skip, nbx, nby, nbz, aux);
    else
        hipLaunchKernelGGL((k_backward<T, EPI, TZ>), grid, dim3(256), 0, st, g, proj, out, out_z, sc, partials, skip,
                           nbx, nby, nbz, aux);
}

template <typename T>
hipError_t launch_backward(const GeoDev &g, const T *proj, T *out, T *out_z, int epi, const Scalars *sc,
                           double *partials, const int *skip, hipStream_t st, const float *aux)
{
    if (g.projector == KCT_PROJECTOR_TT) return launch_backward_tt<T>(g, proj, out, out_z, epi, sc, partials, skip, st, aux);
    if constexpr (std::is_same<T, double>::value) {  // double storage: plain backprojection only
        if (epi != BWD_PLAIN) return hipErrorInvalidValue;
        launch_bwd<T, BWD_PLAIN>(g, proj, out, out_z, sc, partials, skip, aux, st);
    } else {
        switch (epi) {
        case BWD_PLAIN: launch_bwd<T, BWD_PLAIN>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        case BWD_NORM: launch_bwd<T, BWD_NORM>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        case BWD_LSQR0: launch_bwd<T, BWD_LSQR0>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        case BWD_LSQR: launch_bwd<T, BWD_LSQR>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        case BWD_TIK: launch_bwd<T, BWD_TIK>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        case BWD_JACOBI: launch_bwd<T, BWD_JACOBI>(g, proj, out, out_z, sc, partials, skip, aux, st); break;
        default:
            if constexpr (std::is_same<T, float>::value) {  // the diagonal of A^T A is single precision
                if (epi == BWD_DIAG) {
                    launch_bwd<T, BWD_DIAG>(g, proj, out, out_z, sc, partials, skip, aux, st);
                    break;
                }
                if (epi == BWD_DIAG_INV) {
                    launch_bwd<T, BWD_DIAG_INV>(g, proj, out, out_z, sc, partials, skip, aux, st);
                    break;
                }
            }
            return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

#define KCT_BINST(T)                                                                                             \
    template hipError_t launch_backward<T>(const GeoDev &, const T *, T *, T *, int, const Scalars *, double *, \
                                           const int *, hipStream_t, const float *);
KCT_BINST(float)
KCT_BINST(bf16)
KCT_BINST(_Float16)
KCT_BINST(double)

}  // namespace kct
