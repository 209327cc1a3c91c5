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
static_assert(BX == 16 && BY == 16, "the shadow table (ShadowParam) is built for columns of 16 x 16 voxels");

__device__ __forceinline__ double bwd_block_sum(double v)
{
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((__builtin_amdgcn_workitem_id_x() & 63) == 0) red[__builtin_amdgcn_workitem_id_x() >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (__builtin_amdgcn_workitem_id_x() == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
    return r;
}

// The element of type E at byte offset off from base.
template <typename E> __device__ __forceinline__ const E *byte_at(const void *base, unsigned off)
{
    return reinterpret_cast<const E *>(static_cast<const char *>(base) + off);
}

// backward_block runs workgroup w (0 <= w < nbx * nby * nbz) of the
// backprojection into one volume; its partial sum goes to partials[w].
// s_pix / s_col: LDS for ch_rows(TZB) x CHC staged pixels (plus two zero rows and a
// spare record) and CHC columns.
template <typename T, int EPI, int TZB, int CHC>
__device__ __forceinline__ void backward_block(const GeoDev &g, int w, const T *__restrict__ proj,
                                               T *__restrict__ out, T *__restrict__ out_z,
                                               const Scalars *__restrict__ sc, double *__restrict__ partials,
                                               int nbx, int nby, int nbz, const float *__restrict__ aux,
                                               PixStage<acc_t<T>> *s_pix, ColStage *s_col)
{
    using A = acc_t<T>;
    constexpr int CHR = ch_rows(TZB);  // staged rows per chunk
    constexpr bool SQ = EPI == BWD_DIAG || EPI == BWD_DIAG_INV;  // squared weights, e not read

    // XCD-aware brick assignment
    const int nb = nbx * nby * nbz;
    const int b = (nb % NXCD == 0) ? (w % NXCD) * (nb / NXCD) + w / NXCD : w;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int ix = bx * BX + (int)(__builtin_amdgcn_workitem_id_x() % BX);
    const int iy = by * BY + (int)(__builtin_amdgcn_workitem_id_x() / BX);
    const int iz0 = bz * TZB;
    const int nzb = g.nz - iz0 < TZB ? g.nz - iz0 : TZB;
    const bool valid = ix < g.nx && iy < g.ny;

    // the brick's column in the shadow table, and its lowest and highest plane
    // (heights above the source plane, mm)
    const int sbi = __builtin_amdgcn_readfirstlane(by * g.sbx + bx);  // uniform: the table row stays scalar
    const size_t sbxy = (size_t)g.sbx * g.sby;
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
        // 1. shadow of the brick: its column's detector columns from the table
        //    (uniform: scalar loads), its rows from the heights of its lowest and
        //    highest plane seen at the column's extreme inverse depths, widened
        //    by 0.01 row against rounding
        int u0, u1, v0, v1;
        {
            const ShadowParam sh = g.shadows[(size_t)k * sbxy + sbi];
            u0 = sh.u0;
            u1 = sh.u1;
            const float p0 = wz0 * sh.rmin, p1 = wz0 * sh.rmax, p2 = wz1 * sh.rmin, p3 = wz1 * sh.rmax;
            const float zlo = fminf(fminf(p0, p1), fminf(p2, p3)), zhi = fmaxf(fmaxf(p0, p1), fmaxf(p2, p3));
            const int b0 = (int)ceilf(__builtin_fmaf(zlo, g.kv, g.fv0) - 0.01f);
            const int b1 = (int)floorf(__builtin_fmaf(zhi, g.kv, g.fv0) + 0.01f);
            v0 = __builtin_amdgcn_readfirstlane(b0 < 0 ? 0 : b0);
            v1 = __builtin_amdgcn_readfirstlane(b1 > g.nv - 1 ? g.nv - 1 : b1);
        }
        const T *pk = SQ ? proj : proj + (size_t)k * g.nv * g.nu;  // not read when SQ
        const ColParam *ck = g.cols + (size_t)k * g.nu;
        for (int cu0 = u0; cu0 <= u1; cu0 += CHC) {
            const int ncol = u1 - cu0 + 1 < CHC ? u1 - cu0 + 1 : CHC;
            for (int cv0 = v0; cv0 <= v1; cv0 += CHR) {
                const int nrow = v1 - cv0 + 1 < CHR ? v1 - cv0 + 1 : CHR;
                // the thread index read here (an empty asm keeps the compiler from
                // hoisting what is derived from it out of the brick loops of the
                // persistent form, where it spilled)
                unsigned tid = __builtin_amdgcn_workitem_id_x();
                asm volatile("" : "+v"(tid));
                // 2. stage the chunk: per pixel the z-parameters of its ray and L * e,
                //    per column the in-plane parameters
                //    (pixel t = r * ncol + c; t steps by 256: r by dr, c by dc, with carry)
                {
                    // tid / ncol through a reciprocal: (t + 0.5) / ncol lies at least
                    // 0.5 / ncol >= 0.01 from an integer, the product's rounding below 1e-4
                    const float rn = __builtin_amdgcn_rcpf((float)ncol);
                    int r = (int)(((float)tid + 0.5f) * rn), c = (int)tid - r * ncol;
                    const int dr = 256 / ncol, dc = 256 - dr * ncol;
                    for (int t = (int)tid; t < ncol * nrow; t += 256) {
                        // the projection value first: its load overlaps the parameter loads.
                        // All three are addressed as a uniform base plus a 32-bit byte offset
                        // (one view's projection values span < 2^31 bytes: a detector has
                        // < 2^28 pixels)
                        const unsigned pix = (unsigned)(cv0 + r) * (unsigned)g.nu + (unsigned)(cu0 + c);
                        const A ev = SQ ? (A)0 : to_acc(*byte_at<T>(pk, pix * (unsigned)sizeof(T)));
                        const ColParam cp = *byte_at<ColParam>(ck, (unsigned)(cu0 + c) * (unsigned)sizeof(ColParam));
                        const RowParam rp = *byte_at<RowParam>(g.rows, (unsigned)(cv0 + r) * (unsigned)sizeof(RowParam));
                        const bool par = rp.inv_qz == 0.0f;
                        PixStage<A> ps;
                        ps.czr = par ? PAR_INV : zeta_inv_slope(rp.inv_qz, cp.kz);
                        ps.nzc = zeta_offset(zeta_centre(rp.qz, cp.tcv, g.zc) + (par ? pzadd : 0.0f), ps.czr);
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
                if (tid < ncol) s_col[tid] = stage_column(g, vp.dom, ck[cu0 + tid]);
                // two zero rows after the chunk's: the gather reads a voxel's first
                // candidate row without a branch, and these have weight 0 for any voxel
                if (tid < 2 * ncol) {
                    const int zr = tid < ncol ? nrow : nrow + 1;
                    const int zcol = tid < ncol ? (int)tid : (int)tid - ncol;
                    // the zero made here (an empty asm keeps the compiler from
                    // hoisting the record out of the view loop and spilling it)
                    float zero = 0.0f;
                    asm volatile("" : "+v"(zero));
                    PixStage<A> z{};
                    z.nzc = zero;
                    z.czr = zero;
                    z.le = (A)zero;
                    s_pix[zr * CHC + zcol] = z;
                }
                __syncthreads();
                // 3. gather
                // the lane's column indices laundered per chunk: the few values derived
                // from them are recomputed here instead of being kept live (and spilled)
                // through the view loop
                int ixv = ix, iyv = iy;
                asm volatile("" : "+v"(ixv), "+v"(iyv));
                if (valid) gather_chunk<A, SQ, CHC>(g, vp, ixv, iyv, iz0, nzb, s_pix, s_col, cu0, ncol, cv0, nrow, acc);
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
        if (__builtin_amdgcn_workitem_id_x() == 0) partials[w] = bs;
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
    constexpr int CHC = ch_cols(TZB);
    __shared__ PixStage<acc_t<T>> s_pix[(ch_rows(TZB) + 2) * CHC + NH - 1];
    __shared__ ColStage s_col[CHC];
    backward_block<T, EPI, TZB, CHC>(g, __builtin_amdgcn_workgroup_id_x(), proj, out, out_z, sc, partials, nbx, nby, nbz, aux, s_pix,
                                     s_col);
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

// Backprojection variants of the batched form (BwdVariant): brick depth and
// staged chunk width.
__host__ __device__ constexpr int variant_depth(int v) { return v == BWD_VDEEP ? TZ_DEEP : TZ; }
constexpr int VARIANT_LDS_COLS = 48;  // the widest chunk of the variants
// staged records of the largest chunk of the variants
constexpr int VARIANT_LDS_RECORDS =
    ((ch_rows(TZ_DEEP) + 2) * ch_cols(TZ_DEEP) > (ch_rows(TZ) + 2) * ch_cols(TZ) ? (ch_rows(TZ_DEEP) + 2) * ch_cols(TZ_DEEP)
                                                                                  : (ch_rows(TZ) + 2) * ch_cols(TZ)) +
    NH - 1;

int64_t backward_variant_grid(const GeoDev &g, int variant, int &nbx, int &nby, int &nbz)
{
    bwd_grid(g, variant_depth(variant), nbx, nby, nbz);
    return (int64_t)nbx * nby * nbz;
}

// The variant a single solve would use: its block decomposition (and so its
// partial sums) is that of kct_cgls_solve.
int backward_default_variant(const GeoDev &g) { return bwd_depth(g) == TZ_DEEP ? BWD_VDEEP : BWD_VSHALLOW; }

// One tile (brick) of variant v of instance bi's r = A^T e with |r|^2 partials.
__device__ __forceinline__ void batch_backward_tile(const BatchInst *bi, int lw, PixStage<float> *s_pix,
                                                    ColStage *s_col)
{
    if (bi->bwd_v == BWD_VDEEP)
        backward_block<float, BWD_NORM, TZ_DEEP, 32>(bi->g, lw, bi->e, bi->r, nullptr, bi->sc, bi->part, bi->nbx,
                                                    bi->nby, bi->nbz, nullptr, s_pix, s_col);
    else
        backward_block<float, BWD_NORM, TZ, 48>(bi->g, lw, bi->e, bi->r, nullptr, bi->sc, bi->part, bi->nbx, bi->nby,
                                               bi->nbz, nullptr, s_pix, s_col);
}

// Persistent batched r = A^T e: every workgroup takes items from the queue
// until it is empty (see BatchInst); each item is up to BATCH_ITEM_BWD bricks
// of one instance.
__global__ __launch_bounds__(256, 6) void kp_backward(const BatchInst *__restrict__ B,
                                                      const int64_t *__restrict__ off, int count,
                                                      BatchQueue *__restrict__ q)
{
    __shared__ PixStage<float> s_pix[VARIANT_LDS_RECORDS];
    __shared__ ColStage s_col[VARIANT_LDS_COLS];
    const int64_t total = off[count];
    for (;;) {
        const int64_t item = batch_pop(q);
        if (item >= total) break;
        const int i = batch_find(off, count, item);
        const BatchInst *bi = B + i;
        if (bi->sc->done) continue;
        const int64_t t0 = (item - off[i]) * BATCH_ITEM_BWD;
        const int64_t t1 = t0 + BATCH_ITEM_BWD < bi->nbk ? t0 + BATCH_ITEM_BWD : bi->nbk;
        for (int64_t t = t0; t < t1; ++t) {
            batch_backward_tile(bi, (int)t, s_pix, s_col);
            __syncthreads();  // the tile's block sum is read before the next tile writes it
        }
    }
    batch_exit(q);
}

hipError_t batch_backward_occupancy(int &per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kp_backward, 256, 0);
}

hipError_t launch_batch_backward(const BatchInst *B, const int64_t *off, int count, BatchQueue *q, int grid,
                                 hipStream_t st)
{
    hipLaunchKernelGGL(kp_backward, dim3((unsigned)grid), dim3(256), 0, st, B, off, count, q);
    return hipGetLastError();
}

// A single plain backprojection with batched-form variant v (the tuner times these).
template <int TZB, int CHC>
__global__ __launch_bounds__(256, 6) void k_backward_v(GeoDev g, const float *__restrict__ proj,
                                                       float *__restrict__ out, int nbx, int nby, int nbz)
{
    __shared__ PixStage<float> s_pix[(ch_rows(TZB) + 2) * CHC + NH - 1];
    __shared__ ColStage s_col[CHC];
    backward_block<float, BWD_PLAIN, TZB, CHC>(g, __builtin_amdgcn_workgroup_id_x(), proj, out, nullptr, nullptr, nullptr, nbx, nby, nbz,
                                               nullptr, s_pix, s_col);
}

hipError_t launch_backward_variant(const GeoDev &g, int variant, const float *proj, float *out, hipStream_t st)
{
    int nbx, nby, nbz;
    const int64_t nb = backward_variant_grid(g, variant, nbx, nby, nbz);
    if (variant == BWD_VDEEP)
        hipLaunchKernelGGL((k_backward_v<TZ_DEEP, 32>), dim3((unsigned)nb), dim3(256), 0, st, g, proj, out, nbx, nby,
                           nbz);
    else
        hipLaunchKernelGGL((k_backward_v<TZ, 48>), dim3((unsigned)nb), dim3(256), 0, st, g, proj, out, nbx, nby, nbz);
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
