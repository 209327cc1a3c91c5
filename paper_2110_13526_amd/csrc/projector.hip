// projector.hip -- the forward cone-beam projector for gfx950.
//
//   forward  p = A x    (Section 2, Eq. 1): ray-driven.  One lane per ray; the
//            lanes of a wavefront hold neighbouring detector rows of one
//            column (R rows per lane).  Their rays share the in-plane part of the walk (identical
//            work in every lane, no divergence), differ only in z, and read a
//            copy of the volume stored z-fastest, so one gather instruction of
//            the wavefront touches a few neighbouring cache lines.  Each lane
//            accumulates w_ij * x_j in single precision (kct_ray.h).
// The backprojector (the voxel-driven gather that evaluates the same weights)
// is in backproject.hip.
//
// The kernel can fuse a double-precision partial sum of the squares of its
// outputs (|p|^2 of Algorithm 1) and the LSQR bidiagonalisation update.
#include <type_traits>

#include "kct_batch.h"
#include "kct_epilogue.h"
#include "kct_internal.h"
#include "kct_ray.h"
#include "kct_weights.h"

namespace kct {

constexpr int FWD_COLS = 4;    // detector columns per workgroup (one per wavefront)
constexpr int FWD_R = 4;       // detector rows per lane (the batched form's tuner chooses 1 or 2)
constexpr int NXCD = 8;

// Sum of v over the 256 threads of the workgroup, in a fixed order.  Result is
// valid in thread 0.
__device__ __forceinline__ double block_sum_256(double v)
{
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = __builtin_amdgcn_workitem_id_x() >> 6;
    if ((__builtin_amdgcn_workitem_id_x() & 63) == 0) red[w] = v;
    __syncthreads();
    double r = 0.0;
    if (__builtin_amdgcn_workitem_id_x() == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
    return r;
}

struct FwdGrid {
    int ncg, nbands, nviews;
    int64_t nblocks;
};

__host__ __device__ __forceinline__ FwdGrid fwd_grid(const GeoDev &g, int rows_per_lane)
{
    FwdGrid f;
    const int rows = 64 * rows_per_lane;  // detector rows per wavefront
    f.ncg = (g.nu + FWD_COLS - 1) / FWD_COLS;
    f.nbands = (g.nv + rows - 1) / rows;
    f.nviews = g.nviews;
    f.nblocks = (int64_t)f.ncg * f.nbands * f.nviews;
    return f;
}

// Workgroup order: column group fastest, then view, then row band, so the
// workgroups in flight cover one band of detector rows (one z-slab of the
// volume) over many views.  Dispatch fills the eight XCDs round-robin; within
// every 64 consecutive workgroups the order is permuted so that each XCD gets 8
// neighbouring column groups, which share voxels in that XCD's L2.
//
// forward_block runs workgroup w (0 <= w < fwd_grid(g, R).nblocks) of the
// projection of one volume; R rows per lane.  Its partial sum goes to
// partials[w].
template <typename TV, typename TP, int EPI, int R>
__device__ __forceinline__ void forward_block(const GeoDev &g, int64_t w, const TV *__restrict__ vol,
                                              const TV *__restrict__ vol_z, TP *__restrict__ out,
                                              const TP *__restrict__ aux, const Scalars *__restrict__ sc,
                                              double *__restrict__ partials)
{
    constexpr int FWD_ROWS = 64 * R;
    const FwdGrid fg = fwd_grid(g, R);
    const int64_t full = fg.nblocks & ~(int64_t)63;
    const int64_t L = w < full ? (w & ~(int64_t)63) + (w % NXCD) * 8 + (w / NXCD) % 8 : w;
    const int cg = (int)(L % fg.ncg);
    const int64_t rest = L / fg.ncg;
    const int k = (int)(rest % fg.nviews);
    const int band = (int)(rest / fg.nviews);
    // the wavefront's column, made provably uniform so that the in-plane walk
    // (a function of the column) runs on scalar registers and branches
    const int iu = cg * FWD_COLS + __builtin_amdgcn_readfirstlane((int)(__builtin_amdgcn_workitem_id_x() >> 6));
    const int lane = (int)(__builtin_amdgcn_workitem_id_x() & 63);
    ViewParam vp = g.views[k];
    vp.dom = __builtin_amdgcn_readfirstlane(vp.dom);  // uniform: the volume's base and strides follow it

    int nxi, neta, sxi, seta, sz;
    float hxi, heta;
    const TV *base;
    if (vp.dom == 0) {  // xi = x, eta = y
        nxi = g.nx; neta = g.ny; hxi = g.hx; heta = g.hy;
        if (vol_z) { base = vol_z; sz = 1; sxi = g.nz; seta = g.nx * g.nz; }
        else { base = vol; sz = g.nx * g.ny; sxi = 1; seta = g.nx; }
    } else {            // xi = y, eta = x
        nxi = g.ny; neta = g.nx; hxi = g.hy; heta = g.hx;
        if (vol_z) { base = vol_z; sz = 1; sxi = g.nx * g.nz; seta = g.nz; }
        else { base = vol; sz = g.nx * g.ny; sxi = g.nx; seta = 1; }
    }

    // lane rows: band * FWD_ROWS + lane + 64 r
    using A = acc_t<TV>;
    float zc[R], czr[R], Ls[R];
    A p[R];
    bool ok[R];
    const bool col_ok = iu < g.nu;
    ColParam cp{};
    if (col_ok) cp = g.cols[(size_t)k * g.nu + iu];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iv = band * FWD_ROWS + lane + 64 * r;
        ok[r] = col_ok && iv < g.nv;
        const RowParam rp = ok[r] ? g.rows[iv] : RowParam{0.0f, 0.0f};
        zc[r] = zeta_centre(rp.qz, cp.tcv, g.zc);
        czr[r] = zeta_inv_slope(rp.inv_qz, cp.kz);
        Ls[r] = ray_length_per_xi(cp.lxy2, rp.qz, cp.gp);
        if (!ok[r]) czr[r] = 1.0f, zc[r] = 3.0e30f;  // far outside: an inert ray
    }
    if (col_ok) {
        A s[R];
        if (sz == 1)
            trace_rays<TV, R, 1>(base, sxi, seta, sz, nxi, neta, g.nz, hxi, heta, g.hz, cp.eta_c, cp.inv_a, cp.a, zc,
                                 czr, s);
        else
            trace_rays<TV, R, 0>(base, sxi, seta, sz, nxi, neta, g.nz, hxi, heta, g.hz, cp.eta_c, cp.inv_a, cp.a, zc,
                                 czr, s);
#pragma unroll
        for (int r = 0; r < R; ++r) p[r] = (A)Ls[r] * s[r];
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) p[r] = 0;
    }
    double sq = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!ok[r]) continue;
        const int iv = band * FWD_ROWS + lane + 64 * r;
        const size_t ray = ((size_t)k * g.nv + iv) * g.nu + iu;
        sq += fwd_store<TP, EPI, A>(out, aux, sc, ray, p[r]);
    }
    if (EPI != FWD_PLAIN) {
        const double bs = block_sum_256(sq);
        if (__builtin_amdgcn_workitem_id_x() == 0) partials[w] = bs;
    }
}

template <typename TV, typename TP, int EPI>
__global__ __launch_bounds__(256, sizeof(acc_t<TV>) != 4 ? 1 : (sizeof(TV) == 4 ? 7 : 8)) void k_forward(GeoDev g, const TV *__restrict__ vol, const TV *__restrict__ vol_z,
                                                 TP *__restrict__ out, const TP *__restrict__ aux,
                                                 const Scalars *__restrict__ sc, double *__restrict__ partials,
                                                 const int *__restrict__ skip)
{
    if (skip && *skip) return;
    forward_block<TV, TP, EPI, FWD_R>(g, __builtin_amdgcn_workgroup_id_x(), vol, vol_z, out, aux, sc, partials);
}

// One explicit rows-per-lane variant, plain epilogue (the batched form's tuner times these).
template <typename TV, typename TP, int EPI, int R>
__global__ __launch_bounds__(256) void k_forward_r(GeoDev g, const TV *__restrict__ vol, const TV *__restrict__ vol_z,
                                                   TP *__restrict__ out)
{
    forward_block<TV, TP, EPI, R>(g, __builtin_amdgcn_workgroup_id_x(), vol, vol_z, out, nullptr, nullptr, nullptr);
}

int64_t forward_num_blocks(const GeoDev &g)
{
    return g.projector == KCT_PROJECTOR_TT ? tt_forward_num_blocks(g) : fwd_grid(g, FWD_R).nblocks;
}
int64_t forward_num_blocks_r(const GeoDev &g, int rows_per_lane) { return fwd_grid(g, rows_per_lane).nblocks; }

template <typename TV, typename TP>
hipError_t launch_forward(const GeoDev &g, const TV *vol, const TV *vol_z, TP *out, const TP *aux, int epi,
                          const Scalars *sc, double *partials, const int *skip, hipStream_t st)
{
    if (g.projector == KCT_PROJECTOR_TT) return launch_forward_tt<TV, TP>(g, vol, vol_z, out, aux, epi, sc, partials, skip, st);
    dim3 grid((unsigned)fwd_grid(g, FWD_R).nblocks);
    dim3 block(256);
    if constexpr (std::is_same<TV, double>::value) {  // double storage: plain projection only
        if (epi != FWD_PLAIN) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_forward<TV, TP, FWD_PLAIN>), grid, block, 0, st, g, vol, vol_z, out, aux, sc, partials,
                           skip);
    } else {
        switch (epi) {
        case FWD_PLAIN:
            hipLaunchKernelGGL((k_forward<TV, TP, FWD_PLAIN>), grid, block, 0, st, g, vol, vol_z, out, aux, sc, partials, skip);
            break;
        case FWD_NORM:
            hipLaunchKernelGGL((k_forward<TV, TP, FWD_NORM>), grid, block, 0, st, g, vol, vol_z, out, aux, sc, partials, skip);
            break;
        case FWD_BMINUS:
            hipLaunchKernelGGL((k_forward<TV, TP, FWD_BMINUS>), grid, block, 0, st, g, vol, vol_z, out, aux, sc, partials,
                               skip);
            break;
        case FWD_LSQR:
            hipLaunchKernelGGL((k_forward<TV, TP, FWD_LSQR>), grid, block, 0, st, g, vol, vol_z, out, aux, sc, partials, skip);
            break;
        default:
            return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_forward_r(const GeoDev &g, const float *vol, const float *vol_z, float *out, int rows_per_lane,
                            hipStream_t st)
{
    dim3 grid((unsigned)fwd_grid(g, rows_per_lane).nblocks);
    if (rows_per_lane == 1)
        hipLaunchKernelGGL((k_forward_r<float, float, FWD_PLAIN, 1>), grid, dim3(256), 0, st, g, vol, vol_z, out);
    else if (rows_per_lane == 2)
        hipLaunchKernelGGL((k_forward_r<float, float, FWD_PLAIN, 2>), grid, dim3(256), 0, st, g, vol, vol_z, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Persistent batched p = A d with |p|^2 partials for every instance (CGLS
// steps of a batched solve): every workgroup takes items from the queue until
// it is empty; an item is up to BATCH_ITEM_FWD workgroup tiles of one
// instance's forward grid, in its own rows-per-lane variant.
__global__ __launch_bounds__(256, 8) void kp_forward(const BatchInst *__restrict__ B, const int64_t *__restrict__ off,
                                                  int count, BatchQueue *__restrict__ q)
{
    const int64_t total = off[count];
    for (;;) {
        const int64_t item = batch_pop(q);
        if (item >= total) break;
        const int i = batch_find(off, count, item);
        const BatchInst *bi = B + i;
        if (bi->sc->done) continue;
        const int64_t t0 = (item - off[i]) * BATCH_ITEM_FWD;
        const int64_t t1 = t0 + BATCH_ITEM_FWD < bi->nf ? t0 + BATCH_ITEM_FWD : bi->nf;
        for (int64_t t = t0; t < t1; ++t) {
            if (bi->fwd_r == 1)
                forward_block<float, float, FWD_NORM, 1>(bi->g, t, bi->d, bi->dz, bi->p, nullptr, bi->sc, bi->part);
            else
                forward_block<float, float, FWD_NORM, 2>(bi->g, t, bi->d, bi->dz, bi->p, nullptr, bi->sc, bi->part);
            __syncthreads();  // the tile's block sum is read before the next tile writes it
        }
    }
    batch_exit(q);
}

hipError_t launch_batch_forward(const BatchInst *B, const int64_t *off, int count, BatchQueue *q, int grid,
                                hipStream_t st)
{
    hipLaunchKernelGGL(kp_forward, dim3((unsigned)grid), dim3(256), 0, st, B, off, count, q);
    return hipGetLastError();
}

// Resident workgroups of the persistent batched kernels: the device's compute
// units times the workgroups one of them holds.
hipError_t batch_persistent_grids(int &fwd, int &bwd, int &dir)
{
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int nf = 0, nb = 0, nd = 0;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nf, kp_forward, 256, 0);
    if (e == hipSuccess) e = batch_backward_occupancy(nb);
    if (e == hipSuccess) e = batch_dir_occupancy(nd);
    if (e != hipSuccess) return e;
    fwd = cus * (nf > 0 ? nf : 1);
    bwd = cus * (nb > 0 ? nb : 1);
    dir = cus * (nd > 0 ? nd : 1);
    return hipSuccess;
}

#define KCT_INST(TV, TP)                                                                                       \
    template hipError_t launch_forward<TV, TP>(const GeoDev &, const TV *, const TV *, TP *, const TP *, int,   \
                                               const Scalars *, double *, const int *, hipStream_t);
KCT_INST(float, float)
KCT_INST(bf16, bf16)
KCT_INST(_Float16, _Float16)
KCT_INST(float, bf16)
KCT_INST(float, _Float16)
KCT_INST(double, double)

}  // namespace kct
