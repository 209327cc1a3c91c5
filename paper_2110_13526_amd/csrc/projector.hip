// projector.hip -- the forward cone-beam projector for gfx950.
//
//   forward  p = A x    (Section 2, Eq. 1): ray-driven.  One lane per ray; the
//            64 lanes of a wavefront are 64 neighbouring detector columns of one
//            row, so their voxel reads fall on neighbouring addresses when the
//            volume is stored with the eta axis (the non-dominant in-plane axis)
//            fastest.  Each lane walks the voxels of its ray in increasing xi,
//            merging the crossings of the three families of voxel planes
//            (Siddon's traversal), and accumulates w_ij * x_j in single
//            precision.
// The backprojector (the voxel-driven gather that evaluates the same weights)
// is in backproject.hip.
//
// The kernel can fuse a double-precision partial sum of the squares of its
// outputs (|p|^2 of Algorithm 1) and the LSQR bidiagonalisation update.
#include "kct_internal.h"
#include "kct_ray.h"
#include "kct_weights.h"

namespace kct {

constexpr int FWD_COLS = 64;  // detector columns per workgroup (one wavefront)
constexpr int FWD_ROWS = 4;   // detector rows per workgroup (one per wavefront)

// Sum of v over the 256 threads of the workgroup, in a fixed order.  Result is
// valid in thread 0.
__device__ __forceinline__ double block_sum_256(double v)
{
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
    return r;
}

template <typename T, int EPI>
__global__ __launch_bounds__(256) void k_forward(GeoDev g, const T *__restrict__ vol, const T *__restrict__ vol_t,
                                                 T *__restrict__ out, const T *__restrict__ aux,
                                                 const Scalars *__restrict__ sc, double *__restrict__ partials,
                                                 const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const int k = blockIdx.z;
    const int iu = blockIdx.x * FWD_COLS + (threadIdx.x & 63);
    const int iv = blockIdx.y * FWD_ROWS + (threadIdx.x >> 6);
    const ViewParam vp = g.views[k];
    const bool valid = iu < g.nu && iv < g.nv;

    const int szeta = g.nx * g.ny;
    int nxi, neta, sxi, seta;
    float hxi, heta;
    const T *base;
    if (vp.dom == 0) {
        nxi = g.nx; neta = g.ny; hxi = g.hx; heta = g.hy;
        if (vol_t) { base = vol_t; sxi = g.ny; seta = 1; }
        else { base = vol; sxi = 1; seta = g.nx; }
    } else {
        nxi = g.ny; neta = g.nx; hxi = g.hy; heta = g.hx;
        base = vol; sxi = g.nx; seta = 1;
    }

    float p = 0.0f;
    if (valid) {
        const ColParam cp = g.cols[(size_t)k * g.nu + iu];
        const RowParam rp = g.rows[iv];
        const float zeta_c = zeta_centre(rp.qz, cp.tcv, g.zc);
        const float czr = zeta_inv_slope(rp.inv_qz, cp.kz);
        const float L = ray_length_per_xi(cp.lxy2, rp.qz, cp.gp);
        const float s = trace_ray<T>(base, sxi, seta, szeta, nxi, neta, g.nz, hxi, heta, g.hz, cp.eta_c, cp.inv_a,
                                     cp.a, zeta_c, czr);
        p = L * s;
    }
    const size_t ray = ((size_t)k * g.nv + iv) * g.nu + iu;
    double sq = 0.0;
    if (valid) {
        float o;
        if (EPI == FWD_BMINUS) o = to_f32(aux[ray]) - p;
        else if (EPI == FWD_LSQR) o = (float)sc->fwd_c1 * p - (float)sc->fwd_c2 * to_f32(out[ray]);
        else o = p;
        const T st = from_f32<T>(o);
        out[ray] = st;
        const double od = (double)to_f32(st);
        sq = od * od;
    }
    if (EPI != FWD_PLAIN) {
        const double bs = block_sum_256(sq);
        if (threadIdx.x == 0)
            partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = bs;
    }
}

int64_t forward_num_blocks(const GeoDev &g)
{
    return (int64_t)((g.nu + FWD_COLS - 1) / FWD_COLS) * ((g.nv + FWD_ROWS - 1) / FWD_ROWS) * g.nviews;
}

template <typename T>
hipError_t launch_forward(const GeoDev &g, const T *vol, const T *vol_t, T *out, const T *aux, int epi,
                          const Scalars *sc, double *partials, const int *skip, hipStream_t st)
{
    dim3 grid((g.nu + FWD_COLS - 1) / FWD_COLS, (g.nv + FWD_ROWS - 1) / FWD_ROWS, g.nviews);
    dim3 block(256);
    switch (epi) {
    case FWD_PLAIN:
        hipLaunchKernelGGL((k_forward<T, FWD_PLAIN>), grid, block, 0, st, g, vol, vol_t, out, aux, sc, partials, skip);
        break;
    case FWD_NORM:
        hipLaunchKernelGGL((k_forward<T, FWD_NORM>), grid, block, 0, st, g, vol, vol_t, out, aux, sc, partials, skip);
        break;
    case FWD_BMINUS:
        hipLaunchKernelGGL((k_forward<T, FWD_BMINUS>), grid, block, 0, st, g, vol, vol_t, out, aux, sc, partials,
                           skip);
        break;
    case FWD_LSQR:
        hipLaunchKernelGGL((k_forward<T, FWD_LSQR>), grid, block, 0, st, g, vol, vol_t, out, aux, sc, partials, skip);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define KCT_INST(T)                                                                                              \
    template hipError_t launch_forward<T>(const GeoDev &, const T *, const T *, T *, const T *, int,            \
                                          const Scalars *, double *, const int *, hipStream_t);
KCT_INST(float)
KCT_INST(bf16)
KCT_INST(_Float16)

}  // namespace kct
