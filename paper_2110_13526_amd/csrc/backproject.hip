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

template <typename T, int EPI>
__global__ __launch_bounds__(256, 4) void k_backward(GeoDev g, const T *__restrict__ proj, T *__restrict__ out,
                                                  T *__restrict__ out_z, const Scalars *__restrict__ sc,
                                                  double *__restrict__ partials, const int *__restrict__ skip, int nbx,
                                                  int nby, int nbz)
{
    if (skip && *skip) return;
    __shared__ PixStage s_pix[CH_ROWS * CH_COLS];
    __shared__ ColStage s_col[CH_COLS];
    __shared__ int s_fp[4];

    // XCD-aware brick assignment
    const int nb = nbx * nby * nbz;
    const int w = blockIdx.x;
    const int b = (nb % NXCD == 0) ? (w % NXCD) * (nb / NXCD) + w / NXCD : w;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int ix = bx * BX + (int)(threadIdx.x % BX);
    const int iy = by * BY + (int)(threadIdx.x / BX);
    const int iz0 = bz * TZ;
    const int nzb = g.nz - iz0 < TZ ? g.nz - iz0 : TZ;
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

    float acc[TZ];
#pragma unroll
    for (int j = 0; j < TZ; ++j) acc[j] = 0.0f;

    for (int k = 0; k < g.nviews; ++k) {
        const ViewParam vp = g.views[k];
        // 1. shadow of the brick: lanes 0..7 of wave 0 project one corner each
        if (threadIdx.x < 64) {
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
            if (threadIdx.x == 0) {
                int u0 = (int)floorf(umin) - 1, u1 = (int)ceilf(umax) + 1;
                int v0 = (int)floorf(vmin) - 1, v1 = (int)ceilf(vmax) + 1;
                s_fp[0] = u0 < 0 ? 0 : u0;
                s_fp[1] = u1 > g.nu - 1 ? g.nu - 1 : u1;
                s_fp[2] = v0 < 0 ? 0 : v0;
                s_fp[3] = v1 > g.nv - 1 ? g.nv - 1 : v1;
            }
        }
        __syncthreads();
        const int u0 = s_fp[0], u1 = s_fp[1], v0 = s_fp[2], v1 = s_fp[3];
        __syncthreads();
        const T *pk = proj + (size_t)k * g.nv * g.nu;
        const ColParam *ck = g.cols + (size_t)k * g.nu;
        for (int cu0 = u0; cu0 <= u1; cu0 += CH_COLS) {
            const int ncol = u1 - cu0 + 1 < CH_COLS ? u1 - cu0 + 1 : CH_COLS;
            for (int cv0 = v0; cv0 <= v1; cv0 += CH_ROWS) {
                const int nrow = v1 - cv0 + 1 < CH_ROWS ? v1 - cv0 + 1 : CH_ROWS;
                // 2. stage the chunk: per pixel the z-parameters of its ray and L * e,
                //    per column the in-plane parameters
                for (int t = threadIdx.x; t < ncol * nrow; t += 256) {
                    const int r = t / ncol, c = t - r * ncol;
                    const ColParam cp = ck[cu0 + c];
                    const RowParam rp = g.rows[cv0 + r];
                    const bool par = rp.inv_qz == 0.0f;
                    PixStage ps;
                    ps.zc = zeta_centre(rp.qz, cp.tcv, g.zc) + (par ? pzadd : 0.0f);
                    ps.czr = zeta_inv_slope(par ? INFINITY : rp.inv_qz, cp.kz);
                    ps.le = ray_length_per_xi(cp.lxy2, rp.qz, cp.gp) * to_f32(pk[(size_t)(cv0 + r) * g.nu + cu0 + c]);
                    ps.pad = 0.0f;
                    s_pix[r * CH_COLS + c] = ps;
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
                if (valid) gather_chunk(g, vp, ix, iy, iz0, nzb, s_pix, s_col, cu0, ncol, cv0, nrow, acc);
                __syncthreads();
            }
        }
    }

    double sq = 0.0;
    if (valid) {
#pragma unroll
        for (int j = 0; j < TZ; ++j) {
            if (j >= nzb) continue;
            const int iz = iz0 + j;
            const size_t vox = ((size_t)iz * g.ny + iy) * g.nx + ix;
            float o;
            if (EPI == BWD_LSQR0) o = (float)sc->bwd_c1 * acc[j];
            else if (EPI == BWD_LSQR) o = (float)sc->bwd_c1 * acc[j] - (float)sc->bwd_c2 * to_f32(out[vox]);
            else if (EPI == BWD_NORM) o = sc->bwd_scale * acc[j];
            else o = acc[j];
            const T st = from_f32<T>(o);
            out[vox] = st;
            if (EPI == BWD_LSQR0 || EPI == BWD_LSQR) out_z[((size_t)iy * g.nx + ix) * g.nz + iz] = st;
            const double od = (double)to_f32(st);
            sq += od * od;
        }
    }
    if (EPI != BWD_PLAIN) {
        const double bs = bwd_block_sum(sq);
        if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    }
}

static void bwd_grid(const GeoDev &g, int &nbx, int &nby, int &nbz)
{
    nbx = (g.nx + BX - 1) / BX;
    nby = (g.ny + BY - 1) / BY;
    nbz = (g.nz + TZ - 1) / TZ;
}

int64_t backward_num_blocks(const GeoDev &g)
{
    int nbx, nby, nbz;
    bwd_grid(g, nbx, nby, nbz);
    return (int64_t)nbx * nby * nbz;
}

template <typename T>
hipError_t launch_backward(const GeoDev &g, const T *proj, T *out, T *out_z, int epi, const Scalars *sc,
                           double *partials, const int *skip, hipStream_t st)
{
    int nbx, nby, nbz;
    bwd_grid(g, nbx, nby, nbz);
    dim3 grid((unsigned)(nbx * nby * nbz));
    dim3 block(256);
    switch (epi) {
    case BWD_PLAIN:
        hipLaunchKernelGGL((k_backward<T, BWD_PLAIN>), grid, block, 0, st, g, proj, out, out_z, sc, partials, skip,
                           nbx, nby, nbz);
        break;
    case BWD_NORM:
        hipLaunchKernelGGL((k_backward<T, BWD_NORM>), grid, block, 0, st, g, proj, out, out_z, sc, partials, skip,
                           nbx, nby, nbz);
        break;
    case BWD_LSQR0:
        hipLaunchKernelGGL((k_backward<T, BWD_LSQR0>), grid, block, 0, st, g, proj, out, out_z, sc, partials, skip,
                           nbx, nby, nbz);
        break;
    case BWD_LSQR:
        hipLaunchKernelGGL((k_backward<T, BWD_LSQR>), grid, block, 0, st, g, proj, out, out_z, sc, partials, skip,
                           nbx, nby, nbz);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define KCT_BINST(T)                                                                                             \
    template hipError_t launch_backward<T>(const GeoDev &, const T *, T *, T *, int, const Scalars *, double *, \
                                           const int *, hipStream_t);
KCT_BINST(float)
KCT_BINST(bf16)
KCT_BINST(_Float16)

}  // namespace kct
