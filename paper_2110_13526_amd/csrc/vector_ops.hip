// vector_ops.hip -- the streaming vector updates and the double-precision
// scalar steps of CGLS (Section 2, Algorithm 1) and LSQR on gfx950.
//
// Reductions are deterministic: every producing kernel writes one partial sum
// per workgroup, and a one-workgroup finalize kernel adds the partials in a
// fixed order and performs the scalar algebra (norms, alpha, beta, Givens
// rotation, stop tests) in double precision on the device.  No atomics.
//
// Kernels on the iteration path take a pointer to the solver's "done" flag and
// return at once when it is set, so a solve can be enqueued in full without
// host synchronisation and still stop early (tolerance reached, breakdown).
#include "kct_batch.h"
#include "kct_internal.h"
#include "kct_weights.h"

namespace kct {

constexpr int STREAM_BLOCKS = 2048;  // grid of the streaming kernels (8 per CU)
constexpr int TB = 256;

int64_t stream_num_blocks() { return STREAM_BLOCKS; }

__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double red[TB / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
    return r;
}

template <typename T>
__global__ __launch_bounds__(TB) void k_norm2(const T *__restrict__ v, int64_t n, double *__restrict__ partials,
                                              const int *__restrict__ skip)
{
    if (skip && *skip) return;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        double x = (double)to_f32(v[i]);
        s += x * x;
    }
    double b = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

template <typename T>
__global__ __launch_bounds__(TB) void k_fill_zero(T *__restrict__ v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB)
        v[i] = from_f32<T>(0.0f);
}

template <typename T>
__global__ __launch_bounds__(TB) void k_copy(const T *__restrict__ s, T *__restrict__ d, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) d[i] = s[i];
}

// x += alpha d
template <typename T>
__global__ __launch_bounds__(TB) void k_cgls_x(float *__restrict__ x, const T *__restrict__ d,
                                               const Scalars *__restrict__ sc, int64_t n)
{
    if (sc->done) return;
    const float alpha = (float)sc->x_alpha;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB)
        x[i] = x[i] + alpha * to_f32(d[i]);
}

// e -= alpha p, partial |e|^2
template <typename T>
__global__ __launch_bounds__(TB) void k_cgls_e(T *__restrict__ e, const T *__restrict__ p,
                                               const Scalars *__restrict__ sc, int64_t n,
                                               double *__restrict__ partials)
{
    if (sc->done) return;
    const float alpha = (float)sc->e_alpha;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        const T v = from_f32<T>(to_f32(e[i]) - alpha * to_f32(p[i]));
        e[i] = v;
        const double dv = (double)to_f32(v);
        s += dv * dv;
    }
    double b = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

// d = r + beta d (first: d = r), and dz = d stored z-fastest.  A workgroup
// takes a 32 (z) x 32 (x) tile of one y-plane through LDS, so the plain and
// the z-fastest stores both coalesce.  With dpart, also the workgroup's partial
// sum of the stored d^2 (the Tikhonov term of NP2).
template <typename T, int FIRST>
__device__ __forceinline__ void cgls_d_tile(int nx, int ny, int nz, const T *__restrict__ r, T *__restrict__ d,
                                            T *__restrict__ dz, const Scalars *__restrict__ sc,
                                            double *__restrict__ dpart, int tx_blk, int tz_blk, int y,
                                            int64_t blk)
{
    __shared__ float tile[32][33];
    const float beta = FIRST ? 0.0f : (float)sc->beta;
    const int bx = tx_blk * 32, bz = tz_blk * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    double sq = 0.0;
    for (int j = ty; j < 32; j += 8) {
        const int x = bx + tx, z = bz + j;
        if (x < nx && z < nz) {
            const size_t i = ((size_t)z * ny + y) * nx + x;
            float v = to_f32(r[i]);
            if (!FIRST) v = v + beta * to_f32(d[i]);
            const T st = from_f32<T>(v);
            d[i] = st;
            tile[j][tx] = to_f32(st);
            const double dv = (double)to_f32(st);
            sq += dv * dv;
        }
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int z = bz + tx, x = bx + j;
        if (x < nx && z < nz) dz[((size_t)y * nx + x) * nz + z] = from_f32<T>(tile[tx][j]);
    }
    if (dpart) {
        const double b = block_sum(sq);
        if (threadIdx.x == 0) dpart[blk] = b;
    }
}

template <typename T, int FIRST>
__global__ __launch_bounds__(TB) void k_cgls_d(int nx, int ny, int nz, const T *__restrict__ r, T *__restrict__ d,
                                               T *__restrict__ dz, const Scalars *__restrict__ sc,
                                               double *__restrict__ dpart)
{
    if (sc->done) return;
    cgls_d_tile<T, FIRST>(nx, ny, nz, r, d, dz, sc, dpart, blockIdx.x, blockIdx.y, blockIdx.z,
                          ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x);
}

template <typename TS, typename TD>
__global__ __launch_bounds__(TB) void k_zfast_copy(int nx, int ny, int nz, const TS *__restrict__ s,
                                                   TD *__restrict__ dz)
{
    __shared__ acc_t<TS> tile[32][33];
    const int bx = blockIdx.x * 32, bz = blockIdx.y * 32, y = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int j = ty; j < 32; j += 8) {
        const int x = bx + tx, z = bz + j;
        if (x < nx && z < nz) tile[j][tx] = to_acc(s[((size_t)z * ny + y) * nx + x]);
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int z = bz + tx, x = bx + j;
        if (x < nx && z < nz) dz[((size_t)y * nx + x) * nz + z] = store_as<TD>(tile[tx][j]);
    }
}

// LSQR: init: w = w_vcoef v.  Iteration: x += x_coef w; w = w_vcoef v - w_coef w.
template <typename T, int INIT>
__global__ __launch_bounds__(TB) void k_lsqr_xw(float *__restrict__ x, T *__restrict__ w, const T *__restrict__ v,
                                                const Scalars *__restrict__ sc, int64_t n)
{
    if (sc->done) return;
    const float vc = (float)sc->w_vcoef;
    if (INIT) {
        for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB)
            w[i] = from_f32<T>(vc * to_f32(v[i]));
        return;
    }
    const float xc = (float)sc->x_coef, wc = (float)sc->w_coef;
    const bool upd_w = sc->w_vcoef != 0.0 || sc->w_coef != 0.0;
    for (int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TB) {
        const float wi = to_f32(w[i]);
        x[i] = x[i] + xc * wi;
        if (upd_w) w[i] = from_f32<T>(vc * to_f32(v[i]) - wc * wi);
    }
}

// Fixed-order sum of the partials followed by one scalar step.
__device__ double fixed_order_sum(const double *__restrict__ partials, int64_t np, double *red)
{
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < np; i += TB) s += partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// One scalar step of a solve, run by one workgroup: the fixed-order sums of
// the partials, then the step (thread 0).  partials2 (optional): a second set
// of partials, used by F_ALPHA for the Tikhonov term |d|^2.
__device__ __forceinline__ void finalize_step(Scalars *__restrict__ sc, const double *__restrict__ partials,
                                              int64_t np, int op, const double *__restrict__ partials2,
                                              int64_t np2)
{
    if (op != F_NB0 && sc->done) return;
    __shared__ double red[TB];
    const double S = fixed_order_sum(partials, np, red);
    const double S2 = partials2 ? fixed_order_sum(partials2, np2, red) : 0.0;
    if (threadIdx.x != 0) return;
    auto stop = [&](int reason) {
        sc->done = 1;
        sc->stop = reason;
        sc->skip_bwd = 1;
        sc->t_done = wall_clock64();  // the solve's completion time on the device clock
    };
    switch (op) {
    case F_NB0:  // NB0 = |b|
        sc->nb0 = sqrt(S);
        sc->nb = sc->nb0;
        sc->phibar = sc->nb0;
        if (sc->maxiter <= 0) stop(KCT_STOP_MAXITER);
        break;
    case F_NB_INIT:  // NB of e = b - A x0 (reported if the first step breaks down)
        sc->nb = sqrt(S);
        if (!isfinite(sc->nb)) stop(KCT_STOP_NUMERIC);
        break;
    case F_NR2_INIT: {  // NR2_old = |r|^2 (r is stored divided by sr)
        const double nr2 = S * (sc->sr * sc->sr);
        sc->nr2_old = nr2;
        sc->nr2_now = nr2;
        if (!isfinite(nr2)) stop(KCT_STOP_NUMERIC);
        else if (nr2 == 0.0) stop(KCT_STOP_BREAKDOWN);
        break;
    }
    case F_ALPHA: {  // NP2 = |p|^2 (+ lambda^2 |d|^2), alpha = NR2_old / NP2 (p is stored divided by sp)
        const double np2 = S * (sc->sp * sc->sp) + sc->tik_d2 * S2;
        sc->np2 = np2;
        if (!isfinite(np2)) stop(KCT_STOP_NUMERIC);
        else if (np2 == 0.0) stop(KCT_STOP_BREAKDOWN);
        else {
            sc->alpha = sc->nr2_old / np2;
            sc->x_alpha = sc->alpha * sc->sr;
            sc->e_alpha = sc->alpha * sc->sp;
        }
        break;
    }
    case F_NB: {  // NB = |e|, i = i + 1, stop test of the while loop
        const double nb = sqrt(S);
        sc->nb = nb;
        sc->iters += 1;
        if (sc->history) sc->history[sc->iters - 1] = sc->nb0 > 0.0 ? nb / sc->nb0 : 0.0;
        if (!isfinite(nb)) stop(KCT_STOP_NUMERIC);
        else if (!(nb > sc->err * sc->nb0)) stop(sc->iters >= sc->maxiter ? KCT_STOP_MAXITER : KCT_STOP_TOL);
        else if (sc->iters >= sc->maxiter) stop(KCT_STOP_MAXITER);
        break;
    }
    case F_BETA: {  // NR2_now = |r|^2, beta = NR2_now / NR2_old, NR2_old = NR2_now
        const double nr2 = S * (sc->sr * sc->sr);
        sc->nr2_now = nr2;
        if (!isfinite(nr2)) stop(KCT_STOP_NUMERIC);
        else if (nr2 == 0.0) stop(KCT_STOP_BREAKDOWN);
        else {
            sc->beta = nr2 / sc->nr2_old;
            sc->nr2_old = nr2;
        }
        break;
    }
    case F_L_BETA0: {  // beta_1 = |u_hat|, u = u_hat / beta_1
        const double b = sqrt(S);
        sc->l_beta = b;
        sc->phibar = b;
        sc->nb = b;
        if (!isfinite(b)) stop(KCT_STOP_NUMERIC);
        else if (b == 0.0) stop(KCT_STOP_BREAKDOWN);
        else { sc->bwd_c1 = 1.0 / b; sc->bwd_c2 = 0.0; }
        break;
    }
    case F_L_ALPHA0: {  // alpha_1 = |v_hat|, w_1 = v_hat / alpha_1
        const double a = sqrt(S);
        sc->l_alpha = a;
        sc->rhobar = a;
        sc->nr2_now = S;
        if (!isfinite(a)) stop(KCT_STOP_NUMERIC);
        else if (a == 0.0) stop(KCT_STOP_BREAKDOWN);
        else {
            sc->w_vcoef = 1.0 / (a * sc->sw);  // w is stored divided by sw
            sc->fwd_c1 = 1.0 / a;
            sc->fwd_c2 = a / sc->l_beta;
        }
        break;
    }
    case F_L_BETA: {  // beta_{i+1} = |A v - alpha u| (u_hat' already formed by the forward epilogue)
        const double b = sqrt(S);
        sc->l_beta = b;
        if (!isfinite(b)) { stop(KCT_STOP_NUMERIC); break; }
        // the backprojection of this iteration is skipped on the last iteration
        // and when beta = 0 (then the rotation ends the solve anyway)
        sc->skip_bwd = (b == 0.0 || sc->iters + 1 >= sc->maxiter) ? 1 : 0;
        if (b != 0.0) { sc->bwd_c1 = 1.0 / b; sc->bwd_c2 = b / sc->l_alpha; }
        break;
    }
    case F_L_ALPHA: {  // alpha_{i+1} = |A^T u - beta v| (0 when the backprojection was skipped)
        const double a = sc->skip_bwd ? 0.0 : sqrt(S);
        sc->nr2_now = a * a;
        if (!isfinite(a)) { stop(KCT_STOP_NUMERIC); break; }
        // damping rotation (Tikhonov term), then the Givens rotation (Paige & Saunders)
        if (sc->damp != 0.0) {
            const double rhobar1 = sqrt(sc->rhobar * sc->rhobar + sc->damp * sc->damp);
            const double psi = (sc->damp / rhobar1) * sc->phibar;
            sc->res2 += psi * psi;
            sc->phibar = (sc->rhobar / rhobar1) * sc->phibar;
            sc->rhobar = rhobar1;
        }
        const double beta = sc->l_beta;
        const double rho = sqrt(sc->rhobar * sc->rhobar + beta * beta);
        const double c = sc->rhobar / rho, s = beta / rho;
        const double theta = s * a;
        sc->rho = rho;
        sc->cg = c;
        sc->sg = s;
        sc->theta = theta;
        sc->rhobar = -c * a;
        sc->phi = c * sc->phibar;
        sc->phibar = s * sc->phibar;
        sc->x_coef = (sc->phi / rho) * sc->sw;
        sc->w_coef = theta / rho;
        sc->w_vcoef = a != 0.0 ? 1.0 / (a * sc->sw) : 0.0;
        if (a == 0.0) sc->w_coef = 0.0;
        sc->l_alpha = a;
        if (a != 0.0) { sc->fwd_c1 = 1.0 / a; sc->fwd_c2 = a / beta; }
        break;
    }
    case F_L_GIVENS: {  // after x and w are updated: i = i + 1, stop tests
        sc->iters += 1;
        const double nb = sqrt(sc->phibar * sc->phibar + sc->res2);  // |phibar| without damping
        sc->nb = nb;
        if (sc->history) sc->history[sc->iters - 1] = sc->nb0 > 0.0 ? nb / sc->nb0 : 0.0;
        if (!isfinite(nb)) stop(KCT_STOP_NUMERIC);
        else if (sc->l_beta == 0.0 || (sc->iters < sc->maxiter && sc->l_alpha == 0.0)) stop(KCT_STOP_BREAKDOWN);
        else if (!(nb > sc->err * sc->nb0)) stop(sc->iters >= sc->maxiter ? KCT_STOP_MAXITER : KCT_STOP_TOL);
        else if (sc->iters >= sc->maxiter) stop(KCT_STOP_MAXITER);
        break;
    }
    default:
        break;
    }
}

__global__ __launch_bounds__(TB) void k_finalize(Scalars *__restrict__ sc, const double *__restrict__ partials,
                                                 int64_t np, int op, const double *__restrict__ partials2,
                                                 int64_t np2)
{
    finalize_step(sc, partials, np, op, partials2, np2);
}

// ---------------------------------------------------------------- batched
// Batched streaming steps: workgroup w serves instance w / STREAM_BLOCKS as
// workgroup w % STREAM_BLOCKS of that instance's own streaming grid, so every
// instance sees the block decomposition (and the partial sums) of a single solve.
__global__ __launch_bounds__(TB) void kb_vec(const BatchInst *__restrict__ B, int op, int maxiter, double err)
{
    const int i = blockIdx.x / STREAM_BLOCKS;
    const int lb = blockIdx.x % STREAM_BLOCKS;
    const BatchInst *bi = B + i;
    Scalars *sc = bi->sc;
    const int64_t stride = (int64_t)STREAM_BLOCKS * TB;
    const int64_t i0 = (int64_t)lb * TB + threadIdx.x;
    if (op == BV_INIT) {  // scalars of a plain FP32 CGLS solve (all storage scales 1)
        if (lb == 0 && threadIdx.x == 0) {
            Scalars s;
            memset(&s, 0, sizeof(s));
            s.maxiter = maxiter;
            s.err = err;
            s.sr = s.sp = s.sw = 1.0;
            s.fwd_scale = s.bwd_scale = 1.0f;
            s.t_start = wall_clock64();
            *sc = s;
        }
        return;
    }
    if (op == BV_NORM_B) {  // partials of |b|^2
        double q = 0.0;
        for (int64_t k = i0; k < bi->m; k += stride) {
            const double v = (double)bi->b[k];
            q += v * v;
        }
        const double bs = block_sum(q);
        if (threadIdx.x == 0) bi->part[lb] = bs;
        return;
    }
    if (op == BV_X0_E) {  // x0 = 0 (also when the solve stopped at once: K = 0 or b = 0), e = b
        for (int64_t k = i0; k < bi->n; k += stride) bi->x[k] = 0.0f;
        if (sc->done) return;
        for (int64_t k = i0; k < bi->m; k += stride) bi->e[k] = bi->b[k];
        return;
    }
    if (sc->done) return;
    if (op == BV_CGLS_X) {  // x += alpha d
        const float alpha = (float)sc->x_alpha;
        for (int64_t k = i0; k < bi->n; k += stride) bi->x[k] = bi->x[k] + alpha * bi->d[k];
    } else if (op == BV_CGLS_E) {  // e -= alpha p, partials of |e|^2
        const float alpha = (float)sc->e_alpha;
        double q = 0.0;
        for (int64_t k = i0; k < bi->m; k += stride) {
            const float v = bi->e[k] - alpha * bi->p[k];
            bi->e[k] = v;
            q += (double)v * (double)v;
        }
        const double bs = block_sum(q);
        if (threadIdx.x == 0) bi->part[lb] = bs;
    }
}

// Persistent batched d = r + beta d with its z-fastest copy: every workgroup
// takes items from the queue until it is empty; an item is up to
// BATCH_ITEM_DIR 32 x 32 tiles of one instance (tile numbering of k_cgls_d).
template <int FIRST>
__global__ __launch_bounds__(TB) void kp_dir(const BatchInst *__restrict__ B, const int64_t *__restrict__ off,
                                             int count, BatchQueue *__restrict__ q)
{
    const int64_t total = off[count];
    for (;;) {
        const int64_t item = batch_pop(q);
        if (item >= total) break;
        const int i = batch_find(off, count, item);
        const BatchInst *bi = B + i;
        if (bi->sc->done) continue;
        const int gx = (bi->g.nx + 31) / 32, gz = (bi->g.nz + 31) / 32;
        const int64_t t0 = (item - off[i]) * BATCH_ITEM_DIR;
        const int64_t t1 = t0 + BATCH_ITEM_DIR < bi->ndir ? t0 + BATCH_ITEM_DIR : bi->ndir;
        for (int64_t t = t0; t < t1; ++t) {
            cgls_d_tile<float, FIRST>(bi->g.nx, bi->g.ny, bi->g.nz, bi->r, bi->d, bi->dz, bi->sc, nullptr,
                                      (int)(t % gx), (int)((t / gx) % gz), (int)(t / ((int64_t)gx * gz)), t);
            __syncthreads();  // the LDS tile is read before the next tile writes it
        }
    }
    batch_exit(q);
}

hipError_t batch_dir_occupancy(int &per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kp_dir<0>, TB, 0);
}

__global__ __launch_bounds__(TB) void kb_finalize(const BatchInst *__restrict__ B, int op, int kind)
{
    const BatchInst *bi = B + blockIdx.x;
    const int64_t np = kind == BG_FWD ? bi->nf : (kind == BG_BWD ? bi->nbk : (int64_t)STREAM_BLOCKS);
    finalize_step(bi->sc, bi->part, np, op, nullptr, 0);
}

hipError_t launch_batch_vec(const BatchInst *B, int count, int op, int maxiter, double err, hipStream_t st)
{
    hipLaunchKernelGGL(kb_vec, dim3((unsigned)(count * STREAM_BLOCKS)), dim3(TB), 0, st, B, op, maxiter, err);
    return hipGetLastError();
}

hipError_t launch_batch_dir(const BatchInst *B, const int64_t *off, int count, BatchQueue *q, int grid, int first,
                            hipStream_t st)
{
    if (first) hipLaunchKernelGGL(kp_dir<1>, dim3((unsigned)grid), dim3(TB), 0, st, B, off, count, q);
    else hipLaunchKernelGGL(kp_dir<0>, dim3((unsigned)grid), dim3(TB), 0, st, B, off, count, q);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchInst *B, int count, int op, int kind, hipStream_t st)
{
    hipLaunchKernelGGL(kb_finalize, dim3((unsigned)count), dim3(TB), 0, st, B, op, kind);
    return hipGetLastError();
}

static dim3 sgrid(int64_t n)
{
    int64_t b = (n + TB - 1) / TB;
    if (b > STREAM_BLOCKS) b = STREAM_BLOCKS;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

template <typename TS, typename TD>
hipError_t launch_zfast_copy(const GeoDev &g, const TS *src, TD *dst, hipStream_t st)
{
    dim3 grid((g.nx + 31) / 32, (g.nz + 31) / 32, g.ny);
    hipLaunchKernelGGL((k_zfast_copy<TS, TD>), grid, dim3(TB), 0, st, g.nx, g.ny, g.nz, src, dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_norm2(const T *v, int64_t n, double *partials, const int *skip, hipStream_t st)
{
    // always STREAM_BLOCKS partials so the finalize step reads a fixed count
    hipLaunchKernelGGL(k_norm2<T>, dim3(STREAM_BLOCKS), dim3(TB), 0, st, v, n, partials, skip);
    return hipGetLastError();
}

hipError_t launch_finalize(Scalars *sc, const double *partials, int64_t nparts, int op, hipStream_t st,
                           const double *partials2, int64_t nparts2)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(TB), 0, st, sc, partials, nparts, op, partials2, nparts2);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_zero(T *v, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_zero<T>, sgrid(n), dim3(TB), 0, st, v, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(const T *src, T *dst, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy<T>, sgrid(n), dim3(TB), 0, st, src, dst, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cgls_x(float *x, const T *d, const Scalars *sc, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_cgls_x<T>, sgrid(n), dim3(TB), 0, st, x, d, sc, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cgls_d(const GeoDev &g, const T *r, T *d, T *dz, const Scalars *sc, int first, hipStream_t st,
                         double *dpart)
{
    dim3 grid((g.nx + 31) / 32, (g.nz + 31) / 32, g.ny);
    if (first) hipLaunchKernelGGL((k_cgls_d<T, 1>), grid, dim3(TB), 0, st, g.nx, g.ny, g.nz, r, d, dz, sc, dpart);
    else hipLaunchKernelGGL((k_cgls_d<T, 0>), grid, dim3(TB), 0, st, g.nx, g.ny, g.nz, r, d, dz, sc, dpart);
    return hipGetLastError();
}

int64_t cgls_d_num_blocks(const GeoDev &g) { return (int64_t)((g.nx + 31) / 32) * ((g.nz + 31) / 32) * g.ny; }

template <typename T>
hipError_t launch_cgls_e(T *e, const T *p, const Scalars *sc, int64_t n, double *partials, hipStream_t st)
{
    hipLaunchKernelGGL(k_cgls_e<T>, dim3(STREAM_BLOCKS), dim3(TB), 0, st, e, p, sc, n, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lsqr_xw(float *x, T *w, const T *v, const Scalars *sc, int init, int64_t n, hipStream_t st)
{
    if (init) hipLaunchKernelGGL((k_lsqr_xw<T, 1>), sgrid(n), dim3(TB), 0, st, x, w, v, sc, n);
    else hipLaunchKernelGGL((k_lsqr_xw<T, 0>), sgrid(n), dim3(TB), 0, st, x, w, v, sc, n);
    return hipGetLastError();
}

#define KCT_VINST(T)                                                                                       \
    template hipError_t launch_norm2<T>(const T *, int64_t, double *, const int *, hipStream_t);          \
    template hipError_t launch_fill_zero<T>(T *, int64_t, hipStream_t);                                   \
    template hipError_t launch_copy<T>(const T *, T *, int64_t, hipStream_t);                             \
    template hipError_t launch_cgls_x<T>(float *, const T *, const Scalars *, int64_t, hipStream_t);      \
    template hipError_t launch_cgls_d<T>(const GeoDev &, const T *, T *, T *, const Scalars *, int,       \
                                         hipStream_t, double *);                                          \
    template hipError_t launch_cgls_e<T>(T *, const T *, const Scalars *, int64_t, double *, hipStream_t); \
    template hipError_t launch_lsqr_xw<T>(float *, T *, const T *, const Scalars *, int, int64_t, hipStream_t);
KCT_VINST(float)
KCT_VINST(bf16)
KCT_VINST(_Float16)

#define KCT_ZINST(TS, TD) template hipError_t launch_zfast_copy<TS, TD>(const GeoDev &, const TS *, TD *, hipStream_t);
KCT_ZINST(float, float)
KCT_ZINST(bf16, bf16)
KCT_ZINST(_Float16, _Float16)
KCT_ZINST(double, double)

}  // namespace kct
