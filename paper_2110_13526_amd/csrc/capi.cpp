// capi.cpp -- the extern "C" entry points of kct.h: argument validation,
// workspace layout and the CGLS / LSQR drivers (sequences of kernel launches on
// the caller's stream, no host synchronisation until the final result read).
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kct_internal.h"

namespace kct {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

kct_status geometry_build(const kct_volume_desc &vol, const kct_cone_desc &cone, Geometry *g);

namespace {

// Launch timing of the solvers' projector steps (kct_timing_enable): one HIP
// event pair around every forward and backward launch of a CGLS / LSQR
// iteration, recorded on the solve's stream.  Process-wide; events are
// created on first use and reused.
struct LaunchTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<std::pair<size_t, size_t>> pairs[2];  // per kind (0 forward, 1 backward): start, stop
    hipError_t next(size_t &i)
    {
        if (used == pool.size()) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            pool.push_back(e);
        }
        i = used++;
        return hipSuccess;
    }
    hipError_t begin(hipStream_t st, size_t &i0)
    {
        hipError_t r = next(i0);
        return r != hipSuccess ? r : hipEventRecord(pool[i0], st);
    }
    hipError_t end(int kind, hipStream_t st, size_t i0)
    {
        size_t i1;
        hipError_t r = next(i1);
        if (r == hipSuccess) r = hipEventRecord(pool[i1], st);
        if (r == hipSuccess) pairs[kind].push_back({i0, i1});
        return r;
    }
};
LaunchTimer g_timer;

size_t elem_size(kct_dtype t)
{
    switch (t) {
    case KCT_F32: return 4;
    case KCT_BF16: return 2;
    case KCT_F16: return 2;
    case KCT_F64: return 8;
    default: return 0;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t nvox(const Geometry *g) { return (int64_t)g->dev.nx * g->dev.ny * g->dev.nz; }
int64_t nrays(const Geometry *g) { return (int64_t)g->dev.nviews * g->dev.nv * g->dev.nu; }

int64_t num_partials(const Geometry *g)
{
    // the largest forward grid of every projector and variant (the workspace may
    // be sized before the projector is chosen)
    int64_t a = forward_num_blocks_r(g->dev, 1), b = backward_num_blocks(g->dev), c = stream_num_blocks();
    const int64_t t = tt_forward_num_blocks(g->dev);
    if (t > a) a = t;
    int nbx, nby, nbz;
    const int64_t tb = tt_backward_grid_dims(g->dev, nbx, nby, nbz);
    if (tb > b) b = tb;
    int64_t m = a > b ? a : b;
    return m > c ? m : c;
}

struct SolverLayout {
    size_t scal, part, part2, v0, v1, v2, p0, p1, m2, total;
};

// [Scalars][partials][partials of |d|^2][3 volumes][2 (CGLS) or 1 (LSQR)
// projections][CGLS with Jacobi: one float volume, the preconditioner]
SolverLayout solver_layout(const Geometry *g, kct_dtype t, int solver)
{
    SolverLayout L{};
    const bool jacobi = (solver & KCT_SOLVER_WITH_JACOBI) != 0;
    solver &= ~KCT_SOLVER_WITH_JACOBI;
    size_t es = elem_size(t);
    size_t V = align256((size_t)nvox(g) * es), P = align256((size_t)nrays(g) * es);
    L.scal = 0;
    L.part = align256(sizeof(Scalars));
    L.part2 = L.part + align256((size_t)num_partials(g) * sizeof(double));
    L.v0 = L.part2 + align256((size_t)cgls_d_num_blocks(g->dev) * sizeof(double));
    L.v1 = L.v0 + V;
    L.v2 = L.v1 + V;
    L.p0 = L.v2 + V;
    L.p1 = L.p0 + P;
    L.m2 = (solver == KCT_SOLVER_CGLS) ? L.p1 + P : L.p1;
    L.total = jacobi ? L.m2 + align256((size_t)nvox(g) * sizeof(float)) : L.m2;
    return L;
}

kct_status check_geometry(kct_geometry h, const char *fn)
{
    if (!h) {
        set_error(std::string(fn) + ": geometry is NULL");
        return KCT_ERR_INVALID_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error(std::string(fn) + ": hipGetDevice failed");
        return KCT_ERR_HIP;
    }
    const Geometry *g = reinterpret_cast<const Geometry *>(h);
    if (dev != g->device) {
        set_error(std::string(fn) + ": the current device differs from the device the geometry was created on");
        return KCT_ERR_INVALID_ARG;
    }
    return KCT_OK;
}

kct_status check_dtype(kct_dtype t, const char *fn)
{
    if (elem_size(t) == 0) {
        set_error(std::string(fn) + ": unknown storage type");
        return KCT_ERR_UNSUPPORTED;
    }
    return KCT_OK;
}

// The solvers run on the 32- and 16-bit storage types; double storage is
// offered for the projector pair only.
kct_status check_solver_dtype(kct_dtype t, const char *fn)
{
    kct_status s = check_dtype(t, fn);
    if (s != KCT_OK) return s;
    if (t == KCT_F64) {
        set_error(std::string(fn) + ": the solvers do not support double storage (use F32, BF16 or F16)");
        return KCT_ERR_UNSUPPORTED;
    }
    return KCT_OK;
}

bool misaligned(const void *p) { return ((uintptr_t)p & 15u) != 0; }

template <typename T> kct_dtype dtype_of();
template <> kct_dtype dtype_of<float>() { return KCT_F32; }
template <> kct_dtype dtype_of<bf16>() { return KCT_BF16; }
template <> kct_dtype dtype_of<_Float16>() { return KCT_F16; }

#define KCT_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            set_error(std::string(fn) + ": " #expr " failed: " + hipGetErrorString(e_));         \
            return KCT_ERR_HIP;                                                                  \
        }                                                                                        \
    } while (0)

// A projector launch of a solver iteration, timed when kct_timing_enable is on
// (kind 0 forward, 1 backward).
#define KCT_TIMED(kind, st, expr)                                                                \
    do {                                                                                         \
        size_t i0_ = 0;                                                                          \
        if (g_timer.on) KCT_TRY(g_timer.begin(st, i0_));                                         \
        KCT_TRY(expr);                                                                           \
        if (g_timer.on) KCT_TRY(g_timer.end(kind, st, i0_));                                     \
    } while (0)

struct StorageScales {
    double sr, sp, sw;
};

// Scalars at the start of a solve.  lambda: CGLS Tikhonov parameter (tik,
// applied through r and NP2) or LSQR damping (damp).
__global__ void k_init_scalars(Scalars *sc, int maxiter, double err, double *history, StorageScales ss,
                               double tik, double damp)
{
    if (threadIdx.x != 0) return;
    Scalars s;
    memset(&s, 0, sizeof(s));
    s.maxiter = maxiter;
    s.err = err;
    s.history = history;
    s.sr = ss.sr;
    s.sp = ss.sp;
    s.sw = ss.sw;
    s.fwd_scale = (float)(ss.sr / ss.sp);
    s.bwd_scale = (float)(1.0 / ss.sr);
    s.tik_r = (float)(tik * tik / ss.sr);   // r_stored = A^T e / sr - (lambda^2 / sr) x
    s.tik_d2 = tik * tik * ss.sr * ss.sr;   // lambda^2 |d|^2 with d = sr * d_stored
    s.damp = damp;
    *sc = s;
}

double pow2_at_least(double v) { return std::exp2(std::ceil(std::log2(v))); }

// Storage scales of the solvers' work vectors.  FP32 and BF16 have the range
// of single precision and use 1 (every scaling is then an exact no-op).  FP16
// (largest finite 65504, smallest normal 6.1e-5) stores, as powers of two:
//  - CGLS r and d divided by a bound C on the column sums of A, so that
//    |r| <= C |e|_inf stays on the scale of e (and b); p divided by C R,
//    with R a bound on the row sums of A, so |p| <= R |d| does too;
//  - LSQR w, which is a unit-norm vector of n elements, multiplied by
//    about sqrt(n) so its elements are of order one.
// Bounds: a ray crosses the volume over at most its diagonal (R); in one view
// a voxel meets the rays of at most (footprint columns) x (footprint rows)
// pixels, each over at most the voxel diagonal (C).
StorageScales storage_scales(const Geometry *g, kct_dtype t)
{
    StorageScales s{1.0, 1.0, 1.0};
    if (t != KCT_F16) return s;
    const kct_volume_desc &v = g->vol;
    const kct_cone_desc &c = g->cone;
    const double ex = v.nx * v.vx, ey = v.ny * v.vy, ez = v.nz * v.vz;
    const double R = std::sqrt(ex * ex + ey * ey + ez * ez);
    double rmax = 0.0;  // largest distance of a volume corner from the rotation axis
    for (int i = 0; i < 4; ++i) {
        const double x = v.cx + ((i & 1) ? 0.5 : -0.5) * ex, y = v.cy + ((i & 2) ? 0.5 : -0.5) * ey;
        rmax = std::fmax(rmax, std::sqrt(x * x + y * y));
    }
    const double mag = c.sdd / std::fmax(c.sid - rmax, 1e-6 * c.sid);  // the volume lies inside the orbit
    const double dvox = std::sqrt(v.vx * v.vx + v.vy * v.vy + v.vz * v.vz);
    const double dxy = std::sqrt(v.vx * v.vx + v.vy * v.vy);
    const double cols = std::ceil(mag * dxy / c.du) + 1.0, rows = std::ceil(mag * dvox / c.dv) + 1.0;
    const double C = (double)c.n_views * cols * rows * dvox;
    s.sr = pow2_at_least(C);
    s.sp = s.sr * pow2_at_least(R);
    s.sw = 1.0 / pow2_at_least(std::sqrt((double)nvox(g)));
    return s;
}

template <typename T>
kct_status project_t(const Geometry *g, const void *x, void *b, void *ws, hipStream_t st)
{
    const char *fn = "kct_project";
    const T *vol = (const T *)x;
    T *vz = nullptr;
    if (ws) {
        vz = (T *)ws;
        KCT_TRY((launch_zfast_copy<T, T>(g->dev, vol, vz, st)));
    }
    KCT_TRY((launch_forward<T, T>(g->dev, vol, vz, (T *)b, nullptr, FWD_PLAIN, nullptr, nullptr, nullptr, st)));
    return KCT_OK;
}

template <typename T>
kct_status backproject_t(const Geometry *g, const void *b, void *x, hipStream_t st)
{
    const char *fn = "kct_backproject";
    KCT_TRY(launch_backward<T>(g->dev, (const T *)b, (T *)x, nullptr, BWD_PLAIN, nullptr, nullptr, nullptr, st));
    return KCT_OK;
}

template <typename T>
kct_status read_info(Scalars *sc, kct_solve_info *info, hipStream_t st, const char *fn, int solver)
{
    Scalars h;
    KCT_TRY(hipMemcpyAsync(&h, sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    KCT_TRY(hipStreamSynchronize(st));
    if (info) {
        info->iterations = h.iters;
        info->nb0 = h.nb0;
        info->nb = h.nb;
        info->nr2 = solver == KCT_SOLVER_CGLS ? h.nr2_old : h.nr2_now;
        info->stop_reason = h.done ? h.stop : KCT_STOP_MAXITER;
    }
    if (h.done && h.stop == KCT_STOP_NUMERIC) {
        set_error(std::string(fn) + ": a solver norm became NaN or Inf");
        return KCT_ERR_NUMERIC;
    }
    return KCT_OK;
}

// CGLS with delayed residual computation (Algorithm 1), with the options of
// kct_solve_opts: Tikhonov term (CGLS on [A; lambda I]: r = A^T e - lambda^2 x,
// NP2 = |A d|^2 + lambda^2 |d|^2), Jacobi right preconditioning (r = M^2 A^T e
// is stored, so d and x stay in the unpreconditioned space and NR2 = |M A^T e|^2
// comes from the epilogue's partials), periodic recomputation of e.
template <typename T>
kct_status cgls_t(const Geometry *g, const void *bv, void *xv, const kct_solve_opts *o, void *ws,
                  kct_solve_info *info, hipStream_t st)
{
    const char *fn = "kct_cgls_solve";
    const bool jacobi = o->jacobi != 0;
    const double lambda = o->tikhonov;
    const int re = o->recompute_every;
    const SolverLayout L =
        solver_layout(g, dtype_of<T>(), KCT_SOLVER_CGLS | (jacobi ? KCT_SOLVER_WITH_JACOBI : 0));
    char *w = (char *)ws;
    Scalars *sc = (Scalars *)(w + L.scal);
    double *part = (double *)(w + L.part);
    double *dpart = lambda > 0.0 ? (double *)(w + L.part2) : nullptr;
    T *d = (T *)(w + L.v0), *dz = (T *)(w + L.v1), *r = (T *)(w + L.v2);
    T *e = (T *)(w + L.p0), *p = (T *)(w + L.p1);
    float *m2 = jacobi ? (float *)(w + L.m2) : nullptr;
    const T *b = (const T *)bv;
    float *x = (float *)xv;
    const GeoDev &G = g->dev;
    const int64_t n = nvox(g), m = nrays(g);
    const int64_t nf = forward_num_blocks(G), nbk = backward_num_blocks(G), ns = stream_num_blocks();
    const int64_t nd = lambda > 0.0 ? cgls_d_num_blocks(G) : 0;
    const int K = o->max_iter;
    const int *done = &sc->done;
    // r = A^T e in the variant's form; aux is x (Tikhonov) or M^2 (Jacobi)
    const int repi = jacobi ? BWD_JACOBI : (lambda > 0.0 ? BWD_TIK : BWD_NORM);
    const float *raux = jacobi ? m2 : (lambda > 0.0 ? x : nullptr);

    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, st, sc, K, o->err_tol, o->history,
                       storage_scales(g, dtype_of<T>()), lambda, 0.0);
    KCT_TRY(hipGetLastError());
    if (jacobi)  // M^2 = 1 / diag(A^T A), 0 where the diagonal is 0
        KCT_TRY(launch_backward<float>(G, nullptr, m2, nullptr, BWD_DIAG_INV, nullptr, nullptr, nullptr, st));
    // NB0 = |b|
    KCT_TRY(launch_norm2<T>(b, m, part, nullptr, st));
    KCT_TRY(launch_finalize(sc, part, ns, F_NB0, st));
    // x = x0; p = A x; e = b - p
    if (o->x0_is_zero) {
        KCT_TRY(launch_fill_zero<float>(x, n, st));
        KCT_TRY(launch_copy<T>(b, e, m, st));
    } else {
        // single-precision z-fastest copy of x0 in the (not yet used) d and d_z space
        float *xz0 = (float *)(w + L.v0);
        KCT_TRY((launch_zfast_copy<float, float>(G, x, xz0, st)));
        KCT_TRY((launch_forward<float, T>(G, x, xz0, e, b, FWD_BMINUS, sc, part, done, st)));
        KCT_TRY(launch_finalize(sc, part, nf, F_NB_INIT, st));
    }
    // x += alpha d; e -= alpha p (or e = b - A x every re-th iteration); NB; i = i + 1
    auto step_end = [&](int i) -> kct_status {
        KCT_TRY(launch_cgls_x<T>(x, d, sc, n, st));
        if (re > 0 && i % re == 0) {
            KCT_TRY((launch_forward<float, T>(G, x, nullptr, e, b, FWD_BMINUS, sc, part, done, st)));
            KCT_TRY(launch_finalize(sc, part, nf, F_NB, st));
        } else {
            KCT_TRY(launch_cgls_e<T>(e, p, sc, m, part, st));
            KCT_TRY(launch_finalize(sc, part, ns, F_NB, st));
        }
        return KCT_OK;
    };
    // r = A^T e; d = r; NR2_old = |r|^2
    KCT_TIMED(1, st, (launch_backward<T>(G, e, r, nullptr, repi, sc, part, done, st, raux)));
    KCT_TRY(launch_finalize(sc, part, nbk, F_NR2_INIT, st));
    KCT_TRY(launch_cgls_d<T>(G, r, d, dz, sc, 1, st, dpart));
    // p = A d; NP2 = |p|^2 (+ lambda^2 |d|^2); alpha = NR2_old / NP2
    KCT_TIMED(0, st, (launch_forward<T, T>(G, d, dz, p, nullptr, FWD_NORM, sc, part, done, st)));
    KCT_TRY(launch_finalize(sc, part, nf, F_ALPHA, st, dpart, nd));
    kct_status s = step_end(1);
    if (s != KCT_OK) return s;
    for (int it = 1; it < K; ++it) {
        // r = A^T e; NR2_now = |r|^2; beta = NR2_now / NR2_old; NR2_old = NR2_now
        KCT_TIMED(1, st, (launch_backward<T>(G, e, r, nullptr, repi, sc, part, done, st, raux)));
        KCT_TRY(launch_finalize(sc, part, nbk, F_BETA, st));
        // d = r + beta d
        KCT_TRY(launch_cgls_d<T>(G, r, d, dz, sc, 0, st, dpart));
        // p = A d; NP2; alpha
        KCT_TIMED(0, st, (launch_forward<T, T>(G, d, dz, p, nullptr, FWD_NORM, sc, part, done, st)));
        KCT_TRY(launch_finalize(sc, part, nf, F_ALPHA, st, dpart, nd));
        if ((s = step_end(it + 1)) != KCT_OK) return s;
    }
    return read_info<T>(sc, info, st, fn, KCT_SOLVER_CGLS);
}

// LSQR (Paige & Saunders) with the normalisations of u and v folded into the
// fused epilogues: u = u_hat / beta and v = v_hat / alpha are never formed.
template <typename T>
kct_status lsqr_t(const Geometry *g, const void *bv, void *xv, const kct_solve_opts *o, void *ws,
                  kct_solve_info *info, hipStream_t st)
{
    const char *fn = "kct_lsqr_solve";
    const SolverLayout L = solver_layout(g, dtype_of<T>(), KCT_SOLVER_LSQR);
    char *wp = (char *)ws;
    Scalars *sc = (Scalars *)(wp + L.scal);
    double *part = (double *)(wp + L.part);
    T *v = (T *)(wp + L.v0), *vz = (T *)(wp + L.v1), *w = (T *)(wp + L.v2);
    T *u = (T *)(wp + L.p0);
    const T *b = (const T *)bv;
    float *x = (float *)xv;
    const GeoDev &G = g->dev;
    const int64_t n = nvox(g), m = nrays(g);
    const int64_t nf = forward_num_blocks(G), nbk = backward_num_blocks(G), ns = stream_num_blocks();
    const int K = o->max_iter;
    const int *done = &sc->done;

    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, st, sc, K, o->err_tol, o->history,
                       storage_scales(g, dtype_of<T>()), 0.0, o->tikhonov);
    KCT_TRY(hipGetLastError());
    KCT_TRY(launch_norm2<T>(b, m, part, nullptr, st));
    KCT_TRY(launch_finalize(sc, part, ns, F_NB0, st));
    // beta u = b - A x0
    if (o->x0_is_zero) {
        KCT_TRY(launch_fill_zero<float>(x, n, st));
        KCT_TRY(launch_copy<T>(b, u, m, st));
        KCT_TRY(launch_norm2<T>(u, m, part, done, st));
        KCT_TRY(launch_finalize(sc, part, ns, F_L_BETA0, st));
    } else {
        // single-precision z-fastest copy of x0 in the (not yet used) v and v_z space
        float *xz0 = (float *)(wp + L.v0);
        KCT_TRY((launch_zfast_copy<float, float>(G, x, xz0, st)));
        KCT_TRY((launch_forward<float, T>(G, x, xz0, u, b, FWD_BMINUS, sc, part, done, st)));
        KCT_TRY(launch_finalize(sc, part, nf, F_L_BETA0, st));
    }
    // alpha v = A^T u; w = v
    KCT_TIMED(1, st, (launch_backward<T>(G, u, v, vz, BWD_LSQR0, sc, part, done, st)));
    KCT_TRY(launch_finalize(sc, part, nbk, F_L_ALPHA0, st));
    KCT_TRY(launch_lsqr_xw<T>(x, w, v, sc, 1, n, st));
    for (int it = 0; it < K; ++it) {
        // beta u = A v - alpha u
        KCT_TIMED(0, st, (launch_forward<T, T>(G, v, vz, u, nullptr, FWD_LSQR, sc, part, done, st)));
        KCT_TRY(launch_finalize(sc, part, nf, F_L_BETA, st));
        // alpha v = A^T u - beta v (skipped on the last iteration), Givens rotation
        KCT_TIMED(1, st, (launch_backward<T>(G, u, v, vz, BWD_LSQR, sc, part, &sc->skip_bwd, st)));
        KCT_TRY(launch_finalize(sc, part, nbk, F_L_ALPHA, st));
        // x += (phi / rho) w; w = v - (theta / rho) w
        KCT_TRY(launch_lsqr_xw<T>(x, w, v, sc, 0, n, st));
        KCT_TRY(launch_finalize(sc, part, 0, F_L_GIVENS, st));
    }
    return read_info<T>(sc, info, st, fn, KCT_SOLVER_LSQR);
}

kct_status check_solve_args(kct_geometry h, kct_dtype t, const void *b, void *x, const kct_solve_opts *o, void *ws,
                            size_t ws_bytes, int solver, const char *fn)
{
    kct_status s = check_geometry(h, fn);
    if (s != KCT_OK) return s;
    if ((s = check_solver_dtype(t, fn)) != KCT_OK) return s;
    if (!b || !x || !o) {
        set_error(std::string(fn) + ": b, x and opts must not be NULL");
        return KCT_ERR_INVALID_ARG;
    }
    if (misaligned(b) || misaligned(x) || misaligned(ws)) {
        set_error(std::string(fn) + ": buffers must be 16-byte aligned");
        return KCT_ERR_INVALID_ARG;
    }
    if (o->max_iter < 0 || !(o->err_tol >= 0.0) || !std::isfinite(o->err_tol)) {
        set_error(std::string(fn) + ": max_iter must be >= 0 and err_tol finite and >= 0");
        return KCT_ERR_INVALID_ARG;
    }
    if (!(o->tikhonov >= 0.0) || !std::isfinite(o->tikhonov) || o->recompute_every < 0) {
        set_error(std::string(fn) + ": tikhonov must be finite and >= 0, recompute_every >= 0");
        return KCT_ERR_INVALID_ARG;
    }
    if (solver == KCT_SOLVER_LSQR && (o->jacobi || o->recompute_every)) {
        set_error(std::string(fn) + ": jacobi and recompute_every are CGLS options");
        return KCT_ERR_INVALID_ARG;
    }
    if (solver == KCT_SOLVER_LSQR && o->tikhonov > 0.0 && !o->x0_is_zero) {
        set_error(std::string(fn) + ": LSQR with tikhonov > 0 needs x0 = 0 (its damping penalises x - x0)");
        return KCT_ERR_UNSUPPORTED;
    }
    if (o->jacobi && (o->tikhonov > 0.0 || t == KCT_F16)) {
        set_error(std::string(fn) + ": jacobi is not available with tikhonov > 0 or F16 storage");
        return KCT_ERR_UNSUPPORTED;
    }
    const Geometry *g = reinterpret_cast<const Geometry *>(h);
    if (o->jacobi) solver |= KCT_SOLVER_WITH_JACOBI;
    size_t need = solver_layout(g, t, solver).total;
    if (!ws || ws_bytes < need) {
        set_error(std::string(fn) + ": workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                  std::to_string(need));
        return KCT_ERR_WORKSPACE;
    }
    return KCT_OK;
}

}  // namespace
}  // namespace kct

using namespace kct;

extern "C" {

kct_status kct_geometry_create(const kct_volume_desc *vol, const kct_cone_desc *cone, kct_geometry *out)
{
    if (!vol || !cone || !out) {
        set_error("kct_geometry_create: NULL argument");
        return KCT_ERR_INVALID_ARG;
    }
    *out = nullptr;
    Geometry *g = new (std::nothrow) Geometry();
    if (!g) {
        set_error("kct_geometry_create: out of host memory");
        return KCT_ERR_INVALID_ARG;
    }
    kct_status s = geometry_build(*vol, *cone, g);
    if (s != KCT_OK) {
        delete g;
        return s;
    }
    *out = reinterpret_cast<kct_geometry>(g);
    return KCT_OK;
}

void kct_geometry_destroy(kct_geometry h)
{
    if (!h) return;
    Geometry *g = reinterpret_cast<Geometry *>(h);
    if (g->d_tables) (void)hipFree(g->d_tables);
    delete g;
}

kct_status kct_geometry_set_projector(kct_geometry h, int32_t projector)
{
    if (!h) {
        set_error("kct_geometry_set_projector: geometry is NULL");
        return KCT_ERR_INVALID_ARG;
    }
    if (projector != KCT_PROJECTOR_SIDDON && projector != KCT_PROJECTOR_TT) {
        set_error("kct_geometry_set_projector: unknown projector");
        return KCT_ERR_INVALID_ARG;
    }
    reinterpret_cast<Geometry *>(h)->dev.projector = projector;
    return KCT_OK;
}

kct_status kct_geometry_dims(kct_geometry h, int64_t *n_vox, int64_t *n_rays)
{
    if (!h) {
        set_error("kct_geometry_dims: geometry is NULL");
        return KCT_ERR_INVALID_ARG;
    }
    const Geometry *g = reinterpret_cast<const Geometry *>(h);
    if (n_vox) *n_vox = nvox(g);
    if (n_rays) *n_rays = nrays(g);
    return KCT_OK;
}

kct_status kct_project_workspace_size(kct_geometry h, kct_dtype t, size_t *bytes)
{
    if (!h || !bytes) {
        set_error("kct_project_workspace_size: NULL argument");
        return KCT_ERR_INVALID_ARG;
    }
    kct_status s = check_dtype(t, "kct_project_workspace_size");
    if (s != KCT_OK) return s;
    *bytes = (size_t)nvox(reinterpret_cast<const Geometry *>(h)) * elem_size(t);
    return KCT_OK;
}

kct_status kct_project(kct_geometry h, kct_dtype t, const void *x, void *b, void *ws, size_t ws_bytes,
                       hipStream_t stream)
{
    const char *fn = "kct_project";
    kct_status s = check_geometry(h, fn);
    if (s != KCT_OK) return s;
    if ((s = check_dtype(t, fn)) != KCT_OK) return s;
    if (!x || !b) {
        set_error("kct_project: x and b must not be NULL");
        return KCT_ERR_INVALID_ARG;
    }
    if (misaligned(x) || misaligned(b) || misaligned(ws)) {
        set_error("kct_project: buffers must be 16-byte aligned");
        return KCT_ERR_INVALID_ARG;
    }
    const Geometry *g = reinterpret_cast<const Geometry *>(h);
    if (ws && ws_bytes < (size_t)nvox(g) * elem_size(t)) {
        set_error("kct_project: workspace smaller than kct_project_workspace_size");
        return KCT_ERR_WORKSPACE;
    }
    switch (t) {
    case KCT_F32: return project_t<float>(g, x, b, ws, stream);
    case KCT_BF16: return project_t<bf16>(g, x, b, ws, stream);
    case KCT_F16: return project_t<_Float16>(g, x, b, ws, stream);
    default: return project_t<double>(g, x, b, ws, stream);
    }
}

kct_status kct_backproject(kct_geometry h, kct_dtype t, const void *b, void *x, hipStream_t stream)
{
    const char *fn = "kct_backproject";
    kct_status s = check_geometry(h, fn);
    if (s != KCT_OK) return s;
    if ((s = check_dtype(t, fn)) != KCT_OK) return s;
    if (!x || !b) {
        set_error("kct_backproject: b and x must not be NULL");
        return KCT_ERR_INVALID_ARG;
    }
    if (misaligned(x) || misaligned(b)) {
        set_error("kct_backproject: buffers must be 16-byte aligned");
        return KCT_ERR_INVALID_ARG;
    }
    const Geometry *g = reinterpret_cast<const Geometry *>(h);
    switch (t) {
    case KCT_F32: return backproject_t<float>(g, b, x, stream);
    case KCT_BF16: return backproject_t<bf16>(g, b, x, stream);
    case KCT_F16: return backproject_t<_Float16>(g, b, x, stream);
    default: return backproject_t<double>(g, b, x, stream);
    }
}

kct_status kct_solver_workspace_size(kct_geometry h, kct_dtype t, int32_t solver, size_t *bytes)
{
    if (!h || !bytes) {
        set_error("kct_solver_workspace_size: NULL argument");
        return KCT_ERR_INVALID_ARG;
    }
    kct_status s = check_solver_dtype(t, "kct_solver_workspace_size");
    if (s != KCT_OK) return s;
    if (solver != KCT_SOLVER_CGLS && solver != KCT_SOLVER_LSQR &&
        solver != (KCT_SOLVER_CGLS | KCT_SOLVER_WITH_JACOBI)) {
        set_error("kct_solver_workspace_size: unknown solver");
        return KCT_ERR_INVALID_ARG;
    }
    *bytes = solver_layout(reinterpret_cast<const Geometry *>(h), t, solver).total;
    return KCT_OK;
}

kct_status kct_cgls_solve(kct_geometry h, kct_dtype t, const void *b, void *x, const kct_solve_opts *opts, void *ws,
                          size_t ws_bytes, kct_solve_info *info, hipStream_t stream)
{
    kct_status s = check_solve_args(h, t, b, x, opts, ws, ws_bytes, KCT_SOLVER_CGLS, "kct_cgls_solve");
    if (s != KCT_OK) return s;
    const Geometry *g = reinterpret_cast<const Geometry *>(h);
    switch (t) {
    case KCT_F32: return cgls_t<float>(g, b, x, opts, ws, info, stream);
    case KCT_BF16: return cgls_t<bf16>(g, b, x, opts, ws, info, stream);
    default: return cgls_t<_Float16>(g, b, x, opts, ws, info, stream);
    }
}

kct_status kct_lsqr_solve(kct_geometry h, kct_dtype t, const void *b, void *x, const kct_solve_opts *opts, void *ws,
                          size_t ws_bytes, kct_solve_info *info, hipStream_t stream)
{
    kct_status s = check_solve_args(h, t, b, x, opts, ws, ws_bytes, KCT_SOLVER_LSQR, "kct_lsqr_solve");
    if (s != KCT_OK) return s;
    const Geometry *g = reinterpret_cast<const Geometry *>(h);
    switch (t) {
    case KCT_F32: return lsqr_t<float>(g, b, x, opts, ws, info, stream);
    case KCT_BF16: return lsqr_t<bf16>(g, b, x, opts, ws, info, stream);
    default: return lsqr_t<_Float16>(g, b, x, opts, ws, info, stream);
    }
}

kct_status kct_diag_normal(kct_geometry h, float *out, hipStream_t stream)
{
    const char *fn = "kct_diag_normal";
    kct_status s = check_geometry(h, fn);
    if (s != KCT_OK) return s;
    if (!out || misaligned(out)) {
        set_error("kct_diag_normal: out must be a 16-byte aligned device pointer");
        return KCT_ERR_INVALID_ARG;
    }
    const Geometry *g = reinterpret_cast<const Geometry *>(h);
    KCT_TRY(launch_backward<float>(g->dev, nullptr, out, nullptr, BWD_DIAG, nullptr, nullptr, nullptr, stream));
    return KCT_OK;
}

kct_status kct_timing_enable(int32_t on)
{
    g_timer.on = on != 0;
    g_timer.used = 0;
    g_timer.pairs[0].clear();
    g_timer.pairs[1].clear();
    return KCT_OK;
}

kct_status kct_timing_get(int32_t kind, int32_t *count, double *avg_ms, double *min_ms, double *max_ms)
{
    const char *fn = "kct_timing_get";
    if ((kind != 0 && kind != 1) || !count || !avg_ms || !min_ms || !max_ms) {
        set_error("kct_timing_get: kind must be 0 or 1 and the outputs non-NULL");
        return KCT_ERR_INVALID_ARG;
    }
    double sum = 0.0, lo = 0.0, hi = 0.0;
    int32_t n = 0;
    for (const auto &pr : g_timer.pairs[kind]) {
        KCT_TRY(hipEventSynchronize(g_timer.pool[pr.second]));
        float ms = 0.0f;
        KCT_TRY(hipEventElapsedTime(&ms, g_timer.pool[pr.first], g_timer.pool[pr.second]));
        lo = n == 0 ? ms : (ms < lo ? ms : lo);
        hi = n == 0 ? ms : (ms > hi ? ms : hi);
        sum += ms;
        ++n;
    }
    *count = n;
    *avg_ms = n ? sum / n : 0.0;
    *min_ms = lo;
    *max_ms = hi;
    return KCT_OK;
}

const char *kct_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
