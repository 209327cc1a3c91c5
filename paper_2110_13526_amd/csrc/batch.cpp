// batch.cpp -- batched CGLS (Section 2, Algorithm 1) over many independent
// reconstructions: the kct_batch_* entry points of kct.h.
//
// Every step of an iteration is one launch that covers all instances (the
// batched kernels of projector.hip, backproject.hip and vector_ops.hip); each
// instance keeps its own FP64 scalars, partial sums and stop flag, so a batch
// computes exactly what the instances' separate solves compute.  The steps of
// one iteration are recorded once as a HIP graph on the batch's own stream and
// replayed K - 1 times.  Instances are laid out in the batched grids largest
// first, so the small ones fill the tail of each launch.
//
// The autotuner picks, per instance, the forward variant (1 or 2 detector rows
// per lane) by timing both on the instance's geometry, and can keep its choices
// in a text file keyed by the instance's sizes.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "kct_internal.h"

namespace kct {

void set_error(const std::string &msg);

struct Batch {
    std::vector<const Geometry *> geoms;
    std::vector<int> fwd_r;   // per instance, 1 or 2
    std::vector<int> order;   // grid order: instance indices, largest work first
    int device = -1;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t pad64(int64_t x) { return (x + 63) & ~(int64_t)63; }

int64_t inst_n(const Geometry *g) { return (int64_t)g->dev.nx * g->dev.ny * g->dev.nz; }
int64_t inst_m(const Geometry *g) { return (int64_t)g->dev.nviews * g->dev.nv * g->dev.nu; }

int64_t inst_partials(const Geometry *g)
{
    int64_t a = std::max(forward_num_blocks_r(g->dev, 1), forward_num_blocks_r(g->dev, 2));
    int nbx, nby, nbz;
    int64_t b = backward_grid_dims(g->dev, nbx, nby, nbz);  // the batched backprojection's grid
    return std::max(std::max(a, b), stream_num_blocks());
}

// [BatchInst table][offset tables][per instance: Scalars | partials | d | dz | r | e | p]
struct BatchLayout {
    size_t table, offs, total;
    std::vector<size_t> base;  // start of each instance's block
    std::vector<size_t> part, d, dz, r, e, p;
};

BatchLayout batch_layout(const Batch *b)
{
    BatchLayout L;
    const size_t c = b->geoms.size();
    L.table = 0;
    L.offs = a256(c * sizeof(BatchInst));
    size_t at = L.offs + a256((size_t)BG_COUNT * (c + 1) * sizeof(int64_t));
    for (size_t i = 0; i < c; ++i) {
        const Geometry *g = b->geoms[i];
        const size_t V = a256((size_t)inst_n(g) * sizeof(float)), P = a256((size_t)inst_m(g) * sizeof(float));
        L.base.push_back(at);
        L.part.push_back(at + a256(sizeof(Scalars)));
        L.d.push_back(L.part.back() + a256((size_t)inst_partials(g) * sizeof(double)));
        L.dz.push_back(L.d.back() + V);
        L.r.push_back(L.dz.back() + V);
        L.e.push_back(L.r.back() + V);
        L.p.push_back(L.e.back() + P);
        at = L.p.back() + P;
    }
    L.total = at;
    return L;
}

std::string size_key(const Geometry *g)
{
    std::ostringstream o;
    o << g->dev.nx << 'x' << g->dev.ny << 'x' << g->dev.nz << '/' << g->dev.nviews << 'x' << g->dev.nv << 'x'
      << g->dev.nu;
    return o.str();
}

kct_status fail(const char *fn, const std::string &what, kct_status s)
{
    set_error(std::string(fn) + ": " + what);
    return s;
}

#define KCT_BTRY(expr)                                                                                   \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return fail(fn, std::string(#expr " failed: ") + hipGetErrorString(e_), KCT_ERR_HIP); \
    } while (0)

kct_status check_batch(kct_batch h, const char *fn, Batch *&b)
{
    b = reinterpret_cast<Batch *>(h);
    if (!b) return fail(fn, "batch is NULL", KCT_ERR_INVALID_ARG);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(fn, "hipGetDevice failed", KCT_ERR_HIP);
    if (dev != b->device) return fail(fn, "the current device differs from the batch's device", KCT_ERR_INVALID_ARG);
    return KCT_OK;
}

// One batched iteration after the init block: r = A^T e, beta, d = r + beta d,
// p = A d, alpha, x += alpha d, e -= alpha p, NB.
hipError_t batch_iteration(const BatchInst *T, const int64_t *off, int c, const int64_t *nblk, hipStream_t st)
{
    hipError_t e;
    if ((e = launch_batch_backward(T, off + BG_BWD * (c + 1), c, nblk[BG_BWD], st)) != hipSuccess) return e;
    if ((e = launch_batch_finalize(T, c, F_BETA, BG_BWD, st)) != hipSuccess) return e;
    if ((e = launch_batch_dir(T, off + BG_DIR * (c + 1), c, nblk[BG_DIR], 0, st)) != hipSuccess) return e;
    if ((e = launch_batch_forward(T, off + BG_FWD * (c + 1), c, nblk[BG_FWD], st)) != hipSuccess) return e;
    if ((e = launch_batch_finalize(T, c, F_ALPHA, BG_FWD, st)) != hipSuccess) return e;
    if ((e = launch_batch_vec(T, c, BV_CGLS_X, 0, 0.0, st)) != hipSuccess) return e;
    if ((e = launch_batch_vec(T, c, BV_CGLS_E, 0, 0.0, st)) != hipSuccess) return e;
    return launch_batch_finalize(T, c, F_NB, BG_STREAM, st);
}

}  // namespace
}  // namespace kct

using namespace kct;

extern "C" {

kct_status kct_batch_create(const kct_geometry *geoms, int32_t count, kct_batch *out)
{
    const char *fn = "kct_batch_create";
    if (!geoms || !out || count <= 0) return fail(fn, "geoms and out must be given and count > 0", KCT_ERR_INVALID_ARG);
    *out = nullptr;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(fn, "hipGetDevice failed", KCT_ERR_HIP);
    Batch *b = new (std::nothrow) Batch();
    if (!b) return fail(fn, "out of host memory", KCT_ERR_INVALID_ARG);
    b->device = dev;
    for (int i = 0; i < count; ++i) {
        const Geometry *g = reinterpret_cast<const Geometry *>(geoms[i]);
        if (!g || g->device != dev || g->dev.projector != KCT_PROJECTOR_SIDDON) {
            delete b;
            return fail(fn, "geometry " + std::to_string(i) + " is NULL, on another device or not a Siddon geometry",
                        KCT_ERR_INVALID_ARG);
        }
        b->geoms.push_back(g);
        b->fwd_r.push_back(2);
        b->order.push_back(i);
    }
    // largest work (rays x voxels along a ray ~ rays * side) first
    std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) {
        const double wa = (double)inst_m(b->geoms[a]) * b->geoms[a]->dev.nx;
        const double wc = (double)inst_m(b->geoms[c]) * b->geoms[c]->dev.nx;
        return wa > wc;
    });
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) {
        if (b->stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return fail(fn, "stream or event creation failed", KCT_ERR_HIP);
    }
    *out = reinterpret_cast<kct_batch>(b);
    return KCT_OK;
}

void kct_batch_destroy(kct_batch h)
{
    Batch *b = reinterpret_cast<Batch *>(h);
    if (!b) return;
    if (b->stream) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipStreamDestroy(b->stream);
    }
    if (b->ev) (void)hipEventDestroy(b->ev);
    delete b;
}

kct_status kct_batch_workspace_size(kct_batch h, size_t *bytes)
{
    const char *fn = "kct_batch_workspace_size";
    Batch *b = nullptr;
    kct_status s = check_batch(h, fn, b);
    if (s != KCT_OK) return s;
    if (!bytes) return fail(fn, "bytes is NULL", KCT_ERR_INVALID_ARG);
    *bytes = batch_layout(b).total;
    return KCT_OK;
}

kct_status kct_batch_tune(kct_batch h, void *ws, size_t ws_bytes, const char *cache_path, hipStream_t stream)
{
    const char *fn = "kct_batch_tune";
    Batch *b = nullptr;
    kct_status s = check_batch(h, fn, b);
    if (s != KCT_OK) return s;
    const BatchLayout L = batch_layout(b);
    if (!ws || ws_bytes < L.total) return fail(fn, "workspace smaller than kct_batch_workspace_size", KCT_ERR_WORKSPACE);
    std::map<std::string, int> known;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string key;
        int r;
        while (in >> key >> r)
            if (r == 1 || r == 2) known[key] = r;
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    KCT_BTRY(hipEventCreate(&t0));
    KCT_BTRY(hipEventCreate(&t1));
    std::vector<std::string> fresh;
    kct_status rc = KCT_OK;
    char *w = (char *)ws;
    for (size_t i = 0; i < b->geoms.size() && rc == KCT_OK; ++i) {
        const Geometry *g = b->geoms[i];
        const std::string key = size_key(g);
        auto it = known.find(key);
        if (it != known.end()) {
            b->fwd_r[i] = it->second;
            continue;
        }
        float *d = (float *)(w + L.d[i]), *dz = (float *)(w + L.dz[i]), *p = (float *)(w + L.p[i]);
        hipError_t e = launch_fill_zero<float>(d, inst_n(g), stream);
        if (e == hipSuccess) e = launch_zfast_copy<float, float>(g->dev, d, dz, stream);
        float best = 0.0f;
        int best_r = 2;
        for (int r = 1; r <= 2 && e == hipSuccess; ++r) {
            e = launch_forward_r(g->dev, d, dz, p, r, stream);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(t0, stream);
            for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) e = launch_forward_r(g->dev, d, dz, p, r, stream);
            if (e == hipSuccess) e = hipEventRecord(t1, stream);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e == hipSuccess && (r == 1 || ms < best)) {
                best = ms;
                best_r = r;
            }
        }
        if (e != hipSuccess) {
            rc = fail(fn, std::string("timing failed: ") + hipGetErrorString(e), KCT_ERR_HIP);
            break;
        }
        b->fwd_r[i] = best_r;
        known[key] = best_r;
        fresh.push_back(key);
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (rc == KCT_OK && cache_path && !fresh.empty()) {
        std::ofstream o(cache_path, std::ios::app);
        for (const auto &k : fresh) o << k << ' ' << known[k] << '\n';
    }
    return rc;
}

kct_status kct_batch_cgls_solve(kct_batch h, const float *const *bs, float *const *xs, const kct_solve_opts *opts,
                                int32_t use_graph, void *ws, size_t ws_bytes, kct_solve_info *infos,
                                hipStream_t stream)
{
    const char *fn = "kct_batch_cgls_solve";
    Batch *b = nullptr;
    kct_status s = check_batch(h, fn, b);
    if (s != KCT_OK) return s;
    const int c = (int)b->geoms.size();
    if (!bs || !xs || !opts || !infos) return fail(fn, "bs, xs, opts and infos must not be NULL", KCT_ERR_INVALID_ARG);
    if (opts->max_iter < 0 || !(opts->err_tol >= 0.0) || opts->history || opts->tikhonov != 0.0 || opts->jacobi ||
        opts->recompute_every || !opts->x0_is_zero)
        return fail(fn, "batched CGLS takes max_iter >= 0, err_tol >= 0 and x0 = 0 only", KCT_ERR_INVALID_ARG);
    for (int i = 0; i < c; ++i)
        if (!bs[i] || !xs[i] || ((uintptr_t)bs[i] & 15u) || ((uintptr_t)xs[i] & 15u))
            return fail(fn, "instance " + std::to_string(i) + ": b and x must be 16-byte aligned device pointers",
                        KCT_ERR_INVALID_ARG);
    const BatchLayout L = batch_layout(b);
    if (!ws || ws_bytes < L.total || ((uintptr_t)ws & 255u))
        return fail(fn, "workspace missing, misaligned or smaller than kct_batch_workspace_size", KCT_ERR_WORKSPACE);
    char *w = (char *)ws;
    BatchInst *T = (BatchInst *)(w + L.table);
    int64_t *off = (int64_t *)(w + L.offs);

    // host tables in grid order
    std::vector<BatchInst> tab(c);
    std::vector<int64_t> offs((size_t)BG_COUNT * (c + 1), 0);
    for (int j = 0; j < c; ++j) {
        const int i = b->order[j];
        const Geometry *g = b->geoms[i];
        BatchInst &t = tab[j];
        memset(&t, 0, sizeof(t));
        t.g = g->dev;
        t.n = inst_n(g);
        t.m = inst_m(g);
        t.fwd_r = b->fwd_r[i];
        t.nbk = backward_grid_dims(g->dev, t.nbx, t.nby, t.nbz);
        t.nf = forward_num_blocks_r(g->dev, t.fwd_r);
        t.b = bs[i];
        t.x = xs[i];
        t.sc = (Scalars *)(w + L.base[i]);
        t.part = (double *)(w + L.part[i]);
        t.d = (float *)(w + L.d[i]);
        t.dz = (float *)(w + L.dz[i]);
        t.r = (float *)(w + L.r[i]);
        t.e = (float *)(w + L.e[i]);
        t.p = (float *)(w + L.p[i]);
        const int64_t dir = (int64_t)((g->dev.nx + 31) / 32) * ((g->dev.nz + 31) / 32) * g->dev.ny;
        offs[BG_FWD * (c + 1) + j + 1] = offs[BG_FWD * (c + 1) + j] + pad64(t.nf);
        offs[BG_BWD * (c + 1) + j + 1] = offs[BG_BWD * (c + 1) + j] + pad64(t.nbk);
        offs[BG_DIR * (c + 1) + j + 1] = offs[BG_DIR * (c + 1) + j] + dir;
        offs[BG_STREAM * (c + 1) + j + 1] = offs[BG_STREAM * (c + 1) + j] + stream_num_blocks();
    }
    int64_t nblk[BG_COUNT];
    for (int k = 0; k < BG_COUNT; ++k) nblk[k] = offs[k * (c + 1) + c];
    if (nblk[BG_FWD] > 0x7fffffff || nblk[BG_BWD] > 0x7fffffff || nblk[BG_DIR] > 0x7fffffff ||
        (int64_t)c * stream_num_blocks() > 0x7fffffff)
        return fail(fn, "batch too large for one launch", KCT_ERR_INVALID_ARG);

    hipStream_t st = b->stream;
    // order after the caller's earlier work
    KCT_BTRY(hipEventRecord(b->ev, stream));
    KCT_BTRY(hipStreamWaitEvent(st, b->ev, 0));
    KCT_BTRY(hipMemcpyAsync(T, tab.data(), sizeof(BatchInst) * c, hipMemcpyHostToDevice, st));
    KCT_BTRY(hipMemcpyAsync(off, offs.data(), sizeof(int64_t) * offs.size(), hipMemcpyHostToDevice, st));
    KCT_BTRY(hipStreamSynchronize(st));  // the host tables may go out of scope below

    const int K = opts->max_iter;
    // init block of Algorithm 1 for every instance
    KCT_BTRY(launch_batch_vec(T, c, BV_INIT, K, opts->err_tol, st));
    KCT_BTRY(launch_batch_vec(T, c, BV_NORM_B, 0, 0.0, st));
    KCT_BTRY(launch_batch_finalize(T, c, F_NB0, BG_STREAM, st));
    KCT_BTRY(launch_batch_vec(T, c, BV_X0_E, 0, 0.0, st));
    KCT_BTRY(launch_batch_backward(T, off + BG_BWD * (c + 1), c, nblk[BG_BWD], st));
    KCT_BTRY(launch_batch_finalize(T, c, F_NR2_INIT, BG_BWD, st));
    KCT_BTRY(launch_batch_dir(T, off + BG_DIR * (c + 1), c, nblk[BG_DIR], 1, st));
    KCT_BTRY(launch_batch_forward(T, off + BG_FWD * (c + 1), c, nblk[BG_FWD], st));
    KCT_BTRY(launch_batch_finalize(T, c, F_ALPHA, BG_FWD, st));
    KCT_BTRY(launch_batch_vec(T, c, BV_CGLS_X, 0, 0.0, st));
    KCT_BTRY(launch_batch_vec(T, c, BV_CGLS_E, 0, 0.0, st));
    KCT_BTRY(launch_batch_finalize(T, c, F_NB, BG_STREAM, st));
    if (K > 1) {
        if (use_graph) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            KCT_BTRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            const hipError_t ce = batch_iteration(T, off, c, nblk, st);
            const hipError_t ee = hipStreamEndCapture(st, &graph);
            if (ce != hipSuccess || ee != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(fn, std::string("graph capture failed: ") + hipGetErrorString(ce != hipSuccess ? ce : ee),
                            KCT_ERR_HIP);
            }
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            for (int it = 1; it < K && ie == hipSuccess; ++it) ie = hipGraphLaunch(exec, st);
            if (ie == hipSuccess) ie = hipStreamSynchronize(st);
            if (exec) (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) return fail(fn, std::string("graph replay failed: ") + hipGetErrorString(ie), KCT_ERR_HIP);
        } else {
            for (int it = 1; it < K; ++it) KCT_BTRY(batch_iteration(T, off, c, nblk, st));
        }
    }
    // results
    std::vector<Scalars> sc(c);
    for (int j = 0; j < c; ++j) KCT_BTRY(hipMemcpyAsync(&sc[j], tab[j].sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    KCT_BTRY(hipStreamSynchronize(st));
    bool numeric = false;
    for (int j = 0; j < c; ++j) {
        const int i = b->order[j];
        kct_solve_info &inf = infos[i];
        inf.iterations = sc[j].iters;
        inf.nb0 = sc[j].nb0;
        inf.nb = sc[j].nb;
        inf.nr2 = sc[j].nr2_old;
        inf.stop_reason = sc[j].done ? sc[j].stop : KCT_STOP_MAXITER;
        numeric = numeric || (sc[j].done && sc[j].stop == KCT_STOP_NUMERIC);
    }
    if (numeric) return fail(fn, "a solver norm became NaN or Inf in at least one instance", KCT_ERR_NUMERIC);
    return KCT_OK;
}

}  // extern "C"
