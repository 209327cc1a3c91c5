// batch.cpp -- batched CGLS (Section 2, Algorithm 1) over many independent
// reconstructions: the kct_batch_* entry points of kct.h.
//
// Every step of an iteration is one launch that covers all instances; the
// heavy steps (backprojection, direction update, forward projection) are
// persistent launches that drain a device work queue of (instance, tiles)
// items, largest instance first (BatchInst in kct_internal.h).  Each instance
// keeps its own FP64 scalars, partial sums and stop flag, so a batch computes
// exactly what the instances' separate solves compute.  The steps of one
// iteration are recorded once per batch (and workspace) as a HIP graph on the
// batch's own stream and replayed K - 1 times per solve.  The scalar steps
// stamp each instance's set-up and completion on the device clock, so the
// latency of every instance inside the batch is measured.
//
// The autotuner picks, per instance, the forward variant (1 or 2 detector rows
// per lane) and the backprojection variant (brick depth and staged chunk
// width) by timing them on the instance's geometry, and can keep its choices
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
    std::vector<int> bwd_v;   // per instance, a BwdVariant
    std::vector<int> order;   // grid order: instance indices, largest work first
    int device = -1;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    int grid_fwd = 0, grid_bwd = 0, grid_dir = 0;  // resident workgroups of the persistent steps
    // the recorded iteration (valid for the workspace it was recorded with)
    hipGraphExec_t exec = nullptr;
    const void *exec_ws = nullptr;
    // device-clock stamps of the last solve, per instance (set-up, completion)
    std::vector<unsigned long long> t_start, t_done;
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t inst_n(const Geometry *g) { return (int64_t)g->dev.nx * g->dev.ny * g->dev.nz; }
int64_t inst_m(const Geometry *g) { return (int64_t)g->dev.nviews * g->dev.nv * g->dev.nu; }

int64_t inst_ndir(const Geometry *g)
{
    return (int64_t)((g->dev.nx + 31) / 32) * ((g->dev.nz + 31) / 32) * g->dev.ny;
}

int64_t inst_partials(const Geometry *g)
{
    int64_t a = std::max(forward_num_blocks_r(g->dev, 1), forward_num_blocks_r(g->dev, 2));
    int nbx, nby, nbz;
    int64_t bmax = 0;
    for (int v = 0; v < BWD_VARIANTS; ++v) bmax = std::max(bmax, backward_variant_grid(g->dev, v, nbx, nby, nbz));
    return std::max(std::max(a, bmax), stream_num_blocks());
}

int64_t items_of(int64_t tiles, int per_item) { return (tiles + per_item - 1) / per_item; }

// [BatchInst table][item tables][queues][per instance: Scalars | partials | d | dz | r | e | p]
struct BatchLayout {
    size_t table, offs, queues, total;
    std::vector<size_t> base;  // start of each instance's block
    std::vector<size_t> part, d, dz, r, e, p;
};

constexpr int BATCH_QUEUES = 3;  // backprojection, direction update, forward projection

BatchLayout batch_layout(const Batch *b)
{
    BatchLayout L;
    const size_t c = b->geoms.size();
    L.table = 0;
    L.offs = a256(c * sizeof(BatchInst));
    L.queues = L.offs + a256((size_t)BG_COUNT * (c + 1) * sizeof(int64_t));
    size_t at = L.queues + a256(BATCH_QUEUES * sizeof(BatchQueue));
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
hipError_t batch_iteration(const Batch *b, const BatchInst *T, const int64_t *off, BatchQueue *q, int c,
                           hipStream_t st)
{
    hipError_t e;
    if ((e = launch_batch_backward(T, off + BG_BWD * (c + 1), c, q + 0, b->grid_bwd, st)) != hipSuccess) return e;
    if ((e = launch_batch_finalize(T, c, F_BETA, BG_BWD, st)) != hipSuccess) return e;
    if ((e = launch_batch_dir(T, off + BG_DIR * (c + 1), c, q + 1, b->grid_dir, 0, st)) != hipSuccess) return e;
    if ((e = launch_batch_forward(T, off + BG_FWD * (c + 1), c, q + 2, b->grid_fwd, st)) != hipSuccess) return e;
    if ((e = launch_batch_finalize(T, c, F_ALPHA, BG_FWD, st)) != hipSuccess) return e;
    if ((e = launch_batch_vec(T, c, BV_CGLS_X, 0, 0.0, st)) != hipSuccess) return e;
    if ((e = launch_batch_vec(T, c, BV_CGLS_E, 0, 0.0, st)) != hipSuccess) return e;
    return launch_batch_finalize(T, c, F_NB, BG_STREAM, st);
}

void drop_graph(Batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->exec_ws = nullptr;
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
        b->fwd_r.push_back(2);  // two rows per lane until the tuner has timed the instance
        b->bwd_v.push_back(backward_default_variant(g->dev));
        b->order.push_back(i);
    }
    if (batch_persistent_grids(b->grid_fwd, b->grid_bwd, b->grid_dir) != hipSuccess) {
        delete b;
        return fail(fn, "occupancy query of the persistent kernels failed", KCT_ERR_HIP);
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
    drop_graph(b);
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
    // cache lines: "<sizes> <rows per lane> [<backprojection variant>]"
    std::map<std::string, std::pair<int, int>> known;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string key;
            int r = 0, v = -1;
            if (!(ls >> key >> r) || (r != 1 && r != 2)) continue;
            if (!(ls >> v) || v < 0 || v >= BWD_VARIANTS) v = -1;
            known[key] = {r, v};
        }
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    KCT_BTRY(hipEventCreate(&t0));
    KCT_BTRY(hipEventCreate(&t1));
    // average time of `reps` launches of fn after one warm-up
    auto time_it = [&](auto launch, float &ms) -> hipError_t {
        hipError_t e = launch();
        if (e == hipSuccess) e = hipEventRecord(t0, stream);
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) e = launch();
        if (e == hipSuccess) e = hipEventRecord(t1, stream);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        return e;
    };
    std::vector<std::string> fresh;
    kct_status rc = KCT_OK;
    char *w = (char *)ws;
    for (size_t i = 0; i < b->geoms.size() && rc == KCT_OK; ++i) {
        const Geometry *g = b->geoms[i];
        const std::string key = size_key(g);
        auto it = known.find(key);
        if (it != known.end() && it->second.second >= 0) {
            b->fwd_r[i] = it->second.first;
            b->bwd_v[i] = it->second.second;
            continue;
        }
        float *d = (float *)(w + L.d[i]), *dz = (float *)(w + L.dz[i]), *p = (float *)(w + L.p[i]);
        float *r = (float *)(w + L.r[i]);
        hipError_t e = launch_fill_zero<float>(d, inst_n(g), stream);
        if (e == hipSuccess) e = launch_zfast_copy<float, float>(g->dev, d, dz, stream);
        if (e == hipSuccess) e = launch_fill_zero<float>(p, inst_m(g), stream);
        float best = 0.0f;
        int best_r = 2;
        for (int rr = 1; rr <= 2 && e == hipSuccess; ++rr) {
            float ms = 0.0f;
            e = time_it([&] { return launch_forward_r(g->dev, d, dz, p, rr, stream); }, ms);
            if (e == hipSuccess && (rr == 1 || ms < best)) {
                best = ms;
                best_r = rr;
            }
        }
        int best_v = b->bwd_v[i];
        for (int v = 0; v < BWD_VARIANTS && e == hipSuccess; ++v) {
            float ms = 0.0f;
            e = time_it([&] { return launch_backward_variant(g->dev, v, p, r, stream); }, ms);
            if (e == hipSuccess && (v == 0 || ms < best)) {
                best = ms;
                best_v = v;
            }
        }
        if (e != hipSuccess) {
            rc = fail(fn, std::string("timing failed: ") + hipGetErrorString(e), KCT_ERR_HIP);
            break;
        }
        b->fwd_r[i] = best_r;
        b->bwd_v[i] = best_v;
        known[key] = {best_r, best_v};
        fresh.push_back(key);
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (rc == KCT_OK && cache_path && !fresh.empty()) {
        std::ofstream o(cache_path, std::ios::app);
        for (const auto &k : fresh) o << k << ' ' << known[k].first << ' ' << known[k].second << '\n';
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
    BatchQueue *q = (BatchQueue *)(w + L.queues);

    // host tables in grid order: per instance its tiles per step, and the item
    // numbering of the persistent steps (instances in order, largest first)
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
        t.bwd_v = b->bwd_v[i];
        t.nbk = backward_variant_grid(g->dev, t.bwd_v, t.nbx, t.nby, t.nbz);
        t.nf = forward_num_blocks_r(g->dev, t.fwd_r);
        t.ndir = inst_ndir(g);
        t.b = bs[i];
        t.x = xs[i];
        t.sc = (Scalars *)(w + L.base[i]);
        t.part = (double *)(w + L.part[i]);
        t.d = (float *)(w + L.d[i]);
        t.dz = (float *)(w + L.dz[i]);
        t.r = (float *)(w + L.r[i]);
        t.e = (float *)(w + L.e[i]);
        t.p = (float *)(w + L.p[i]);
        offs[BG_FWD * (c + 1) + j + 1] = offs[BG_FWD * (c + 1) + j] + items_of(t.nf, BATCH_ITEM_FWD);
        offs[BG_BWD * (c + 1) + j + 1] = offs[BG_BWD * (c + 1) + j] + items_of(t.nbk, BATCH_ITEM_BWD);
        offs[BG_DIR * (c + 1) + j + 1] = offs[BG_DIR * (c + 1) + j] + items_of(t.ndir, BATCH_ITEM_DIR);
        offs[BG_STREAM * (c + 1) + j + 1] = offs[BG_STREAM * (c + 1) + j] + stream_num_blocks();
    }
    for (int k = 0; k < BG_COUNT; ++k)
        if (offs[k * (c + 1) + c] > 0x7fffffff) return fail(fn, "batch too large for one launch", KCT_ERR_INVALID_ARG);
    if ((int64_t)c * stream_num_blocks() > 0x7fffffff)
        return fail(fn, "batch too large for one launch", KCT_ERR_INVALID_ARG);
    const BatchQueue zero_q[BATCH_QUEUES] = {};

    hipStream_t st = b->stream;
    // order after the caller's earlier work
    KCT_BTRY(hipEventRecord(b->ev, stream));
    KCT_BTRY(hipStreamWaitEvent(st, b->ev, 0));
    KCT_BTRY(hipMemcpyAsync(T, tab.data(), sizeof(BatchInst) * c, hipMemcpyHostToDevice, st));
    KCT_BTRY(hipMemcpyAsync(off, offs.data(), sizeof(int64_t) * offs.size(), hipMemcpyHostToDevice, st));
    KCT_BTRY(hipMemcpyAsync(q, zero_q, sizeof(zero_q), hipMemcpyHostToDevice, st));
    KCT_BTRY(hipStreamSynchronize(st));  // the host tables may go out of scope below

    const int K = opts->max_iter;
    // init block of Algorithm 1 for every instance
    KCT_BTRY(launch_batch_vec(T, c, BV_INIT, K, opts->err_tol, st));
    KCT_BTRY(launch_batch_vec(T, c, BV_NORM_B, 0, 0.0, st));
    KCT_BTRY(launch_batch_finalize(T, c, F_NB0, BG_STREAM, st));
    KCT_BTRY(launch_batch_vec(T, c, BV_X0_E, 0, 0.0, st));
    KCT_BTRY(launch_batch_backward(T, off + BG_BWD * (c + 1), c, q + 0, b->grid_bwd, st));
    KCT_BTRY(launch_batch_finalize(T, c, F_NR2_INIT, BG_BWD, st));
    KCT_BTRY(launch_batch_dir(T, off + BG_DIR * (c + 1), c, q + 1, b->grid_dir, 1, st));
    KCT_BTRY(launch_batch_forward(T, off + BG_FWD * (c + 1), c, q + 2, b->grid_fwd, st));
    KCT_BTRY(launch_batch_finalize(T, c, F_ALPHA, BG_FWD, st));
    KCT_BTRY(launch_batch_vec(T, c, BV_CGLS_X, 0, 0.0, st));
    KCT_BTRY(launch_batch_vec(T, c, BV_CGLS_E, 0, 0.0, st));
    KCT_BTRY(launch_batch_finalize(T, c, F_NB, BG_STREAM, st));
    if (K > 1) {
        if (use_graph) {
            // the iteration's launches depend only on the workspace (tables, queues,
            // instance blocks) and the count: recorded once per workspace
            if (!b->exec || b->exec_ws != ws) {
                drop_graph(b);
                hipGraph_t graph = nullptr;
                KCT_BTRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                const hipError_t ce = batch_iteration(b, T, off, q, c, st);
                const hipError_t ee = hipStreamEndCapture(st, &graph);
                hipError_t ie = ce != hipSuccess ? ce : ee;
                if (ie == hipSuccess) ie = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
                if (graph) (void)hipGraphDestroy(graph);
                if (ie != hipSuccess) {
                    b->exec = nullptr;
                    return fail(fn, std::string("graph capture failed: ") + hipGetErrorString(ie), KCT_ERR_HIP);
                }
                b->exec_ws = ws;
            }
            hipError_t ie = hipSuccess;
            for (int it = 1; it < K && ie == hipSuccess; ++it) ie = hipGraphLaunch(b->exec, st);
            if (ie == hipSuccess) ie = hipStreamSynchronize(st);
            if (ie != hipSuccess) return fail(fn, std::string("graph replay failed: ") + hipGetErrorString(ie), KCT_ERR_HIP);
        } else {
            for (int it = 1; it < K; ++it) KCT_BTRY(batch_iteration(b, T, off, q, c, st));
        }
    }
    // results
    std::vector<Scalars> sc(c);
    for (int j = 0; j < c; ++j) KCT_BTRY(hipMemcpyAsync(&sc[j], tab[j].sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    b->t_start.assign(c, 0);
    b->t_done.assign(c, 0);
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
        b->t_start[i] = sc[j].t_start;
        b->t_done[i] = sc[j].t_done;
        numeric = numeric || (sc[j].done && sc[j].stop == KCT_STOP_NUMERIC);
    }
    if (numeric) return fail(fn, "a solver norm became NaN or Inf in at least one instance", KCT_ERR_NUMERIC);
    return KCT_OK;
}

kct_status kct_batch_latencies(kct_batch h, double *seconds)
{
    const char *fn = "kct_batch_latencies";
    Batch *b = nullptr;
    kct_status s = check_batch(h, fn, b);
    if (s != KCT_OK) return s;
    if (!seconds) return fail(fn, "seconds is NULL", KCT_ERR_INVALID_ARG);
    const int c = (int)b->geoms.size();
    if ((int)b->t_done.size() != c) return fail(fn, "no batched solve has run on this batch", KCT_ERR_INVALID_ARG);
    int khz = 0;
    KCT_BTRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device));
    if (khz <= 0) return fail(fn, "the device reports no wall-clock rate", KCT_ERR_UNSUPPORTED);
    unsigned long long t0 = ~0ull;
    for (int i = 0; i < c; ++i) t0 = std::min(t0, b->t_start[i]);
    for (int i = 0; i < c; ++i)
        seconds[i] = b->t_done[i] >= t0 ? (double)(b->t_done[i] - t0) / (1e3 * (double)khz) : -1.0;
    return KCT_OK;
}

}  // extern "C"
