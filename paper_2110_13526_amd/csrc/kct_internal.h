// kct_internal.h -- types shared by the host side and the kernels of the
// cone-beam projector library (not part of the public C ABI).
//
// The geometry is reduced on the host, in double precision, to per-view,
// per-detector-column and per-detector-row parameters of the rays, rounded once
// to single precision.  Every kernel that needs the weight w_ij of a ray and a
// voxel reads these same numbers and evaluates the same inline functions
// (kct_weights.h), which is what makes the backprojector the exact transpose of
// the forward projector.
//
// Ray parametrisation.  For each view one in-plane axis is "dominant" (x when
// |cos t| / vx >= |sin t| / vy, else y); call it xi and the other in-plane axis
// eta.  Coordinates are voxel-index units: along an axis with n cells plane m
// (m = 0..n) sits at m - h, where the plane offset h is the multiple of 1/2 in
// [0, n] nearest to the isocentre's index (h = n/2 for a volume centred on the
// isocentre, so the origin is the volume centre).  A ray of detector column iu
// and row iv is then
//     eta(xi)  = eta_c + a * xi                       (column parameters)
//     zeta(xi) = zeta_c + xi / czr,  zeta_c = qz * tcv - zc,  czr = inv_qz * kz
// and its length in mm per unit of xi is L = sqrt(lxy2 + (qz * gp)^2).
// The ray crosses eta-plane mb (index frame) at xi = (mb - eta_c) * inv_a and
// zeta-plane mb at xi = (mb - zeta_c) * czr.  Parametrising by the voxel
// index along the dominant axis keeps every quantity O(volume size), so single
// precision resolves a crossing to about 1e-5 of a voxel.  Rays nearly
// parallel to an axis' planes (the most sensitive crossings: an error in the
// coordinate moves the crossing by error / slope) pass near the isocentre; with
// the origin there their coordinates are small and so are their roundings,
// also for off-centre volumes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kct.h"

namespace kct {

struct ColParam {    // per (view, detector column)
    float eta_c;     // eta (index frame) where the ray meets the plane xi = 0
    float inv_a;     // d xi / d eta; 0 when the ray is parallel to the eta planes
    float a;         // d eta / d xi
    float tcv;       // (fraction of the source->pixel segment at xi = 0) / vz
    float kz;        // vz * (xi extent of the segment in mm) / vxi
    float gp;        // fraction of the source->pixel segment per unit of xi
    float lxy2;      // in-plane part of (mm per unit xi)^2
    float pad;
};

struct RowParam {    // per detector row
    float qz;        // z of the pixel centre [mm] (the source is at z = 0)
    float inv_qz;    // 1 / qz, 0 when qz == 0
};

struct ViewParam {   // per view
    float sx, sy;    // source position [mm]
    float c, s;      // cos and sin of the view angle
    int dom;         // 0: xi = x, eta = y;  1: xi = y, eta = x
    float dn, dd;    // half extent of a voxel's square across (e_u) and along the central ray [mm]
    int pad;
};

// Per (view, column of 16 x 16 voxel bricks): the detector columns that the
// brick column's rays can meet (its shadow, clamped to the detector; u0 > u1
// when none), and the extreme inverse depths of its four in-plane corners, from
// which a brick of any z-extent bounds its detector rows.
struct ShadowParam {
    int u0, u1;
    float rmin, rmax;  // 1 / depth along the central ray [1/mm]
};

// Everything the kernels need, passed by value.
struct GeoDev {
    int nx, ny, nz, nviews, nu, nv;
    float vx, vy, vz;
    float x0, y0, z0;        // world coordinates of the volume's lower corner [mm]
    float hx, hy, hz;        // plane offsets: plane m of an axis at m - h (n/2 when centred)
    float zc;                // z / vz of the zeta frame's origin (0 when centred)
    float inv_vz;
    float sdd, du, dv, off_u, off_v;
    float inv_du, inv_dv;
    float cu, cv;            // (nu - 1)/2, (nv - 1)/2
    // Detector coordinates as fractional pixel indices, for bounds:
    // column = ku * (lateral / depth) + fu0, row = kv * (height / depth) + fv0
    float ku, kv;            // sdd / du, sdd / dv
    float fu0, fv0;          // cu - off_u / du, cv - off_v / dv
    int projector;           // KCT_PROJECTOR_SIDDON or KCT_PROJECTOR_TT (host-side dispatch)
    float sid;               // source to rotation axis [mm]
    const ColParam *cols;    // [nviews][nu]
    const RowParam *rows;    // [nv]
    const ViewParam *views;  // [nviews]
    const ShadowParam *shadows;  // [nviews][sby][sbx] (16 x 16 brick columns)
    int sbx, sby;
};

// Double-precision solver state kept on the device (one per solve).
struct Scalars {
    // CGLS (Algorithm 1)
    double nb0, nb, nr2_old, nr2_now, np2, alpha, beta;
    // LSQR (Paige & Saunders)
    double l_alpha, l_beta, rhobar, phibar, rho, phi, theta, cg, sg;
    double fwd_c1, fwd_c2;   // u_hat' = c1 * (A v_hat) - c2 * u_hat
    double bwd_c1, bwd_c2;   // v_hat' = c1 * (A^T u_hat) - c2 * v_hat
    double x_coef, w_coef, w_vcoef;  // x += x_coef w;  w = w_vcoef v_hat - w_coef w
    // Storage scales (powers of two; 1 unless the storage type is FP16): a
    // stored element s represents sigma * s.  CGLS: r and d use sr, p uses sp
    // (e and b are stored as they are); LSQR: w uses sw.
    double sr, sp, sw;
    double x_alpha, e_alpha;         // CGLS: x += x_alpha d;  e -= e_alpha p
    double tik_d2;                   // CGLS Tikhonov: lambda^2 * sr^2 (weight of |d_stored|^2 in NP2)
    double damp, res2;               // LSQR damping lambda and the sum of psi^2 of its rotations
    float tik_r, pad_f;              // CGLS Tikhonov: r = bwd_scale * A^T e - tik_r * x
    float fwd_scale, bwd_scale;      // CGLS epilogues: p = fwd_scale * (A d), r = bwd_scale * (A^T e)
    double err;
    double *history;
    int iters, done, stop, maxiter;
    int skip_bwd, pad0, pad1, pad2;
    // device wall-clock stamps (batched solves): set up, and stopped
    unsigned long long t_start, t_done;
};

enum FinalizeOp {
    F_NB0 = 0,
    F_NB_INIT,
    F_NR2_INIT,
    F_ALPHA,
    F_NB,
    F_BETA,
    F_L_BETA0,
    F_L_ALPHA0,
    F_L_BETA,
    F_L_ALPHA,
    F_L_GIVENS,
};

// Forward-projection epilogues.
enum FwdEpi {
    FWD_PLAIN = 0,  // out = A x
    FWD_NORM,       // out = A x, partial |out|^2
    FWD_BMINUS,     // out = aux - A x, partial |out|^2
    FWD_LSQR,       // out = c1 * A x - c2 * out, partial |out|^2 (reads scalars)
};

// Backprojection epilogues.
enum BwdEpi {
    BWD_PLAIN = 0,  // out = A^T y
    BWD_NORM,       // out = A^T y, partial |out|^2
    BWD_LSQR0,      // out = c1 * A^T y, also z-fastest copy, partial |out|^2
    BWD_LSQR,       // out = c1 * A^T y - c2 * out, also z-fastest copy, partial |out|^2
    BWD_TIK,        // out = bwd_scale * A^T y - tik_r * aux, partial |out|^2   (aux = x, Tikhonov)
    BWD_JACOBI,     // out = aux * A^T y, partial aux * (A^T y)^2             (aux = 1 / diag(A^T A))
    BWD_DIAG,       // out = sum_i w_ij^2 = diag(A^T A) (proj not read)
    BWD_DIAG_INV,   // out = 1 / diag(A^T A), 0 where the diagonal is 0 (proj not read)
};

struct Geometry {
    kct_volume_desc vol;
    kct_cone_desc cone;
    int device;
    GeoDev dev;
    void *d_tables;  // one allocation holding cols, rows and views
    size_t table_bytes;
};

// bfloat16 storage: the upper 16 bits of an IEEE single (raw bits).
struct bf16 {
    uint16_t bits;
};

// Kernel launchers (defined in the .hip files).
// Forward projection with volume storage TV and projection storage TP.
template <typename TV, typename TP>
hipError_t launch_forward(const GeoDev &g, const TV *vol, const TV *vol_z, TP *out, const TP *aux, int epi,
                          const Scalars *sc, double *partials, const int *skip, hipStream_t st);
// vol_z (optional): the same volume stored z-fastest, vol_z[(iy * nx + ix) * nz + iz].
// out_z (LSQR epilogues only): receives the output in that layout as well.
template <typename T>
hipError_t launch_backward(const GeoDev &g, const T *proj, T *out, T *out_z, int epi, const Scalars *sc,
                           double *partials, const int *skip, hipStream_t st, const float *aux = nullptr);
int64_t forward_num_blocks(const GeoDev &g);                         // the default variant
int64_t forward_num_blocks_r(const GeoDev &g, int rows_per_lane);     // rows_per_lane 1 or 2
int64_t backward_num_blocks(const GeoDev &g);

// Vector kernels (vector_ops.hip).
int64_t stream_num_blocks();
// dst[(iy * nx + ix) * nz + iz] = src[(iz * ny + iy) * nx + ix]
template <typename TS, typename TD>
hipError_t launch_zfast_copy(const GeoDev &g, const TS *src, TD *dst, hipStream_t st);
template <typename T>
hipError_t launch_norm2(const T *v, int64_t n, double *partials, const int *skip, hipStream_t st);
hipError_t launch_finalize(Scalars *sc, const double *partials, int64_t nparts, int op, hipStream_t st,
                           const double *partials2 = nullptr, int64_t nparts2 = 0);
template <typename T>
hipError_t launch_fill_zero(T *v, int64_t n, hipStream_t st);
// The solvers keep the iterate x in single precision whatever the storage type
// of the other vectors (16-bit iterates stagnate).
template <typename T>
hipError_t launch_copy(const T *src, T *dst, int64_t n, hipStream_t st);
// x += alpha d
template <typename T>
hipError_t launch_cgls_x(float *x, const T *d, const Scalars *sc, int64_t n, hipStream_t st);
// d = r (+ beta d) and its z-fastest copy
template <typename T>
hipError_t launch_cgls_d(const GeoDev &g, const T *r, T *d, T *dz, const Scalars *sc, int first,
                         hipStream_t st, double *dpart = nullptr);
int64_t cgls_d_num_blocks(const GeoDev &g);
// e -= alpha p, partial |e|^2
template <typename T>
hipError_t launch_cgls_e(T *e, const T *p, const Scalars *sc, int64_t n, double *partials, hipStream_t st);
// LSQR: w = w_vcoef v (init) or x += x_coef w; w = w_vcoef v - w_coef w
template <typename T>
hipError_t launch_lsqr_xw(float *x, T *w, const T *v, const Scalars *sc, int init, int64_t n, hipStream_t st);
// the TT footprint pair (tt.hip); launch_forward / launch_backward dispatch to
// them for geometries whose projector is KCT_PROJECTOR_TT
template <typename TV, typename TP>
hipError_t launch_forward_tt(const GeoDev &g, const TV *vol, const TV *vol_z, TP *out, const TP *aux, int epi,
                             const Scalars *sc, double *partials, const int *skip, hipStream_t st);
template <typename T>
hipError_t launch_backward_tt(const GeoDev &g, const T *proj, T *out, T *out_z, int epi, const Scalars *sc,
                              double *partials, const int *skip, hipStream_t st, const float *aux);
int64_t tt_forward_num_blocks(const GeoDev &g);
// forward with an explicit rows-per-lane variant (1 or 2), plain epilogue
hipError_t launch_forward_r(const GeoDev &g, const float *vol, const float *vol_z, float *out, int rows_per_lane,
                            hipStream_t st);

// ---------------------------------------------------------------- batched CGLS
// One instance of a batched solve as the batched kernels see it (single
// precision storage).  The heavy steps of an iteration (backprojection,
// direction update, forward projection) run as persistent launches: a grid
// sized to the resident capacity of the device drains a queue of items, an
// item being up to a fixed number of consecutive tiles (workgroups of the
// instance's own single-solve grid) of one instance; items are numbered
// instance by instance in the batch's order (largest work first), so
// item q belongs to the instance i with off[i] <= q < off[i + 1].  Each tile
// is processed exactly as the instance's own solve would process it, with
// that instance's partial sums and scalars, so a batched solve returns the
// bits of the separate solves; an instance whose solve has stopped skips its
// items.
struct BatchInst {
    GeoDev g;
    int64_t n, m;               // voxels, rays
    int fwd_r;                  // rows per lane of its forward variant (1 or 2)
    int bwd_v;                  // its backprojection variant (BWD_VARIANTS)
    int nbx, nby, nbz;          // backward brick grid of that variant
    int64_t nf, nbk, ndir;      // tiles of its forward, backward and direction grids (partials per launch)
    const float *b;
    float *x;
    Scalars *sc;
    double *part;
    float *d, *dz, *r, *e, *p;
};

// Backprojection variants of the batched form: brick depth and staged chunk
// width (columns).  0: 16-deep bricks, 48-column chunks; 1: 20-deep bricks,
// 32-column chunks (the single solve's choice for large volumes).
enum BwdVariant { BWD_VSHALLOW = 0, BWD_VDEEP = 1, BWD_VARIANTS = 2 };

enum BatchGrid { BG_FWD = 0, BG_BWD, BG_DIR, BG_STREAM, BG_COUNT };  // item tables, each count + 1 long
// Tiles per queue item of each persistent step: items must far outnumber the
// resident workgroups for the queue to balance the load (a brick of the
// backprojection is a long task, a forward or direction tile a short one).
constexpr int BATCH_ITEM_FWD = 16, BATCH_ITEM_BWD = 1, BATCH_ITEM_DIR = 8;
// Queue state of one persistent step: the next item, and the workgroups that
// have left (the last one resets both for the next launch).
struct BatchQueue {
    unsigned next, exited, pad0, pad1;
};

hipError_t launch_batch_forward(const BatchInst *B, const int64_t *off, int count, BatchQueue *q, int grid,
                                hipStream_t st);
hipError_t launch_batch_backward(const BatchInst *B, const int64_t *off, int count, BatchQueue *q, int grid,
                                 hipStream_t st);
// op: one of the batched vector steps below
enum BatchVecOp { BV_INIT = 0, BV_NORM_B, BV_X0_E, BV_CGLS_X, BV_CGLS_E };
hipError_t launch_batch_vec(const BatchInst *B, int count, int op, int maxiter, double err, hipStream_t st);
hipError_t launch_batch_dir(const BatchInst *B, const int64_t *off, int count, BatchQueue *q, int grid, int first,
                            hipStream_t st);
// finalize of every instance; kind: which grid produced the partials (BatchGrid)
hipError_t launch_batch_finalize(const BatchInst *B, int count, int op, int kind, hipStream_t st);
// resident workgroups of the persistent kernels on the current device
hipError_t batch_persistent_grids(int &fwd, int &bwd, int &dir);
hipError_t batch_backward_occupancy(int &per_cu);
hipError_t batch_dir_occupancy(int &per_cu);
// a single backprojection (plain epilogue) with one of the batched form's variants (tuner)
hipError_t launch_backward_variant(const GeoDev &g, int variant, const float *proj, float *out, hipStream_t st);
int64_t backward_variant_grid(const GeoDev &g, int variant, int &nbx, int &nby, int &nbz);
int backward_default_variant(const GeoDev &g);
int64_t tt_backward_grid_dims(const GeoDev &g, int &nbx, int &nby, int &nbz);

}  // namespace kct
