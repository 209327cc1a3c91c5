/*
 * kct.h -- C ABI of the MI355X (gfx950) cone-beam projector pair and the CGLS /
 * LSQR solvers built around it.
 *
 * Method: Kulvait & Rose, "Software Implementation of the Krylov Methods Based
 * Reconstruction for the 3D Cone Beam CT Operator" (Fully3D 2021,
 * arXiv 2110.13526).  The operator A maps a voxel volume x to projection data
 * b = A x (Section 2, Eq. 1); the reconstruction solves the least-squares
 * problem through the normal equations A^T A x = A^T b (Section 2, Eq. 2) with
 * CGLS (Section 2, Algorithm 1, CGLS with delayed residual computation) or LSQR
 * (Section 2; Paige & Saunders 1982).  The projector is the Siddon ray model
 * (Section 3): w_ij is the length in mm of the segment from the source to the
 * centre of detector pixel i that lies inside voxel j.  A and A^T evaluate the
 * same weight function on the same single-precision ray parameters, so A^T is
 * the exact transpose of A up to accumulation rounding.
 *
 * Geometry convention (the paper fixes only SID, SDD, pixel pitch and the
 * number of views, Section 4): world frame in mm, rotation axis +z; view k has
 * source s = (SID cos t_k, SID sin t_k, 0), detector centre s - SDD (cos t_k,
 * sin t_k, 0), detector axes e_u = (-sin t_k, cos t_k, 0) and e_v = (0, 0, 1);
 * pixel (iv, iu) has its centre at u = (iu - (nu-1)/2) du + off_u,
 * v = (iv - (nv-1)/2) dv + off_v.  Voxel (ix, iy, iz) spans
 * [cx - nx vx/2 + ix vx, ... + vx] and likewise in y and z (off-centre volumes
 * are allowed, Section 3).  The volume must lie strictly between the source and
 * the detector for every view.
 *
 * Memory layout (dense, no padding): volume x[iz][iy][ix] (ix fastest),
 * projections b[k][iv][iu] (iu fastest).  Storage type is chosen per call
 * (kct_dtype); ray and voxel accumulation is single precision (double for
 * KCT_F64), solver scalars (norms, step lengths, Givens rotations) are double
 * precision on the device, and the solvers' iterate x is always single
 * precision.
 *
 * Conventions for every function below:
 *  - Data pointers are DEVICE pointers of the current HIP device unless marked
 *    (host).  Buffers are contiguous, 16-byte aligned and must not alias.
 *  - Outputs are overwritten, never accumulated into.
 *  - Work is enqueued on the given stream (0 = legacy default stream) and is
 *    asynchronous unless stated otherwise.
 *  - Arguments are validated before anything is enqueued.  On failure nothing
 *    runs, a status other than KCT_OK is returned and kct_last_error() holds a
 *    message for the calling thread.  No function aborts or throws.
 *  - The library allocates only the geometry's small tables (kct_geometry_
 *    create); every large buffer (volumes, projections, workspaces) belongs to
 *    the caller.
 */
#ifndef KCT_H
#define KCT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KCT_OK = 0,
    KCT_ERR_INVALID_ARG = 1, /* null pointer, bad size, degenerate geometry        */
    KCT_ERR_UNSUPPORTED = 2, /* storage type or option not available               */
    KCT_ERR_HIP = 3,         /* a HIP runtime call failed                           */
    KCT_ERR_WORKSPACE = 4,   /* workspace missing or smaller than required          */
    KCT_ERR_NUMERIC = 5      /* a solver norm became NaN or Inf                     */
} kct_status;

/* Storage type of volumes, projections and workspace vectors.  The weights
 * are single precision in every case; F32, BF16 and F16 accumulate in single
 * precision, F64 in double (F64 is for the projector pair only: it evaluates
 * the same matrix to double-precision rounding, e.g. for gradient checks). */
typedef enum { KCT_F32 = 0, KCT_BF16 = 1, KCT_F16 = 2, KCT_F64 = 3 } kct_dtype;

/* Voxel grid: counts, voxel size [mm] and the volume centre [mm] (off-centre
 * reconstruction, Section 3). */
typedef struct {
    int32_t nx, ny, nz;
    double vx, vy, vz;
    double cx, cy, cz;
} kct_volume_desc;

/* Circular cone-beam orbit and flat detector (Section 4 gives SID, SDD, pixel
 * pitch and number of views).  View angles are t_k = angle0 + k * arc / n_views
 * unless `angles` (host, n_views values in radians) is given. */
typedef struct {
    int32_t n_views;
    double angle0, arc;
    const double *angles; /* (host, optional) */
    double sid, sdd;      /* source-isocentre and source-detector distance [mm] */
    int32_t nu, nv;       /* detector columns (u) and rows (v) */
    double du, dv;        /* pixel pitch [mm] */
    double off_u, off_v;  /* detector offset [mm] */
} kct_cone_desc;

/* Opaque geometry handle.  It owns small device tables on the device that was
 * current at creation; use it only with that device current. */
typedef struct kct_geometry_s *kct_geometry;

/* Validate the description and upload the per-view / per-column / per-row ray
 * tables (computed in double precision on the host and rounded once to single).
 * Errors: KCT_ERR_INVALID_ARG for non-positive sizes or pitches, SDD <= SID, a
 * volume that is not strictly between source and detector, a volume of 2^31
 * voxels or more (or a side above 2^20), projection data of 2^31 rays or more,
 * or a detector of 2^28 pixels or more; KCT_ERR_HIP if the upload fails.
 * Synchronous. */
kct_status kct_geometry_create(const kct_volume_desc *vol, const kct_cone_desc *cone, kct_geometry *out);

/* Free the tables (NULL is ignored).  The caller must ensure no enqueued work
 * still uses the geometry. */
void kct_geometry_destroy(kct_geometry g);

/* Projector models (Section 3).  KCT_PROJECTOR_SIDDON (the default): w_ij is
 * the length of ray i inside voxel j.  KCT_PROJECTOR_TT: the separable
 * footprint model with trapezoid transaxial and trapezoid axial footprints
 * (the projector of the paper's experiments, Section 4):
 * w_ij = L_i F_u F_v, F_u and F_v the pixel means of unit trapezoids whose
 * breakpoints are the detector coordinates of the voxel's in-plane corners
 * (transaxial) and of its z extent seen from its nearest and farthest in-plane
 * corner (axial), L_i = min(vx/|d_x|, vy/|d_y|, vz/|d_z|) for ray i's unit
 * direction d.  Both pairs evaluate identical weights in the projector and the
 * backprojector. */
enum { KCT_PROJECTOR_SIDDON = 0, KCT_PROJECTOR_TT = 1 };

/* Select the projector model used by every later call with g (project,
 * backproject, diag_normal, the solvers).  Batched solves take Siddon
 * geometries only.  Errors: INVALID_ARG. */
kct_status kct_geometry_set_projector(kct_geometry g, int32_t projector);

/* Number of voxels (n) and rays (m) of A in R^{m x n} (Section 2, Eq. 1). */
kct_status kct_geometry_dims(kct_geometry g, int64_t *n_vox, int64_t *n_rays);

/* Bytes of workspace kct_project needs for its best layout: one volume in
 * the storage type (a copy of x stored z-fastest, which lets the rays of one
 * detector column, held by neighbouring lanes, read neighbouring addresses). */
kct_status kct_project_workspace_size(kct_geometry g, kct_dtype dtype, size_t *bytes);

/* Forward projection b := A x (Section 2, Eq. 1; standalone projection,
 * Section 3).  x: n_vox elements, b: n_rays elements, both of `dtype`.  `ws`
 * may be NULL (then x is read in its own layout by every view, which is
 * correct but slower); otherwise ws_bytes must be at least
 * kct_project_workspace_size.  Errors: INVALID_ARG, UNSUPPORTED, WORKSPACE,
 * HIP. */
kct_status kct_project(kct_geometry g, kct_dtype dtype, const void *x, void *b, void *ws, size_t ws_bytes,
                       hipStream_t stream);

/* Size of the fixed device array that kct_project_noalloc uses (64 MiB): a
 * volume of up to 16 Mi FP32 voxels (256^3), 32 Mi 16-bit or 8 Mi FP64 voxels. */
#define KCT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* kct_project without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Computes exactly what kct_project computes with a
 * workspace (the same kernels, the same bits), but takes the z-fastest copy of
 * x in a fixed array of the library (KCT_NOALLOC_SCRATCH_BYTES; each device the
 * library runs on holds it from the first use until the process ends) instead
 * of a caller workspace.  It calls no hipMalloc / hipFree and no allocating
 * library routine.  Every call on one device shares that array and overwrites
 * what it needs, so calls that overlap in time on one device (different
 * streams or threads) race; serialise them.  Errors: as kct_project, and
 * WORKSPACE when n_vox * element size exceeds KCT_NOALLOC_SCRATCH_BYTES. */
kct_status kct_project_noalloc(kct_geometry g, kct_dtype dtype, const void *x, void *b, hipStream_t stream);

/* Backprojection x := A^T b (Section 2, Eq. 2; standalone backprojection,
 * Section 3), the exact transpose of kct_project.  Voxel-driven gather: no
 * atomics, deterministic.  Errors: INVALID_ARG, UNSUPPORTED, HIP. */
kct_status kct_backproject(kct_geometry g, kct_dtype dtype, const void *b, void *x, hipStream_t stream);

/* Solver options (Algorithm 1 inputs besides b and x0, and the variants the
 * paper describes in Sections 3, 5 and 7).  Zero-initialise the struct for plain CGLS /
 * LSQR. */
typedef struct {
    int32_t max_iter;   /* K >= 0; K = 0 returns x0 unchanged                           */
    double err_tol;     /* ERR >= 0: stop once NB <= ERR * NB0 (NB0 = |b|, Eq. 3)        */
    int32_t x0_is_zero; /* nonzero: x is not read, the solve starts from x0 = 0          */
    double *history;    /* (device, optional) max_iter doubles: NB_i / NB0 per iteration  */
    double tikhonov;    /* lambda >= 0: minimise |b - A x|^2 + lambda^2 |x|^2 (the Tikhonov
                           / L2 regularisation of Sections 3 and 7).  CGLS runs on the
                           stacked system [A; lambda I]; LSQR uses Paige & Saunders'
                           damping and then needs x0 = 0.  With lambda > 0, LSQR's NB is
                           the norm of the stacked residual [b - A x; -lambda x]; CGLS's
                           NB stays |b - A x|.                                             */
    int32_t jacobi;     /* CGLS only, nonzero: Jacobi preconditioning (Sections 3, 5): CGLS on
                           A M with M = diag(A^T A)^(-1/2) (0 where the diagonal is 0),
                           x = M z.  Needs the workspace of KCT_SOLVER_CGLS |
                           KCT_SOLVER_WITH_JACOBI; not with tikhonov > 0 or F16 storage. */
    int32_t recompute_every; /* CGLS only, k > 0: after every k-th iteration e = b - A x is
                           recomputed instead of updated (Section 5 discusses the drift
                           of the updated discrepancy); costs one more A per k iterations. */
} kct_solve_opts;

/* Stop reasons. */
enum { KCT_STOP_MAXITER = 0, KCT_STOP_TOL = 1, KCT_STOP_BREAKDOWN = 2, KCT_STOP_NUMERIC = 3 };

/* Solver result (host).  For CGLS nb is the updated discrepancy norm NB of
 * Algorithm 1; for LSQR it is the estimate |phibar| of |b - A x|. */
typedef struct {
    int32_t iterations;  /* i of Algorithm 1 (updates of x)                   */
    double nb0, nb;      /* |b| and the final discrepancy norm                 */
    double nr2;          /* CGLS: last |A^T e|^2; LSQR: last alpha^2           */
    int32_t stop_reason; /* KCT_STOP_*                                          */
} kct_solve_info;

enum { KCT_SOLVER_CGLS = 0, KCT_SOLVER_LSQR = 1, KCT_SOLVER_WITH_JACOBI = 0x100 };

/* Workspace bytes for a solver (KCT_SOLVER_CGLS or KCT_SOLVER_LSQR, for CGLS
 * optionally | KCT_SOLVER_WITH_JACOBI).  CGLS holds d, r and a z-fastest copy
 * of d (volumes) and e, p (projections): the paper's three volumes and three
 * projection vectors with x and b (Section 5) plus the copy, and a small block
 * of double-precision scalars and reduction partials; with Jacobi one more
 * single-precision volume (the preconditioner).  LSQR holds v, w and a
 * z-fastest copy of v (volumes) and u (projections). */
kct_status kct_solver_workspace_size(kct_geometry g, kct_dtype dtype, int32_t solver, size_t *bytes);

/* CGLS with delayed residual computation (Section 2, Algorithm 1), with the
 * direction update d = r + beta d.  b: n_rays elements of `dtype`; x: n_vox
 * single-precision (float) elements whatever `dtype` is (a 16-bit iterate
 * stagnates), x0 on entry (unless opts->x0_is_zero), x_K on return.  The
 * workspace vectors use `dtype`.  Breakdown (NR2 = 0 or
 * NP2 = 0, e.g. b = 0) stops with the current x.  The whole iteration runs on
 * the device without host synchronisation; the call synchronises `stream` once
 * at the end to fill *info (host).  Errors: INVALID_ARG, UNSUPPORTED,
 * WORKSPACE, HIP; KCT_ERR_NUMERIC when NB became NaN/Inf (info is still
 * filled). */
kct_status kct_cgls_solve(kct_geometry g, kct_dtype dtype, const void *b, void *x, const kct_solve_opts *opts,
                          void *ws, size_t ws_bytes, kct_solve_info *info, hipStream_t stream);

/* LSQR (Section 2, Paige & Saunders 1982): Golub-Kahan bidiagonalisation with
 * Givens QR, iterations aligned with CGLS (K products with A and K with A^T).
 * Same arguments, ownership and errors as kct_cgls_solve. */
kct_status kct_lsqr_solve(kct_geometry g, kct_dtype dtype, const void *b, void *x, const kct_solve_opts *opts,
                          void *ws, size_t ws_bytes, kct_solve_info *info, hipStream_t stream);

/* diag(A^T A): out_j = sum_i w_ij^2, the squared column norms of A (the
 * diagonal that Jacobi preconditioning inverts, Section 5), computed by the
 * backprojector's gather with squared weights.  out: n_vox floats (device),
 * volume layout.  Errors: INVALID_ARG, HIP. */
kct_status kct_diag_normal(kct_geometry g, float *out, hipStream_t stream);

/* ---------------------------------------------------------------- batched CGLS
 * Many independent reconstructions, each with its own geometry (volume,
 * detector, views, distances), solved together by CGLS (Section 2,
 * Algorithm 1).  Every step of an iteration is one launch that covers all
 * instances; the backprojection, the direction update and the forward
 * projection are persistent launches (as many workgroups as the device holds
 * at once) that drain a device work queue of (instance, tiles) items, largest
 * instance first.  Each instance keeps its own double-precision scalars,
 * partial sums and stop flag, so it gets exactly the result of its own
 * kct_cgls_solve when both use the same forward and backprojection variants
 * (the defaults).  The steps of one iteration are recorded as a HIP graph once
 * per batch and workspace and replayed.  FP32 storage. */
typedef struct kct_batch_s *kct_batch;

/* geoms: count geometry handles (host array), all created on the current
 * device; they must outlive the batch.  The batch owns one stream of its own
 * (default priority) for graph capture.  Errors: INVALID_ARG, HIP. */
kct_status kct_batch_create(const kct_geometry *geoms, int32_t count, kct_batch *out);

/* Synchronises the batch's stream and frees it (NULL is ignored). */
void kct_batch_destroy(kct_batch b);

/* Bytes of workspace of kct_batch_cgls_solve and kct_batch_tune: a small table
 * plus, per instance, CGLS's d, its z-fastest copy, r (volumes), e, p
 * (projections), scalars and partial sums. */
kct_status kct_batch_workspace_size(kct_batch b, size_t *bytes);

/* Autotuner: for each instance, time its forward projection with one and with
 * two detector rows per lane, and its backprojection with each brick shape
 * (16-deep bricks staged in 48-column chunks, 20-deep bricks in 32-column
 * chunks), 3 launches each after a warm-up (HIP events), and keep the faster of
 * each for the batch's solves (a tuned instance may then differ from its own
 * kct_cgls_solve by the rounding of regrouped partial sums).  cache_path
 * (host, optional): a text file of "<sizes> <rows per lane> <brick shape>"
 * lines; instances whose sizes are listed are not timed, new choices are
 * appended.  ws is scratch (kct_batch_workspace_size bytes, contents
 * overwritten).  Synchronous.  Errors: INVALID_ARG, WORKSPACE, HIP. */
kct_status kct_batch_tune(kct_batch b, void *ws, size_t ws_bytes, const char *cache_path, hipStream_t stream);

/* For every instance i: x_i := K iterations of CGLS (Algorithm 1) on b_i from
 * x0 = 0.  opts: max_iter and err_tol apply to every instance; x0_is_zero must
 * be nonzero and the other fields zero.  bs, xs: host arrays of count device
 * pointers (n_rays_i and n_vox_i floats, 16-byte aligned).  use_graph nonzero:
 * iterations 2..K replay one recorded HIP graph (the same results as plain
 * launches).  ws: 256-byte aligned.  infos: host array of count results.  The
 * solve is ordered after earlier work on `stream` and synchronises before it
 * returns.  Errors: INVALID_ARG, WORKSPACE, HIP; KCT_ERR_NUMERIC if NB became
 * NaN/Inf in some instance (infos still filled). */
kct_status kct_batch_cgls_solve(kct_batch b, const float *const *bs, float *const *xs, const kct_solve_opts *opts,
                                int32_t use_graph, void *ws, size_t ws_bytes, kct_solve_info *infos,
                                hipStream_t stream);

/* Per-instance latency of the last kct_batch_cgls_solve on this batch:
 * seconds[i] (host, count values) = time on the device clock from the batch's
 * set-up (the first step of the solve) to the step at which instance i's solve
 * stopped (K iterations, tolerance, breakdown).  Errors: INVALID_ARG (no solve
 * yet), UNSUPPORTED (no device wall clock), HIP. */
kct_status kct_batch_latencies(kct_batch b, double *seconds);

/* Launch timing of the solvers' projector steps, for measurement (not part of
 * the method).  kct_timing_enable(1) clears the record and from then on every
 * forward (p = A d in CGLS, the u update in LSQR) and backward (r = A^T e, the
 * v update) launch of a kct_cgls_solve / kct_lsqr_solve iteration is
 * bracketed by a HIP event pair on the solve's stream; kct_timing_enable(0)
 * stops recording (and clears).  Process-wide, not thread-safe: time one solve
 * at a time.  Events are created on first use and reused.  Errors: HIP (from
 * the solve that records). */
kct_status kct_timing_enable(int32_t on);

/* The launches recorded since kct_timing_enable(1) of one kind (0 forward,
 * 1 backward): their number and the average, smallest and largest duration in
 * milliseconds (host outputs; 0 when none).  Waits for the recorded events.
 * Errors: INVALID_ARG (other kind, NULL output), HIP. */
kct_status kct_timing_get(int32_t kind, int32_t *count, double *avg_ms, double *min_ms, double *max_ms);

/* Message describing the last failure on the calling thread ("" if none). */
const char *kct_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KCT_H */
