"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test names what fixes the expected value: brute force on tiny inputs,
closed forms, invariants of the operator, library routines on an independently
assembled matrix, and the claims the paper makes about CGLS and LSQR.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import kct_inputs as ki
import oracle
from tests import bruteforce as bf


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------------ operator

@pytest.fixture(scope="module", params=["base", "offcenter", "aniso", "odd"])
def t16_pair(request):
    g = ki.t16(request.param)
    return g, bf.matrix(g)


def test_bruteforce_matrix_forward(t16_pair):
    """A x from the oracle's Siddon traversal equals the pair-by-pair slab matrix (Eq. 1)."""
    g, A = t16_pair
    for seed in (1, 2):
        x = ki.random_volume(g, seed)
        assert rel(oracle.project(g, x), A @ x.ravel()) < 1e-12
    x = ki.phantom(g, 6, 7, dtype=np.float64)
    assert rel(oracle.project(g, x), A @ x.ravel()) < 1e-12


def test_bruteforce_matrix_transpose(t16_pair):
    """A^T y from the oracle's slab-parallel scatter equals the brute-force transpose (Eq. 2)."""
    g, A = t16_pair
    for seed in (3, 4):
        y = ki.random_projections(g, seed)
        assert rel(oracle.backproject(g, y), A.T @ y.ravel()) < 1e-12


def test_bruteforce_structure(t16_pair):
    """Same set of weights above rounding level (structural nonzeros) as brute force.
    Pieces shorter than 1e-9 mm are rounding artefacts of coincident crossings."""
    g, A = t16_pair
    B = oracle.assemble(g)  # duplicate (ray, voxel) pieces are summed here
    assert B.nnz <= oracle.count_nnz(g) <= B.nnz + 64
    assert (B.data > 1e-9).sum() == (A.data > 1e-9).sum()
    assert abs(B - A).max() < 1e-12


def test_sampled_rays_and_voxels(t16_pair):
    g, A = t16_pair
    x = ki.random_volume(g, 5)
    y = ki.random_projections(g, 6)
    rng = np.random.default_rng(0)
    rays = rng.choice(g.n_rays, 64, replace=False)
    vox = rng.choice(g.n_vox, 64, replace=False)
    np.testing.assert_allclose(oracle.project_rays(g, x, rays), (A @ x.ravel())[rays], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.backproject_voxels(g, y, vox), (A.T @ y.ravel())[vox], rtol=1e-12,
                               atol=1e-12)


@pytest.mark.parametrize("variant", ["base", "offcenter", "aniso"])
def test_uniform_volume_is_box_chord(variant):
    """x = 1 gives the chord of each ray through the whole volume box (closed form)."""
    g = ki.t16(variant)
    lo = np.array([g.cx - g.nx * g.vx / 2, g.cy - g.ny * g.vy / 2, g.cz - g.nz * g.vz / 2])
    hi = lo + np.array([g.nx * g.vx, g.ny * g.vy, g.nz * g.vz])
    b = oracle.project(g, np.ones(g.vol_shape))
    np.testing.assert_allclose(b, bf.box_chord(g, lo, hi), rtol=1e-13, atol=1e-12)
    assert b.max() > 0


@pytest.mark.parametrize("vox", [(0, 0, 0), (5, 9, 3), (15, 15, 15), (8, 8, 8), (2, 13, 11)])
def test_single_voxel_is_box_chord(vox):
    """x = e_j gives the chord of each ray through one voxel box (closed form)."""
    g = ki.t16("offcenter")
    ix, iy, iz = vox
    x = np.zeros(g.vol_shape)
    x[iz, iy, ix] = 1.0
    lo = np.array([g.cx - g.nx * g.vx / 2 + ix * g.vx, g.cy - g.ny * g.vy / 2 + iy * g.vy,
                   g.cz - g.nz * g.vz / 2 + iz * g.vz])
    hi = lo + np.array([g.vx, g.vy, g.vz])
    np.testing.assert_allclose(oracle.project(g, x), bf.box_chord(g, lo, hi), rtol=1e-13, atol=1e-13)


def test_orientation_sign():
    """At view angle 0 an object at +y lands on +u (magnification SDD/SID) and +z on +v."""
    g = ki.t16().replace(n_views=1)
    x = np.zeros(g.vol_shape)
    x[8, 12, 8] = 1.0  # voxel centre at (+0.5, +4.5, +0.5) mm
    b = oracle.project(g, x)[0]
    iv, iu = np.unravel_index(np.argmax(b), b.shape)
    u = (iu - (g.nu - 1) / 2) * g.du
    v = (iv - (g.nv - 1) / 2) * g.dv
    mag = g.sdd / (g.sid - 0.5)
    assert abs(u - 4.5 * mag) <= 1.0 and abs(v - 0.5 * mag) <= 1.0


def test_rotation_symmetry():
    """Rotating the volume by +90 degrees about z and every view angle by +90 degrees
    leaves the projections unchanged (rotation sense of the orbit)."""
    g = ki.t16().replace(n_views=5, angle0=0.3, arc=1.0)
    g90 = g.replace(angle0=0.3 + math.pi / 2)
    x = ki.random_volume(g, 9)
    xr = np.rot90(x, k=-1, axes=(1, 2))  # new[iy, ix] = old[n-1-ix, iy]
    assert rel(oracle.project(g90, xr.copy()), oracle.project(g, x)) < 1e-12


def test_linearity_and_nonnegativity():
    g = ki.t16("offcenter")
    x1, x2 = ki.random_volume(g, 11), ki.random_volume(g, 12)
    a, b = 1.7, -0.4
    assert rel(oracle.project(g, a * x1 + b * x2),
               a * oracle.project(g, x1) + b * oracle.project(g, x2)) < 1e-12
    xp = np.abs(x1)
    assert oracle.project(g, xp).min() >= 0.0


@pytest.mark.parametrize("variant", ["base", "offcenter", "odd"])
def test_adjoint_dot_product(variant):
    """<A x, y> = <x, A^T y>."""
    g = ki.t16(variant)
    x = ki.random_volume(g, 21)
    y = ki.random_projections(g, 22)
    lhs = float((oracle.project(g, x) * y).sum())
    rhs = float((x * oracle.backproject(g, y)).sum())
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y))


def test_ellipsoid_line_integrals_converge_linearly():
    """A applied to a 4^3-supersampled voxelised ellipsoid tends to the analytic
    ellipsoid line integrals with error O(h): halving the voxel size halves the error."""
    errs = []
    for n in (16, 32, 64):
        vox = 32.0 / n
        g = ki.ConeGeometry(n, n, n, vox, vox, vox, n_views=8, nu=40, nv=40, du=1.6, dv=1.6,
                            cx=0.7, cy=-1.1, cz=0.4, angle0=0.2)
        q = np.array([0.3, -0.5, 0.6, 0.55])
        q /= np.linalg.norm(q)
        e = ki.Ellipsoid(np.array([1.5, -2.0, 1.0]), np.array([11.0, 7.0, 9.0]), ki._quat_to_rot(q), 1.0)
        x = ki.voxelize(g, [e], supersample=4, dtype=np.float64)
        ref = bf.ellipsoid_chords(g, e)
        errs.append(rel(oracle.project(g, x), ref))
    assert errs[0] < 0.15 and errs[-1] < 0.04
    for a, b in zip(errs, errs[1:]):
        assert 1.4 < a / b < 2.8, errs


# ------------------------------------------------------------------ CGLS / LSQR

def small_geom():
    return ki.ConeGeometry(8, 8, 8, 2.0, 2.0, 2.0, n_views=8, nu=24, nv=20, du=1.5, dv=1.5,
                           cx=0.3, cy=-0.2, cz=0.1)


@pytest.fixture(scope="module")
def small_problem():
    g = small_geom()
    A = bf.matrix(g)
    xt = ki.phantom(g, 5, 31, dtype=np.float64)
    b = (A @ xt.ravel()).reshape(g.proj_shape)
    b = ki.gaussian_noise(b, 0.01, 32)
    return g, A, b


def krylov_minimiser(A, b, x0, K):
    """argmin |b - A x| over x0 + span{r0, (A^T A) r0, ..., (A^T A)^(K-1) r0}, dense FP64.
    The basis is built by Lanczos with full re-orthogonalisation."""
    r0 = A.T @ (b - A @ x0)
    V = np.zeros((A.shape[1], K))
    v = r0 / np.linalg.norm(r0)
    for j in range(K):
        for _ in range(2):
            v = v - V[:, :j] @ (V[:, :j].T @ v)
        v = v / np.linalg.norm(v)
        V[:, j] = v
        v = A.T @ (A @ v)
    AV = A @ V
    y, *_ = np.linalg.lstsq(AV, b - A @ x0, rcond=None)
    return x0 + V @ y


def test_cgls_first_iterate_closed_form(small_problem):
    """x_1 = x0 + alpha r0, r0 = A^T (b - A x0), alpha = |r0|^2 / |A r0|^2."""
    g, A, b = small_problem
    bb = b.ravel()
    x0 = ki.random_volume(g, 33).ravel() * 0.1
    r0 = A.T @ (bb - A @ x0)
    alpha = (r0 @ r0) / np.linalg.norm(A @ r0) ** 2
    res = oracle.cgls(g, b, 1, x0=x0)
    assert res.iterations == 1
    assert rel(res.x, x0 + alpha * r0) < 1e-12
    assert abs(res.nb - np.linalg.norm(bb - A @ res.x.ravel())) < 1e-10 * res.nb


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 6])
def test_cgls_and_lsqr_are_krylov_minimisers(small_problem, K):
    """Both iterates minimise the residual over the same Krylov space (brute force)."""
    g, A, b = small_problem
    x0 = ki.random_volume(g, 34).ravel() * 0.05
    ref = krylov_minimiser(A, b.ravel(), x0, K)
    assert rel(oracle.cgls(g, b, K, x0=x0).x, ref) < 1e-9
    assert rel(oracle.lsqr(g, b, K, x0=x0).x, ref) < 1e-9
    assert rel(oracle.cgls(g, b, K).x, krylov_minimiser(A, b.ravel(), np.zeros(g.n_vox), K)) < 1e-9


def test_printed_direction_update_is_not_cg(small_problem):
    """The direction update as printed (d = d + beta r) leaves the Krylov minimiser,
    which is why the oracle reads it as d = r + beta d."""
    g, A, b = small_problem
    ref = krylov_minimiser(A, b.ravel(), np.zeros(g.n_vox), 4)
    assert rel(oracle.cgls(g, b, 4).x, ref) < 1e-9
    assert rel(oracle.cgls(g, b, 4, literal_update=True).x, ref) > 1e-3


@pytest.mark.parametrize("K", [10, 20])
def test_lsqr_matches_scipy(small_problem, K):
    """The oracle's LSQR and CGLS against scipy.sparse.linalg.lsqr on the brute-force matrix."""
    g, A, b = small_problem
    ref = spla.lsqr(A, b.ravel(), damp=0.0, atol=0.0, btol=0.0, conlim=0.0, iter_lim=K)[0]
    assert rel(oracle.lsqr(g, b, K).x, ref) < 1e-9
    assert rel(oracle.cgls(g, b, K).x, ref) < 1e-8


def test_cgls_matches_cg_on_normal_equations(small_problem):
    """CGLS = CG on A^T A x = A^T b (Eq. 2), via scipy.sparse.linalg.cg."""
    g, A, b = small_problem
    K = 8
    ATA = spla.aslinearoperator(A.T @ A)
    ref, _ = spla.cg(ATA, A.T @ b.ravel(), x0=np.zeros(g.n_vox), rtol=0.0, atol=0.0, maxiter=K)
    assert rel(oracle.cgls(g, b, K).x, ref) < 1e-8


def test_cgls_lsqr_practically_identical():
    """The paper reports that LSQR and CGLS give practically identical results on
    CT data.  In FP64 they agree to 1e-8 while the Krylov basis stays orthogonal
    (20 iterations here); at 40 iterations both have drifted from the exact
    Krylov minimiser by loss of orthogonality, yet their discrepancies still
    agree within 1 % and their iterates within 1 %."""
    g = ki.config("c1").replace(nx=32, ny=32, nz=32, vx=2.0, vy=2.0, vz=2.0, n_views=30, nu=48, nv=48,
                                du=2.0, dv=2.0)
    xt = ki.phantom(g, 10, 101, dtype=np.float64)
    b = ki.gaussian_noise(oracle.project(g, xt), 0.005, 1000101)
    c = oracle.cgls(g, b, 20)
    s = oracle.lsqr(g, b, 20)
    assert c.iterations == s.iterations == 20
    assert rel(c.x, s.x) < 1e-8
    np.testing.assert_allclose(c.history, s.history, rtol=1e-8)
    c = oracle.cgls(g, b, 40)
    s = oracle.lsqr(g, b, 40)
    assert rel(c.x, s.x) < 1e-2
    np.testing.assert_allclose(c.history, s.history, rtol=1e-2)


@pytest.fixture(scope="module")
def c1_small():
    g = ki.config("c1").replace(nx=32, ny=32, nz=32, vx=2.0, vy=2.0, vz=2.0, n_views=45, nu=48, nv=48,
                                du=2.0, dv=2.0)
    xt = ki.phantom(g, 10, 101, dtype=np.float64)
    b = oracle.project(g, xt)
    return g, xt, b


def test_cgls_monotone(c1_small):
    """CG on the normal equations: |b - A x_k| non-increasing and |x_k - x0| non-decreasing."""
    g, xt, b = c1_small
    res = oracle.cgls(g, b, 12)
    h = res.history
    assert np.all(np.diff(h) <= 1e-14)
    norms = [np.linalg.norm(oracle.cgls(g, b, k).x) for k in range(1, 9)]
    assert np.all(np.diff(norms) >= -1e-12)


def test_cgls_updated_residual_drift(c1_small):
    """The paper finds the updated and the recomputed discrepancy differ by less
    than 0.0001 % after 10 iterations."""
    g, xt, b = c1_small
    res = oracle.cgls(g, b, 10)
    true_nb = np.linalg.norm(b - oracle.project(g, res.x))
    assert abs(res.nb - true_nb) / true_nb < 1e-6


def test_cgls_converges_on_consistent_data(c1_small):
    """Loose sanity check of the paper's convergence finding: on noise-free,
    consistent data the relative discrepancy falls below 1 % within a few dozen
    iterations and keeps falling."""
    g, xt, b = c1_small
    res = oracle.cgls(g, b, 30)
    e = res.history
    assert e[-1] < 0.01
    assert np.argmax(e < 0.01) < 30


def test_cgls_edge_cases():
    g = small_geom()
    zero = np.zeros(g.proj_shape)
    res = oracle.cgls(g, zero, 5)
    assert res.iterations == 0 and res.stop_reason == oracle.STOP_BREAKDOWN and not res.x.any()
    res = oracle.lsqr(g, zero, 5)
    assert res.iterations == 0 and res.stop_reason == oracle.STOP_BREAKDOWN and not res.x.any()
    b = oracle.project(g, ki.phantom(g, 3, 1, dtype=np.float64))
    x0 = ki.random_volume(g, 2)
    res = oracle.cgls(g, b, 0, x0=x0)
    assert res.iterations == 0 and np.array_equal(res.x.ravel(), x0.ravel())
    # tolerance stop
    res = oracle.cgls(g, b, 50, err=0.2)
    assert res.stop_reason == oracle.STOP_TOL and res.history[-1] <= 0.2 and res.iterations < 50
    res = oracle.lsqr(g, b, 50, err=0.2)
    assert res.stop_reason == oracle.STOP_TOL and res.history[-1] <= 0.2 and res.iterations < 50


# ------------------------------------------------- variants (Sections 3, 5, 7)

@pytest.mark.parametrize("variant", ["base", "offcenter", "aniso", "odd"])
def test_diag_normal_is_squared_column_norms(variant):
    """diag(A^T A)_j = sum_i w_ij^2, against the brute-force matrix."""
    g = ki.t16(variant)
    A = bf.matrix(g)
    ref = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    assert rel(oracle.diag_normal(g).ravel(), ref) < 1e-12


@pytest.mark.parametrize("K", [3, 8])
@pytest.mark.parametrize("lam", [0.5, 3.0])
def test_tikhonov_cgls_and_damped_lsqr_match_scipy(small_problem, K, lam):
    """min |b - A x|^2 + lambda^2 |x|^2: scipy's LSQR with damp, the oracle's damped
    LSQR and the oracle's CGLS on [A; lambda I] give the same K-th iterate."""
    g, A, b = small_problem
    ref = spla.lsqr(A, b.ravel(), damp=lam, atol=0.0, btol=0.0, conlim=0.0, iter_lim=K)[0]
    rl = oracle.lsqr(g, b, K, damp=lam)
    rc = oracle.cgls(g, b, K, tikhonov=lam)
    assert rel(rl.x, ref) < 1e-8
    assert rel(rc.x, ref) < 1e-8
    # LSQR's residual estimate is the stacked residual, CGLS's NB the data residual
    x = rl.x.ravel()
    stacked = np.sqrt(np.linalg.norm(b.ravel() - A @ x) ** 2 + lam ** 2 * np.linalg.norm(x) ** 2)
    assert abs(rl.nb - stacked) <= 1e-9 * stacked
    assert abs(rc.nb - np.linalg.norm(b.ravel() - A @ rc.x.ravel())) <= 1e-9 * rc.nb


def test_tikhonov_cgls_converges_to_regularised_solution(small_problem):
    """With a strong penalty the normal matrix A^T A + lambda^2 I is well conditioned
    and the iterate reaches the dense solution of the regularised normal equations."""
    g, A, b = small_problem
    lam = 4.0
    Ad = A.toarray()
    ref = np.linalg.solve(Ad.T @ Ad + lam ** 2 * np.eye(Ad.shape[1]), Ad.T @ b.ravel())
    assert rel(oracle.cgls(g, b, 80, tikhonov=lam).x, ref) < 1e-9
    assert rel(oracle.lsqr(g, b, 80, damp=lam).x, ref) < 1e-9


@pytest.mark.parametrize("every", [1, 3])
def test_recomputed_discrepancy_gives_the_same_iterates(small_problem, every):
    """Recomputing e = b - A x every k iterations instead of updating it changes
    nothing in exact arithmetic (Section 5: the drift is below 1e-6)."""
    g, A, b = small_problem
    r0 = oracle.cgls(g, b, 10)
    r1 = oracle.cgls(g, b, 10, recompute_every=every)
    assert rel(r1.x, r0.x) < 1e-10
    np.testing.assert_allclose(r1.history, r0.history, rtol=1e-9)


def krylov_minimiser_jacobi(A, b, x0, K, M):
    """argmin |b - A x| over x0 + M span{r0, (M A^T A M) r0, ...}, r0 = M A^T (b - A x0)."""
    AM = A @ sp.diags(M)
    z = krylov_minimiser(AM, b - A @ x0, np.zeros(A.shape[1]), K)
    return x0 + M * z


@pytest.mark.parametrize("K", [1, 2, 4, 6])
def test_jacobi_cgls_is_preconditioned_krylov_minimiser(small_problem, K):
    g, A, b = small_problem
    dg = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    M = np.where(dg > 0, 1.0 / np.sqrt(np.where(dg > 0, dg, 1.0)), 0.0)
    x0 = ki.random_volume(g, 35).ravel() * 0.05
    assert rel(oracle.cgls_jacobi(g, b, K, x0=x0).x.ravel(), krylov_minimiser_jacobi(A, b.ravel(), x0, K, M)) < 1e-9
    # and the same iterate as scipy's LSQR on A M
    z = spla.lsqr(A @ sp.diags(M), b.ravel(), atol=0.0, btol=0.0, conlim=0.0, iter_lim=K)[0]
    assert rel(oracle.cgls_jacobi(g, b, K).x.ravel(), M * z) < 1e-8


def _tt_matrix(g):
    """The TT matrix, column by column: the TT oracle's projection of every unit vector."""
    cols = []
    e = np.zeros(g.n_vox)
    for j in range(g.n_vox):
        e[j] = 1.0
        cols.append(sp.csc_matrix(oracle.tt_project(g, e.reshape(g.vol_shape)).reshape(-1, 1)))
        e[j] = 0.0
    return sp.hstack(cols).tocsr()


@pytest.mark.parametrize("K", [1, 3, 6])
def test_tt_jacobi_cgls_is_preconditioned_krylov_minimiser(small_problem, K):
    """Jacobi CGLS on the TT operator (Section 5's preconditioner with the
    projector of Section 4): the iterate minimises |b - A_TT x| over
    x0 + M span{r0, (M A^T A M) r0, ...} with M = diag(A_TT^T A_TT)^(-1/2) taken
    from the explicitly formed TT matrix."""
    g, _, b = small_problem
    A = _tt_matrix(g)
    dg = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    assert rel(oracle.tt_diag_normal(g).ravel(), dg) < 1e-12
    M = np.where(dg > 0, 1.0 / np.sqrt(np.where(dg > 0, dg, 1.0)), 0.0)
    x0 = ki.random_volume(g, 36).ravel() * 0.05
    got = oracle.cgls_jacobi(g, b, K, x0=x0, projector="tt").x.ravel()
    assert rel(got, krylov_minimiser_jacobi(A, b.ravel(), x0, K, M)) < 1e-9
    z = spla.lsqr(A @ sp.diags(M), b.ravel(), atol=0.0, btol=0.0, conlim=0.0, iter_lim=K)[0]
    assert rel(oracle.cgls_jacobi(g, b, K, projector="tt").x.ravel(), M * z) < 1e-8


def test_tikhonov_cgls_with_initial_guess(small_problem):
    """With x0 the Tikhonov CGLS is CGLS on the stacked system [A; lambda I] x = [b; 0]
    started at x0: scipy's LSQR on the explicitly stacked matrix gives the same iterate."""
    g, A, b = small_problem
    lam, K = 1.5, 5
    x0 = ki.random_volume(g, 36).ravel() * 0.05
    S = sp.vstack([A, lam * sp.identity(A.shape[1], format="csr")]).tocsr()
    rhs = np.concatenate([b.ravel(), np.zeros(A.shape[1])])
    ref = spla.lsqr(S, rhs, atol=0.0, btol=0.0, conlim=0.0, iter_lim=K, x0=x0)[0]
    assert rel(oracle.cgls(g, b, K, x0=x0, tikhonov=lam).x.ravel(), ref) < 1e-8


# ------------------------------------------------------ TT footprint projector

def test_tt_uniform_volume_is_exact_chord():
    """Neighbouring voxels' trapezoids sum to one, so for a uniform volume every
    ray that enters and leaves through the two faces normal to its dominant axis
    gets exactly its chord (the same value as the Siddon projector)."""
    g = ki.t16("base").replace(n_views=2, explicit_angles=[0.0, np.pi / 2])
    ones = np.ones(g.vol_shape)
    bt = oracle.tt_project(g, ones)
    bs = oracle.project(g, ones)
    c = slice(20, 28)  # central rays: they cross the volume between the x (view 0) or y (view 1) faces
    assert np.abs(bt[:, c, c] - bs[:, c, c]).max() < 1e-12 * bs[:, c, c].max()
    # and they are the closed-form chords through the volume box
    lo = np.array([g.cx - g.nx * g.vx / 2, g.cy - g.ny * g.vy / 2, g.cz - g.nz * g.vz / 2])
    hi = lo + np.array([g.nx * g.vx, g.ny * g.vy, g.nz * g.vz])
    chord = bf.box_chord(g, lo, hi)
    assert np.abs(bt[:, c, c] - chord[:, c, c]).max() < 1e-12 * chord[:, c, c].max()


@pytest.mark.parametrize("variant", ["base", "offcenter", "aniso", "odd"])
def test_tt_support_contains_every_ray_through_the_voxel(variant):
    """The TT footprint of a voxel is its exact shadow (widened by the linear
    ramps only inside it): every ray that crosses the voxel (positive Siddon
    weight) has a positive TT weight, and no ray far outside the shadow has one."""
    g = ki.t16(variant)
    rng = np.random.default_rng(11)
    for j in rng.choice(g.n_vox, 12, replace=False):
        e = np.zeros(g.n_vox)
        e[j] = 1.0
        bs = oracle.project(g, e.reshape(g.vol_shape))
        bt = oracle.tt_project(g, e.reshape(g.vol_shape))
        assert np.all(bt[bs > 1e-9] > 0)
        assert np.all(bt >= 0)
        # TT's support is at most one pixel wider than the shadow of the rays
        ks, vs, us = np.nonzero(bt > 0)
        ks2, vs2, us2 = np.nonzero(bs > 0)
        for k in set(ks2.tolist()):
            assert us[ks == k].min() >= us2[ks2 == k].min() - 1 and us[ks == k].max() <= us2[ks2 == k].max() + 1
            assert vs[ks == k].min() >= vs2[ks2 == k].min() - 1 and vs[ks == k].max() <= vs2[ks2 == k].max() + 1


@pytest.mark.parametrize("variant", ["base", "offcenter", "odd"])
def test_tt_adjoint(variant):
    """The scatter (forward) and the gather (backward) of the TT oracle are
    each other's transpose."""
    g = ki.t16(variant)
    rng = np.random.default_rng(12)
    x = rng.standard_normal(g.vol_shape)
    y = rng.standard_normal(g.proj_shape)
    lhs = float((oracle.tt_project(g, x) * y).sum())
    rhs = float((x * oracle.tt_backproject(g, y)).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_tt_pixel_means_by_quadrature():
    """F_u F_v of single voxels against a midpoint-rule quadrature of the two
    trapezoids over each pixel (2000 x 2000 samples per pixel would be
    needless; the trapezoids are separable, so 4000 samples per axis)."""
    g = ki.ConeGeometry(4, 4, 4, 2.0, 2.0, 2.0, 3, 14, 12, 1.3, 1.1, sid=60.0, sdd=120.0, cx=0.4, cy=-0.3, cz=0.2)
    src_all, Q = bf.rays(g)
    for j in [0, 21, 42, 63]:
        iz, iy, ix = np.unravel_index(j, g.vol_shape)
        e = np.zeros(g.vol_shape)
        e[iz, iy, ix] = 1.0
        bt = oracle.tt_project(g, e)
        lo = np.array([g.cx - g.nx * g.vx / 2 + ix * g.vx, g.cy - g.ny * g.vy / 2 + iy * g.vy,
                       g.cz - g.nz * g.vz / 2 + iz * g.vz])
        for k in range(g.n_views):
            th = g.angles()[k]
            c, s = np.cos(th), np.sin(th)
            src = np.array([g.sid * c, g.sid * s, 0.0])
            corners = [(lo[0] + a * g.vx, lo[1] + b * g.vy) for a in (0, 1) for b in (0, 1)]
            dep = [-(c * (px - src[0]) + s * (py - src[1])) for px, py in corners]
            tu = sorted(g.sdd * (-s * (px - src[0]) + c * (py - src[1])) / d for (px, py), d in zip(corners, dep))
            tv = sorted(g.sdd * z / d for z in (lo[2], lo[2] + g.vz) for d in (min(dep), max(dep)))

            def trap(t, u):
                up = np.clip((u - t[0]) / max(t[1] - t[0], 1e-300), 0, 1)
                dn = np.clip((t[3] - u) / max(t[3] - t[2], 1e-300), 0, 1)
                return np.minimum(up, dn)

            for iv in range(g.nv):
                for iu in range(g.nu):
                    uc = (iu - (g.nu - 1) / 2) * g.du + g.off_u
                    vc = (iv - (g.nv - 1) / 2) * g.dv + g.off_v
                    us = uc + ((np.arange(4000) + 0.5) / 4000 - 0.5) * g.du
                    vs = vc + ((np.arange(4000) + 0.5) / 4000 - 0.5) * g.dv
                    fu, fv = trap(tu, us).mean(), trap(tv, vs).mean()
                    d = Q[k, iv, iu] - src_all[k]
                    L = min(vox / abs(di) for vox, di in zip((g.vx, g.vy, g.vz), d / np.linalg.norm(d)) if di != 0)
                    assert abs(bt[k, iv, iu] - L * fu * fv) <= 1e-6 * L, (j, k, iv, iu)


def test_tt_approaches_siddon_with_resolution():
    """Both projectors approximate the same line integrals; on a fixed smooth
    object their difference shrinks as the voxels get finer."""
    diffs = []
    for n in (16, 32, 64):
        g = ki.ConeGeometry(n, n, n, 32.0 / n, 32.0 / n, 32.0 / n, 8, 64, 64, 1.0, 1.0)
        x = ki.voxelize(g, ki.draw_ellipsoids(g, 6, 7))
        bt, bs = oracle.tt_project(g, x), oracle.project(g, x)
        diffs.append(rel(bt, bs))
    assert diffs[0] > diffs[1] > diffs[2] and diffs[2] < 0.025, diffs


@pytest.mark.parametrize("variant", ["base", "offcenter", "aniso", "odd"])
def test_tt_diag_normal_is_squared_column_norms(variant):
    """diag(A_TT^T A_TT)_j = sum_i a_ij^2 (Section 5's Jacobi diagonal for the
    TT projector), against the squared norms of the columns of A_TT formed one
    by one as the TT projection of every unit vector e_j (the matrix entries
    themselves are pinned by the quadrature test above)."""
    g = ki.t16(variant)
    ref = np.empty(g.n_vox)
    e = np.zeros(g.n_vox)
    for j in range(g.n_vox):
        e[j] = 1.0
        col = oracle.tt_project(g, e.reshape(g.vol_shape)).ravel()
        ref[j] = col @ col
        e[j] = 0.0
    got = oracle.tt_diag_normal(g).ravel()
    assert ref.min() >= 0 and ref.max() > 0
    assert np.abs(got - ref).max() <= 1e-12 * ref.max()
    assert rel(got, ref) < 1e-12


# ------------------------------------------------------------------ single-precision storage form

@pytest.mark.parametrize("solver", ["cgls", "lsqr"])
@pytest.mark.parametrize("K", [1, 3, 6])
def test_store32_iterates_are_floats_near_the_krylov_minimiser(small_problem, solver, K):
    """The storage form that keeps the solver vectors in single precision
    (Section 5) rounds every stored element: its iterate is exactly a float
    array, and it departs from the brute-force Krylov minimiser only by
    single-precision rounding (a dropped term or a misplaced update would move
    it by O(1))."""
    g, A, b = small_problem
    b32 = b.astype(np.float32).astype(np.float64)
    ref = krylov_minimiser(A, b32.ravel(), np.zeros(g.n_vox), K)
    res = getattr(oracle, solver)(g, b32, K, store32=True)
    x = res.x.ravel()
    assert np.array_equal(x, x.astype(np.float32).astype(np.float64))
    assert 0.0 < rel(x, ref) < 1e-5
    full = getattr(oracle, solver)(g, b32, K)
    assert rel(full.x, ref) < 1e-9
    np.testing.assert_allclose(res.history, full.history, rtol=1e-5)


def test_store32_first_iterate_closed_form(small_problem):
    """K = 1 with single-precision storage: x_1 = fl(alpha fl(r0)) with
    r0 = fl(A^T fl(b - fl(A x0))), alpha = |fl(r0)|^2 / |fl(A fl(r0))|^2 in
    double (the closed form of the first step, rounded where it is stored)."""
    g, A, b = small_problem
    b32 = b.astype(np.float32).astype(np.float64).ravel()
    f = lambda v: v.astype(np.float32).astype(np.float64)  # noqa: E731
    r0 = f(A.T @ f(b32))
    p = f(A @ r0)
    alpha = (r0 @ r0) / (p @ p)
    res = oracle.cgls(g, b32, 1, store32=True)
    # the brute-force matrix and the traversal differ by ~1e-13, which can move
    # an element across a float rounding boundary: allow a few such flips
    assert rel(res.x, f(alpha * r0)) < 1e-7


def test_results_do_not_depend_on_thread_count():
    """The oracle's projector, scatter backprojector and CGLS give the same bits
    with one thread as with all (the CPU baseline times both)."""
    g = ki.t16("offcenter")
    x = ki.random_volume(g, 5)
    y = ki.random_projections(g, 6)
    n = oracle.num_threads()
    try:
        oracle.set_num_threads(1)
        a1, r1, c1 = oracle.project(g, x), oracle.backproject(g, y), oracle.cgls(g, y, 3).x
        oracle.set_num_threads(max(n, 3))
        a2, r2, c2 = oracle.project(g, x), oracle.backproject(g, y), oracle.cgls(g, y, 3).x
    finally:
        oracle.set_num_threads(n)
    assert np.array_equal(a1, a2) and np.array_equal(r1, r2) and np.array_equal(c1, c2)


U32 = 2.0 ** -24  # unit roundoff of single precision


def _gamma(k):
    """gamma_k = k u / (1 - k u): the bound on the relative error of k
    successive single-precision roundings (Higham, Accuracy and Stability of
    Numerical Algorithms, Lemma 3.1)."""
    return k * U32 / (1.0 - k * U32)


@pytest.mark.parametrize("variant", ["base", "odd", "offcenter"])
def test_single_precision_projector_within_the_summation_bound(variant):
    """The single-precision form of the pair (Section 5: the GPU projectors
    compute in float) rounds every weight and input element once and every
    partial sum once per term, so per ray |A32 x - A x| <= gamma_(n+2) (|A| |x|)
    with n the ray's nonzeros, and per voxel likewise over its column (the
    standard bound for recursive fused multiply-add summation of rounded
    products).  A dropped, doubled or misplaced term breaks the bound by a
    factor ~1e6; a no-op (double arithmetic) is caught by the rounding checks."""
    g = ki.t16(variant)
    A = oracle.assemble(g)
    absA = abs(A)
    x = ki.random_volume(g, 21) - 0.5
    y = ki.random_projections(g, 22) - 0.5
    b64, b32 = oracle.project(g, x).ravel(), oracle.project32(g, x).ravel()
    r64, r32 = oracle.backproject(g, y).ravel(), oracle.backproject32(g, y).ravel()
    n_row = np.diff(A.indptr)
    n_col = np.diff(A.tocsc().indptr)
    bound_b = np.array([_gamma(k + 2) for k in n_row]) * (absA @ np.abs(x.ravel())) * (1 + 1e-9) + 1e-300
    bound_r = np.array([_gamma(k + 2) for k in n_col]) * (absA.T @ np.abs(y.ravel())) * (1 + 1e-9) + 1e-300
    assert np.all(np.abs(b32 - b64) <= bound_b)
    assert np.all(np.abs(r32 - r64) <= bound_r)
    # single precision in fact: every result is a float, and the results differ
    assert np.array_equal(b32, b32.astype(np.float32).astype(np.float64))
    assert np.array_equal(r32, r32.astype(np.float32).astype(np.float64))
    assert np.any(b32 != b64) and np.any(r32 != r64)


def test_single_precision_solve_stays_near_the_double_solve(small_problem):
    """CGLS and LSQR with the single-precision pair and single-precision storage
    (the precision structure of a float GPU path with double scalars): iterates
    are floats, within single-precision rounding of the FP64 solve at small K,
    and not equal to it; the preconditioned solver refuses the form."""
    g, A, b = small_problem
    b32 = b.astype(np.float32).astype(np.float64)
    for solver in ("cgls", "lsqr"):
        full = getattr(oracle, solver)(g, b32, 4)
        res = getattr(oracle, solver)(g, b32, 4, projector="siddon32", store32=True)
        x = res.x.ravel()
        assert np.array_equal(x, x.astype(np.float32).astype(np.float64))
        assert 0.0 < rel(x, full.x) < 1e-5
        np.testing.assert_allclose(res.history, full.history, rtol=1e-5)
    with pytest.raises(ValueError):
        oracle.cgls_jacobi(g, b32, 2, projector="siddon32")
