"""The separable trapezoid-footprint (TT) projector pair on the GPU against the
FP64 oracle, through the C ABI (Section 3's projector model; the projector of
the experiments in Section 4).

Tolerances as for the Siddon pair: relative L2 error 1e-5 for single-precision
projections and backprojections (also with double storage, whose weights are
the same single-precision numbers; its adjoint identity holds to 1e-12), plus
one storage rounding for BF16 / FP16, and 1e-4 for FP32 solver iterates after K
iterations.
"""
import numpy as np
import pytest

import kct_inputs as ki
import oracle
from tests.gpu_util import dev, rel, say, to_dev, to_np, torch_mod

pytestmark = pytest.mark.gpu

TOL = 1e-5

SMALL = {
    "t16": ki.t16("base"),
    "t16_offcenter": ki.t16("offcenter"),
    "t16_aniso": ki.t16("aniso"),
    "t16_odd": ki.t16("odd"),
    "c1": ki.config("c1"),
    # detector not a multiple of the 64-row / 4-column ray tile, volume not a
    # multiple of the 16^3 brick, views through 45 degrees
    "ragged": ki.ConeGeometry(37, 29, 23, 0.9, 1.1, 1.3, n_views=7, nu=77, nv=19, du=1.3, dv=1.7, cx=1.2,
                              cy=-0.7, cz=2.1, off_u=0.9, off_v=-1.4, angle0=np.pi / 4),
    "one_voxel": ki.ConeGeometry(1, 1, 1, 3.0, 3.0, 3.0, n_views=5, nu=9, nv=7, du=1.0, dv=1.0),
}


def tt_geometry(desc):
    import paper_2110_13526_amd as kct
    return kct.Geometry.from_desc(desc, device=dev(), projector="tt")


@pytest.fixture(scope="module", params=sorted(SMALL))
def case(request):
    name = request.param
    g = SMALL[name]
    say(f"[tt] case {name}: vol {g.vol_shape} proj {g.proj_shape}")
    return name, g, tt_geometry(g)


def test_forward_matches_oracle(case):
    name, g, G = case
    import paper_2110_13526_amd as kct
    for x in (ki.random_volume(g, 1), ki.phantom(g, 8, 2, dtype=np.float64)):
        x32 = x.astype(np.float32)
        b = to_np(kct.project(G, to_dev(x32)))
        ref = oracle.tt_project(g, x32.astype(np.float64))
        err = rel(b, ref)
        say(f"  forward rel {err:.3e}")
        assert err < TOL, (name, err)


def test_backward_matches_oracle(case):
    name, g, G = case
    import paper_2110_13526_amd as kct
    y = (1.0 + 0.5 * ki.random_projections(g, 3)).astype(np.float32)
    r = to_np(kct.backproject(G, to_dev(y)))
    ref = oracle.tt_backproject(g, y.astype(np.float64))
    err = rel(r, ref)
    say(f"  backward rel {err:.3e}")
    assert err < TOL, (name, err)


def test_layouts_and_determinism(case):
    name, g, G = case
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    x = to_dev(ki.phantom(g, 6, 7))
    b1 = kct.project(G, x)
    b2 = kct.project(G, x, transposed_copy=False)
    b3 = kct.project(G, x)
    assert torch.equal(b1, b2) and torch.equal(b1, b3)
    y = to_dev(ki.random_projections(g, 8))
    assert torch.equal(kct.backproject(G, y), kct.backproject(G, y))


def test_double_precision_matches_oracle(case):
    """FP64 storage and accumulation: the pair reproduces the oracle to rounding."""
    name, g, G = case
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    x = ki.random_volume(g, 5).astype(np.float64)
    y = ki.random_projections(g, 6).astype(np.float64)
    b = to_np(kct.project(G, torch.from_numpy(x).to(dev())))
    r = to_np(kct.backproject(G, torch.from_numpy(y).to(dev())))
    eb, er = rel(b, oracle.tt_project(g, x)), rel(r, oracle.tt_backproject(g, y))
    say(f"  f64 forward {eb:.3e} backward {er:.3e}")
    # the weights are formed in single precision on both sides of the pair
    # (bitwise equal in the kernels), the oracle forms them in double
    assert eb < TOL and er < TOL
    lhs = float(np.dot(b.ravel(), y.ravel()))
    rhs = float(np.dot(x.ravel(), r.ravel()))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(b) * np.linalg.norm(y)


@pytest.mark.parametrize("name", ["t16", "t16_odd", "t16_offcenter", "ragged"])
def test_weights_bitwise_identical(name):
    """A column of A (forward of e_j) and a row of A (backprojection of e_i) hold the same weight bits."""
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    g = SMALL[name]
    G = tt_geometry(g)
    rng = np.random.default_rng(12)
    checked = 0
    for j in rng.choice(g.n_vox, 8, replace=False):
        x = torch.zeros(g.n_vox, dtype=torch.float32, device=dev())
        x[j] = 1.0
        col = kct.project(G, x.view(g.vol_shape)).view(-1)
        nz = torch.nonzero(col).view(-1).cpu().numpy()
        for i in rng.choice(nz, min(6, nz.size), replace=False) if nz.size else []:
            y = torch.zeros(g.n_rays, dtype=torch.float32, device=dev())
            y[i] = 1.0
            row = kct.backproject(G, y.view(g.proj_shape)).view(-1)
            assert row[j].view(torch.int32).item() == col[i].view(torch.int32).item()
            checked += 1
    assert checked > 0


@pytest.mark.parametrize("name", ["t16_odd", "t16_offcenter", "ragged"])
def test_backward_takes_every_weight(name):
    """Completeness of the TT backprojector's candidates (detector shadow,
    footprint pixel ranges), voxel by voxel: (A^T y)_j = sum_i A_ij y_i from
    the forward of every unit vector e_j, in double precision for a positive y,
    against the backprojection of y.  Voxels no footprint reaches must be
    exactly zero, the others agree to single-precision summation (1e-5)."""
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    g = SMALL[name]
    G = tt_geometry(g)
    say(f"[tt] explicit A^T y on {name}: {g.n_vox} forward launches")
    rng = np.random.default_rng(18)
    y = torch.from_numpy((1.0 + 0.5 * rng.random(g.proj_shape)).astype(np.float32)).to(dev())
    y64 = y.double().view(-1)
    x = torch.zeros(g.n_vox, dtype=torch.float32, device=dev())
    ref = torch.empty(g.n_vox, dtype=torch.float64, device=dev())
    for j in range(g.n_vox):
        x.zero_()
        x[j] = 1.0
        ref[j] = (kct.project(G, x.view(g.vol_shape)).view(-1).double() * y64).sum()
    r = kct.backproject(G, y).view(-1).double()
    miss = ref == 0
    assert torch.equal(r[miss], ref[miss])
    err = ((r[~miss] - ref[~miss]).abs() / ref[~miss]).max().item()
    say(f"  voxels reached {int((~miss).sum())} of {g.n_vox}, max relative error {err:.3e}")
    assert err < 1e-5


@pytest.mark.parametrize("name", ["t16_offcenter", "ragged", "c1"])
def test_diag_normal(name):
    import paper_2110_13526_amd as kct
    g = SMALL[name]
    G = tt_geometry(g)
    err = rel(to_np(kct.diag_normal(G)), oracle.tt_diag_normal(g))
    say(f"[tt] diag {name}: rel {err:.3e}")
    assert err < TOL


def test_projector_switch_and_reject():
    """Switching the model changes the operator; unknown models are rejected."""
    import paper_2110_13526_amd as kct
    g = SMALL["t16"]
    G = tt_geometry(g)
    x = to_dev(ki.phantom(g, 6, 3))
    bt = to_np(kct.project(G, x))
    G.set_projector("siddon")
    bs = to_np(kct.project(G, x))
    assert rel(bs, oracle.project(g, to_np(x))) < TOL
    assert rel(bt, bs) > 1e-3
    with pytest.raises(ValueError):
        G.set_projector("joseph")
    from paper_2110_13526_amd import _lib
    assert _lib.load().kct_geometry_set_projector(G.handle, 7) == _lib.KCT_ERR_INVALID_ARG
    with pytest.raises(Exception):
        kct.Batch([tt_geometry(g)])


@pytest.fixture(scope="module")
def c1_tt():
    g = ki.config("c1")
    x_true = ki.phantom(g, ki.N_ELLIPSOIDS["c1"], ki.SEEDS["c1"])
    b = oracle.tt_project(g, x_true.astype(np.float64))
    b = ki.gaussian_noise(b, 0.005, ki.SEEDS["c1"] + 1_000_000).astype(np.float32)
    return g, tt_geometry(g), b


@pytest.mark.parametrize("solver", ["cgls", "lsqr"])
def test_solvers_match_oracle(c1_tt, solver):
    import paper_2110_13526_amd as kct
    g, G, b = c1_tt
    K = 10
    ref = getattr(oracle, solver)(g, b.astype(np.float64), K, projector="tt")
    x, info = getattr(kct, solver)(G, to_dev(b), K, history=True)
    err = rel(to_np(x), ref.x)
    herr = float(np.max(np.abs(to_np(info.history) - ref.history) / ref.history))
    say(f"[tt] {solver}: x rel {err:.3e}, history {herr:.3e}")
    assert err < 1e-4 and herr < 1e-4


def test_cgls_jacobi(c1_tt):
    """Jacobi-preconditioned CGLS (Section 5) with the TT pair and the TT
    diagonal, against the oracle's Jacobi CGLS on the TT operator: the
    discrepancy history and z = diag^(1/2) x over every voxel within the FP32
    solver bound (the tiny diagonal entries at the cone boundary amplify
    weight rounding in x itself, see the Siddon test)."""
    import paper_2110_13526_amd as kct
    g, G, b = c1_tt
    K = 10
    ref = oracle.cgls_jacobi(g, b.astype(np.float64), K, projector="tt")
    x, info = kct.cgls(G, to_dev(b), K, jacobi=True, history=True)
    assert info.iterations == ref.iterations == K
    diag = oracle.tt_diag_normal(g)
    sw = np.sqrt(diag)
    xn = to_np(x)
    mask = diag >= 1e-3 * diag.max()
    err_z = rel(sw * xn, sw * ref.x)
    err = rel(xn[mask], ref.x[mask])
    herr = float(np.max(np.abs(to_np(info.history) - ref.history) / ref.history))
    say(f"[tt] cgls jacobi: z rel {err_z:.3e} (all voxels), x rel {err:.3e} on {mask.mean():.3f} of the voxels "
        f"({rel(xn, ref.x):.3e} on all), history {herr:.3e}")
    assert err_z < 1e-4 and err < 1e-4 and herr < 1e-4


def test_cgls_tikhonov_and_recompute(c1_tt):
    import paper_2110_13526_amd as kct
    g, G, b = c1_tt
    ref = oracle.cgls(g, b.astype(np.float64), 8, tikhonov=20.0, projector="tt")
    x, _ = kct.cgls(G, to_dev(b), 8, tikhonov=20.0)
    assert rel(to_np(x), ref.x) < 1e-4
    ref = oracle.cgls(g, b.astype(np.float64), 8, recompute_every=3, projector="tt")
    x, _ = kct.cgls(G, to_dev(b), 8, recompute_every=3)
    assert rel(to_np(x), ref.x) < 1e-4


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("name", ["t16_offcenter", "c1"])
def test_storage_types(name, dt):
    """16-bit storage with FP32 accumulation: the oracle gets the storage-rounded
    input, so the error is the FP32 weight bound plus one rounding of each output
    (2^-9 for BF16, 2^-11 for FP16)."""
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    tdt = {"bf16": torch.bfloat16, "f16": torch.float16}[dt]
    bound = TOL + {"bf16": 2.0 ** -9, "f16": 2.0 ** -11}[dt]
    g = SMALL[name]
    G = tt_geometry(g)
    x = torch.from_numpy(ki.phantom(g, 8, 5)).to(dev()).to(tdt)
    b = kct.project(G, x)
    assert b.dtype == tdt
    eb = rel(to_np(b), oracle.tt_project(g, to_np(x)))
    y = torch.from_numpy(np.abs(ki.random_projections(g, 9)).astype(np.float32)).to(dev()).to(tdt)
    r = kct.backproject(G, y)
    er = rel(to_np(r), oracle.tt_backproject(g, to_np(y)))
    say(f"[tt] {name} {dt}: forward {eb:.3e} backward {er:.3e} (bound {bound:.3e})")
    assert eb < bound and er < bound


def test_autograd_pair_is_adjoint():
    """The autograd wrappers on a TT geometry: the gradient of <A x, y> is A^T y."""
    import paper_2110_13526_amd as kct
    from paper_2110_13526_amd.autograd import project_fn
    torch = torch_mod()
    g = SMALL["t16_offcenter"]
    G = tt_geometry(g)
    x = torch.from_numpy(ki.random_volume(g, 3).astype(np.float64)).to(dev()).requires_grad_(True)
    y = torch.from_numpy(ki.random_projections(g, 4).astype(np.float64)).to(dev())
    (project_fn(G, x) * y).sum().backward()
    ref = oracle.tt_backproject(g, to_np(y))
    err = rel(to_np(x.grad), ref)
    say(f"[tt] autograd grad vs oracle A^T y: {err:.3e}")
    assert err < TOL
    assert rel(to_np(x.grad), to_np(kct.backproject(G, y))) == 0.0
