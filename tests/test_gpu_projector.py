"""GPU parity of the projector pair against the FP64 oracle (through the C ABI).

Tolerance: relative L2 error 1e-5 for single-precision projections and
backprojections (storage and accumulation in float32; the oracle in float64).
"""
import numpy as np
import pytest

import kct_inputs as ki
import oracle
from tests.gpu_util import dev, geometry, rel, say, to_dev, to_np, torch_mod

pytestmark = pytest.mark.gpu

TOL = 1e-5

SMALL = {
    "t16": ki.t16("base"),
    "t16_offcenter": ki.t16("offcenter"),
    "t16_aniso": ki.t16("aniso"),
    "t16_odd": ki.t16("odd"),
    "c1": ki.config("c1"),
    # ragged: detector not a multiple of the 64 x 4 ray tile, volume not a
    # multiple of the 16 x 16 voxel tile, views at 45 degrees (dominant-axis switch)
    "ragged": ki.ConeGeometry(37, 29, 23, 0.9, 1.1, 1.3, n_views=7, nu=77, nv=19, du=1.3, dv=1.7, cx=1.2,
                              cy=-0.7, cz=2.1, off_u=0.9, off_v=-1.4, angle0=np.pi / 4),
    "one_voxel": ki.ConeGeometry(1, 1, 1, 3.0, 3.0, 3.0, n_views=5, nu=9, nv=7, du=1.0, dv=1.0),
    "one_column": ki.ConeGeometry(8, 8, 8, 1.0, 1.0, 1.0, n_views=3, nu=1, nv=1, du=1.0, dv=1.0),
}


@pytest.fixture(scope="module", params=sorted(SMALL))
def case(request):
    name = request.param
    g = SMALL[name]
    say(f"[projector] case {name}: vol {g.vol_shape} proj {g.proj_shape}")
    return name, g, geometry(g)


def test_forward_matches_oracle(case):
    name, g, G = case
    import paper_2110_13526_amd as kct
    # white noise (every crossing error shows) and phantom data, off-centre geometries included
    for x in (ki.random_volume(g, 1), ki.phantom(g, 8, 2, dtype=np.float64)):
        x32 = x.astype(np.float32)
        b = to_np(kct.project(G, to_dev(x32)))
        ref = oracle.project(g, x32.astype(np.float64))
        if np.linalg.norm(ref) == 0:
            assert np.abs(b).max() == 0
        else:
            assert rel(b, ref) < TOL, (name, rel(b, ref))


def test_backward_matches_oracle(case):
    """Positive projection values (no cancellation inside a voxel's sum)."""
    name, g, G = case
    import paper_2110_13526_amd as kct
    y = (1.0 + 0.5 * ki.random_projections(g, 3)).astype(np.float32)
    r = to_np(kct.backproject(G, to_dev(y)))
    ref = oracle.backproject(g, y.astype(np.float64))
    if np.linalg.norm(ref) == 0:
        assert np.abs(r).max() == 0
    else:
        assert rel(r, ref) < TOL, (name, rel(r, ref))


def test_backward_signed_matches_oracle(case):
    """Signed projection values (uniform in [-1, 1]), voxel by voxel.

    With cancellation inside a voxel's sum a relative L2 bound says little, so
    each voxel is held to the size of the terms around it.  A single-precision
    crossing position is off by ~1e-6 of a voxel (its absolute rounding), which
    moves a piece of the ray's length between the two voxels that share the
    crossed plane: negligible against a voxel's own sum sum_i |w_ij| |y_i| unless
    the voxel holds only tiny clips of rays (the edge of the truncated field of
    view of the 64^3 problem: such a voxel is off by up to 2.2e-3 of its own tiny
    sum, ~1e-6 absolute).  The neighbour across the crossed plane holds the
    longer piece of those rays, so every voxel's error is bounded by 1e-5 times
    the largest sum_i |w_ik| |y_i| over its 3 x 3 x 3 neighbourhood; voxels
    that no ray reaches are exactly zero."""
    from scipy.ndimage import maximum_filter
    name, g, G = case
    import paper_2110_13526_amd as kct
    y = ki.random_projections(g, 9).astype(np.float32)  # uniform in [-1, 1]
    r = to_np(kct.backproject(G, to_dev(y)))
    ref = oracle.backproject(g, y.astype(np.float64))
    own = oracle.backproject(g, np.abs(y).astype(np.float64))
    near = maximum_filter(own, size=3, mode="constant", cval=0.0)
    err = np.abs(r - ref)
    q_own = err / np.maximum(own, 1e-300)
    say(f"[projector] signed backward {name}: max |err| / own sum {float(q_own.max()):.2e}, "
        f"/ neighbourhood sum {float((err / np.maximum(near, 1e-300)).max()):.2e}, "
        f"voxels above 1e-5 of their own sum: {int((q_own > 1e-5).sum())} of {g.n_vox}")
    assert np.all(err <= 1e-5 * near), (name, float((err / np.maximum(near, 1e-300)).max()))
    assert np.all(r[own == 0] == 0)


def test_adjoint_identity(case):
    """<A x, y> = <x, A^T y> on the GPU (weights are shared, only summation order differs)."""
    name, g, G = case
    import paper_2110_13526_amd as kct
    x = ki.random_volume(g, 4).astype(np.float32)
    y = ki.random_projections(g, 5).astype(np.float32)
    ax = to_np(kct.project(G, to_dev(x)))
    aty = to_np(kct.backproject(G, to_dev(y)))
    lhs = float((ax * y).sum())
    rhs = float((x.astype(np.float64) * aty).sum())
    scale = np.linalg.norm(ax) * np.linalg.norm(y) + 1e-30
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_layouts_and_determinism(case):
    """The transposed-copy layout and the plain layout give bitwise equal projections;
    repeated runs are bitwise equal."""
    name, g, G = case
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    x = to_dev(ki.phantom(g, 6, 7))
    b1 = kct.project(G, x)
    b2 = kct.project(G, x, transposed_copy=False)
    b3 = kct.project(G, x)
    assert torch.equal(b1, b2) and torch.equal(b1, b3)
    y = to_dev(ki.random_projections(g, 8))
    r1 = kct.backproject(G, y)
    r2 = kct.backproject(G, y)
    assert torch.equal(r1, r2)


@pytest.mark.parametrize("name", ["t16", "t16_odd", "t16_offcenter", "ragged"])
def test_weights_bitwise_identical(name):
    """A e_j (a column of A) and A^T e_i (a row of A) contain the same weight bits:
    the forward kernel returns L_i * w_ij, the backprojector w_ij * (L_i * 1)."""
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    g = SMALL[name]
    G = geometry(g)
    rng = np.random.default_rng(11)
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
            # same sparsity: the ray's row has a positive entry exactly where its walk found one
            checked += 1
    assert checked > 0


@pytest.mark.parametrize("name", ["t16_odd", "t16_offcenter", "t16_aniso", "ragged"])
def test_backward_takes_every_weight(name):
    """Completeness of the backprojector's candidate search (detector shadow,
    hit columns, candidate rows), voxel by voxel: with the columns of A from
    the forward of every unit vector e_j, (A^T y)_j = sum_i A_ij y_i is formed
    in double precision for a positive y and compared with the backprojection
    of y in every voxel.  A voxel the rays miss must come out exactly zero; any
    other differs only by single-precision summation of its few dozen terms
    (relative 1e-5), so a weight the candidate search dropped shows up in its
    voxel unless it is below that fraction of the voxel's total."""
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    g = {"t16_odd": ki.t16("odd"), "t16_offcenter": ki.t16("offcenter"), "t16_aniso": ki.t16("aniso"),
         "ragged": SMALL["ragged"]}[name]
    G = geometry(g)
    say(f"[projector] explicit A^T y on {name}: {g.n_vox} forward launches")
    rng = np.random.default_rng(17)
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
    say(f"  voxels hit {int((~miss).sum())} of {g.n_vox}, max relative error {err:.3e}")
    assert err < 1e-5


def test_orientation_on_gpu():
    """At view angle 0 an object at +y lands on +u and +z on +v (as the oracle)."""
    import paper_2110_13526_amd as kct
    g = ki.t16().replace(n_views=1)
    x = np.zeros(g.vol_shape, np.float32)
    x[12, 12, 8] = 1.0
    b = to_np(kct.project(geometry(g), to_dev(x)))[0]
    iv, iu = np.unravel_index(np.argmax(b), b.shape)
    assert iu > g.nu / 2 and iv > g.nv / 2


def test_invalid_arguments_rejected():
    import paper_2110_13526_amd as kct
    from paper_2110_13526_amd import _lib
    torch = torch_mod()
    g = ki.t16()
    with pytest.raises(kct.KctError) as ei:
        kct.Geometry.from_desc(g.replace(sdd=400.0), device=dev())  # SDD < SID
    assert ei.value.status == _lib.KCT_ERR_INVALID_ARG
    with pytest.raises(kct.KctError):
        kct.Geometry.from_desc(g.replace(nx=0), device=dev())
    with pytest.raises(kct.KctError):
        kct.Geometry.from_desc(g.replace(vx=400.0), device=dev())  # volume reaches the source
    G = geometry(g)
    b = to_dev(np.zeros(g.proj_shape, np.float32))
    ws = torch.empty(16, dtype=torch.uint8, device=dev())
    with pytest.raises(kct.KctError) as ei:
        kct.cgls(G, b, 3, workspace=ws)
    assert ei.value.status == _lib.KCT_ERR_WORKSPACE
    with pytest.raises(ValueError):
        kct.project(G, to_dev(np.zeros((3, 3, 3), np.float32)))


# ------------------------------------------------------------------ full sizes

FULL = ["c2", "c3"]


@pytest.mark.parametrize("name", FULL)
def test_full_size_sampled_parity(name):
    """At the benchmark sizes: sampled rays of A x_true and sampled voxels of A^T e
    against the oracle evaluated one output at a time."""
    import paper_2110_13526_amd as kct
    g = ki.config(name)
    say(f"[projector] full size {name}: phantom")
    x = ki.phantom(g, ki.N_ELLIPSOIDS[name], ki.SEEDS[name])
    G = geometry(g)
    xd = to_dev(x)
    b = kct.project(G, xd)
    rng = np.random.default_rng(99)
    rays = rng.choice(g.n_rays, 2000, replace=False)
    torch = torch_mod()
    bs = to_np(b.view(-1)[torch.from_numpy(rays).to(dev())])
    say(f"[projector] full size {name}: oracle rays")
    ref = oracle.project_rays(g, x.astype(np.float64), rays)
    assert rel(bs, ref) < TOL, rel(bs, ref)
    # backprojection of a smooth, fully supported projection set
    e = (b / b.max()).contiguous()
    r = kct.backproject(G, e)
    vox = rng.choice(g.n_vox, 300, replace=False)
    rs = to_np(r.view(-1)[torch.from_numpy(vox).to(dev())])
    say(f"[projector] full size {name}: oracle voxels")
    e64 = to_np(e)
    refv = oracle.backproject_voxels(g, e64, vox)
    assert rel(rs, refv) < TOL, rel(rs, refv)
    del b, r, e, xd
    torch.cuda.empty_cache()
