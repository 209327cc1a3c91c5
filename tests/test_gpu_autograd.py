"""Differentiable form: autograd through the projector pair and unrolled CGLS.

Checks, with the double-precision instantiation of the kernels (float64
tensors: the same single-precision weights, double accumulation):
  * torch.autograd.gradcheck of A and A^T on a tiny geometry (full Jacobian);
  * on the 24^3 instance (2 mm voxels, 24 views, 48 x 48 detector of 2 mm):
    the directional derivative of L(x) = |A x - y|^2 / 2 by central finite
    differences against <grad L, v> (L is quadratic, so central differences
    are exact up to rounding), and grad L against the FP64 oracle's
    A^T (A x - y) (the GPU matrix has single-precision weights: 1e-5);
  * 8 unrolled CGLS iterations, loss |x_8 - x_true|^2, gradient in b:
    checkpointed and plain backward agree, the forward equals the library's
    CGLS, and the directional derivative matches central finite differences
    of the GPU unrolled CGLS and of the FP64 oracle CGLS.
"""
import numpy as np
import pytest

import kct_inputs as ki
import oracle
from tests.gpu_util import dev, geometry, rel, say, to_np, torch_mod

pytestmark = pytest.mark.gpu


def _t(a, dtype):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev()).to(dtype)


def tiny():
    return ki.ConeGeometry(nx=5, ny=4, nz=3, vx=2.0, vy=2.5, vz=3.0, n_views=3, nu=7, nv=5, du=2.0, dv=2.5,
                           sid=200.0, sdd=400.0, cx=0.7, cy=-0.4, cz=0.3)


def test_gradcheck_tiny_fp64():
    torch = torch_mod()
    from paper_2110_13526_amd.autograd import backproject_fn, project_fn
    g = tiny()
    G = geometry(g)
    say("[autograd] gradcheck tiny")
    rng = np.random.default_rng(3)
    x = _t(rng.standard_normal(g.vol_shape), torch.float64).requires_grad_(True)
    y = _t(rng.standard_normal(g.proj_shape), torch.float64).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: project_fn(G, t), (x,), eps=1e-6, atol=1e-9, rtol=1e-7)
    assert torch.autograd.gradcheck(lambda t: backproject_fn(G, t), (y,), eps=1e-6, atol=1e-9, rtol=1e-7)
    # batched input: a leading batch dimension is projected item by item
    xb = _t(rng.standard_normal((2,) + g.vol_shape), torch.float64).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: project_fn(G, t), (xb,), eps=1e-6, atol=1e-9, rtol=1e-7)


@pytest.fixture(scope="module")
def fd24():
    g = ki.config("fd24")
    x_true = ki.phantom(g, 10, ki.SEEDS["fd24"])
    b = oracle.project(g, x_true.astype(np.float64))
    b = ki.gaussian_noise(b, 0.005, ki.SEEDS["fd24"] + 1_000_000)
    return g, geometry(g), x_true, b


def test_quadratic_loss_gradient_fd_and_oracle(fd24):
    torch = torch_mod()
    from paper_2110_13526_amd.autograd import project_fn
    g, G, x_true, b = fd24
    rng = np.random.default_rng(5)
    x0 = 0.5 * x_true + 0.1 * rng.standard_normal(g.vol_shape)
    v = rng.standard_normal(g.vol_shape)
    yt = _t(b, torch.float64)

    def loss(xt):
        res = project_fn(G, xt) - yt
        return 0.5 * (res * res).sum()

    x = _t(x0, torch.float64).requires_grad_(True)
    L = loss(x)
    (grad,) = torch.autograd.grad(L, x)
    gn = to_np(grad)
    eps = 1e-3
    with torch.no_grad():
        lp = loss(_t(x0 + eps * v, torch.float64)).item()
        lm = loss(_t(x0 - eps * v, torch.float64)).item()
    fd = (lp - lm) / (2 * eps)
    an = float((gn * v).sum())
    say(f"[autograd] fd24 quadratic: fd {fd:.12e} autograd {an:.12e}")
    assert abs(fd - an) <= 1e-9 * abs(an)
    ref = oracle.backproject(g, oracle.project(g, x0) - b)
    err = rel(gn, ref)
    say(f"[autograd] fd24 gradient vs oracle A^T(Ax - b): rel {err:.3e}")
    assert err < 1e-5


def test_unrolled_cgls_checkpoint_forward_and_fd(fd24):
    torch = torch_mod()
    import paper_2110_13526_amd as kct
    from paper_2110_13526_amd.autograd import cgls_unrolled
    g, G, x_true, b = fd24
    K = 8
    xt64 = _t(x_true, torch.float64)

    def loss_of(bt, checkpoint=True):
        xk = cgls_unrolled(G, bt, K, checkpoint=checkpoint)
        return ((xk - xt64) ** 2).sum(), xk

    b64 = _t(b, torch.float64).requires_grad_(True)
    L1, xk = loss_of(b64, True)
    (g1,) = torch.autograd.grad(L1, b64)
    b64b = _t(b, torch.float64).requires_grad_(True)
    L2, _ = loss_of(b64b, False)
    (g2,) = torch.autograd.grad(L2, b64b)
    say(f"[autograd] unrolled K={K}: checkpoint vs plain grad rel {rel(to_np(g1), to_np(g2)):.3e}")
    assert rel(to_np(g1), to_np(g2)) < 1e-12

    # forward: the library's CGLS (FP32 vectors) and the FP64 oracle
    xlib, _ = kct.cgls(G, _t(b, torch.float32), K)
    ref = oracle.cgls(g, b, K)
    say(f"[autograd] x_K vs library cgls {rel(to_np(xk), to_np(xlib)):.3e}, vs oracle {rel(to_np(xk), ref.x):.3e}")
    assert rel(to_np(xk), to_np(xlib)) < 1e-4
    assert rel(to_np(xk), ref.x) < 1e-5

    # directional derivative in b: autograd vs central differences (GPU, FP64)
    rng = np.random.default_rng(9)
    v = rng.standard_normal(g.proj_shape) * np.abs(b).mean()
    an = float((to_np(g1) * v).sum())
    h = 1e-5
    with torch.no_grad():
        lp = loss_of(_t(b + h * v, torch.float64))[0].item()
        lm = loss_of(_t(b - h * v, torch.float64))[0].item()
    fd = (lp - lm) / (2 * h)
    say(f"[autograd] unrolled d/dh: autograd {an:.10e} fd {fd:.10e}")
    assert abs(fd - an) <= 1e-6 * abs(an)

    # the same directional derivative from the FP64 oracle's CGLS
    def oracle_loss(bb):
        xo = oracle.cgls(g, bb, K).x
        return float(((xo - x_true) ** 2).sum())

    fdo = (oracle_loss(b + h * v) - oracle_loss(b - h * v)) / (2 * h)
    say(f"[autograd] unrolled d/dh oracle fd {fdo:.10e}")
    assert abs(fdo - an) <= 1e-4 * abs(an)


def test_batched_c5_shape_adjoint():
    """The differentiable form's batch: 4 volumes of 192^3, 180 views, 256 x 256
    detector; the backward of a projection is the backprojection of the output
    gradient, so <A x, w> = <x, A^T w> per item through autograd.  The two sides
    share their weights bit for bit and differ only by single-precision summation,
    so the difference is bounded relative to |A x| |w| (the Cauchy-Schwarz bound of
    the dot product), as in the projector's own adjoint test; relative to the
    cancelling sum <A x, w> of a zero-mean w it is ~1e-5."""
    torch = torch_mod()
    from paper_2110_13526_amd.autograd import project_fn
    g = ki.config("c5")
    G = geometry(g)
    say("[autograd] c5 batch")
    x = torch.stack([_t(ki.phantom(g, 10, ki.SEEDS["c5"] + i), torch.float32) for i in range(4)])
    x.requires_grad_(True)
    b = project_fn(G, x)
    w = torch.randn(b.shape, generator=torch.Generator(device=dev()).manual_seed(1), device=dev())
    (gx,) = torch.autograd.grad((b * w).sum(), x)
    lhs = (b.double() * w.double()).sum(dim=(1, 2, 3))
    rhs = (x.detach().double() * gx.double()).sum(dim=(1, 2, 3))
    scale = b.detach().double().flatten(1).norm(dim=1) * w.double().flatten(1).norm(dim=1)
    err = ((lhs - rhs).abs() / scale).max().item()
    say(f"[autograd] c5 adjoint max |lhs - rhs| / (|Ax| |w|) {err:.3e}, "
        f"relative to |lhs| {((lhs - rhs).abs() / lhs.abs()).max().item():.3e}")
    assert err < 1e-5


def test_unrolled_cgls_c5_fp32_checkpointed():
    """The differentiable form at its configured size: a batch of 4 volumes of
    192^3 (0.5 mm), 180 views, 256 x 256 detector (0.8 mm), float32 tensors, 8
    unrolled CGLS iterations (Algorithm 1) with per-iteration checkpointing,
    loss |x_8 - x_true|^2, gradient in b.  The checkpointed and the plain
    backward recompute the same deterministic kernels, so their gradients agree;
    x_8 of every item equals the library's CGLS (FP32 vectors, FP64 scalars in
    both) within the solver bound 1e-4.  Peak device memory of both backward
    passes is reported."""
    torch = torch_mod()
    import paper_2110_13526_amd as kct
    from paper_2110_13526_amd.autograd import cgls_unrolled
    g = ki.config("c5")
    G = geometry(g)
    K, n = 8, 4
    say("[autograd] c5 unrolled CGLS: phantoms")
    xs = torch.stack([_t(ki.phantom(g, 10, ki.SEEDS["c5"] + i), torch.float32) for i in range(n)])
    with torch.no_grad():
        bc = torch.stack([kct.project(G, xs[i]) for i in range(n)])
    gen = torch.Generator(device=dev()).manual_seed(5)
    sigma = 0.005 * bc.flatten(1).max(dim=1).values.view(n, 1, 1, 1)
    b = (bc + sigma * torch.randn(bc.shape, generator=gen, device=dev())).contiguous()
    del bc
    grads, peaks = {}, {}
    for ck in (True, False):
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        bb = b.clone().requires_grad_(True)
        xk = cgls_unrolled(G, bb, K, checkpoint=ck)
        loss = ((xk - xs) ** 2).sum()
        (gb,) = torch.autograd.grad(loss, bb)
        torch.cuda.synchronize()
        peaks[ck] = (torch.cuda.max_memory_allocated() - base) / 2 ** 20
        grads[ck] = gb
        if ck:
            x_ck = xk.detach()
        del xk, loss, bb
    err_g = (torch.linalg.vector_norm((grads[True] - grads[False]).double())
             / torch.linalg.vector_norm(grads[False].double())).item()
    say(f"[autograd] c5 K={K}: checkpointed vs plain gradient rel {err_g:.3e}; peak memory above inputs "
        f"{peaks[True]:.0f} MiB checkpointed, {peaks[False]:.0f} MiB plain")
    assert err_g < 1e-6
    assert peaks[True] < peaks[False]
    for i in range(n):
        xl, info = kct.cgls(G, b[i].contiguous(), K)
        e = rel(to_np(x_ck[i]), to_np(xl))
        say(f"[autograd] c5 item {i}: x_8 vs library CGLS rel {e:.3e}")
        assert e < 1e-4
