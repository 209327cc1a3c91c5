"""Differentiable form of the projector pair and of CGLS (Algorithm 1).

    b = project_fn(g, x)        # forward A x, backward A^T (hand-written gather)
    r = backproject_fn(g, y)    # forward A^T y, backward A
    x_K = cgls_unrolled(g, b, K, checkpoint=True)

A is linear, so the derivative of x -> A x is A itself and its adjoint is
A^T: the backward of ``project_fn`` is one backprojection and the backward of
``backproject_fn`` one projection, both through the C ABI.  Because the two
kernels evaluate bitwise identical weights, the gradient is the exact adjoint
of the forward map up to accumulation rounding (with float64 tensors the
accumulation is double precision, so finite differences in double precision
see the same matrix).

Leading batch dimensions are allowed: ``x`` of shape (..., nz, ny, nx) is
projected item by item with the one geometry ``g``.

``cgls_unrolled`` runs K iterations of CGLS with delayed residual computation
(Section 2, Algorithm 1; direction update d = r + beta d) from x0 = 0 as torch
operations around ``project_fn`` / ``backproject_fn``, so autograd
differentiates x_K with respect to b (and anything upstream of b).  With
``checkpoint=True`` each iteration is a checkpointed block: the forward pass
keeps only the iteration's inputs (x, r, d, e and the scalar |r|^2), and the
backward pass recomputes the iteration (one A and one A^T) before
differentiating it, so memory grows by four vectors per iteration instead of
every intermediate.
"""
from __future__ import annotations

import torch

from . import backproject, project

__all__ = ["project_fn", "backproject_fn", "cgls_unrolled", "ProjectFn", "BackprojectFn"]


def _aligned(t):
    """Contiguous, with the 16-byte alignment the C ABI requires (autograd may
    hand over views at arbitrary offsets)."""
    t = t.contiguous()
    return t if t.data_ptr() % 16 == 0 else t.clone()


def _batched(fn, g, t, out_shape):
    lead = t.shape[: t.dim() - 3]
    flat = t.reshape((-1,) + tuple(t.shape[-3:]))
    outs = [fn(g, _aligned(flat[i])) for i in range(flat.shape[0])]
    if not outs:
        return t.new_empty(tuple(lead) + tuple(out_shape))
    return torch.stack(outs).reshape(tuple(lead) + tuple(out_shape))


class ProjectFn(torch.autograd.Function):
    """b = A x; grad_x = A^T grad_b."""

    @staticmethod
    def forward(ctx, x, g):
        ctx.g = g
        return _batched(project, g, x, g.proj_shape)

    @staticmethod
    def backward(ctx, grad_b):
        g = ctx.g
        return _batched(backproject, g, grad_b, g.vol_shape), None


class BackprojectFn(torch.autograd.Function):
    """r = A^T y; grad_y = A grad_r."""

    @staticmethod
    def forward(ctx, y, g):
        ctx.g = g
        return _batched(backproject, g, y, g.vol_shape)

    @staticmethod
    def backward(ctx, grad_r):
        g = ctx.g
        return _batched(project, g, grad_r, g.proj_shape), None


def project_fn(g, x):
    """Differentiable b = A x (x: (..., nz, ny, nx) on the geometry's device)."""
    return ProjectFn.apply(x, g)


def backproject_fn(g, y):
    """Differentiable r = A^T y (y: (..., n_views, nv, nu))."""
    return BackprojectFn.apply(y, g)


def _sq(t):
    """|t|^2 per batch item in double precision, keeping dimensions for
    broadcasting.  CGLS's scalars (NR2, |p|^2, alpha, beta) are formed in
    double precision whatever the vectors' type, like the library's solver;
    only the vector updates use the vectors' type."""
    t = t.double()
    return (t * t).sum(dim=(-3, -2, -1), keepdim=True)


def _iteration(g, x, r, d, e, nr2_old, first: bool, last: bool):
    """One CGLS step from (x, r = A^T e, d, e, NR2_old); returns the next state.

    first: d = r (the init block of Algorithm 1), otherwise beta = NR2 / NR2_old
    and d = r + beta d.  Then p = A d, alpha = NR2 / |p|^2, x += alpha d,
    e -= alpha p, and, unless this is the last step, the delayed residual
    r = A^T e of the next step (so K steps cost K products with A and K with
    A^T, as in Algorithm 1)."""
    nr2 = _sq(r)
    if first:
        d = r
    else:
        d = r + (nr2 / nr2_old).to(r.dtype) * d
    p = project_fn(g, d)
    alpha = nr2 / _sq(p)
    x = x + alpha.to(x.dtype) * d
    e = e - alpha.to(e.dtype) * p
    if not last:
        r = backproject_fn(g, e)
    return x, r, d, e, nr2


def cgls_unrolled(g, b, K: int, checkpoint: bool = True):
    """K CGLS iterations (Algorithm 1, x0 = 0, no early stop) differentiable in b.

    b: (..., n_views, nv, nu), float32 or float64.  Returns x_K with b's dtype;
    the scalars of every iteration are double precision.
    Iterations that would divide by zero (b = 0) are the caller's concern: the
    differentiable form has no breakdown test."""
    if K < 1:
        raise ValueError("K must be >= 1")
    lead = tuple(b.shape[: b.dim() - 3])
    x = torch.zeros(lead + tuple(g.vol_shape), dtype=b.dtype, device=b.device)
    e = b
    r = backproject_fn(g, e)
    d = torch.zeros_like(x)
    nr2 = torch.ones(lead + (1, 1, 1), dtype=torch.float64, device=b.device)
    for it in range(K):
        first, last = it == 0, it == K - 1
        if checkpoint:
            from torch.utils.checkpoint import checkpoint as ckpt
            x, r, d, e, nr2 = ckpt(_iteration, g, x, r, d, e, nr2, first, last, use_reentrant=False)
        else:
            x, r, d, e, nr2 = _iteration(g, x, r, d, e, nr2, first, last)
    return x
