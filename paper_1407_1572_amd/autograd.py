"""Gradients through the IFMM solve (torch.autograd).

For the covariance kernel of Section 1's table, A(theta) = K_ell + sigma^2 I
with K_ell(r) = exp(-r / ell), the Gaussian-process quantities need
x = A^-1 b and derivatives with respect to b, ell and sigma^2.  With
x = A^-1 b and an upstream gradient g_x:
    d/db        = A^-T g_x,
    d/d sigma^2 = -(A^-T g_x)^T x,
    d/d ell     = -(A^-T g_x)^T (dA/d ell) x,
summed over right-hand-side columns.  Every kernel here is symmetric, so
A^-T = A^-1: the backward reuses the forward's factor for a second solve (the
transposed solve), and dA/d ell x is one FMM product of the kernel
derivative (r / ell^2) exp(-r / ell) on the factor's own tree and Chebyshev
bases (ifmm_matvec_kernel).  The interpolation is linear in the kernel, so
that product is exactly the derivative of the factored FMM matrix, and the
gradients are those of the matrix the solver inverts (checked against
central finite differences and a dense-matrix gradient).

Everything runs in the gfx950 library; this module only marshals tensors.
"""
from __future__ import annotations

import torch

from .ifmm import IFMMSolver


class _ExpSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, ell, sigma2, points, opts):
        ell_v, s2_v = float(ell), float(sigma2)
        s = IFMMSolver(points, "exp", ell_v, "const", 1.0 + s2_v, opts["eps"], opts["leaf_size"], opts["rank"],
                       refine_tol=opts["refine_tol"], precision=opts["precision"], box=opts["box"],
                       r_max=opts["r_max"])
        x = s.solve(b)
        ctx.solver = s
        ctx.ell = ell_v
        ctx.dev = (ell.device if torch.is_tensor(ell) else None, sigma2.device if torch.is_tensor(sigma2) else None)
        ctx.save_for_backward(x)
        ctx.info = s.last_info
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        s = ctx.solver
        g = s.solve(gx.contiguous())  # A^-T g_x = A^-1 g_x (A symmetric)
        grad_b = g
        grad_s2 = grad_ell = None
        if ctx.needs_input_grad[2]:
            grad_s2 = (-(g * x).sum()).to(ctx.dev[1])
        if ctx.needs_input_grad[1]:
            dAx = s.matvec_kernel(x, "dexp_dell", ctx.ell, "const", 0.0)
            grad_ell = (-(g * dAx).sum()).to(ctx.dev[0])
        s.close()
        ctx.solver = None
        return grad_b, grad_ell, grad_s2, None, None


def exp_kernel_solve(points, b, ell, sigma2, eps: float = 1e-10, leaf_size: int = 64, rank: int = 36,
                     refine_tol: float = 1e-12, precision: str = "fp64", box=None, r_max: int = 0):
    """x = A^-1 b for A = exp(-r/ell) + sigma^2 I on ``points`` ([N, 2] float64
    on the GPU), differentiable in b ([N] or [N, nrhs]), ell and sigma2 (0-dim
    tensors or floats).  The factor is built in the forward pass and freed after
    the backward pass (which reuses it); refinement to ``refine_tol`` makes x
    the solution of the FMM matrix to that residual."""
    ell_t = ell if torch.is_tensor(ell) else torch.tensor(float(ell), dtype=torch.float64)
    s2_t = sigma2 if torch.is_tensor(sigma2) else torch.tensor(float(sigma2), dtype=torch.float64)
    opts = dict(eps=eps, leaf_size=leaf_size, rank=rank, refine_tol=refine_tol, precision=precision,
                box=box, r_max=r_max)
    return _ExpSolve.apply(b, ell_t, s2_t, points, opts)


def gp_loss(points, y, ell, sigma2, **kw):
    """L = 1/2 y^T A(ell, sigma^2)^-1 y (the data-fit term of a Gaussian-process
    marginal likelihood); its gradients are dL/dy = alpha, dL/d sigma^2 =
    -1/2 alpha^T alpha and dL/d ell = -1/2 alpha^T (dA/d ell) alpha with
    alpha = A^-1 y."""
    alpha = exp_kernel_solve(points, y, ell, sigma2, **kw)
    return 0.5 * (y * alpha).sum()
