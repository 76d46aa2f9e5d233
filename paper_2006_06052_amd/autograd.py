"""Differentiable solves: torch.autograd.Function wrappers around the C ABI.

The forward pass solves A x = b; the backward pass solves the adjoint system
A^T lambda = dL/dx (mgk_solve_transposed, preconditioned by the transposed
V-cycle) and maps lambda to the parameter gradients with a HIP kernel:

* ``stokes_solve(theta, b, n)`` - A(theta) is the finite-difference Stokes operator
  assembled from the per-cell viscosity theta; dL/dtheta_e = -lambda^T (dA/dtheta_e) x
  (mgk_theta_grad; A is linear in theta, so this is exact), dL/db = lambda.
* ``bsr_solve(rowptr, col, values, b)`` - A given by its BSR values; dL/dA = -lambda x^T
  on every stored block (mgk_bsr_grad), dL/db = lambda.

This module only marshals; all arithmetic runs in libmgk.
"""
from __future__ import annotations

import numpy as np
import torch

from . import AMG_SPAI0, F32, Solver, stokes_bsr, theta_grad


class _StokesSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, b, n, hier, rtol, params):
        ptr, col, val = stokes_bsr(n, theta.detach().to("cpu", torch.float64).numpy())
        s = Solver(ptr, col, val, 4, AMG_SPAI0, stream=torch.cuda.current_stream(b.device),
                   hier=hier, enable_transpose=1, **params)
        b64 = b.detach().to(torch.float64).contiguous()
        x = torch.zeros_like(b64)
        info = s.solve(b64, x, rtol)
        if info["status"] != 0:
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.solver, ctx.n, ctx.rtol = s, n, rtol
        ctx.theta_meta = (theta.device, theta.dtype)
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        lam = torch.zeros_like(x)
        info = ctx.solver.solve_transposed(gx.to(torch.float64).contiguous(), lam, ctx.rtol)
        if info["status"] != 0:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        n = ctx.n
        g = torch.empty((n - 1) ** 3, dtype=torch.float64, device=x.device)
        theta_grad(n, lam, x, g, stream=torch.cuda.current_stream(x.device))
        dev, dt = ctx.theta_meta
        return g.to(dev, dt), lam, None, None, None, None


def stokes_solve(theta: torch.Tensor, b: torch.Tensor, n: int, hier: int = F32,
                 rtol: float = 1e-10, **params) -> torch.Tensor:
    """x = A(theta)^-1 b for the n^3-node stabilized Stokes operator; differentiable in
    theta ((n-1)^3 per-cell viscosities, any device) and b (FP64, on the GPU)."""
    return _StokesSolve.apply(theta, b, n, hier, rtol, params)


class _BsrSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, b, rowptr, col, block, hier, rtol, params):
        val = values.detach().to("cpu", torch.float64).numpy()
        s = Solver(rowptr, col, val, block, AMG_SPAI0, stream=torch.cuda.current_stream(b.device),
                   hier=hier, enable_transpose=1, **params)
        b64 = b.detach().to(torch.float64).contiguous()
        x = torch.zeros_like(b64)
        info = s.solve(b64, x, rtol)
        if info["status"] != 0:
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.solver, ctx.rtol = s, rtol
        ctx.vmeta = (values.device, values.dtype, values.shape)
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        lam = torch.zeros_like(x)
        info = ctx.solver.solve_transposed(gx.to(torch.float64).contiguous(), lam, ctx.rtol)
        if info["status"] != 0:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        dev, dt, shape = ctx.vmeta
        g = torch.empty(int(np.prod(shape)), dtype=torch.float64, device=x.device)
        ctx.solver.bsr_grad(lam, x, g)
        return g.reshape(shape).to(dev, dt), lam, None, None, None, None, None, None


def bsr_solve(rowptr, col, values: torch.Tensor, b: torch.Tensor, block: int, hier: int = F32,
              rtol: float = 1e-10, **params) -> torch.Tensor:
    """x = A^-1 b with A given by BSR (host rowptr/col, differentiable values [nnzb, b, b])."""
    return _BsrSolve.apply(values, b, np.asarray(rowptr, np.int32), np.asarray(col, np.int32),
                           block, hier, rtol, params)
