"""Differentiable diffusion solve: phi = A(k)^-1 f with k = exp(theta) on the links.

Backward runs the library's adjoint path: one extra PCG solve with the same
(symmetric) operator and V-cycle, A lambda = dL/dphi, then the per-link kernel
    dL/dtheta_f = -h^-2 k_f (lambda_p - lambda_q)(phi_p - phi_q),   dL/df = lambda.
The multigrid hierarchy only preconditions the solves and is not differentiated.
"""
from __future__ import annotations

import torch

from .gmg import Solver


class DiffusionSolve(torch.autograd.Function):
    """forward(theta_x, theta_y, theta_z, f, solver, rtol, max_it) -> phi (N,N,N), float64 on the GPU.

    `solver` must have been created with coeff_is_log=True; its coefficients are
    replaced by exp(theta) in forward (and again in backward if another call
    changed them in between)."""

    @staticmethod
    def forward(ctx, theta_x, theta_y, theta_z, f, solver: Solver, rtol: float = 1e-10, max_it: int = 500):
        if not solver.options.coeff_is_log:
            raise ValueError("DiffusionSolve needs a Solver created with coeff_is_log=True")
        solver.set_coefficients(theta_x.detach(), theta_y.detach(), theta_z.detach())
        phi, info = solver.solve(f.detach(), rtol=rtol, max_it=max_it, raise_on_failure=True)
        ctx.solver = solver
        ctx.version = solver.version
        ctx.rtol, ctx.max_it = rtol, max_it
        ctx.info = info
        ctx.save_for_backward(theta_x, theta_y, theta_z, phi)
        return phi

    @staticmethod
    def backward(ctx, grad_phi):
        theta_x, theta_y, theta_z, phi = ctx.saved_tensors
        solver = ctx.solver
        if solver.version != ctx.version:
            solver.set_coefficients(theta_x.detach(), theta_y.detach(), theta_z.detach())
        gx, gy, gz, lam, info = solver.adjoint_gradient(phi, grad_phi.contiguous(), rtol=ctx.rtol,
                                                        max_it=ctx.max_it)
        if info["status"] != "GMG_OK":
            raise RuntimeError(f"adjoint solve failed: {info}")
        return gx, gy, gz, lam, None, None, None


def diffusion_solve(theta_x, theta_y, theta_z, f, solver: Solver, rtol: float = 1e-10, max_it: int = 500):
    return DiffusionSolve.apply(theta_x, theta_y, theta_z, f, solver, rtol, max_it)
