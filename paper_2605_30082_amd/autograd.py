"""Differentiable pressure-Poisson solve.

Forward: p = zero-mean solution of L(beta) p = rhs - mean(rhs).
Backward, for an upstream gradient w = dLoss/dp:
  lambda = zero-mean solution of L lambda = w - mean(w)   (L is symmetric, so the
           adjoint solve reuses the forward hierarchy),
  dLoss/drhs    = lambda,
  dLoss/dbeta_f = (lambda_R - lambda_L)(p_R - p_L) / h^2 on interior faces
                  (one fused face-gradient kernel), 0 on walls.
p is recomputed in the backward pass from the saved (rhs, beta) unless
save_p=True; no V-cycle state is stored.

faces_from_vof chains the gradient one step further, to the VOF fractions the
face coefficients are built from (mixture density, then harmonic-mean faces);
faces_from_density to a cell density.
"""
from __future__ import annotations

import torch

from . import solver as _S
from .solver import Solver


def _check_solver(solver: Solver, rhs: torch.Tensor, precision: str) -> None:
    if solver.closed:
        raise ValueError("the solver passed to poisson_solve has been closed")
    if tuple(solver.cell_shape) != tuple(rhs.shape):
        raise ValueError(f"solver grid {solver.cell_shape} does not match rhs {tuple(rhs.shape)}")
    if solver.precision != precision:
        raise ValueError(f"solver precision {solver.precision!r} differs from {precision!r}")


class PoissonSolve(torch.autograd.Function):
    """Forward and backward each run on one level hierarchy: the caller's
    persistent Solver (its coefficients replaced through mg_update, which
    allocates nothing), else one built for the call and freed at its end.  The
    graph keeps only the saved tensors, so no hierarchy outlives a call and the
    backward can run any number of times (retain_graph)."""

    @staticmethod
    def forward(ctx, rhs, beta_x, beta_y, beta_z, h, tol, precision, save_p, solver):
        rhs = rhs.contiguous()
        if solver is None:
            with Solver(beta_x, beta_y, beta_z, h, precision=precision, zero_guess=True) as s:
                p, _ = s.solve(rhs, tol)
            ctx.solver, ctx.version = None, None
        else:
            _check_solver(solver, rhs, precision)
            solver.update(beta_x, beta_y, beta_z)
            p, _ = solver.solve(rhs, tol, p=torch.zeros_like(rhs))
            ctx.solver, ctx.version = solver, solver.coef_version
        ctx.h, ctx.tol, ctx.precision, ctx.save_p = float(h), float(tol), precision, bool(save_p)
        if save_p:
            ctx.save_for_backward(rhs, beta_x, beta_y, beta_z, p)
        else:
            ctx.save_for_backward(rhs, beta_x, beta_y, beta_z)
        return p

    @staticmethod
    def backward(ctx, grad_p):
        saved = ctx.saved_tensors
        rhs, bx, by, bz = saved[:4]
        need_rhs, need_bx, need_by, need_bz = ctx.needs_input_grad[:4]
        g_rhs = g_x = g_y = g_z = None
        if not (need_rhs or need_bx or need_by or need_bz):
            return g_rhs, g_x, g_y, g_z, None, None, None, None, None
        own = ctx.solver is None or ctx.solver.closed
        if own:
            solver = Solver(bx, by, bz, ctx.h, precision=ctx.precision, zero_guess=True)
        else:
            solver = ctx.solver
            if solver.coef_version != ctx.version:
                # a later forward replaced the coefficients: import this graph's again
                solver.update(bx, by, bz)
                ctx.version = solver.coef_version
        try:
            lam, _ = solver.solve_adjoint(grad_p.contiguous(), ctx.tol, lam=torch.zeros_like(rhs))
            if need_rhs:
                g_rhs = lam
            if need_bx or need_by or need_bz:
                if ctx.save_p:
                    p = saved[4]
                else:
                    p, _ = solver.solve(rhs, ctx.tol, p=torch.zeros_like(rhs))
                gx, gy, gz = solver.face_grad(lam, p)
                g_x = gx if need_bx else None
                g_y = gy if need_by else None
                g_z = gz if need_bz else None
        finally:
            if own:
                solver.close()
        return g_rhs, g_x, g_y, g_z, None, None, None, None, None


def poisson_solve(rhs, beta_x, beta_y, beta_z, h, tol: float = 1e-10, precision: str = "fp64",
                  save_p: bool = False, solver: Solver = None):
    """Differentiable zero-mean solve of div(beta grad p) = rhs - mean(rhs).

    solver: an open Solver of the same grid and precision, re-used by the forward
    and the backward (coefficients replaced without allocating: the per-time-step
    form); without one each call builds and frees its own hierarchy.
    """
    return PoissonSolve.apply(rhs, beta_x, beta_y, beta_z, h, tol, precision, save_p, solver)


class FacesFromVof(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f_drop, f_film, rho_drop, rho_film, rho_gas):
        f_drop, f_film = f_drop.contiguous(), f_film.contiguous()
        ctx.rho = (float(rho_drop), float(rho_film), float(rho_gas))
        ctx.save_for_backward(f_drop, f_film)
        return _S.faces_from_vof(f_drop, f_film, *ctx.rho)

    @staticmethod
    def backward(ctx, g_x, g_y, g_z):
        f_drop, f_film = ctx.saved_tensors
        shapes = _S.face_shapes(tuple(reversed(f_drop.shape)))
        grads = [torch.zeros(s, dtype=torch.float64, device=f_drop.device) if g is None else g.contiguous()
                 for g, s in zip((g_x, g_y, g_z), shapes)]
        g_drop, g_film = _S.vof_grad(f_drop, f_film, *ctx.rho, *grads)
        return (g_drop if ctx.needs_input_grad[0] else None, g_film if ctx.needs_input_grad[1] else None,
                None, None, None)


def faces_from_vof(f_drop, f_film, rho_drop: float, rho_film: float, rho_gas: float):
    """Differentiable face coefficients (beta_x, beta_y, beta_z) from the VOF fractions."""
    return FacesFromVof.apply(f_drop, f_film, rho_drop, rho_film, rho_gas)


class FacesFromDensity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho):
        rho = rho.contiguous()
        ctx.save_for_backward(rho)
        return _S.faces_from_density(rho)

    @staticmethod
    def backward(ctx, g_x, g_y, g_z):
        (rho,) = ctx.saved_tensors
        shapes = _S.face_shapes(tuple(reversed(rho.shape)))
        grads = [torch.zeros(s, dtype=torch.float64, device=rho.device) if g is None else g.contiguous()
                 for g, s in zip((g_x, g_y, g_z), shapes)]
        return _S.density_grad(rho, *grads)


def faces_from_density(rho):
    """Differentiable face coefficients (beta_x, beta_y, beta_z) = 2/(rho_L + rho_R) from a cell density."""
    return FacesFromDensity.apply(rho)
