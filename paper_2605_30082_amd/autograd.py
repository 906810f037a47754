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


class PoissonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rhs, beta_x, beta_y, beta_z, h, tol, precision, save_p):
        solver = Solver(beta_x, beta_y, beta_z, h, precision=precision, zero_guess=True)
        p, _ = solver.solve(rhs.contiguous(), tol)
        ctx.h, ctx.tol, ctx.precision, ctx.save_p = float(h), float(tol), precision, bool(save_p)
        ctx.solver = solver
        if save_p:
            ctx.save_for_backward(rhs, beta_x, beta_y, beta_z, p)
        else:
            ctx.save_for_backward(rhs, beta_x, beta_y, beta_z)
        return p

    @staticmethod
    def backward(ctx, grad_p):
        saved = ctx.saved_tensors
        rhs, bx, by, bz = saved[:4]
        solver = ctx.solver
        need_rhs, need_bx, need_by, need_bz = ctx.needs_input_grad[:4]
        g_rhs = g_x = g_y = g_z = None
        if need_rhs or need_bx or need_by or need_bz:
            lam, _ = solver.solve_adjoint(grad_p.contiguous(), ctx.tol)
            if need_rhs:
                g_rhs = lam
            if need_bx or need_by or need_bz:
                if ctx.save_p:
                    p = saved[4]
                else:
                    p, _ = solver.solve(rhs.contiguous(), ctx.tol)
                gx, gy, gz = solver.face_grad(lam, p)
                g_x = gx if need_bx else None
                g_y = gy if need_by else None
                g_z = gz if need_bz else None
        solver.close()
        ctx.solver = None
        return g_rhs, g_x, g_y, g_z, None, None, None, None


def poisson_solve(rhs, beta_x, beta_y, beta_z, h, tol: float = 1e-10, precision: str = "fp64",
                  save_p: bool = False):
    """Differentiable zero-mean solve of div(beta grad p) = rhs - mean(rhs)."""
    return PoissonSolve.apply(rhs, beta_x, beta_y, beta_z, h, tol, precision, save_p)


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
