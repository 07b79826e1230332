"""torch.autograd.Function through assembly and solve.

forward(alpha, K) -> u = K(alpha, K)^{-1} b on the device (fpde_assemble +
fpde_solve).  backward(gbar) -> lam = K^{-1} gbar with the stored factor
(K is symmetric; fpde_solve_factored), then the adjoint kernel re-walks every
path and returns dJ/dalpha and dJ/dK (fpde_adjoint).

The adjoint sums hold for a load vector that does not depend on alpha or K
(f = 1 or source values given at the Gauss points).  The manufactured source
of the unit cube is a function of both, so it is refused here rather than
differentiated only through the matrix.
"""
from __future__ import annotations

import torch


class FracSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha, K, mesh, quad_points=4, precision=0, source=0, f_gauss=None):
        from . import FPDE_SRC_ONE, FPDE_SRC_USER, params, solve_problem
        if source not in (FPDE_SRC_ONE, FPDE_SRC_USER):
            raise ValueError("FracSolve: the load vector must not depend on alpha or K "
                             "(FPDE_SRC_ONE or FPDE_SRC_USER)")
        a = float(alpha.detach().cpu())
        k = [float(v) for v in K.detach().cpu()]
        p = params(a, k, quad_points=quad_points, precision=precision, source=source)
        u, factor, _ = solve_problem(mesh, p, f_gauss)
        ctx.mesh = mesh
        ctx.p = p
        ctx.factor = factor
        ctx.save_for_backward(u)
        return u.clone()

    @staticmethod
    def backward(ctx, gbar):
        (u,) = ctx.saved_tensors
        lam = torch.empty_like(u)
        ctx.mesh.solve_factored(ctx.p, ctx.factor, gbar.contiguous().to(torch.float64), lam)
        ga, gk = ctx.mesh.adjoint(ctx.p, u, lam)
        da = torch.tensor(ga, dtype=torch.float64)
        dk = torch.tensor(gk, dtype=torch.float64)
        return da, dk, None, None, None, None, None
