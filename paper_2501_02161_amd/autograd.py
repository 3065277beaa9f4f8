"""Differentiable steady solve: J(gamma) as a torch.autograd.Function whose
backward is the discrete adjoint of the paper (Sec. 2.4, Eqs. 53-66).

forward  runs lbm_forward_solve and saves only gamma and the converged
         macroscopic fields (density deviation, u, T), not the populations;
backward recovers the thermal non-equilibrium populations from (u, T) alone
         (lbm_thermal_resolve: the D3Q7 lattice with u frozen), then runs
         lbm_adjoint_solve and lbm_sensitivity and returns grad_J * dJ/dgamma.

All arithmetic runs in the gfx950 library; this module only moves tensors.
"""
from __future__ import annotations

import torch

from . import lbm


class SteadySensitivity(torch.autograd.Function):
    """J = SteadySensitivity.apply(gamma, problem) for a `lbm.Problem`."""

    @staticmethod
    def forward(ctx, gamma: torch.Tensor, problem: "lbm.Problem"):
        g = problem.gamma_tensor(gamma.detach())
        info = problem.forward(g)
        ctx.problem = problem
        ctx.info = info
        T = problem.T.clone() if problem.thermal else None
        ctx.save_for_backward(g, problem.drho.clone(), problem.u.clone(),
                              T if T is not None else torch.empty(0, device=g.device))
        ctx.thermal = problem.thermal
        ctx.shape = gamma.shape
        return torch.tensor(info["J"], dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, grad_J: torch.Tensor):
        g, drho, u, T = ctx.saved_tensors
        p = ctx.problem
        T = T if ctx.thermal else None
        with torch.cuda.device(p.device):
            if ctx.thermal:
                lbm.lbm_thermal_resolve(p.h, g, u, T)
            ctx.adjoint_info = lbm.lbm_adjoint_solve(p.h, g, drho, u, T).as_dict()
            dJ = torch.empty_like(g)
            lbm.lbm_sensitivity(p.h, g, drho, u, T, dJ)
        grad = grad_J.to(torch.float32) * dJ
        return grad.reshape(ctx.shape), None


def objective(gamma: torch.Tensor, problem: "lbm.Problem") -> torch.Tensor:
    """Differentiable steady objective J(gamma) (float64 0-dim tensor)."""
    return SteadySensitivity.apply(gamma, problem)


class SteadyObjective(torch.nn.Module):
    """nn.Module form: holds the problem (geometry, parameters, workspace) and
    maps a design field to J."""

    def __init__(self, spec, device=None):
        super().__init__()
        self.problem = lbm.Problem(spec, device=device)

    def forward(self, gamma: torch.Tensor) -> torch.Tensor:
        return SteadySensitivity.apply(gamma, self.problem)
