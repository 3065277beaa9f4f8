"""Differentiable steady solve: J(gamma) as a torch.autograd.Function whose
backward is the discrete adjoint of the paper (Sec. 2.4, Eqs. 53-66).

forward  runs lbm_forward_solve and saves only gamma and the converged
         macroscopic fields (density deviation, u, T), not the populations;
backward recovers the thermal non-equilibrium populations from (u, T) alone
         (lbm_thermal_resolve: the D3Q7 lattice with u frozen), then runs
         lbm_adjoint_solve and lbm_sensitivity and returns grad_J * dJ/dgamma.

The adjoint is the gradient of the steady problem only at a converged state,
so a sweep that stops at its step cap (status LBM_NOT_CONVERGED) raises an
LBMError by default; with strict=False it warns instead.

All arithmetic runs in the gfx950 library; this module only moves tensors.
"""
from __future__ import annotations

import warnings

import torch

from . import lbm


def _check_converged(what: str, info: dict, strict: bool) -> None:
    if info.get("status", lbm.LBM_OK) == lbm.LBM_OK:
        return
    msg = (f"{what} stopped at its step cap after {info.get('steps')} steps without meeting the "
           f"residual criterion (residuals {info.get('residual')}); the adjoint gradient is exact "
           f"only at a converged state")
    if strict:
        raise lbm.LBMError(lbm.LBM_NOT_CONVERGED, msg)
    warnings.warn(msg, RuntimeWarning, stacklevel=3)


class SteadySensitivity(torch.autograd.Function):
    """J = SteadySensitivity.apply(gamma, problem, strict) for a `lbm.Problem`."""

    @staticmethod
    def forward(ctx, gamma: torch.Tensor, problem: "lbm.Problem", strict: bool = True):
        g = problem.gamma_tensor(gamma.detach())
        info = problem.forward(g)
        _check_converged("forward solve", info, strict)
        ctx.problem = problem
        ctx.strict = strict
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
                ti = lbm.lbm_thermal_resolve(p.h, g, u, T).as_dict()
                _check_converged("thermal re-solve", ti, ctx.strict)
            ctx.adjoint_info = lbm.lbm_adjoint_solve(p.h, g, drho, u, T).as_dict()
            _check_converged("adjoint solve", ctx.adjoint_info, ctx.strict)
            dJ = torch.empty_like(g)
            lbm.lbm_sensitivity(p.h, g, drho, u, T, dJ)
        grad = grad_J.to(torch.float32) * dJ
        return grad.reshape(ctx.shape), None, None


def objective(gamma: torch.Tensor, problem: "lbm.Problem", strict: bool = True) -> torch.Tensor:
    """Differentiable steady objective J(gamma) (float64 0-dim tensor); a
    sweep that does not converge raises (strict) or warns."""
    return SteadySensitivity.apply(gamma, problem, strict)


class SteadyObjective(torch.nn.Module):
    """nn.Module form: holds the problem (geometry, parameters, workspace) and
    maps a design field to J."""

    def __init__(self, spec, device=None, strict: bool = True):
        super().__init__()
        self.problem = lbm.Problem(spec, device=device)
        self.strict = strict

    def forward(self, gamma: torch.Tensor) -> torch.Tensor:
        return SteadySensitivity.apply(gamma, self.problem, self.strict)
