"""Topology optimisation around the steady sensitivity: the level-set method
of Sec. 2.2 (Eqs. 13-15, 67).

Each iteration solves the steady forward problem, the discrete adjoint and
dJ/dgamma (warm-started from the previous iteration's states after the
first), then moves the level set phi by one semi-implicit step of the
reaction-diffusion equation (Eq. 14) with the multiplier of Eq. (67) and maps
it to the binary design (Eq. 15), all in the gfx950 library
(lbm_forward_resume, lbm_adjoint_resume, lbm_sensitivity,
lbm_levelset_update).  The starting design is the empty chamber: every design
node fluid (phi = 1).
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import lbm


def design_length(spec) -> int:
    """Longest side (in nodes) of the bounding box of the design domain."""
    design = (np.asarray(spec.mask).reshape(spec.nz, spec.ny, spec.nx) & 7) == 0
    idx = np.argwhere(design)
    if len(idx) == 0:
        return 1
    return int((idx.max(0) - idx.min(0) + 1).max())


class LevelSetOptimizer:
    """sigma is the dimensionless regularisation coefficient of Eq. (14) on
    the length L of the design domain (its longest side), a scalar or per
    axis (sigma_x, sigma_y, sigma_z) for the anisotropic regularisation of
    Sec. 3.3.4: the library gets sigma L^2 in lattice units."""

    def __init__(self, spec, K: float = 0.1, sigma=1e-3, vmax: float = 0.3, device="cuda:0"):
        self.spec = spec
        self.problem = lbm.Problem(spec, device=device)
        self.K, self.vmax = float(K), float(vmax)
        self.sigma = tuple(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (3,)).tolist())
        self.L = design_length(spec)
        self.sigma_lattice = tuple(v * self.L ** 2 for v in self.sigma)
        self.device = self.problem.device
        design = (np.asarray(spec.mask).reshape(spec.nz, spec.ny, spec.nx) & 7) == 0
        g0 = np.where(design, 1.0, np.asarray(spec.gamma, dtype=np.float64).reshape(design.shape))
        self.gamma = torch.tensor(g0, dtype=torch.float32, device=self.device).contiguous()
        self.phi = torch.where(torch.tensor(design, device=self.device), 1.0, 0.0).float().contiguous()
        self.phi_next = torch.empty_like(self.phi)
        self.history = []
        self.updates = 0  # node updates of all solves

    def iterate(self) -> dict:
        p = self.problem
        t0 = time.perf_counter()
        if not self.history:
            fi = p.forward(self.gamma)
            ai = p.adjoint()
        else:
            fi = p.forward_resume(self.gamma)
            ai = p.adjoint_resume()
        J = p.sensitivity()
        with torch.cuda.device(self.device):
            ls = lbm.lbm_levelset_update(p.h, self.phi, self.phi_next, p.dJ, self.gamma, self.K,
                                         self.sigma_lattice, self.vmax)
        torch.cuda.synchronize(self.device)
        self.phi, self.phi_next = self.phi_next, self.phi
        self.updates += p.N * (fi["steps"] + ai["steps"])
        rec = {"iteration": len(self.history), "J": J, "volume": ls["volume"], "G": ls["G"],
               "lambda": ls["lambda"], "fwd_steps": fi["steps"], "adj_steps": ai["steps"],
               "fwd_status": fi["status"], "adj_status": ai["status"],
               "seconds": time.perf_counter() - t0}
        self.history.append(rec)
        return rec

    def run(self, iterations: int, log=None) -> list:
        for _ in range(iterations):
            r = self.iterate()
            if log:
                log(r)
        return self.history
