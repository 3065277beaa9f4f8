"""The largest grid the library indexes (N = 2^31 / 32 = 67,108,864 nodes, the
32-bit node-index limit with 32 bytes of headroom per node): a plane channel
periodic in y with a uniform design field, 256 x 1024 x 256 nodes.  Its
solution does not depend on y, so after fixed forward and adjoint steps
every y row must hold the same values bit for bit (any indexing error across
the 20 GB of populations would break that), and the y = 0 slice must match
the FP64 oracle's solve of the same channel on 3 periodic y rows."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from _parity import rel
from paper_2501_02161_amd import lbm

pytestmark = pytest.mark.gpu

NX, NY, NZ = 256, 1024, 256
STEPS = 4


def slit(ny):
    w = W.channel_3d_slit(NX, ny, NZ, tau=0.8, u_peak=0.05)
    m = w.mask.copy()
    m[(m & 7) == W.FLUID] = W.DESIGN
    return w.replace(mask=m, gamma=np.full(m.shape, 0.8), alpha_max=0.2, q_brink=0.1,
                     max_steps=STEPS, tol=0.0, check_every=0, name=f"slit_{NX}x{ny}x{NZ}_design")


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


def test_largest_grid_is_y_invariant_and_matches_the_oracle():
    w = slit(NY)
    assert w.N == (1 << 31) // 32
    print(f"[maxsize] {w.nx}x{w.ny}x{w.nz} = {w.N} nodes", flush=True)
    prob = lbm.Problem(w, device="cuda:0")
    gamma = torch.full((NZ, NY, NX), 0.8, dtype=torch.float32, device="cuda:0")
    fw = prob.forward(gamma)
    ad = prob.adjoint()
    J = prob.sensitivity()
    torch.cuda.synchronize()
    assert fw["steps"] == STEPS and ad["steps"] == STEPS and np.isfinite(J)
    drho, u, dJ = prob.drho, prob.u, prob.dJ
    for name, f in (("drho", drho), ("u", u), ("dJ", dJ)):
        ref = f[..., :1, :] if f.dim() == 3 else f[:, :, :1, :]
        same = torch.equal(f, ref.expand_as(f))
        print(f"[maxsize] {name} identical over y: {same}", flush=True)
        assert same, name
        assert torch.isfinite(f).all()
    # the y = 0 slice against the oracle on 3 periodic rows
    ws = slit(3)
    o = oracle.Oracle(ws)
    r = o.solve(fwd_steps=STEPS, adj_steps=STEPS, tol=0.0, check_every=0)
    k = (ws.mask & 7)[:, 0, :]
    live = k < W.WALL
    design = k == W.DESIGN
    g_rho = drho[:, 0, :].cpu().numpy().astype(np.float64)
    g_u = u[:, :, 0, :].cpu().numpy().astype(np.float64)
    g_dJ = dJ[:, 0, :].cpu().numpy().astype(np.float64)
    o_rho = r["rho"].reshape(NZ, 3, NX)[:, 0, :] - ws.rho0
    o_u = r["u"].reshape(NZ, 3, NX, 3)[:, 0, :, :]
    o_dJ = r["dJ"].reshape(NZ, 3, NX)[:, 0, :]
    # J is a mean over the inlet nodes (NY rows on the GPU, 3 in the oracle), so
    # dJ/dgamma of one node scales with 1 / rows
    err = {"p": rel(g_rho[live], o_rho[live]),
           "u": rel(np.moveaxis(g_u, 0, -1)[live], o_u[live]),
           "dJ": rel(g_dJ[design] * (NY / 3.0), o_dJ[design])}
    print(f"[maxsize] y = 0 slice vs oracle: {err}", flush=True)
    assert err["p"] < 1e-5 and err["u"] < 1e-5 and err["dJ"] < 1e-4
