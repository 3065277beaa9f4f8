"""The level-set update and the optimisation loop on the GPU:

* lbm_levelset_update against the numpy oracle of Eqs. 14, 15, 67 on random
  level sets and sensitivities (phi to FP32 rounding, the multiplier, volume
  and G; the binary design follows the GPU's own phi);
* warm restarts converge to the cold solve of the same design;
* a short optimisation of a small 3D pipe bend drives the fluid fraction to
  the limit and lowers J once the constraint holds.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.levelset import levelset_update
from _parity import rel
from paper_2501_02161_amd import lbm, optimize

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


LS_CASES = {
    # name: (workload, sigma in lattice units, K, smooth level set)
    "explicit": (lambda: W.pipe_bend_3d(n=24, port=6), 0.0, 0.2, False),
    "walls_ports": (lambda: W.pipe_bend_3d(n=24, port=6), 2.0, 0.2, False),
    "walls_ports_smooth": (lambda: W.pipe_bend_3d(n=24, port=6), 20.0, 0.02, True),
    "many_sweeps": (lambda: W.periodic_box(24, 3, 0.5), 120.0, 0.1, True),
    # sigma_z = 10 sigma_x, the anisotropic regularisation of Sec. 3.3.4
    "anisotropic": (lambda: W.pipe_bend_3d(n=24, port=6), (2.0, 2.0, 20.0), 0.02, True),
}


@pytest.mark.parametrize("name", list(LS_CASES))
def test_levelset_update_parity(name):
    """K sigma from 0 (no diffusion) over 0.4 (a few dozen sweeps; the design
    domain touches walls, the inlet and the outlet, no flux there) to 12
    (several hundred sweeps); the smooth cases keep the step off the clamp so
    that the solve itself is compared."""
    make, sigma, K, smooth = LS_CASES[name]
    w = make()
    p = lbm.Problem(w, device="cuda:0")
    kinds = w.mask & 7
    design = kinds == W.DESIGN
    if smooth:
        phi = 1.6 * (W.smoothed_noise(design.shape, 3.0, 5) - 0.5)
        dJ = W.smoothed_noise(design.shape, 3.0, 6) - 0.4
    else:
        rng = np.random.default_rng(11)
        phi = rng.uniform(-1, 1, design.shape)
        dJ = rng.normal(size=design.shape)
    phi = np.where(design, phi, 0.0).astype(np.float32)
    dJ = np.where(design, dJ, 0.0).astype(np.float32)
    gam = np.ones(design.shape, dtype=np.float32)
    t = lambda a: torch.tensor(a, device="cuda:0").contiguous()
    phi_d, dJ_d, g_d = t(phi), t(dJ), t(gam)
    out = torch.empty_like(phi_d)
    info = lbm.lbm_levelset_update(p.h, phi_d, out, dJ_d, g_d, K, sigma, 0.35)
    torch.cuda.synchronize()
    ref_phi, ref_alpha, ref = levelset_update(phi.astype(np.float64), dJ.astype(np.float64),
                                              kinds, K, sigma, 0.35)
    got = out.cpu().numpy()
    g = g_d.cpu().numpy()
    unclamped = float(np.mean(np.abs(ref_phi[design]) < 1.0))
    print(f"[levelset] {name}: K sigma {K * np.max(sigma):g}, unclamped {unclamped:.3f}, phi err "
          f"{rel(got[design], ref_phi[design]):.2e} lambda {info['lambda']:.9g} vs "
          f"{ref['lambda']:.9g}", flush=True)
    if smooth:
        assert unclamped > 0.9
    assert rel(got[design], ref_phi[design]) < 1e-5
    assert np.array_equal(got[~design], phi[~design])
    assert info["volume"] == ref["volume"] and abs(info["G"] - ref["G"]) < 1e-15
    assert abs(info["lambda"] - ref["lambda"]) <= 1e-6 * ref["lambda"]
    assert abs(info["scale"] - ref["scale"]) <= 1e-6 * ref["scale"]
    assert np.array_equal(g[design], (got[design] >= 0).astype(np.float32))
    assert np.all(g[~design] == 1.0)


def test_warm_restart_reaches_the_cold_solution():
    w = W.pipe_bend_3d(n=24, tau=0.8, Re=10.0, port=6, objective=W.OBJ_PRESSURE_DROP).replace(
        max_steps=40000, tol=1e-8, check_every=500)
    p = lbm.Problem(w, device="cuda:0")
    p.solve(w.gamma)
    g2 = np.clip(w.gamma + 0.2 * (np.random.default_rng(3).random(w.gamma.shape) - 0.5), 0, 1)
    fw = p.forward_resume(g2)
    ad = p.adjoint_resume()
    J_warm = p.sensitivity()
    dJ_warm = p.dJ.cpu().numpy().copy()
    q = lbm.Problem(w, device="cuda:0")
    res = q.solve(g2)
    d = (w.mask & 7) == W.DESIGN
    print(f"[optimize] warm {fw['steps']}/{ad['steps']} steps vs cold "
          f"{res['forward']['steps']}/{res['adjoint']['steps']}", flush=True)
    assert fw["status"] == 0 and ad["status"] == 0
    assert abs(J_warm - res["J"]) <= 1e-5 * abs(res["J"])
    assert rel(dJ_warm[d], q.dJ.cpu().numpy()[d]) < 1e-4


def test_short_optimisation():
    w = W.pipe_bend_3d(n=32, tau=0.8, Re=10.0, port=8, objective=W.OBJ_PRESSURE_DROP).replace(
        max_steps=40000, tol=1e-6, check_every=500)
    opt = optimize.LevelSetOptimizer(w, K=0.3, sigma=1e-3, vmax=0.3)
    hist = opt.run(25, log=lambda r: print(f"[optimize] {r}", flush=True))
    vols = [h["volume"] for h in hist]
    Js = [h["J"] for h in hist]
    assert all(np.isfinite(Js))
    assert all(h["fwd_status"] == 0 and h["adj_status"] == 0 for h in hist)
    # the empty chamber first (volume is the fraction before each update),
    # then solid is added until the fluid fraction settles at the limit
    assert vols[0] == 1.0 and min(vols[:5]) < 1.0
    assert abs(vols[-1] - 0.3) < 0.1
