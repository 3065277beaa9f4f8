"""GPU: conduction through design layers against its exact steady profile.

The heat-sink lattice with no flow, a heated floor and a Dirichlet top: each
interior layer holds one design value, so its conductivity is the RAMP value
of that gamma (ratio 100, q = 1) and the steady temperature is known in closed
form (each link conducts the floor flux with the harmonic mean of its two
nodes' diffusivities).  This pins the design-dependent relaxation time of the
thermal lattice on the GPU independently of the oracle, and the fixed-step
states are compared with the oracle as well.
"""
import numpy as np
import pytest
import torch

import workloads as W
from _parity import gpu_fields, rel, run_gpu, run_oracle
from paper_2501_02161_amd import lbm
from test_oracle_pins import LAYER_GAMMAS, layered_conduction_profile, ramp_conductivity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    lbm.load_library()
    yield


def layered():
    return W.conduction_layers(5, 5, LAYER_GAMMAS, tau=0.8, Pr=1.0, q_w=0.002, T_top=0.1)


def test_design_layers_closed_form():
    w = layered()
    prob, res = run_gpu(w.replace(max_steps=40000, tol=0.0, check_every=1000))
    T = prob.T.cpu().numpy().astype(np.float64)
    Df = (w.tau - 0.5) / 3.0 / w.Pr
    k = ramp_conductivity(np.array(LAYER_GAMMAS), w.k_ratio, w.q_ramp)
    expect = layered_conduction_profile(w, Df * k, Df)
    e = max(rel(T[1:, y, x] - w.T_in, expect - w.T_in)
            for y in range(1, w.ny - 1) for x in range(1, w.nx - 1))
    emax = max(float(np.abs(T[1:, y, x] - expect).max() / np.abs(expect - w.T_in).max())
               for y in range(1, w.ny - 1) for x in range(1, w.nx - 1))
    print(f"[conduction] design layers: profile error {e:.2e} (pointwise {emax:.2e}), "
          f"max |u| {np.abs(prob.u.cpu().numpy()).max():.1e}", flush=True)
    assert e < 1e-5 and emax < 1e-5


def test_design_layers_fixed_steps_parity():
    w = layered().replace(max_steps=700, tol=0.0, check_every=100)
    prob, res = run_gpu(w)
    o, ref = run_oracle(w, steps=700, tol=0.0, check_every=100)
    live = (w.mask.reshape(-1) & 7) < W.WALL
    design = (w.mask.reshape(-1) & 7) == W.DESIGN
    _, u, T, dJ = gpu_fields(prob)
    e_T = rel(T[live] - w.T_in, ref["T"][live] - w.T_in)
    e_dJ = rel(dJ[design], ref["dJ"][design])
    print(f"[conduction] design layers fixed steps: T {e_T:.2e} dJ {e_dJ:.2e} "
          f"J {res['J']:.9g} vs {ref['J']:.9g}", flush=True)
    assert e_T < 1e-5 and e_dJ < 1e-4 and np.abs(u).max() < 1e-6
