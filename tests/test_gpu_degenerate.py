"""GPU parity on the degenerate designs of the method, against the FP64
oracle and closed forms:

* the empty chamber (gamma = 1 on every design node, the initial geometry of
  the paper's optimisations) in the heat-generation formulation (Eqs. 68-72):
  no solid, no heat, so T = 0 and J = 0 exactly, and dJ/dgamma is the explicit
  term beta_max on every design node (3D quarter domain and 2D half domain,
  fixed steps and converged);
* binary designs (gamma in {0, 1}, the paper's alpha of Eq. 11), the all-solid
  and the all-fluid design domain: whole fields after equal fixed step counts
  against the oracle (1e-5 on the fields, 1e-4 on dJ/dgamma), grids with
  ragged last tiles.
"""
import numpy as np
import pytest
import torch

import workloads as W
from _parity import compare_solution, gpu_fields, kinds, rel, run_gpu, run_oracle
from paper_2501_02161_amd import lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    lbm.load_library()
    yield


def _binary(w):
    return w.replace(gamma=(w.gamma >= 0.5).astype(w.gamma.dtype))


EMPTY = {
    # 40 x 12 x 10 = 4800 nodes (19 tiles, the last ragged)
    "3d_quarter": lambda: W.paper_heat_sink(40, 12, 10, Re=20.0, tau=0.7, beta_max=1e-3,
                                            buffer=2, sigma=1.5),
    # 90 x 33 = 2970 nodes (12 tiles, the last ragged)
    "2d_half": lambda: W.paper_heat_sink_2d(90, 33, Re=20.0, tau=0.7, beta_max=1e-3, buffer=2,
                                            sigma=1.5),
}


@pytest.mark.parametrize("name", list(EMPTY))
def test_empty_chamber_heatgen_closed_form(name):
    w0 = EMPTY[name]()
    w0 = w0.replace(gamma=np.ones_like(w0.gamma))
    design = kinds(w0) == W.DESIGN
    beta = np.float32(w0.beta_max)
    for mode, kw in (("fixed", dict(max_steps=400, tol=0.0, check_every=200)),
                     ("converged", dict(max_steps=100000, tol=1e-7, check_every=500))):
        w = w0.replace(**kw)
        print(f"[degenerate] empty chamber {name} {w.nx}x{w.ny}x{w.nz} {mode}", flush=True)
        prob, res = run_gpu(w)
        drho, u, T, dJ = gpu_fields(prob)
        if mode == "converged":
            assert res["forward"]["status"] == 0 and res["adjoint"]["status"] == 0, res
        assert np.all(T == 0.0) and res["J"] == 0.0
        err = float(np.abs(dJ[design] - beta).max() / beta)
        print(f"[degenerate] {name} {mode}: steps {res['forward']['steps']}/"
              f"{res['adjoint']['steps']}, max |dJ - beta_max| / beta_max {err:.2e}, "
              f"max |u| {np.abs(u).max():.3e}", flush=True)
        assert err <= 1e-6
        assert np.all(dJ[~design] == 0.0)
        if mode == "fixed":
            o, ref = run_oracle(w, steps=400, tol=0.0, check_every=200)
            live = kinds(w) < W.WALL
            assert rel(u[live], ref["u"][live]) < 1e-5
            assert rel(drho[live], ref["rho"][live] - w.rho0) < 1e-5
        prob.close()


DESIGNS = {
    # 24 x 14 x 10 = 3360 nodes (14 tiles, the last ragged)
    "heat_sink_binary": lambda: _binary(W.heat_sink(24, 14, 10, Re=40.0, sigma=2.0, seed=103)),
    "heat_sink_all_solid": lambda: W.heat_sink(24, 14, 10, Re=40.0, sigma=2.0, seed=103).replace(
        gamma=np.zeros((10, 14, 24))),
    "heat_sink_all_fluid": lambda: W.heat_sink(24, 14, 10, Re=40.0, sigma=2.0, seed=103).replace(
        gamma=np.ones((10, 14, 24))),
    # 21^3 = 9261 nodes (37 tiles, the last ragged)
    "pipe_bend_3d_dissipation_binary": lambda: _binary(
        W.pipe_bend_3d(n=21, Re=10.0, tau=0.6, sigma=1.5, seed=104, port=6,
                       objective=W.OBJ_DISSIPATION)),
    # 50 x 50 = 2500 nodes (10 tiles, the last ragged)
    "pipe_bend_2d_binary": lambda: _binary(W.pipe_bend_2d(n=50, sigma=2.0, seed=105,
                                                          outlet=(30, 45))),
    "paper_heat_sink_binary": lambda: _binary(
        W.paper_heat_sink(40, 12, 10, Re=20.0, tau=0.7, beta_max=1e-3, buffer=2, sigma=1.5)),
}


@pytest.mark.parametrize("name", list(DESIGNS))
def test_binary_and_uniform_designs_parity(name):
    w = DESIGNS[name]().replace(max_steps=500, tol=0.0, check_every=250)
    print(f"[degenerate] {name} grid {w.nx}x{w.ny}x{w.nz} tau {w.tau:.4f}", flush=True)
    prob, res = run_gpu(w)
    o, ref = run_oracle(w, steps=500, tol=0.0, check_every=250)
    err = compare_solution(w, prob, ref)
    print(f"[degenerate] {name} errors {err} J {res['J']:.9g} vs {ref['J']:.9g}", flush=True)
    assert abs(res["J"] - ref["J"]) <= 1e-5 * abs(ref["J"])
    prob.close()


SMALLEST = {
    # one-node-wide channel: 45 nodes, 3 design nodes, one tile padded to 64
    "heat_sink_5x3x3": lambda: W.heat_sink(5, 3, 3, Re=0.3, tau=0.8, sigma=1.0, seed=106),
    # 28 nodes: the smallest half domain with a mirror row
    "paper_heat_sink_2d_7x4": lambda: W.paper_heat_sink_2d(7, 4, Re=1.0, tau=0.8, beta_max=1e-2,
                                                           buffer=1, sigma=1.0),
    # 112 nodes: the smallest quarter domain with two mirror planes
    "paper_heat_sink_7x4x4": lambda: W.paper_heat_sink(7, 4, 4, Re=1.0, tau=0.8, beta_max=1e-2,
                                                       buffer=1, sigma=1.0),
}


@pytest.mark.parametrize("name", list(SMALLEST))
def test_smallest_grids_parity(name):
    """Grids of fewer nodes than one wave (a single, padded tile)."""
    w = SMALLEST[name]().replace(max_steps=300, tol=0.0, check_every=100)
    print(f"[degenerate] smallest {name} N {w.nx * w.ny * w.nz}", flush=True)
    prob, res = run_gpu(w)
    o, ref = run_oracle(w, steps=300, tol=0.0, check_every=100)
    err = compare_solution(w, prob, ref)
    print(f"[degenerate] {name} errors {err} J {res['J']:.9g} vs {ref['J']:.9g}", flush=True)
    assert abs(res["J"] - ref["J"]) <= 1e-5 * abs(ref["J"])
    prob.close()
