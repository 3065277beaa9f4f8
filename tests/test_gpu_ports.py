"""GPU parity on a lattice whose ports cover all six inward normals
(`workloads.six_port_box`), against the FP64 oracle: each port rule (forward
Zou-He, its transpose, the continuous adjoint's boundary step, the thermal
Dirichlet and outflow rules) runs in the copy specialised for its normal, so
every copy is checked; with `heated` the heated-wall rule meets every
normal too.  Fields 1e-5, dJ/dgamma 1e-4 (norm-wise relative)."""
import pytest
import torch

import workloads as W
from _parity import compare_solution, gpu_fields, rel, run_gpu, run_oracle
from paper_2501_02161_amd import lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    lbm.load_library()
    yield


VARIANTS = {
    "flow_discrete": dict(),
    "flow_continuous": dict(adjoint_kind=1),
    "heat_generation": dict(thermal=True, objective=W.OBJ_HEATGEN, beta_max=2e-3),
    "2d_flow_discrete": dict(nz=1, nx=16, ny=14),
    "2d_flow_continuous": dict(nz=1, nx=16, ny=14, adjoint_kind=1),
    "2d_heat_generation": dict(nz=1, nx=16, ny=14, thermal=True, objective=W.OBJ_HEATGEN,
                               beta_max=2e-3),
    "heated_walls": dict(thermal=True, objective=W.OBJ_HEATSINK, heated=True),
    "2d_heated_walls": dict(nz=1, nx=16, ny=14, thermal=True, objective=W.OBJ_HEATSINK,
                            heated=True),
    # heat generation beside heated walls: J = -sum Q must not pick up the
    # temperature of the layer next to the heated walls
    "heat_generation_heated_walls": dict(thermal=True, objective=W.OBJ_HEATGEN, beta_max=2e-3,
                                         heated=True),
    "2d_heat_generation_heated_walls": dict(nz=1, nx=16, ny=14, thermal=True,
                                            objective=W.OBJ_HEATGEN, beta_max=2e-3, heated=True),
}


@pytest.mark.parametrize("name", list(VARIANTS))
def test_six_port_fixed_steps_parity(name):
    w = W.six_port_box(**VARIANTS[name]).replace(max_steps=500, tol=0.0, check_every=250)
    print(f"[ports] {name} fixed steps", flush=True)
    prob, res = run_gpu(w)
    o, ref = run_oracle(w, steps=500, tol=0.0, check_every=250)
    err = compare_solution(w, prob, ref)
    print(f"[ports] {name} errors {err} J {res['J']:.9g} vs {ref['J']:.9g}", flush=True)
    assert abs(res["J"] - ref["J"]) <= 1e-5 * abs(ref["J"])
    prob.close()


@pytest.mark.parametrize("name", list(VARIANTS))
def test_six_port_converged_parity(name):
    w = W.six_port_box(**VARIANTS[name]).replace(max_steps=100000, tol=1e-7, check_every=250)
    print(f"[ports] {name} converged", flush=True)
    prob, res = run_gpu(w)
    assert res["forward"]["status"] == 0 and res["adjoint"]["status"] == 0, res
    o, ref = run_oracle(w, steps=400000, tol=1e-11, check_every=250)
    assert ref["fwd_status"] == 0 and ref["adj_status"] == 0
    err = compare_solution(w, prob, ref)
    print(f"[ports] {name} converged steps {res['forward']['steps']}/{res['adjoint']['steps']} "
          f"errors {err}", flush=True)
    prob.close()


def _x_mirrored(**kw):
    """The six-port box cut by a mirror plane before its last x layer (the
    outlet patch on that face gives way to SYM nodes)."""
    w = W.six_port_box(**kw)
    m = w.mask.copy()
    m[:, :, w.nx - 1] = W.SYM
    return w.replace(mask=m, symmetric=(True, False, False), name=w.name + "_xmirror")


@pytest.mark.parametrize("kw", [dict(), dict(thermal=True, objective=W.OBJ_HEATGEN, beta_max=2e-3)],
                         ids=["flow", "heat_generation"])
def test_x_mirror_plane_parity_and_unfolding(kw):
    """A mirror plane across x (the other cases mirror y and z): parity with
    the oracle after fixed steps, and the half domain equals the unfolded full
    domain on the GPU: the fields always, J / 2 and dJ/dgamma for the volume
    objective (the dissipation's edge sum has, in the full domain, edges
    across the plane that the half domain has no counterpart of)."""
    w = _x_mirrored(**kw).replace(max_steps=500, tol=0.0, check_every=250)
    print(f"[ports] x mirror {w.name}", flush=True)
    ph, rh = run_gpu(w)
    o, ref = run_oracle(w, steps=500, tol=0.0, check_every=250)
    err = compare_solution(w, ph, ref)
    wf = W.mirror_full(w)
    pf, rf = run_gpu(wf)
    a, b = gpu_fields(ph), gpu_fields(pf)

    def fold(x, ww):
        x = x.reshape((ww.nz, ww.ny, ww.nx) + x.shape[1:])
        return x[:, :, :w.nx - 1]

    volume = w.objective == W.OBJ_HEATGEN
    unf = {k: rel(fold(x, w), fold(y, wf)) for k, x, y in
           zip(("p", "u", "T", "dJ"), a, b) if x is not None and (volume or k != "dJ")}
    print(f"[ports] x mirror parity {err}, half vs full {unf}, J {rh['J']:.9g} x 2 vs "
          f"{rf['J']:.9g}", flush=True)
    assert all(v < 1e-6 for v in unf.values()), unf
    if volume:
        assert abs(2.0 * rh["J"] - rf["J"]) <= 1e-5 * abs(rf["J"])
    ph.close()
    pf.close()
