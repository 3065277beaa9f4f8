"""Pins of the oracle on a lattice whose ports cover all six inward normals
(`workloads.six_port_box`: pressure inlets on x = 0, y = ny-1, z = 0 and
pressure outlets on x = nx-1, y = 0, z = nz-1), no GPU:

* the steady state balances mass through the six ports (the pressure port
  rules of Eq. 8 generalised to every normal, R7, R32);
* the converged discrete adjoint's dJ/dgamma equals complex-step derivatives
  of the converged J at sampled cells, flow only (dissipation) and coupled
  with heat generation or heated walls on every face (Eqs. 54-66 with every
  normal's transpose), in 3D and in the 2D form (four ports, D2Q9 + D2Q5).
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_adjoint import _complex_step_cell, _converged, _port_fluxes


def test_every_normal_occurs():
    for w, normals in ((W.six_port_box(heated=True), [0, 1, 2, 3, 4, 5]),
                       (W.six_port_box(nz=1, nx=16, ny=14, heated=True), [0, 1, 2, 3])):
        m = w.mask.reshape(-1)
        for kinds in ((W.INLET, W.OUTLET), (W.HEATED,)):
            sel = np.isin(m & 7, kinds)
            assert sorted(set(((m[sel] >> 3) & 7).tolist())) == normals


def test_six_port_mass_balance():
    o = oracle.Oracle(W.six_port_box())
    fw = o.forward(max_steps=200000, tol=1e-14, check_every=250)
    assert fw["status"] == 0
    mass, _ = _port_fluxes(o, fw["f"], None)
    assert mass[W.INLET] > 0.0 and mass[W.OUTLET] < 0.0
    assert abs(mass[W.INLET] + mass[W.OUTLET]) <= 1e-9 * mass[W.INLET]


VARIANTS = {
    "flow_dissipation": dict(),
    # heat generation and heated walls on every face together (one slow 3D
    # thermal case instead of two)
    "heat_generation_heated_walls": dict(thermal=True, objective=W.OBJ_HEATGEN, beta_max=1e-2,
                                         heated=True),
    "2d_flow": dict(nz=1, nx=16, ny=14),
    "2d_heat_generation": dict(nz=1, nx=16, ny=14, thermal=True, objective=W.OBJ_HEATGEN,
                               beta_max=2e-3),
    "2d_heated_walls": dict(nz=1, nx=16, ny=14, thermal=True, objective=W.OBJ_HEATSINK,
                            heated=True),
}


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_six_port_gradient_matches_complex_step(variant):
    w = W.six_port_box(**VARIANTS[variant])
    o = oracle.Oracle(w)
    fw, ad, dJ = _converged(o)
    design = np.nonzero((w.mask.reshape(-1) & 7) == W.DESIGN)[0]
    rng = np.random.default_rng(23)
    cells = list(rng.choice(design, size=2, replace=False)) + [int(design[np.argmax(
        np.abs(dJ[design]))])]
    steps = max(int(2.5 * fw["steps"]), 3000)
    with cf.ThreadPoolExecutor(max_workers=3) as ex:
        ref = list(ex.map(lambda k: _complex_step_cell(o, fw, k, steps), cells))
    scale = np.abs(dJ[design]).max()
    for k, r in zip(cells, ref):
        assert abs(dJ[k] - r) <= 1e-8 * scale, (k, dJ[k], r)


def test_oracle_rejects_outward_port_normals():
    """A port whose normal points out of the box (the mistake of unfolding a
    mirror plane without reversing the normals along it) is refused."""
    w = W.six_port_box()
    m = w.mask.copy()
    m[3:7, 4:8, w.nx - 1] = W.code(W.OUTLET, W.NPX)
    with pytest.raises(ValueError, match="inward normal"):
        oracle.Oracle(w.replace(mask=m))
    m = w.mask.copy()
    m[0, 8:11, 9:12] = W.code(W.HEATED, W.NMZ)
    with pytest.raises(ValueError, match="out of the box"):
        oracle.Oracle(w.replace(mask=m))
