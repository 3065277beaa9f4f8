"""Pins of the oracle's formulation of the paper's own heat sink (Sec. 3.3):
symmetry planes, pressure inlets, volumetric heat generation and the
objective J = -sum Q (Eqs. 68-72).

* a quarter domain with two mirror planes reproduces the unfolded full
  domain node for node (forward state, J x 4, and the adjoint dJ/dgamma);
* uniform solid in a periodic box at rest: 1 - T decays exactly as
  (1 - beta_max)^t (the source of Eq. 71 with Eq. 69);
* a pressure-driven plane channel carries the plane Poiseuille profile whose
  curvature matches the pressure gradient it sets up (exact at
  tau = 1/2 + sqrt(3/16)), with equal mass in- and outflow.
The transposes and the converged gradient of this formulation are pinned by
complex step in test_oracle_adjoint.py (case "paper_heat_sink").
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _fold(a, w, wf):
    """Restrict a full-domain node field to the quarter's non-SYM nodes."""
    sh = (wf.nz, wf.ny, wf.nx) + a.shape[1:]
    a = a.reshape(sh)
    return a[:w.nz - (1 if w.symmetric[2] else 0), :w.ny - (1 if w.symmetric[1] else 0),
             :w.nx - (1 if w.symmetric[0] else 0)]


def _quarter(a, w):
    sh = (w.nz, w.ny, w.nx) + a.shape[1:]
    a = a.reshape(sh)
    return a[:w.nz - (1 if w.symmetric[2] else 0), :w.ny - (1 if w.symmetric[1] else 0),
             :w.nx - (1 if w.symmetric[0] else 0)]


@pytest.mark.parametrize("variant", ["heatgen_pressure_inlet", "flow_velocity_inlet"])
def test_quarter_domain_equals_unfolded_full_domain(variant):
    w = W.tiny_paper_heat_sink()
    if variant == "flow_velocity_inlet":
        # flow only, parabolic velocity inlet continued through the mirror planes
        w = w.replace(thermal=False, objective=W.OBJ_PRESSURE_DROP, inlet_rho=0.0, beta_max=0.0,
                      w_dp=1.0, Re=5.0, L_ref=4.0)
    wf = W.mirror_full(w)
    o, of = oracle.Oracle(w), oracle.Oracle(wf)
    kw = dict(tol=1e-13, check_every=200)
    q, full = o.solve(fwd_steps=40000, adj_steps=40000, **kw), \
        of.solve(fwd_steps=40000, adj_steps=40000, **kw)
    assert q["fwd_status"] == 0 and q["adj_status"] == 0
    assert q["fwd_steps"] == full["fwd_steps"]
    for key in ("rho", "u") + (("T",) if w.thermal else ()):
        a, b = _quarter(q[key], w), _fold(full[key], w, wf)
        assert np.max(np.abs(a - b)) <= 1e-12 * max(np.max(np.abs(b)), 1e-30), key
    # J = -sum Q adds up the four quarters; the mean inlet pressure is the same
    heatgen = variant.startswith("heatgen")
    assert abs(full["J"] - (4.0 if heatgen else 1.0) * q["J"]) <= 1e-12 * abs(full["J"])
    # a design cell of the quarter is four mirror cells of the full domain:
    # dJq/dg = (1/4 or 1) x 4 x dJf/dg of one image
    dq, df = _quarter(q["dJ"], w), _fold(full["dJ"], w, wf)
    factor = 1.0 if heatgen else 4.0
    assert np.max(np.abs(dq - factor * df)) <= 1e-9 * np.max(np.abs(dq))
    assert np.max(np.abs(dq)) > 0


@pytest.mark.parametrize("dim", [2, 3])
def test_heat_generation_decay_closed_form(dim):
    w = W.periodic_box(6, dim=dim, gamma_value=0.0, thermal=True).replace(
        beta_max=0.01, objective=W.OBJ_HEATGEN, T_in=0.0)
    o = oracle.Oracle(w)
    f, g = o.init()
    T0 = 0.0
    for t in range(1, 41):
        f, g = o.step(f, g)
        _, u, T = o.macro(f, g)
        assert np.max(np.abs(u)) == 0.0
        assert np.allclose(1.0 - T, (1.0 - 0.01) ** t * (1.0 - T0), rtol=1e-13, atol=0)


def test_pressure_driven_channel_poiseuille():
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    nx, ny, nz = 48, 3, 13
    w = W.channel_3d_slit(nx, ny, nz, tau, 0.0).replace(inlet_rho=1.0 + 3.0 * 2e-4)
    o = oracle.Oracle(w)
    fw = o.forward(max_steps=400000, tol=1e-14, check_every=500)
    assert fw["status"] == 0
    rho, u, _ = o.macro(fw["f"], fw["g"])
    rho = rho.reshape(w.nz, w.ny, w.nx)[:, 1, :]
    ux = u.reshape(w.nz, w.ny, w.nx, 3)[:, 1, :, 0]
    xs = np.arange(16, 32)
    # mid-channel pressure gradient and the profile it drives
    dpdx = np.polyfit(xs, rho[nz // 2, xs] / 3.0, 1)[0]
    nu = (tau - 0.5) / 3.0
    H = nz - 2                             # midway walls
    z = np.arange(1, nz - 1) - 0.5
    exact = -dpdx / (2.0 * w.rho0 * nu) * z * (H - z)
    assert dpdx < 0
    for x in xs:
        assert np.allclose(ux[1:nz - 1, x], exact, rtol=1e-7, atol=0)
    # mass in = mass out (summed axial velocity equal at every section)
    flux = ux[1:nz - 1, 1:nx - 1].sum(axis=0)
    assert np.allclose(flux, flux.mean(), rtol=1e-10)


def test_half_domain_equals_unfolded_full_domain_2d():
    """The 2D heat sink (D2Q9 + D2Q5) on the half domain below its mirror
    plane reproduces the unfolded full domain: fields, J = -sum Q twice,
    and dJ/dgamma (a cell of the half is two mirror cells)."""
    w = W.tiny_paper_heat_sink_2d()
    wf = W.mirror_full(w)
    o, of = oracle.Oracle(w), oracle.Oracle(wf)
    kw = dict(tol=1e-13, check_every=200)
    h, full = o.solve(fwd_steps=40000, adj_steps=40000, **kw), \
        of.solve(fwd_steps=40000, adj_steps=40000, **kw)
    assert h["fwd_status"] == 0 and h["adj_status"] == 0
    for key in ("rho", "u", "T"):
        a, b = _quarter(h[key], w), _fold(full[key], w, wf)
        assert np.max(np.abs(a - b)) <= 1e-12 * max(np.max(np.abs(b)), 1e-30), key
    assert abs(full["J"] - 2.0 * h["J"]) <= 1e-12 * abs(full["J"])
    dh, df = _quarter(h["dJ"], w), _fold(full["dJ"], w, wf)
    assert np.max(np.abs(dh - df)) <= 1e-9 * np.max(np.abs(dh))
    assert np.max(np.abs(dh)) > 0


@pytest.mark.parametrize("nz", [12, 1], ids=["3d", "2d"])
def test_heat_generation_objective_with_heated_walls(nz):
    """J = -sum over design nodes of beta_max (1 - gamma) (1 - T) (Eqs. 69,
    72) also where heated walls sit beside the design domain: the objective
    is the generated heat alone, recomputed here from the oracle's own
    temperature field; the heated walls change T, not what J sums."""
    kw = dict(nz=1, nx=16, ny=14) if nz == 1 else {}
    w = W.six_port_box(thermal=True, objective=W.OBJ_HEATGEN, beta_max=2e-3, heated=True, **kw)
    o = oracle.Oracle(w)
    r = o.forward(max_steps=400, tol=0.0, check_every=100)
    rho, u, T = o.macro(r["f"], r["g"])
    k = (w.mask & 7).reshape(-1)
    design = k == W.DESIGN
    gam = w.gamma.reshape(-1)
    J = -np.sum(w.beta_max * (1.0 - gam[design]) * (1.0 - T[design]))
    assert np.isclose(o.objective(r["f"], r["g"]), J, rtol=1e-13, atol=0)
    # the heated walls do heat the domain (the case is not degenerate)
    w0 = w.replace(q_w=0.0)
    o0 = oracle.Oracle(w0)
    r0 = o0.forward(max_steps=400, tol=0.0, check_every=100)
    assert abs(o0.objective(r0["f"], r0["g"]) - J) > 1e-6 * abs(J)
