"""GPU parity: the gfx950 library, called through the C ABI, against the FP64
oracle on the same seeded inputs.

Small grids (the oracle finishes in seconds) span several 256-node tiles with
ragged tails and compare whole fields after equal fixed step counts, and after
convergence.  At the full benchmark sizes, in the benchmark's launch
configuration, every step's arithmetic is checked node by node: the oracle
takes the GPU's own state and performs one forward (or adjoint) step and the
sensitivity contraction in FP64.

Tolerances (norm-wise relative): 1e-5 on p - p_out, u and T - T_in over
non-wall nodes, 1e-4 on dJ/dgamma over design nodes.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from _parity import (check_pointwise, compare_solution, fmt_pointwise, gpu_fields, gpu_pops,
                     kinds, pointwise, rel, run_gpu, run_oracle)
from paper_2501_02161_amd import lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    lbm.load_library()
    yield


def small_heat_sink(Re=60.0):
    # 37 x 22 x 13 = 10582 nodes: 42 tiles of 256, the last one ragged
    return W.heat_sink(37, 22, 13, Re=Re, sigma=2.0, seed=101)


def small_pipe_bend(objective):
    w = W.pipe_bend_3d(n=30, Re=20.0, sigma=2.0, seed=102, objective=objective)
    return w


CASES = {
    "heat_sink": lambda: small_heat_sink(),
    "pipe_bend_dissipation": lambda: small_pipe_bend(W.OBJ_DISSIPATION),
    "pipe_bend_pressure_drop": lambda: small_pipe_bend(W.OBJ_PRESSURE_DROP),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fixed_steps_parity(name):
    """Equal fixed step counts (600 forward, 600 adjoint) on both sides."""
    w = CASES[name]().replace(max_steps=600, tol=0.0, check_every=200)
    print(f"[parity] {name} grid {w.nx}x{w.ny}x{w.nz} tau {w.tau:.4f}", flush=True)
    prob, res = run_gpu(w)
    o, ref = run_oracle(w, steps=600, tol=0.0, check_every=200)
    err = compare_solution(w, prob, ref)
    assert res["forward"]["steps"] == 600 and res["adjoint"]["steps"] == 600
    assert math.isclose(res["J"], ref["J"], rel_tol=1e-5)
    print(f"[parity] {name} errors {err} J {res['J']:.9g} vs {ref['J']:.9g}", flush=True)


def test_converged_parity():
    """Both sides run to the residual criterion (tol 1e-7, checks every 500
    steps); FP32 and FP64 may stop at different checks, the converged fields
    still agree."""
    w = W.heat_sink(21, 14, 9, Re=20.0, sigma=1.5, seed=103).replace(max_steps=40000, tol=1e-7,
                                                                    check_every=500)
    prob, res = run_gpu(w)
    assert res["forward"]["status"] == lbm.LBM_OK, res
    assert res["adjoint"]["status"] == lbm.LBM_OK, res
    o, ref = run_oracle(w)
    assert ref["fwd_status"] == 0 and ref["adj_status"] == 0
    err = compare_solution(w, prob, ref)
    print(f"[parity] converged steps gpu {res['forward']['steps']}/{res['adjoint']['steps']} "
          f"oracle {ref['fwd_steps']}/{ref['adj_steps']} errors {err}", flush=True)


def test_poiseuille_slit_periodic_axis():
    """Plane Poiseuille flow with a periodic axis (wrap-around streaming on the
    GPU): exact parabola mid-channel at tau = 1/2 + sqrt(3/16), to FP32."""
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    U = 0.02
    # the FP32 residual settles at a few 1e-8, so converge to 2e-7
    w = W.channel_3d_slit(64, 4, 10, tau, U).replace(max_steps=30000, tol=2e-7,
                                                    check_every=500)
    prob = lbm.Problem(w, device="cuda:0")
    info = prob.forward(w.gamma)
    torch.cuda.synchronize()
    assert info["status"] == lbm.LBM_OK, info
    drho, u, _, _ = gpu_fields(prob)
    ux = u[:, 0].reshape(w.nz, w.ny, w.nx)
    H = w.nz - 2
    zs = np.arange(1, w.nz - 1)
    prof = U * 4 * (zs - 0.5) / H * (1 - (zs - 0.5) / H)
    mid = ux[1:-1, :, 20:w.nx - 24]
    assert rel(mid, np.broadcast_to(prof[:, None, None], mid.shape)) < 1e-5
    p = drho.reshape(w.nz, w.ny, w.nx)[w.nz // 2, 0, :] / 3.0
    G = 8 * w.rho0 * (tau - 0.5) / 3.0 * U / H ** 2
    assert np.allclose(np.diff(p)[20:w.nx - 24], -G, rtol=1e-3)


def test_determinism_and_wall_outputs():
    """Bitwise identical results on repeated solves; walls report zeros."""
    w = small_heat_sink().replace(max_steps=300, tol=0.0, check_every=100)
    p1, r1 = run_gpu(w)
    f1 = [x.copy() for x in gpu_fields(p1)]
    p2, r2 = run_gpu(w)
    f2 = gpu_fields(p2)
    for a, b in zip(f1, f2):
        assert np.array_equal(a, b)
    assert r1["J"] == r2["J"]
    wall = kinds(w) >= W.WALL
    assert np.all(f1[0][wall] == 0) and np.all(f1[1][wall] == 0) and np.all(f1[2][wall] == 0)


@pytest.mark.parametrize("two_d", [False, True])
def test_stream_probe_times_and_drops_state(two_d):
    """The streaming probe reports a positive time per launch, leaves no
    solve state behind, and a later solve is unaffected by it."""
    w = (W.paper_heat_sink_2d(40, 12, Re=10.0, tau=0.7, beta_max=1e-3, buffer=2, sigma=1.5)
         if two_d else small_heat_sink()).replace(max_steps=300, tol=0.0, check_every=100)
    p1, r1 = run_gpu(w)
    ref = [x.copy() for x in gpu_fields(p1)]
    g = p1.gamma_tensor(w.gamma)
    with pytest.raises(lbm.LBMError) as e:
        p1.stream_probe(g, 0)
    assert e.value.code == lbm.LBM_EINVAL
    us = p1.stream_probe(g, 200)
    print(f"[probe] {w.name}: {us:.3f} us per launch", flush=True)
    assert 0.0 < us < 1e4
    for call in (lambda: p1.forward_continue(10), lambda: p1.adjoint_resume(),
                 lambda: p1.sensitivity()):
        with pytest.raises(lbm.LBMError) as e:
            call()
        assert e.value.code == lbm.LBM_ESTATE
    r2 = p1.solve(w.gamma)
    torch.cuda.synchronize()
    for a, b in zip(ref, gpu_fields(p1)):
        if a is not None:
            assert np.array_equal(a, b)
    assert r1["J"] == r2["J"]
    p1.close()


def test_error_paths():
    w = small_heat_sink().replace(max_steps=50, tol=0.0, check_every=0)
    prob = lbm.Problem(w, device="cuda:0")
    g = prob.gamma_tensor(w.gamma)
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_adjoint_solve(prob.h, g, None, prob.u, prob.T)
    assert e.value.code == lbm.LBM_ESTATE
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_sensitivity(prob.h, g, None, prob.u, prob.T, prob.dJ)
    assert e.value.code == lbm.LBM_ESTATE
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_forward_solve(prob.h, g, prob.drho, prob.u, None)
    assert e.value.code == lbm.LBM_EINVAL
    # an unstable set-up (tau near 1/2, inlet speed 0.6) is reported, not hidden
    bad = small_heat_sink().replace(tau=0.501, Re=0.6 * 11 / ((0.501 - 0.5) / 3), max_steps=20000,
                                    check_every=100, tol=0.0)
    pb = lbm.Problem(bad, device="cuda:0")
    with pytest.raises(lbm.LBMError) as e:
        pb.forward(bad.gamma)
    assert e.value.code == lbm.LBM_EDIVERGED


# --------------------------------------------------------------------------
# Full sizes: per-step arithmetic at the benchmark's launch configuration
# --------------------------------------------------------------------------
def _unshift(o, h, lattice, ref_value):
    _, wt = o.lattice(lattice)
    return h + wt[None, :] * ref_value


def _step_check(w, fwd_steps=200, adj_steps=200, tol_point=1e-5, tol_grad_point=1e-4):
    """One forward step, one adjoint step and the sensitivity contraction at
    the benchmark's launch configuration, each from the GPU's own state,
    against the oracle's FP64 step: norm-wise errors (returned) and the
    pointwise report (printed and asserted: every node within tol_point of
    its field's scale, every design node within tol_grad_point of
    max |dJ/dgamma|)."""
    prob = lbm.Problem(w.replace(max_steps=fwd_steps, tol=0.0, check_every=100), device="cuda:0")
    got, want = {}, {}
    o = oracle.Oracle(w)
    k = kinds(w)
    live = k < W.WALL
    design = k == W.DESIGN
    # ---- forward: state after fwd_steps, then one more step on both sides
    prob.forward(w.gamma)
    fC = _unshift(o, gpu_pops(prob, lbm.STATE_FLOW, o), 0, w.rho0)
    gC = _unshift(o, gpu_pops(prob, lbm.STATE_THERMAL, o), 1, w.T_in) if w.thermal else None
    prob.forward_continue(1)
    torch.cuda.synchronize()
    fS, gS = o.stream(fC, gC)
    f1, g1 = o.boundary(fS, gS)
    rho, u, T = o.macro(f1, g1)
    drho_g, u_g, T_g, _ = gpu_fields(prob)
    err = {"step_p": rel(drho_g[live], rho[live] - w.rho0), "step_u": rel(u_g[live], u[live])}
    got.update(step_p=drho_g, step_u=u_g)
    want.update(step_p=rho - w.rho0, step_u=u)
    if w.thermal:
        err["step_T"] = rel(T_g[live], T[live])
        got["step_T"], want["step_T"] = T_g - w.T_in, T - w.T_in
    fC2, gC2 = o.collide(f1, g1)
    _, wf = o.lattice(0)
    hC_g = gpu_pops(prob, lbm.STATE_FLOW, o)
    err["step_fC"] = rel(hC_g[live], (fC2 - wf[None, :] * w.rho0)[live])
    got["step_fC"], want["step_fC"] = hC_g, fC2 - wf[None, :] * w.rho0
    if w.thermal:
        _, wg = o.lattice(1)
        kC_g = gpu_pops(prob, lbm.STATE_THERMAL, o)
        err["step_gC"] = rel(kC_g[live], (gC2 - wg[None, :] * w.T_in)[live])
        got["step_gC"], want["step_gC"] = kC_g, gC2 - wg[None, :] * w.T_in
        # non-equilibrium thermal populations of the last step
        e7, _ = o.lattice(1)
        geq = wg[None, :] * T_g[:, None] * (1.0 + 4.0 * (u_g @ e7.T.astype(float)))
        gneq_g = gpu_pops(prob, lbm.STATE_GNEQ, o)
        err["gneq"] = rel(gneq_g[live], (g1 - geq)[live])
        got["gneq"], want["gneq"] = gneq_g, g1 - geq
    # ---- adjoint about the GPU's own (u, T): state f_eq-like with those moments
    prob.adjoint(w.gamma)
    fs = gpu_pops(prob, lbm.STATE_ADJ_FLOW, o)
    gs = gpu_pops(prob, lbm.STATE_ADJ_THERMAL, o) if w.thermal else None
    prob.adjoint_continue(1)
    torch.cuda.synchronize()
    e19, w19 = o.lattice(0)
    rho_s = w.rho0 + drho_g
    f_state = w19[None, :] * (rho_s[:, None] + 3.0 * w.rho0 * (u_g @ e19.T.astype(float)))
    g_state = None
    if w.thermal:
        e7, w7 = o.lattice(1)
        geq = w7[None, :] * T_g[:, None] * (1.0 + 4.0 * (u_g @ e7.T.astype(float)))
        g_state = geq + gpu_pops(prob, lbm.STATE_GNEQ, o)
    jf, jg, jgam = o.objective_grad(f_state, g_state)
    fsS, gsS = o.adjoint_stream(fs, gs)
    fsC, gsC = o.adjoint_collide(f_state, g_state, fsS, gsS, jf, jg)
    fs1, gs1 = o.adjoint_bc(fsC, gsC)
    a_g = gpu_pops(prob, lbm.STATE_ADJ_FLOW, o)
    err["adj_step_f"] = rel(a_g[live], fs1[live])
    got["adj_step_f"], want["adj_step_f"] = a_g, fs1
    if w.thermal:
        b_g = gpu_pops(prob, lbm.STATE_ADJ_THERMAL, o)
        err["adj_step_g"] = rel(b_g[live], gs1[live])
        got["adj_step_g"], want["adj_step_g"] = b_g, gs1
    # ---- sensitivity from the GPU's final adjoint state
    J = prob.sensitivity()
    torch.cuda.synchronize()
    fsS1, gsS1 = o.adjoint_stream(gpu_pops(prob, lbm.STATE_ADJ_FLOW, o),
                                  gpu_pops(prob, lbm.STATE_ADJ_THERMAL, o) if w.thermal else None)
    c = o.sens_contract(f_state, g_state, fsS1, gsS1)
    dJ_ref = jgam - c
    _, _, _, dJ_g = gpu_fields(prob)
    err["sens"] = rel(dJ_g[design], dJ_ref[design])
    assert np.all(dJ_g[~design] == 0.0)
    got["dJ"], want["dJ"] = dJ_g, dJ_ref
    pw = pointwise(w, got, want, live, design)
    print(f"[pointwise] {w.name} one step: {fmt_pointwise(pw)}", flush=True)
    check_pointwise(pw, tol_point, tol_grad_point)
    return err, J


@pytest.mark.parametrize("name", ["heat_sink_160x80x40_Re200", "pipe_bend_96"])
def test_full_size_step_parity(name):
    w = W.heat_sink(Re=200.0) if name.startswith("heat") else W.pipe_bend_3d()
    print(f"[full] {name} nodes {w.N}", flush=True)
    err, J = _step_check(w)
    print(f"[full] {name} errors {err}", flush=True)
    for key, v in err.items():
        assert v < (1e-4 if key == "sens" else 1e-5), (key, err)
