"""Pins of the oracle's adjoint against its own forward map (no GPU).

The discrete adjoint of the paper (Sec. 2.4) must be the exact transpose of
the linearised forward step and must return the exact gradient of the steady
discrete objective.  These tests check that without trusting the adjoint
code: the forward map is differentiated by complex step (exact to rounding for
the polynomial collision and the affine boundary rules), the steady gradient
by complex step and by central finite differences of converged forward solves.
Conservation and symmetry checks follow.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
import workloads as W

H = 1e-30


def cases():
    return {
        "pipe2d_pressure_drop": W.tiny_pipe_bend_2d(),
        "pipe3d_dissipation": W.tiny_pipe_bend_3d(),
        "pipe3d_pressure_drop": W.tiny_pipe_bend_3d(objective=W.OBJ_PRESSURE_DROP),
        "heat_sink": W.tiny_heat_sink(),
        "paper_heat_sink": W.tiny_paper_heat_sink(),
        "paper_heat_sink_2d": W.tiny_paper_heat_sink_2d(),
    }


def _state(o, steps=150):
    r = o.forward(max_steps=steps, tol=0.0, check_every=0)
    return r["f"], r["g"]


def _rand_like(rng, a):
    return None if a is None else rng.standard_normal(a.shape)


def _dot(a, b):
    return 0.0 if a is None else float(np.sum(a * b))


@pytest.mark.parametrize("name", list(cases()))
def test_step_transpose(name):
    """<w, (dPhi/df) v> == <Phi^T w, v> for one full step Phi = B S C (Eq. 35),
    Phi^T = C^T S^T B^T from Eqs. (54)-(56) without the source."""
    o = oracle.Oracle(cases()[name])
    f, g = _state(o)
    rng = np.random.default_rng(1)
    for _ in range(3):
        vf, vg = rng.standard_normal(f.shape), _rand_like(rng, g)
        wf, wg = rng.standard_normal(f.shape), _rand_like(rng, g)
        fo, go = o.step(f + 1j * H * vf, None if g is None else g + 1j * H * vg)
        Lf, Lg = fo.imag / H, (None if go is None else go.imag / H)
        lhs = _dot(wf, Lf) + _dot(wg, Lg)
        af, ag = o.adjoint_step(f, g, wf, wg)
        rhs = _dot(af, vf) + _dot(ag, vg)
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("name", list(cases()))
def test_design_transpose(name):
    """<w, (dPhi/dgamma) dg> == <C_gamma^T S^T B^T w, dg>: the sensitivity
    contraction of Eq. (66) is the transpose of the design derivative."""
    o = oracle.Oracle(cases()[name])
    f, g = _state(o)
    rng = np.random.default_rng(2)
    dg = rng.standard_normal(o.N)
    wf, wg = rng.standard_normal(f.shape), _rand_like(rng, g)
    fo, go = o.step(f.astype(complex), None if g is None else g.astype(complex),
                    gamma=o.gamma + 1j * H * dg)
    lhs = _dot(wf, fo.imag / H) + (0.0 if go is None else _dot(wg, go.imag / H))
    fs, gs = o.adjoint_bc(wf, wg)
    fsS, gsS = o.adjoint_stream(fs, gs)
    c = o.sens_contract(f, g, fsS, gsS)
    rhs = float(c @ dg)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-30)
    assert abs(lhs) > 0


@pytest.mark.parametrize("name", list(cases()))
def test_stream_transpose_and_permutation(name):
    """S^T is the transpose of S (Eq. 37); for the flow lattice S is a
    permutation, so it also preserves inner products."""
    o = oracle.Oracle(cases()[name])
    rng = np.random.default_rng(3)
    x = rng.standard_normal((o.N, o.Q))
    y = rng.standard_normal((o.N, o.Q))
    xg = rng.standard_normal((o.N, 7)) if o.thermal else None
    yg = rng.standard_normal((o.N, 7)) if o.thermal else None
    Sx, Sxg = o.stream(x, xg)
    STy, STyg = o.adjoint_stream(y, yg)
    assert np.isclose(_dot(Sx, y) + _dot(Sxg, yg), _dot(x, STy) + _dot(xg, STyg), rtol=1e-13)
    assert np.isclose(np.sum(Sx * Sx), np.sum(x * x), rtol=1e-14)
    assert np.array_equal(np.sort(Sx.ravel()), np.sort(x.ravel()))


@pytest.mark.parametrize("name", list(cases()))
def test_objective_gradient(name):
    """dJ/df, dJ/dg and the explicit dJ/dgamma against complex step of J."""
    o = oracle.Oracle(cases()[name])
    f, g = _state(o)
    rng = np.random.default_rng(4)
    vf, vg, dg = rng.standard_normal(f.shape), _rand_like(rng, g), rng.standard_normal(o.N)
    jf, jg, jgam = o.objective_grad(f, g)
    Jz = o.objective(f + 1j * H * vf, None if g is None else g + 1j * H * vg,
                     gamma=o.gamma + 1j * H * dg)
    lhs = Jz.imag / H
    rhs = _dot(jf, vf) + _dot(jg, vg) + float(jgam @ dg)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-30)
    assert np.isclose(Jz.real, o.objective(f, g), rtol=1e-15)


# ----------------------------------------------------------- end to end
def _converged(o, tol=1e-13, check=250, cap=200000):
    fw = o.forward(max_steps=cap, tol=tol, check_every=check)
    assert fw["status"] == 0, fw
    ad = o.adjoint(fw["f"], fw["g"], max_steps=cap, tol=tol, check_every=check)
    assert ad["status"] == 0, ad
    dJ = o.sensitivity(fw["f"], fw["g"], ad["fsC"], ad["gsC"])
    return fw, ad, dJ


def _complex_step_cell(o, fw, k, steps):
    """dJ/dgamma_k from a complex-step forward solve warm-started at the
    converged real state (only the imaginary part has to converge)."""
    gz = o.gamma.astype(complex)
    gz[k] += 1j * H
    g0 = None if fw["g"] is None else fw["g"].astype(complex)
    r = o.forward(gamma=gz, max_steps=steps, tol=0.0, check_every=0,
                  state=(fw["f"].astype(complex), g0))
    return o.objective(r["f"], r["g"], gamma=gz).imag / H


@pytest.mark.parametrize("name", list(cases()))
def test_gradient_matches_complex_step(name):
    """The converged discrete adjoint gives the exact gradient of the steady
    discrete J: adjoint dJ/dgamma equals complex-step derivatives of J over
    converged forward solves, at sampled design cells."""
    o = oracle.Oracle(cases()[name])
    fw, ad, dJ = _converged(o)
    design = np.nonzero((o.w.mask.reshape(-1) & 7) == W.DESIGN)[0]
    rng = np.random.default_rng(5)
    cells = list(rng.choice(design, size=5, replace=False)) + [int(design[np.argmax(
        np.abs(dJ[design]))])]
    steps = max(int(2.5 * fw["steps"]), 3000)
    with cf.ThreadPoolExecutor(max_workers=3) as ex:
        ref = list(ex.map(lambda k: _complex_step_cell(o, fw, k, steps), cells))
    scale = np.abs(dJ[design]).max()
    for k, r in zip(cells, ref):
        assert abs(dJ[k] - r) <= 1e-8 * scale, (k, dJ[k], r)
    assert np.all(dJ[(o.w.mask.reshape(-1) & 7) != W.DESIGN] == 0.0)


def test_gradient_matches_central_differences():
    """Central finite differences (h = 1e-4) of converged J on the coupled
    heat-sink problem agree with the adjoint gradient to the FD truncation."""
    o = oracle.Oracle(W.tiny_heat_sink())
    fw, ad, dJ = _converged(o)
    design = np.nonzero((o.w.mask.reshape(-1) & 7) == W.DESIGN)[0]
    rng = np.random.default_rng(6)
    cells = rng.choice(design, size=4, replace=False)
    h = 1e-4
    scale = np.abs(dJ[design]).max()

    def fd(k):
        out = []
        for s in (+1, -1):
            gm = o.gamma.copy()
            gm[k] += s * h
            r = o.forward(gamma=gm, max_steps=200000, tol=1e-14, check_every=250,
                          state=(fw["f"], fw["g"]))
            out.append(o.objective(r["f"], r["g"], gamma=gm))
        return (out[0] - out[1]) / (2 * h)

    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        ref = list(ex.map(fd, cells))
    for k, r in zip(cells, ref):
        assert abs(dJ[k] - r) <= 1e-6 * scale, (k, dJ[k], r)


def test_mirror_symmetry():
    """A heat sink whose design field is mirror-symmetric in y gives a
    mirror-symmetric gradient."""
    w = W.tiny_heat_sink(10, 9, 6)
    g = w.gamma
    w = w.replace(gamma=0.5 * (g + g[:, ::-1, :]))
    o = oracle.Oracle(w)
    fw, ad, dJ = _converged(o)
    d = dJ.reshape(w.nz, w.ny, w.nx)
    assert np.allclose(d, d[:, ::-1, :], rtol=0, atol=1e-10 * np.abs(d).max())
    assert not np.allclose(d, d[:, :, ::-1], rtol=0, atol=1e-3 * np.abs(d).max())


def _port_fluxes(o, f, g):
    """Net mass and heat leaving the box through each port kind at steady
    state: per port node, (what the boundary rule creates) minus (what streams
    out of the box)."""
    e, _ = o.lattice(0)
    eg, _ = o.lattice(1)
    fC, gC = o.collide(f, g)
    kinds = o.w.mask.reshape(-1) & 7
    codes = (o.w.mask.reshape(-1) >> 3) & 7
    nvs = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])
    mass = {W.INLET: 0.0, W.OUTLET: 0.0}
    heat = {W.INLET: 0.0, W.OUTLET: 0.0}
    for n in np.nonzero((kinds == W.INLET) | (kinds == W.OUTLET))[0]:
        nv = nvs[codes[n]]
        c = e @ nv
        mass[kinds[n]] += f[n, c > 0].sum() - fC[n, c < 0].sum()
        if g is not None:
            cg = eg @ nv
            # inflow slot: set by the boundary rule (inlet) or the node's own
            # post-collision value (outlet, zero-gradient outflow)
            inflow = g[n, cg > 0].sum() if kinds[n] == W.INLET else gC[n, cg > 0].sum()
            heat[kinds[n]] += inflow - gC[n, cg < 0].sum()
    return mass, heat


@pytest.mark.parametrize("name", ["pipe3d_dissipation", "heat_sink"])
def test_steady_mass_and_energy_balance(name):
    """At steady state the mass created by the Zou-He rules balances the mass
    streamed out of the box, and the heat put in by the heated walls leaves
    through the ports."""
    o = oracle.Oracle(cases()[name])
    fw = o.forward(max_steps=200000, tol=1e-14, check_every=250)
    mass, heat = _port_fluxes(o, fw["f"], fw["g"])
    u_in, _ = o.geometry()
    inflow = o.w.rho0 * u_in.sum()
    assert np.isclose(mass[W.INLET], inflow, rtol=1e-6)
    assert abs(mass[W.INLET] + mass[W.OUTLET]) <= 1e-10 * inflow
    if o.thermal:
        kinds = o.w.mask.reshape(-1) & 7
        q_in = o.w.q_w * np.count_nonzero(kinds == W.HEATED)
        assert abs(heat[W.INLET] + heat[W.OUTLET] + q_in) <= 1e-9 * q_in


def test_heat_is_carried_downstream():
    """With a strongly advective flow (peak speed 0.05, cell Peclet 9) most of
    the floor heat (over 3/4) leaves through the outlet: the advection term of the
    thermal equilibrium has the right sign."""
    w = W.heat_sink(24, 8, 6, Re=6.0, Pr=6.0, tau=0.6, sigma=1.0, seed=3).replace(
        alpha_max=0.0)
    o = oracle.Oracle(w)
    fw = o.forward(max_steps=200000, tol=1e-12, check_every=250)
    _, heat = _port_fluxes(o, fw["f"], fw["g"])
    kinds = w.mask.reshape(-1) & 7
    q_in = w.q_w * np.count_nonzero(kinds == W.HEATED)
    assert -heat[W.OUTLET] > 0.75 * q_in
    rho, u, T = o.macro(fw["f"], fw["g"])
    T = T.reshape(w.nz, w.ny, w.nx)
    assert T[2, 4, w.nx - 2] > T[2, 4, 2]


def test_adjoint_converges_like_forward():
    """The adjoint iteration contracts at the asymptotic rate of the linearised
    forward iteration (same spectral radius on the physical populations: the
    paper's claim that the discrete adjoint is as stable as the primal).
    Both iterations start from physical vectors (a design perturbation and
    the objective source), so the pure-permutation cycles of wall populations
    that the periodic streaming creates are never excited."""
    o = oracle.Oracle(W.tiny_pipe_bend_2d().replace(tau=0.6))
    fw = o.forward(max_steps=200000, tol=1e-14, check_every=250)
    f, g = fw["f"], fw["g"]
    live = (o.w.mask.reshape(-1) & 7) < W.WALL
    rng = np.random.default_rng(8)
    fo, _ = o.step(f.astype(complex), gamma=o.gamma + 1j * H * rng.standard_normal(o.N))
    v = fo.imag / H
    wv = o.objective_grad(f)[0]
    rates_f, rates_a = [], []
    for k in range(1500):
        fo, _ = o.step(f + 1j * H * v)
        v2 = fo.imag / H
        a, _ = o.adjoint_step(f, g, wv)
        if k >= 1000:
            rates_f.append(np.linalg.norm(v2[live]) / np.linalg.norm(v[live]))
            rates_a.append(np.linalg.norm(a[live]) / np.linalg.norm(wv[live]))
        v = v2 / np.linalg.norm(v2[live])
        wv = a / np.linalg.norm(a[live])
    rf = np.exp(np.mean(np.log(rates_f)))
    ra = np.exp(np.mean(np.log(rates_a)))
    assert 0.9 < rf < 1.0
    assert abs(rf - ra) < 1e-3 * rf


def test_pipe_bend_2d_config():
    """The 2D pipe-bend configuration (64 x 64 D2Q9, tau 0.6, Re 10, the
    paper's own inlet/outlet layout of Fig. 1 with the printed Eqs. 7/8 and
    59/60): converged adjoint gradient against complex step at two cells, and
    the mass balance at the fixed 5000-step state."""
    w = W.pipe_bend_2d()
    o = oracle.Oracle(w)
    fw, ad, dJ = _converged(o, tol=1e-12, check=500)
    design = np.nonzero((w.mask.reshape(-1) & 7) == W.DESIGN)[0]
    k1 = int(design[np.argmax(np.abs(dJ[design]))])
    k2 = int(design[len(design) // 3])
    steps = int(2.5 * fw["steps"])
    with cf.ThreadPoolExecutor(max_workers=2) as ex:
        ref = list(ex.map(lambda k: _complex_step_cell(o, fw, k, steps), [k1, k2]))
    scale = np.abs(dJ[design]).max()
    for k, r in zip([k1, k2], ref):
        assert abs(dJ[k] - r) <= 1e-8 * scale
    fixed = o.forward()            # 5000 steps, as the configuration states
    mass, _ = _port_fluxes(o, fixed["f"], None)
    assert abs(mass[W.INLET] + mass[W.OUTLET]) <= 1e-6 * mass[W.INLET]
