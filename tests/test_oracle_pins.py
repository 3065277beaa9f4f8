"""Pins of the FP64 oracle against what the paper prints and what the
mathematics fixes (no GPU).

* the paper's printed boundary rules and their transposes (Eqs. 7, 8, 58-60),
  read from tests/golden;
* lattice isotropy (Eq. 5 weights) and the equilibrium moments (Eqs. 4, 6, 12);
* closed forms: Brinkman momentum decay in a periodic box, plane Poiseuille
  flow with midway bounce-back, pure conduction under a heated floor;
* the Zou-He invariants of the 3D generalisation (mass flux, no tangential
  momentum, outlet density) and the moments its transpose annihilates;
* complex-step Jacobians against the hand-written boundary matrices.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from _golden import matrix, rows


def node(w, x, y, z=0):
    return x + w.nx * (y + w.ny * z)


# ----------------------------------------------------------------- lattices
@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_isotropy(dim):
    w = W.tiny_pipe_bend_2d() if dim == 2 else W.tiny_heat_sink()
    o = oracle.Oracle(w)
    e, wt = o.lattice(0)
    e = e.astype(float)
    assert math.isclose(wt.sum(), 1.0, abs_tol=1e-15)
    assert np.allclose(wt @ e, 0.0, atol=1e-15)
    d = dim
    E2 = np.einsum("i,ia,ib->ab", wt, e, e)[:d, :d]
    assert np.allclose(E2, np.eye(d) / 3.0, atol=1e-15)
    E3 = np.einsum("i,ia,ib,ic->abc", wt, e, e, e)
    assert np.allclose(E3, 0.0, atol=1e-15)
    E4 = np.einsum("i,ia,ib,ic,id->abcd", wt, e, e, e, e)[:d, :d, :d, :d]
    I = np.eye(d)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
           + np.einsum("ad,bc->abcd", I, I)) / 9.0
    assert np.allclose(E4, iso, atol=1e-15)
    # every direction has its opposite
    for i in range(len(wt)):
        assert sum(np.all(e[j] == -e[i]) for j in range(len(wt))) == 1
    # thermal lattice (D3Q7, or D2Q5 on a 2D problem): cs2 = 1/4
    wth = W.tiny_paper_heat_sink_2d() if dim == 2 else W.tiny_heat_sink()
    eg, wg = oracle.Oracle(wth).lattice(1)
    assert len(wg) == (5 if dim == 2 else 7)
    eg = eg.astype(float)
    assert math.isclose(wg.sum(), 1.0, abs_tol=1e-15)
    assert np.allclose(wg @ eg, 0.0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", wg, eg, eg)[:dim, :dim], np.eye(dim) / 4.0)


# ------------------------------------------------ printed boundary rules
def _d2q9_ports():
    w = W.tiny_pipe_bend_2d()
    o = oracle.Oracle(w)
    inlet = node(w, 0, 5)
    outlet = node(w, w.nx - 5, 0)
    assert w.mask.reshape(-1)[inlet] & 7 == W.INLET
    assert w.mask.reshape(-1)[outlet] & 7 == W.OUTLET
    return w, o, inlet, outlet


def test_eq58_inlet_jacobian():
    """The generic Zou-He Jacobian at a D2Q9 left-wall inlet is Eq. (58)."""
    w, o, inlet, _ = _d2q9_ports()
    assert np.array_equal(o.bc_matrix(inlet), matrix("eq58_inlet_jacobian.txt"))


@pytest.mark.parametrize("which,fixture", [("inlet", "eq59_adjoint_inlet.txt"),
                                           ("outlet", "eq60_adjoint_outlet.txt")])
def test_eq59_eq60_adjoint_bc(which, fixture):
    """B^T applied at a D2Q9 inlet/outlet reproduces Eqs. (59)/(60) entry by entry."""
    w, o, inlet, outlet = _d2q9_ports()
    n = inlet if which == "inlet" else outlet
    M = matrix(fixture)
    got = np.zeros((9, 9))
    for k in range(9):
        fsC = np.zeros((o.N, 9))
        fsC[n, k] = 1.0
        fs, _ = o.adjoint_bc(fsC)
        got[:, k] = fs[n]
    assert np.allclose(got, M, atol=1e-15, rtol=0)


@pytest.mark.parametrize("which,fixture", [("inlet", "eq7_zouhe_inlet.txt"),
                                           ("outlet", "eq8_zouhe_outlet.txt")])
def test_eq7_eq8_forward_bc(which, fixture):
    """The generic rule gives the printed Zou-He unknowns of Eqs. (7)/(8)."""
    w, o, inlet, outlet = _d2q9_ports()
    n = inlet if which == "inlet" else outlet
    rng = np.random.default_rng(0)
    fS = rng.uniform(0.0, 0.3, size=(o.N, 9))
    f, _ = o.boundary(fS)
    u_in, _ = o.geometry()
    scale = w.rho0 * u_in[n] if which == "inlet" else w.rho0
    for r in rows(fixture):
        i, c, coef = int(r[0]), r[1], np.array(r[2:])
        assert math.isclose(f[n, i], c * scale + coef @ fS[n], rel_tol=0, abs_tol=1e-15)
    # the known populations are untouched
    unknown = {int(r[0]) for r in rows(fixture)}
    for i in range(9):
        if i not in unknown:
            assert f[n, i] == fS[n, i]


# ---------------------------------------------- 3D generalisation invariants
def _port_box(normal_code, kind):
    """7^3 walled box with a 3x3 port in the middle of the face that the
    normal points away from."""
    n = 7
    m = W.walled_box(n, n, n)
    ax = normal_code // 2
    face = 0 if normal_code % 2 == 0 else n - 1
    sl = [slice(2, 5)] * 3
    sl[2 - ax] = face          # mask is [z][y][x]
    m[tuple(sl)] = W.code(kind, normal_code)
    w = W.Workload(name="port", dim=3, nx=n, ny=n, nz=n, thermal=True, tau=0.7, Re=3.0,
                   L_ref=3.0, objective=W.OBJ_DISSIPATION, mask=m,
                   gamma=np.full((n, n, n), 0.5), Pr=1.0)
    c = [3, 3, 3]
    c[ax] = face
    return w, oracle.Oracle(w), node(w, *c)


@pytest.mark.parametrize("normal_code", range(6))
@pytest.mark.parametrize("kind", [W.INLET, W.OUTLET])
def test_zou_he_3d_invariants(normal_code, kind):
    w, o, n = _port_box(normal_code, kind)
    e, wt = o.lattice(0)
    nv = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])[
        normal_code]
    rng = np.random.default_rng(normal_code + 10 * kind)
    fS = wt[None, :] * (1.0 + rng.uniform(-0.05, 0.05, size=(o.N, 19)))
    f, _ = o.boundary(fS)
    u_in, _ = o.geometry()
    mom = e.T.astype(float) @ f[n]
    tang = [a for a in range(3) if nv[a] == 0]
    for a in tang:
        assert abs(mom[a]) < 1e-15
    if kind == W.INLET:
        assert math.isclose(mom @ nv, w.rho0 * u_in[n], abs_tol=1e-15)
        assert u_in[n] > 0
    else:
        assert math.isclose(f[n].sum(), w.rho0, abs_tol=1e-15)
    # B^T annihilates the moments that the rule fixes
    B = o.bc_matrix(n)
    fixed = [e[:, a].astype(float) for a in range(3)] if kind == W.INLET else \
        [np.ones(19)] + [e[:, a].astype(float) for a in tang]
    for m_ in fixed:
        assert np.allclose(B.T @ m_, 0.0, atol=1e-15)
    # unknowns are exactly the directions with e.n > 0
    unknown = (e @ nv) > 0
    assert np.allclose(B[unknown][:, unknown], 0.0)


@pytest.mark.parametrize("normal_code", range(6))
@pytest.mark.parametrize("kind", [W.INLET, W.OUTLET])
def test_bc_matrix_equals_complex_step_jacobian(normal_code, kind):
    """The hand-written B_j (flow and thermal) is the derivative of the
    forward boundary rule, obtained here by complex-step (exact for an affine
    map)."""
    w, o, n = _port_box(normal_code, kind)
    rng = np.random.default_rng(1)
    fS = rng.uniform(0.0, 0.2, size=(o.N, 19))
    gS = rng.uniform(0.0, 0.2, size=(o.N, 7))
    for thermal in (False, True):
        Q = 7 if thermal else 19
        J = np.zeros((Q, Q))
        for j in range(Q):
            ff = fS.astype(complex)
            gg = gS.astype(complex)
            (gg if thermal else ff)[n, j] += 1e-30j
            fo, go = o.boundary(ff, gg)
            J[:, j] = ((go if thermal else fo)[n]).imag / 1e-30
        assert np.allclose(J, o.bc_matrix(n, thermal=thermal), atol=1e-14, rtol=0)
    # walls and the heated wall: swap (symmetric permutation)
    wall = node(w, 0, 0, 0)
    B = o.bc_matrix(wall)
    assert np.array_equal(B, B.T) and np.array_equal(B @ B, np.eye(19))


# ------------------------------------------------------------ equilibrium
@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_moments(dim):
    """With tau = 1 the collision returns f_eq(rho, chi u): its moments are
    rho, rho0 chi u and rho/3 I + rho0 chi^2 u u; the thermal equilibrium has
    moments T and T u."""
    if dim == 2:
        w = W.tiny_pipe_bend_2d().replace(tau=1.0)
    else:
        w = W.tiny_heat_sink().replace(tau=1.0, Pr=1e9)   # thermal relaxes with tau_g ~ 1/2
    o = oracle.Oracle(w)
    rng = np.random.default_rng(3)
    e, wt = o.lattice(0)
    e = e.astype(float)
    f = wt[None, :] * (1.0 + rng.uniform(-0.1, 0.1, size=(o.N, o.Q)))
    fC, _ = o.collide(f, None if dim == 2 else rng.uniform(0.01, 0.1, size=(o.N, 7)))
    gam = o.gamma
    kinds = w.mask.reshape(-1) & 7
    rho = f.sum(1)
    u = f @ e / w.rho0
    ab = w.alpha_max * w.q_brink * (1 - gam) / (w.q_brink + gam)
    chi = np.where(kinds == W.DESIGN, 1.0 - w.tau * ab, 1.0)
    d = dim
    for n in np.nonzero(kinds < W.WALL)[0][:40]:
        assert math.isclose(fC[n].sum(), rho[n], abs_tol=1e-15)
        assert np.allclose(fC[n] @ e, w.rho0 * chi[n] * u[n], atol=1e-15)
        P = np.einsum("i,ia,ib->ab", fC[n], e, e)[:d, :d]
        expect = rho[n] / 3.0 * np.eye(d) + w.rho0 * chi[n] ** 2 * np.outer(u[n], u[n])[:d, :d]
        assert np.allclose(P, expect, atol=1e-14)
    if dim == 3:
        # tau_g -> 1/2: g_C = 2 g_eq - g, so g_eq = (g + g_C)/2
        w2 = w.replace(Pr=1.0)
        o2 = oracle.Oracle(w2)
        g = rng.uniform(0.01, 0.1, size=(o2.N, 7))
        eg, wg = o2.lattice(1)
        fC2, gC2 = o2.collide(f, g)
        Df = (w2.tau - 0.5) / 3.0 / w2.Pr
        for n in np.nonzero(kinds == W.FLUID)[0][:5].tolist() + \
                np.nonzero(kinds == W.INLET)[0][:5].tolist():
            tg = 0.5 + Df / 0.25
            geq = g[n] + (gC2[n] - g[n]) * tg      # from g_C = g - (g - geq)/tg
            T = g[n].sum()
            assert math.isclose(geq.sum(), T, abs_tol=1e-14)
            assert np.allclose(geq @ eg.astype(float), T * u[n], atol=1e-14)


# ------------------------------------------------------------ closed forms
@pytest.mark.parametrize("dim", [2, 3])
def test_periodic_box_brinkman_decay(dim):
    """Uniform design field in a periodic box: total momentum decays exactly as
    (1 - a_B)^t, which pins chi = 1 - tau a_B of the Eq. (12) reading."""
    gval = 0.3
    w = W.periodic_box(6, dim, gval).replace(alpha_max=0.08)
    o = oracle.Oracle(w)
    e, wt = o.lattice(0)
    u0 = np.array([0.03, -0.02, 0.01 if dim == 3 else 0.0])
    rng = np.random.default_rng(5)
    f = wt[None, :] * w.rho0 * (1.0 + 3.0 * (e @ u0)[None, :]) \
        + 1e-3 * rng.standard_normal((o.N, o.Q)) * wt[None, :]
    P0 = (f @ e).sum(0)
    ab = w.alpha_max * w.q_brink * (1 - gval) / (w.q_brink + gval)
    r = o.forward(max_steps=25, tol=0.0, check_every=0, state=(f, None))
    P = (r["f"] @ e).sum(0)
    assert np.allclose(P, P0 * (1.0 - ab) ** 25, rtol=1e-12, atol=1e-15)
    # mass is conserved exactly
    assert math.isclose(r["f"].sum(), f.sum(), rel_tol=1e-14)


TAU_MAGIC = 0.5 + math.sqrt(3.0 / 16.0)


@pytest.mark.parametrize("case", ["2d", "3d_slit"])
def test_poiseuille_closed_form(case):
    """Plane Poiseuille flow between full-way bounce-back walls, driven by a
    Zou-He velocity inlet and pressure outlet.  At tau = 1/2 + sqrt(3/16) the
    steady LBGK solution away from the ports is the exact parabola with the
    walls midway between nodes (He et al. 1997), and the pressure gradient is
    dp/dx = -8 rho0 nu U / H^2.  Away from that tau the mid-channel profile is
    off by ~0.5 %, so the check is sharp."""
    U = 0.02
    if case == "2d":
        w = W.channel_2d(64, 10, TAU_MAGIC, U)
    else:
        w = W.channel_3d_slit(64, 4, 10, TAU_MAGIC, U)
    o = oracle.Oracle(w)
    r = o.forward(max_steps=60000, tol=1e-15, check_every=500)
    assert r["status"] == 0
    rho, u, _ = o.macro(r["f"])
    H = (w.nz if case != "2d" else w.ny) - 2
    nu = (w.tau - 0.5) / 3.0
    kinds = w.mask.reshape(-1) & 7
    shape = (w.nz, w.ny, w.nx)
    ux = u[:, 0].reshape(shape)
    p = (rho / 3.0).reshape(shape)
    mid = range(20, w.nx - 24)          # the port boundary layers decay within ~16 nodes
    c = np.arange(1, H + 1)
    prof = U * 4 * (c - 0.5) / H * (1 - (c - 0.5) / H)
    for x in mid:
        if case == "2d":
            assert np.allclose(ux[0, 1:-1, x], prof, rtol=0, atol=1e-11 * U)
        else:
            for y in range(w.ny):
                assert np.allclose(ux[1:-1, y, x], prof, rtol=0, atol=1e-11 * U)
    pline = p[0, w.ny // 2, :] if case == "2d" else p[w.nz // 2, 0, :]
    G = 8 * w.rho0 * nu * U / H ** 2
    assert np.allclose(np.diff(pline)[20:w.nx - 24], -G, rtol=1e-9, atol=0)
    # the inlet nodes carry the prescribed profile exactly
    inl = ux[..., 0][kinds.reshape(shape)[..., 0] == W.INLET]
    assert np.allclose(np.sort(inl), np.sort(np.resize(prof, inl.shape)), atol=1e-16)
    fluid = (kinds.reshape(shape) < W.WALL)[..., 20:w.nx - 24]
    ut = u[:, 1:].reshape(shape + (2,))[..., 20:w.nx - 24, :][fluid]
    assert np.abs(ut).max() < 1e-9 * U


def test_conduction_linear_profile_2d():
    """The same on D2Q9 + D2Q5: a heated floor row under a Dirichlet top row,
    exactly linear with slope -q_w / D."""
    w = W.conduction_column_2d(5, 12, tau=0.8, Pr=0.5, q_w=0.003, T_top=0.25)
    o = oracle.Oracle(w)
    r = o.forward(max_steps=200000, tol=1e-15, check_every=500)
    assert r["status"] == 0
    rho, u, T = o.macro(r["f"], r["g"])
    assert np.abs(u).max() < 1e-15
    D = (w.tau - 0.5) / 3.0 / w.Pr
    T = T.reshape(w.ny, w.nx)
    ys = np.arange(1, w.ny)
    expect = w.T_in + w.q_w / D * (w.ny - 1 - ys)
    for x in range(1, w.nx - 1):
        assert np.allclose(T[1:, x], expect, rtol=1e-10, atol=0)


def test_conduction_linear_profile():
    """No flow, heated floor (flux q_w per column and step) under a Dirichlet
    top at T_top: the steady D3Q7 solution is exactly linear with slope
    -q_w / D, D = cs2 (tau_g - 1/2) = nu / Pr, and equals T_top on the top."""
    w = W.conduction_column(5, 5, 12, tau=0.8, Pr=0.5, q_w=0.003, T_top=0.25)
    o = oracle.Oracle(w)
    r = o.forward(max_steps=100000, tol=1e-15, check_every=500)
    assert r["status"] == 0
    rho, u, T = o.macro(r["f"], r["g"])
    assert np.abs(u).max() < 1e-15
    D = (w.tau - 0.5) / 3.0 / w.Pr
    T = T.reshape(w.nz, w.ny, w.nx)
    zs = np.arange(1, w.nz)
    expect = w.T_in + w.q_w / D * (w.nz - 1 - zs)
    for y in range(1, w.ny - 1):
        for x in range(1, w.nx - 1):
            assert np.allclose(T[1:, y, x], expect, rtol=1e-10, atol=0)


def ramp_conductivity(gamma, ratio, q):
    """RAMP interpolation of the conductivity between solid (gamma = 0,
    conductivity `ratio` in units of the fluid's) and fluid (gamma = 1, 1):
    k = ratio + (1 - ratio) gamma / (1 + q (1 - gamma))."""
    return ratio + (1.0 - ratio) * gamma / (1.0 + q * (1.0 - gamma))


def layered_conduction_profile(w, D_layer, D_top):
    """Exact steady D3Q7 (or D2Q5) temperature of a column conducting a flux
    q_w per step from the heated floor to a Dirichlet top node, for layer
    diffusivities D_layer[z-1] (z = 1 .. nz-2) and D_top at the top node.

    Derivation (no flow, no dependence on x and y): the in-plane and rest
    populations are then at equilibrium, so the two populations along z
    carry T/4 between them.  The net upward count through every link is the
    same constant F = q_w (the floor injects it, nothing else adds heat);
    collision at a node of relaxation time tau keeps the up/down sum and
    scales their difference, which gives F = (1 - 1/(2 tau)) (U - D) for the
    pre-collision pair (U, D).  Summing the two half-links, the temperature
    drop across the link (z, z+1) is 2 F [1/(tau_z - 1/2) + 1/(tau_{z+1} -
    1/2)] = (F / 2) (1/D_z + 1/D_{z+1}) with tau - 1/2 = D / cs2, cs2 = 1/4:
    each link conducts with the harmonic mean of its two nodes'
    diffusivities."""
    D = np.concatenate([np.asarray(D_layer, dtype=np.float64), [D_top]])
    n = len(D)
    T = np.zeros(n)
    T[-1] = w.T_in
    for i in range(n - 2, -1, -1):
        T[i] = T[i + 1] + 0.5 * w.q_w * (1.0 / D[i] + 1.0 / D[i + 1])
    return T   # T at z = 1 .. nz-1


LAYER_GAMMAS = [0.0, 0.0, 0.25, 0.25, 0.5, 1.0, 1.0, 0.75, 0.1, 0.0]


def test_conduction_through_design_layers_pins_ramp():
    """Design-dependent conductivity (RAMP, ratio 100, q = 1) through the
    exact layered conduction profile: a solid slab (gamma = 0) under partly
    and fully fluid layers.  Fixes k(0) = ratio, k(1) = 1, the RAMP values at
    gamma = 0.25, 0.5, 0.75 and 0.1 (q (1 - gamma) and q gamma differ at
    gamma != 0.5), tau_g = 1/2 + D k / cs2 and the harmonic-mean flux across
    every change of conductivity."""
    w = W.conduction_layers(5, 5, LAYER_GAMMAS, tau=0.8, Pr=1.0, q_w=0.002, T_top=0.1)
    o = oracle.Oracle(w)
    r = o.forward(max_steps=400000, tol=1e-15, check_every=500)
    assert r["status"] == 0
    rho, u, T = o.macro(r["f"], r["g"])
    assert np.abs(u).max() < 1e-15
    Df = (w.tau - 0.5) / 3.0 / w.Pr
    k = ramp_conductivity(np.array(LAYER_GAMMAS), w.k_ratio, w.q_ramp)
    assert k[0] == w.k_ratio and k[5] == 1.0
    expect = layered_conduction_profile(w, Df * k, Df)
    T = T.reshape(w.nz, w.ny, w.nx)
    for y in range(1, w.ny - 1):
        for x in range(1, w.nx - 1):
            assert np.allclose(T[1:, y, x], expect, rtol=1e-10, atol=0)
    # the readings a slip would give differ by far more than the tolerance
    g = np.array(LAYER_GAMMAS)
    wrong_q = w.k_ratio + (1.0 - w.k_ratio) * g / (1.0 + w.q_ramp * g)
    inverted = ramp_conductivity(1.0 - g, w.k_ratio, w.q_ramp)
    for kk in (wrong_q, inverted):
        alt = layered_conduction_profile(w, Df * kk, Df)
        assert np.abs(alt - expect).max() > 1e-3 * np.abs(expect).max()
