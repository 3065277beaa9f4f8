"""Seeded synthetic inputs for the adjoint lattice Boltzmann hot path.

This module is shared by the tests, the benchmark and the scripts that write
stored expected values.  It holds none of the method's arithmetic: it only
builds node-type masks (which nodes are walls, ports, heated walls, design
nodes, with the port/heater inward normal), smoothed random design fields and
the scalar parameter sets of the workloads.  The paper runs on geometric
set-ups only (pipe bends, a microchannel heat sink); there is no dataset, so
these seeded fields stand in for its cases.

Mask byte layout (the input format of the C ABI and of the oracle):
  bits 0-2  node kind: DESIGN 0, FLUID 1, INLET 2, OUTLET 3, WALL 4, HEATED 5
  bits 3-5  inward normal for INLET/OUTLET/HEATED: +x 0, -x 1, +y 2, -y 3, +z 4, -z 5
  bits 6-7  zero
Arrays are indexed [z][y][x] (x fastest); 2D problems have nz == 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy import ndimage

DESIGN, FLUID, INLET, OUTLET, WALL, HEATED, SYM = 0, 1, 2, 3, 4, 5, 6
NPX, NMX, NPY, NMY, NPZ, NMZ = 0, 1, 2, 3, 4, 5

OBJ_PRESSURE_DROP, OBJ_DISSIPATION, OBJ_HEATSINK, OBJ_HEATGEN = 0, 1, 2, 3
OBJECTIVE_NAMES = {OBJ_PRESSURE_DROP: "pressure_drop", OBJ_DISSIPATION: "dissipation",
                   OBJ_HEATSINK: "heatsink"}

SEED_BASE = 20250102


def code(kind: int, normal: int = 0) -> int:
    """Pack a node kind and an inward-normal code into one mask byte."""
    return (kind & 7) | ((normal & 7) << 3)


@dataclasses.dataclass
class Workload:
    """One synthetic problem: grid, physical parameters, mask and design field."""
    name: str
    dim: int
    nx: int
    ny: int
    nz: int
    thermal: bool
    tau: float
    Re: float
    L_ref: float
    objective: int
    mask: np.ndarray                      # uint8 [nz, ny, nx]
    gamma: np.ndarray                     # float64 [nz, ny, nx]
    rho0: float = 1.0
    alpha_max: float = 0.05
    q_brink: float = 0.1
    Pr: float = 6.0
    k_ratio: float = 100.0
    q_ramp: float = 1.0
    q_w: float = 0.01
    T_in: float = 0.0
    w_dp: float = 1.0
    periodic: tuple = (False, False, False)
    max_steps: int = 20000
    tol: float = 1e-7
    check_every: int = 1000
    seed: int = 0
    adjoint_kind: int = 0                 # 0 discrete (Sec. 2.4), 1 continuous (Sec. 2.3)
    symmetric: tuple = (False, False, False)  # mirror plane before the last layer of an axis
    inlet_rho: float = 0.0                # > 0: pressure inlets at this density
    beta_max: float = 0.0                 # volumetric heat generation coefficient

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def smoothed_noise(shape, sigma: float, seed: int) -> np.ndarray:
    """Uniform [0,1) noise from PCG64(seed), Gaussian-smoothed (truncated at
    4 sigma, reflecting edges), then min-max rescaled to [0, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.random(shape)
    if sigma > 0:
        a = ndimage.gaussian_filter(a, sigma=sigma, mode="reflect", truncate=4.0)
    lo, hi = float(a.min()), float(a.max())
    if hi > lo:
        a = (a - lo) / (hi - lo)
    return np.clip(a, 0.0, 1.0)


def walled_box(nx: int, ny: int, nz: int, dim: int = 3,
               periodic=(False, False, False), interior: int = DESIGN) -> np.ndarray:
    """Mask with WALL on the outer layer of every non-periodic axis and
    `interior` elsewhere."""
    m = np.full((nz, ny, nx), interior, dtype=np.uint8)
    if not periodic[0]:
        m[:, :, 0] = WALL
        m[:, :, -1] = WALL
    if not periodic[1]:
        m[:, 0, :] = WALL
        m[:, -1, :] = WALL
    if dim == 3 and not periodic[2]:
        m[0, :, :] = WALL
        m[-1, :, :] = WALL
    return m


# --------------------------------------------------------------------------
# The workloads of the benchmark and of the parity tests
# --------------------------------------------------------------------------

def pipe_bend_2d(n: int = 64, tau: float = 0.6, Re: float = 10.0, sigma: float = 3.0,
                 seed: Optional[int] = None, inlet=(8, 23), outlet=(40, 55),
                 steps: int = 5000) -> Workload:
    """2D pipe bend, flow only, D2Q9 on n x n: parabolic velocity inlet on the
    left wall (x=0, rows inlet[0]..inlet[1]), pressure outlet on the bottom
    wall (y=0, columns outlet[0]..outlet[1]), bounce-back elsewhere.  The
    objective is the static pressure drop inlet-to-outlet; fixed step counts."""
    seed = SEED_BASE + 0 if seed is None else seed
    m = walled_box(n, n, 1, dim=2)
    m[0, inlet[0]:inlet[1] + 1, 0] = code(INLET, NPX)
    m[0, 0, outlet[0]:outlet[1] + 1] = code(OUTLET, NPY)
    gamma = smoothed_noise((1, n, n), sigma, seed)
    L = inlet[1] - inlet[0] + 1
    return Workload(name=f"pipe_bend_2d_{n}x{n}", dim=2, nx=n, ny=n, nz=1, thermal=False,
                    tau=tau, Re=Re, L_ref=float(L), objective=OBJ_PRESSURE_DROP, mask=m,
                    gamma=gamma, alpha_max=0.1, q_brink=0.1, w_dp=1.0, max_steps=steps,
                    tol=0.0, check_every=1000, seed=seed)


def pipe_bend_3d(n: int = 96, tau: float = 0.55, Re: float = 100.0, sigma: float = 4.0,
                 seed: Optional[int] = None, port: int = 16, objective: int = OBJ_DISSIPATION
                 ) -> Workload:
    """3D pipe bend, flow only, D3Q19 on n^3: a port x port square velocity
    inlet on face x=0 (y and z in [n/12, n/12+port) and [5n/12, 5n/12+port)),
    a square pressure outlet on face y=0 (x in [3n/4, 3n/4+port), same z
    range), bounce-back elsewhere.  Objective: viscous dissipation."""
    seed = SEED_BASE + 1 if seed is None else seed
    m = walled_box(n, n, n)
    y0 = max(1, round(n * 8 / 96))
    z0 = max(1, round(n * 40 / 96))
    x0 = max(1, round(n * 72 / 96))
    p = min(port, n - 2 - max(y0, z0, x0) + 1)
    m[z0:z0 + p, y0:y0 + p, 0] = code(INLET, NPX)
    m[z0:z0 + p, 0, x0:x0 + p] = code(OUTLET, NPY)
    gamma = smoothed_noise((n, n, n), sigma, seed)
    return Workload(name=f"pipe_bend_3d_{n}^3", dim=3, nx=n, ny=n, nz=n, thermal=False,
                    tau=tau, Re=Re, L_ref=float(p), objective=objective, mask=m, gamma=gamma,
                    alpha_max=0.05, q_brink=0.1, seed=seed)


def heat_sink(nx: int = 160, ny: int = 80, nz: int = 40, Re: float = 200.0,
              Pr: float = 6.0, u_peak: float = 0.1, sigma: float = 5.0,
              seed: Optional[int] = None, tau: Optional[float] = None,
              name: Optional[str] = None, buffer: int = 0) -> Workload:
    """3D microchannel heat sink, coupled D3Q19 flow + D3Q7 heat: velocity
    inlet over the whole interior of face x=0, pressure outlet over the whole
    interior of face x=nx-1, uniform heat flux through the floor z=0, walls
    elsewhere.  Conductivity ratio 100 by RAMP(q=1).  Objective: mean
    temperature of the layer on the heated floor + 0.1 x pressure drop.

    The relaxation time is not given for this case; unless `tau` is passed
    the peak inlet speed is fixed to `u_peak` and tau follows from
    Re = u_peak L / nu with L = nz - 2 (the channel height between the
    midway walls).  u_peak = 0.1 gives tau = 0.728, 0.557, 0.5285 at
    Re 50, 200, 400; with u_peak = 0.05 (tau 0.5285 at Re 200) the BGK flow
    lattice blows up near the inlet corners on the full grid.

    `buffer` > 0 makes the last `buffer` interior layers before the outlet
    plain fluid (not design): a jet leaving a design pore straight through
    the pressure outlet can lock into a period-2 oscillation there."""
    seed = SEED_BASE + 2 if seed is None else seed
    m = walled_box(nx, ny, nz)
    m[1:nz - 1, 1:ny - 1, 0] = code(INLET, NPX)
    m[1:nz - 1, 1:ny - 1, nx - 1] = code(OUTLET, NMX)
    m[0, 1:ny - 1, 1:nx - 1] = code(HEATED, NPZ)
    if buffer > 0:
        m[1:nz - 1, 1:ny - 1, nx - 1 - buffer:nx - 1] = FLUID
    L = float(nz - 2)
    if tau is None:
        tau = 0.5 + 3.0 * u_peak * L / Re
    gamma = smoothed_noise((nz, ny, nx), sigma, seed)
    return Workload(name=name or f"heat_sink_{nx}x{ny}x{nz}_Re{Re:g}", dim=3, nx=nx, ny=ny,
                    nz=nz, thermal=True, tau=tau, Re=Re, L_ref=L, objective=OBJ_HEATSINK,
                    mask=m, gamma=gamma, alpha_max=0.05, q_brink=0.1, Pr=Pr, k_ratio=100.0,
                    q_ramp=1.0, q_w=0.01, T_in=0.0, w_dp=0.1, seed=seed)


def differentiable_case(seed: Optional[int] = None) -> Workload:
    """The autograd workload: coupled heat sink on 128 x 64 x 32 at Re 200.
    Peak inlet speed 0.15 (tau 0.5675): with 0.1 (tau 0.545) the BGK flow
    lattice blows up after ~1500 steps on this grid.  Six fluid layers
    before the outlet: without them a jet through a design pore at the
    outlet (|u| 0.16) oscillates with period 2, which a residual taken over
    an even number of steps cannot see, and the adjoint of that non-steady
    state diverges."""
    seed = SEED_BASE + 3 if seed is None else seed
    return heat_sink(128, 64, 32, Re=200.0, u_peak=0.15, seed=seed, buffer=6,
                     name="heat_sink_128x64x32_Re200")


def paper_heat_sink(nx: int = 128, ny: int = 33, nz: int = 25, Re: float = 60.0,
                    tau: float = 0.6, Pr: float = 7.1, beta_max: float = 1e-5,
                    k_ratio: float = 100.0, alpha_max: float = 0.1, buffer: int = 4,
                    sigma: float = 3.0, seed: Optional[int] = None,
                    name: Optional[str] = None) -> Workload:
    """The paper's own 3D microchannel heat sink (Sec. 3.3, Eqs. 68-72) on a
    quarter of the domain: mirror planes before the last y and z layers (SYM
    nodes), no-slip adiabatic walls at y = 0 and z = 0, a pressure inlet over
    face x = 0 and a pressure outlet over face x = nx-1 (their interiors),
    `buffer` fluid layers after the inlet and before the outlet, the design
    domain between them.  Heat is generated in the solid, Q = beta(gamma)
    (1 - T) with beta = beta_max (1 - gamma) (Eq. 69); the inlet fluid is at
    T = 0; objective J = -sum Q (Eq. 72).  Re follows Eq. (70): the velocity
    scale sqrt(dp / rho0) of the pressure drop, length L = the full channel
    height between the walls, 2 (nz - 2) + 1 nodes; at the given tau the inlet
    density is rho0 + 3 dp with dp = rho0 (Re nu / L)^2."""
    seed = SEED_BASE + 7 if seed is None else seed
    m = np.full((nz, ny, nx), DESIGN, dtype=np.uint8)
    m[0, :, :] = WALL
    m[:, 0, :] = WALL
    m[:, :, 0] = WALL
    m[:, :, nx - 1] = WALL
    m[1:nz - 1, 1:ny - 1, 0] = code(INLET, NPX)
    m[1:nz - 1, 1:ny - 1, nx - 1] = code(OUTLET, NMX)
    if buffer > 0:
        m[1:nz - 1, 1:ny - 1, 1:1 + buffer] = FLUID
        m[1:nz - 1, 1:ny - 1, nx - 1 - buffer:nx - 1] = FLUID
    m[nz - 1, :, :] = SYM
    m[:, ny - 1, :] = SYM
    L = float(2 * (nz - 2) + 1)
    nu = (tau - 0.5) / 3.0
    dp = (Re * nu / L) ** 2
    gamma = smoothed_noise((nz, ny, nx), sigma, seed)
    return Workload(name=name or f"paper_heat_sink_{nx}x{ny}x{nz}_Re{Re:g}", dim=3, nx=nx, ny=ny,
                    nz=nz, thermal=True, tau=tau, Re=Re, L_ref=L, objective=OBJ_HEATGEN, mask=m,
                    gamma=gamma, alpha_max=alpha_max, q_brink=0.1, Pr=Pr, k_ratio=k_ratio,
                    q_ramp=1.0, q_w=0.0, T_in=0.0, w_dp=0.0, seed=seed,
                    symmetric=(False, True, True), inlet_rho=1.0 + 3.0 * dp, beta_max=beta_max)


def mirror_full(w: Workload) -> Workload:
    """The full-domain problem whose quarter (or half) is w: every symmetric
    axis is unfolded about its mirror plane (the SYM layer dropped, the rest
    reflected, with the inward normals along that axis reversed in the
    reflected copy), mask and design field alike."""
    m, g = w.mask, w.gamma
    for a, ax in ((0, 2), (1, 1), (2, 0)):   # x, y, z -> array axes 2, 1, 0
        if not w.symmetric[a]:
            continue
        sl = [slice(None)] * 3
        sl[ax] = slice(0, m.shape[ax] - 1)
        m, g = m[tuple(sl)], g[tuple(sl)]
        # the reflected copy: inward normals along the axis change sign
        r = np.flip(m, axis=ax).copy()
        kind, nc = r & 7, (r >> 3) & 7
        along = np.isin(kind, (INLET, OUTLET, HEATED)) & (nc // 2 == a)
        r[along] = (kind[along] | ((nc[along] ^ 1) << 3)).astype(np.uint8)
        m = np.concatenate([m, r], axis=ax)
        g = np.concatenate([g, np.flip(g, axis=ax)], axis=ax)
    nz, ny, nx = m.shape
    return w.replace(mask=np.ascontiguousarray(m), gamma=np.ascontiguousarray(g), nx=nx, ny=ny,
                     nz=nz, symmetric=(False, False, False), name=w.name + "_full")


def tiny_paper_heat_sink(nx: int = 12, ny: int = 6, nz: int = 5, Re: float = 10.0,
                         tau: float = 0.8, beta_max: float = 2e-3, seed: int = 9) -> Workload:
    """A small quarter-domain heat sink of the paper's formulation, for pins."""
    return paper_heat_sink(nx, ny, nz, Re=Re, tau=tau, Pr=1.0, beta_max=beta_max,
                           alpha_max=0.2, buffer=1, sigma=1.0, seed=seed,
                           name=f"tiny_paper_heat_sink_{nx}x{ny}x{nz}")


SERVING_GRIDS = ((64, 32, 16), (128, 64, 32), (192, 96, 48))
# Poisson arrival rate of the serving stream (requests/s): 0.8 of what plain
# back-to-back solves sustain on one MI355X (mean service 0.559 s per request
# over the first 256 requests of the stream, all arriving at once).
SERVING_RATE = 1.43
SERVING_BUDGET_BYTES = 200 * 10**9


# Smallest relaxation time per serving grid (by channel height nz - 2) at
# which the coupled BGK lattices (D3Q19 flow, D3Q7 heat at Pr 6) converge on
# the serving heat sinks: a sweep of tau in [0.52, 0.65] against peak inlet
# speeds 0.02-0.1 diverged at every speed below these (the thermal relaxation
# time 1/2 + 4 nu / Pr approaches 1/2 there).
SERVING_TAU_MIN = {14: 0.55, 30: 0.57, 46: 0.57}


def serving_request(i: int, base_seed: int = SEED_BASE + 4) -> Workload:
    """Request i of the serving stream: grid uniform over SERVING_GRIDS, Re
    uniform in [50, 400], tau uniform in [0.52, 0.8], own smoothed design
    field.  Re and tau are drawn independently, which is not always a
    problem these lattices can solve: tau is raised to the grid's stability
    floor SERVING_TAU_MIN and the peak inlet speed Re nu / L capped at 0.1,
    and the request carries the effective tau and Re (`tau`, `Re`) beside
    the drawn ones (`tau_drawn`, `Re_drawn`)."""
    rng = np.random.Generator(np.random.PCG64(base_seed * 1000 + i))
    nx, ny, nz = SERVING_GRIDS[int(rng.integers(0, len(SERVING_GRIDS)))]
    Re = float(rng.uniform(50.0, 400.0))
    tau_drawn = float(rng.uniform(0.52, 0.8))
    L = float(nz - 2)
    tau = max(tau_drawn, SERVING_TAU_MIN[int(L)])
    nu = (tau - 0.5) / 3.0
    u = min(Re * nu / L, 0.1)
    Re_eff = u * L / nu
    w = heat_sink(nx, ny, nz, Re=Re_eff, tau=tau, sigma=5.0, seed=base_seed * 1000 + i,
                  name=f"req{i}_{nx}x{ny}x{nz}")
    w.tau_drawn, w.Re_drawn = tau_drawn, Re
    return w


def stability_case(n: int, tau: float, u_peak: float, adjoint_kind: int, seed: int = SEED_BASE + 6,
                   max_steps: int = 1000000, tol: float = 1e-9, dim: int = 3) -> Workload:
    """One point of the stability test: the pipe bend (3D on n^3, or 2D D2Q9
    on n x n) at relaxation time tau and peak inlet speed u_peak,
    pressure-drop objective, given adjoint kind; Re = u_peak L / nu with L
    the port width."""
    if dim == 2:
        w = pipe_bend_2d(n=n, tau=tau, Re=1.0, sigma=max(1.0, n / 24.0), seed=seed,
                         inlet=(n // 8, (23 * n) // 64), outlet=((5 * n) // 8, (55 * n) // 64))
    else:
        w = pipe_bend_3d(n=n, tau=tau, Re=1.0, sigma=max(1.0, n / 24.0), seed=seed,
                         port=max(4, n // 6), objective=OBJ_PRESSURE_DROP)
    nu = (tau - 0.5) / 3.0
    return w.replace(Re=u_peak * w.L_ref / nu, adjoint_kind=adjoint_kind, max_steps=max_steps,
                     tol=tol, check_every=1000,
                     name=f"stability_{dim}d_{n}_tau{tau:g}_u{u_peak:g}_k{adjoint_kind}")


def poisson_arrivals(n: int, rate: float, seed: int = SEED_BASE + 5) -> np.ndarray:
    """Arrival times (seconds) of n requests with exponential gaps at `rate`/s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


# --------------------------------------------------------------------------
# Small geometries for pins and parity tests
# --------------------------------------------------------------------------

def channel_2d(nx: int, ny: int, tau: float, u_peak: float) -> Workload:
    """Straight 2D channel (D2Q9): walls at y=0 and y=ny-1, parabolic velocity
    inlet on x=0, pressure outlet on x=nx-1, fluid (non-design) inside."""
    m = walled_box(nx, ny, 1, dim=2, interior=FLUID)
    m[0, 1:ny - 1, 0] = code(INLET, NPX)
    m[0, 1:ny - 1, nx - 1] = code(OUTLET, NMX)
    L = float(ny - 2)
    nu = (tau - 0.5) / 3.0
    return Workload(name=f"channel_2d_{nx}x{ny}", dim=2, nx=nx, ny=ny, nz=1, thermal=False,
                    tau=tau, Re=u_peak * L / nu, L_ref=L, objective=OBJ_PRESSURE_DROP,
                    mask=m, gamma=np.ones((1, ny, nx)), alpha_max=0.0)


def channel_3d_slit(nx: int, ny: int, nz: int, tau: float, u_peak: float) -> Workload:
    """Plane channel in 3D (D3Q19): walls at z=0 and z=nz-1, periodic in y,
    velocity inlet on x=0, pressure outlet on x=nx-1, fluid inside."""
    per = (False, True, False)
    m = walled_box(nx, ny, nz, periodic=per, interior=FLUID)
    m[1:nz - 1, :, 0] = code(INLET, NPX)
    m[1:nz - 1, :, nx - 1] = code(OUTLET, NMX)
    L = float(nz - 2)
    nu = (tau - 0.5) / 3.0
    return Workload(name=f"slit_{nx}x{ny}x{nz}", dim=3, nx=nx, ny=ny, nz=nz, thermal=False,
                    tau=tau, Re=u_peak * L / nu, L_ref=L, objective=OBJ_PRESSURE_DROP,
                    mask=m, gamma=np.ones((nz, ny, nx)), alpha_max=0.0, periodic=per)


def periodic_box(n: int, dim: int, gamma_value: float, thermal: bool = False) -> Workload:
    """Fully periodic box of design nodes with a uniform design field."""
    nz = n if dim == 3 else 1
    per = (True, True, True)
    m = np.full((nz, n, n), DESIGN, dtype=np.uint8)
    return Workload(name=f"periodic_{dim}d_{n}", dim=dim, nx=n, ny=n, nz=nz,
                    thermal=thermal, tau=0.8, Re=0.0, L_ref=1.0, objective=OBJ_DISSIPATION,
                    mask=m, gamma=np.full((nz, n, n), gamma_value), periodic=per)


def conduction_column(nx: int, ny: int, nz: int, tau: float, Pr: float, q_w: float,
                      T_top: float) -> Workload:
    """Pure conduction: closed box with a heated floor (z=0, heat flux q_w),
    a zero-velocity inlet on the top face acting as a Dirichlet T_top
    boundary, adiabatic walls elsewhere, fluid inside (no flow)."""
    m = walled_box(nx, ny, nz, interior=FLUID)
    m[0, 1:ny - 1, 1:nx - 1] = code(HEATED, NPZ)
    m[nz - 1, 1:ny - 1, 1:nx - 1] = code(INLET, NMZ)
    return Workload(name=f"conduction_{nx}x{ny}x{nz}", dim=3, nx=nx, ny=ny, nz=nz,
                    thermal=True, tau=tau, Re=0.0, L_ref=1.0, objective=OBJ_HEATSINK, mask=m,
                    gamma=np.ones((nz, ny, nx)), Pr=Pr, q_w=q_w, T_in=T_top, w_dp=0.0)


def conduction_layers(nx: int, ny: int, gammas, tau: float, Pr: float, q_w: float,
                      T_top: float, k_ratio: float = 100.0, q_ramp: float = 1.0) -> Workload:
    """Pure conduction through layers of design nodes: the closed box of
    `conduction_column` (heated floor z = 0, zero-velocity inlet on the top
    face as a Dirichlet T_top boundary, adiabatic side walls) whose interior
    layers z = 1 .. nz-2 are DESIGN nodes, layer z holding the uniform design
    value gammas[z - 1] (so nz = len(gammas) + 2).  No flow: the design field
    enters only through the conductivity of each layer."""
    g = np.asarray(gammas, dtype=np.float64)
    nz = len(g) + 2
    m = walled_box(nx, ny, nz, interior=DESIGN)
    m[0, 1:ny - 1, 1:nx - 1] = code(HEATED, NPZ)
    m[nz - 1, 1:ny - 1, 1:nx - 1] = code(INLET, NMZ)
    gamma = np.ones((nz, ny, nx))
    gamma[1:nz - 1] = g[:, None, None]
    return Workload(name=f"conduction_layers_{nx}x{ny}x{nz}", dim=3, nx=nx, ny=ny, nz=nz,
                    thermal=True, tau=tau, Re=0.0, L_ref=1.0, objective=OBJ_HEATSINK, mask=m,
                    gamma=gamma, Pr=Pr, q_w=q_w, T_in=T_top, w_dp=0.0, k_ratio=k_ratio,
                    q_ramp=q_ramp)


def conduction_column_2d(nx: int, ny: int, tau: float, Pr: float, q_w: float,
                         T_top: float) -> Workload:
    """Pure conduction in 2D (D2Q9 + D2Q5): a heated floor (y = 0, heat flux
    q_w), a zero-velocity inlet on the top row acting as a Dirichlet T_top
    boundary, adiabatic side walls, fluid inside (no flow)."""
    m = walled_box(nx, ny, 1, dim=2, interior=FLUID)
    m[0, 0, 1:nx - 1] = code(HEATED, NPY)
    m[0, ny - 1, 1:nx - 1] = code(INLET, NMY)
    return Workload(name=f"conduction_2d_{nx}x{ny}", dim=2, nx=nx, ny=ny, nz=1, thermal=True,
                    tau=tau, Re=0.0, L_ref=1.0, objective=OBJ_HEATSINK, mask=m,
                    gamma=np.ones((1, ny, nx)), Pr=Pr, q_w=q_w, T_in=T_top, w_dp=0.0)


def paper_heat_sink_2d(nx: int = 512, ny: int = 129, Re: float = 60.0, tau: float = 0.6,
                       Pr: float = 7.1, beta_max: float = 1e-5, k_ratio: float = 100.0,
                       alpha_max: float = 0.1, buffer: int = 4, sigma: float = 3.0,
                       seed: Optional[int] = None, name: Optional[str] = None) -> Workload:
    """The 2D form of the paper's heat sink (the planform that Sec. 3.3.5
    designs in 2D and extrudes): D2Q9 flow and D2Q5 heat on the half domain
    below the mirror plane of the channel, wall at y = 0, SYM nodes on the
    last row, pressure inlet over x = 0 and outlet over x = nx-1, `buffer`
    fluid columns after the inlet and before the outlet, the design domain
    between; heat Q = beta(gamma)(1 - T) in the solid (Eq. 69), J = -sum Q
    (Eq. 72); Re from Eq. (70) with L the full width between the walls,
    2 (ny - 2) + 1 nodes."""
    seed = SEED_BASE + 8 if seed is None else seed
    m = np.full((1, ny, nx), DESIGN, dtype=np.uint8)
    m[0, 0, :] = WALL
    m[0, :, 0] = WALL
    m[0, :, nx - 1] = WALL
    m[0, 1:ny - 1, 0] = code(INLET, NPX)
    m[0, 1:ny - 1, nx - 1] = code(OUTLET, NMX)
    if buffer > 0:
        m[0, 1:ny - 1, 1:1 + buffer] = FLUID
        m[0, 1:ny - 1, nx - 1 - buffer:nx - 1] = FLUID
    m[0, ny - 1, :] = SYM
    L = float(2 * (ny - 2) + 1)
    nu = (tau - 0.5) / 3.0
    dp = (Re * nu / L) ** 2
    gamma = smoothed_noise((1, ny, nx), sigma, seed)
    return Workload(name=name or f"paper_heat_sink_2d_{nx}x{ny}_Re{Re:g}", dim=2, nx=nx, ny=ny,
                    nz=1, thermal=True, tau=tau, Re=Re, L_ref=L, objective=OBJ_HEATGEN, mask=m,
                    gamma=gamma, alpha_max=alpha_max, q_brink=0.1, Pr=Pr, k_ratio=k_ratio,
                    q_ramp=1.0, q_w=0.0, T_in=0.0, w_dp=0.0, seed=seed,
                    symmetric=(False, True, False), inlet_rho=1.0 + 3.0 * dp, beta_max=beta_max)


def tiny_paper_heat_sink_2d(nx: int = 14, ny: int = 7, Re: float = 10.0, tau: float = 0.8,
                            beta_max: float = 2e-3, seed: int = 11) -> Workload:
    """A small 2D heat sink of the paper's formulation, for pins."""
    return paper_heat_sink_2d(nx, ny, Re=Re, tau=tau, Pr=1.0, beta_max=beta_max, alpha_max=0.2,
                              buffer=1, sigma=1.0, seed=seed,
                              name=f"tiny_paper_heat_sink_2d_{nx}x{ny}")


def six_port_box(nx: int = 14, ny: int = 13, nz: int = 12, thermal: bool = False,
                 objective: int = OBJ_DISSIPATION, adjoint_kind: int = 0, tau: float = 0.8,
                 drho_in: float = 3e-3, beta_max: float = 0.0, heated: bool = False,
                 seed: Optional[int] = None) -> Workload:
    """A walled box with one port patch on each of its six faces, so that
    every inward normal of the port rules occurs on one lattice: pressure
    inlets (at rho0 + drho_in) on x = 0, y = ny-1 and z = 0, pressure outlets
    on x = nx-1, y = 0 and z = nz-1, each a 4 x 4 patch inside its face;
    seeded smoothed design field in the interior.  With nz = 1 the 2D form:
    four ports of 4 nodes, one per edge (D2Q9, every 2D normal).  `heated`
    adds a HEATED patch (q_w = 0.01) beside the port on every face or edge,
    so the heated-wall rule also meets every inward normal."""
    seed = SEED_BASE + 10 if seed is None else seed
    if nz == 1:
        # the 2D form: four ports, one per edge (D2Q9 + D2Q5)
        m = walled_box(nx, ny, 1, dim=2)
        m[0, 3:7, 0] = code(INLET, NPX)
        m[0, 4:8, nx - 1] = code(OUTLET, NMX)
        m[0, 0, 3:7] = code(OUTLET, NPY)
        m[0, ny - 1, 5:9] = code(INLET, NMY)
        if heated:
            m[0, 8:11, 0] = code(HEATED, NPX)
            m[0, 9:12, nx - 1] = code(HEATED, NMX)
            m[0, 0, 9:12] = code(HEATED, NPY)
            m[0, ny - 1, 10:13] = code(HEATED, NMY)
    else:
        m = walled_box(nx, ny, nz)
        m[3:7, 3:7, 0] = code(INLET, NPX)
        m[3:7, 4:8, nx - 1] = code(OUTLET, NMX)
        m[4:8, 0, 3:7] = code(OUTLET, NPY)
        m[4:8, ny - 1, 5:9] = code(INLET, NMY)
        m[0, 3:7, 4:8] = code(INLET, NPZ)
        m[nz - 1, 5:9, 3:7] = code(OUTLET, NMZ)
        if heated:
            m[8:10, 8:11, 0] = code(HEATED, NPX)
            m[8:10, 8:11, nx - 1] = code(HEATED, NMX)
            m[8:10, 0, 8:11] = code(HEATED, NPY)
            m[1:3, ny - 1, 9:12] = code(HEATED, NMY)
            m[0, 8:11, 9:12] = code(HEATED, NPZ)
            m[nz - 1, 1:4, 9:12] = code(HEATED, NMZ)
    gamma = smoothed_noise((nz, ny, nx), 1.5, seed)
    return Workload(name=f"six_port_box_{nx}x{ny}x{nz}", dim=2 if nz == 1 else 3, nx=nx, ny=ny, nz=nz,
                    thermal=thermal, tau=tau, Re=0.0, L_ref=1.0, objective=objective, mask=m,
                    gamma=gamma, alpha_max=0.1, q_brink=0.1, Pr=1.0, k_ratio=10.0, q_ramp=1.0,
                    q_w=0.01 if heated else 0.0, T_in=0.0, w_dp=0.0, seed=seed,
                    adjoint_kind=adjoint_kind,
                    inlet_rho=1.0 + drho_in, beta_max=beta_max)


def tiny_heat_sink(nx: int = 10, ny: int = 8, nz: int = 6, seed: int = 7, Re: float = 5.0,
                   Pr: float = 1.0, tau: float = 0.8, alpha_max: float = 0.2,
                   sigma: float = 1.0) -> Workload:
    """A small coupled heat-sink problem with fast convergence, for gradient
    checks (same boundary set-up as `heat_sink`)."""
    w = heat_sink(nx, ny, nz, Re=Re, Pr=Pr, tau=tau, sigma=sigma, seed=seed,
                  name=f"tiny_heat_sink_{nx}x{ny}x{nz}")
    return w.replace(alpha_max=alpha_max)


def tiny_pipe_bend_3d(n: int = 10, seed: int = 11, Re: float = 2.0, tau: float = 0.8,
                      objective: int = OBJ_DISSIPATION, alpha_max: float = 0.2) -> Workload:
    """A small 3D pipe bend (inlet on x=0, outlet on y=0) for gradient checks."""
    m = walled_box(n, n, n)
    lo, hi = 2, n - 4
    m[lo:hi + 1, lo:hi + 1, 0] = code(INLET, NPX)
    m[lo:hi + 1, 0, n - 1 - (hi - lo + 1) - 1:n - 2] = code(OUTLET, NPY)
    gamma = smoothed_noise((n, n, n), 1.0, seed)
    return Workload(name=f"tiny_pipe_bend_{n}", dim=3, nx=n, ny=n, nz=n, thermal=False,
                    tau=tau, Re=Re, L_ref=float(hi - lo + 1), objective=objective, mask=m,
                    gamma=gamma, alpha_max=alpha_max, q_brink=0.1, w_dp=1.0, seed=seed)


def tiny_pipe_bend_2d(nx: int = 16, ny: int = 12, seed: int = 5, Re: float = 2.0,
                      tau: float = 0.8, alpha_max: float = 0.2) -> Workload:
    """A small 2D pipe bend (D2Q9) for gradient checks."""
    m = walled_box(nx, ny, 1, dim=2)
    m[0, 3:8, 0] = code(INLET, NPX)
    m[0, 0, nx - 7:nx - 2] = code(OUTLET, NPY)
    gamma = smoothed_noise((1, ny, nx), 1.0, seed)
    return Workload(name=f"tiny_pipe_bend_2d_{nx}x{ny}", dim=2, nx=nx, ny=ny, nz=1,
                    thermal=False, tau=tau, Re=Re, L_ref=5.0, objective=OBJ_PRESSURE_DROP,
                    mask=m, gamma=gamma, alpha_max=alpha_max, q_brink=0.1, seed=seed)


def config_workloads():
    """The benchmark configurations at their full sizes."""
    return {
        "pipe_bend_2d": pipe_bend_2d(),
        "pipe_bend_3d": pipe_bend_3d(),
        "heat_sink_Re50": heat_sink(Re=50.0),
        "heat_sink_Re200": heat_sink(Re=200.0),
        "heat_sink_Re400": heat_sink(Re=400.0),
        "differentiable": differentiable_case(),
    }


def nu_of(tau: float) -> float:
    """Lattice viscosity for relaxation time tau (used only to pick inputs)."""
    return (tau - 0.5) / 3.0


def describe(w: Workload) -> dict:
    """Short JSON-able description of a workload (no arrays)."""
    return {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "nodes": w.N, "tau": w.tau,
            "Re": w.Re, "thermal": w.thermal, "objective": OBJECTIVE_NAMES[w.objective],
            "seed": w.seed}


__all__ = [n for n in dir() if not n.startswith("_") and n not in ("annotations", "math",
                                                                   "dataclasses", "Optional")]
