"""Level-set design update of the topology-optimisation loop, plain numpy.

TEST INFRASTRUCTURE ONLY: used by the test suite to check the library's
update; the library never calls it.

Sec. 2.2 of the paper: the design is a level set phi in [-1, 1] (Eq. 13),
moved by the reaction-diffusion equation d phi / d xi = -K (J' - sigma lap phi)
(Eq. 14) with J' = J'_W + lambda, lambda = exp(G) mean |J'_W - sigma lap phi|
(Eq. 67), G the volume-constraint value of Eq. (10); the binary design is
alpha = 1 where phi >= 0, else 0 (Eq. 15).

Readings taken here (the text leaves them open):
* one step of Eq. (14) per optimisation iteration, semi-implicit: the
  reaction term J'_W + lambda at the current phi, the diffusion term at the
  new phi, i.e. (I - K sigma lap) phi_new = phi - K (J'_W / s + lambda);
  then phi_new is clamped to [-1, 1] (the range of Eq. 13);
* J'_W is divided by s = mean |J'_W| over the design domain (K scale free);
* lap is the 7-point Laplacian (5-point in 2D) in lattice units on the
  design nodes; a neighbour that is not a design node (or lies outside the
  box) counts as the node itself: no flux out of the design domain;
* lambda uses lap of the current phi;
* an anisotropic sigma (Sec. 3.3.4: a diagonal matrix) weights each axis'
  second difference by its own coefficient;
* G is the fluid fraction of the design domain (phi >= 0) minus V_max.
kinds are the node kinds of the mask (DESIGN = 0).
"""
import numpy as np
import scipy.sparse
import scipy.sparse.linalg

_DESIGN = 0
# (offset, axis): axis 0 x, 1 y, 2 z
_OFFSETS = (((0, 0, -1), 0), ((0, 0, 1), 0), ((0, -1, 0), 1), ((0, 1, 0), 1),
            ((-1, 0, 0), 2), ((1, 0, 0), 2))


def _sigma3(sigma):
    s = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (3,))
    return tuple(float(v) for v in s)


def _design_neighbours(kinds, z, y, x):
    """(index, axis) of the axis neighbours of a node that are design nodes."""
    nz, ny, nx = kinds.shape
    out = []
    for (dz, dy, dx), ax in _OFFSETS:
        zz, yy, xx = z + dz, y + dy, x + dx
        if 0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx and kinds[zz, yy, xx] == _DESIGN:
            out.append(((zz, yy, xx), ax))
    return out


def laplacian(phi, kinds, sigma=1.0):
    """sigma-weighted Laplacian sum_a sigma_a d_aa phi of phi [nz, ny, nx] on
    the design nodes (0 elsewhere); sigma a scalar or (sigma_x, sigma_y,
    sigma_z)."""
    sg = _sigma3(sigma)
    phi = np.asarray(phi, dtype=np.float64)
    out = np.zeros_like(phi)
    nz, ny, nx = phi.shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if kinds[z, y, x] != _DESIGN:
                    continue
                c = phi[z, y, x]
                out[z, y, x] = sum(sg[ax] * (phi[idx] - c)
                                   for idx, ax in _design_neighbours(kinds, z, y, x))
    return out


def implicit_matrix(kinds, K, sigma):
    """The matrix of the semi-implicit step over the design nodes,
    A = I - K lap_sigma restricted to design unknowns (CSR, in the order of
    np.flatnonzero(kinds == DESIGN))."""
    sg = _sigma3(sigma)
    d = np.asarray(kinds) == _DESIGN
    ids = -np.ones(kinds.shape, dtype=np.int64)
    nodes = np.argwhere(d)
    ids[d] = np.arange(len(nodes))
    rows, cols, vals = [], [], []
    for r, (z, y, x) in enumerate(nodes):
        diag = 1.0
        for idx, ax in _design_neighbours(kinds, z, y, x):
            rows.append(r)
            cols.append(ids[idx])
            vals.append(-K * sg[ax])
            diag += K * sg[ax]
        rows.append(r)
        cols.append(r)
        vals.append(diag)
    return scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(len(nodes), len(nodes)))


def levelset_update(phi, dJ, kinds, K, sigma, vmax):
    """One design update: returns (phi_new, alpha, info) with info the
    lambda of Eq. (67), the fluid fraction before the step, G and the scale
    of J'.  sigma (lattice units) is a scalar or per axis (sigma_x, sigma_y,
    sigma_z): the anisotropic regularisation of Sec. 3.3.4, sigma lap
    becoming sum_a sigma_a d_aa.  Non-design entries of phi_new copy phi;
    alpha is returned on the design nodes only (others 0)."""
    sg = _sigma3(sigma)
    phi = np.asarray(phi, dtype=np.float64)
    dJ = np.asarray(dJ, dtype=np.float64)
    kinds = np.asarray(kinds)
    d = kinds == _DESIGN
    nd = int(d.sum())
    scale = np.abs(dJ[d]).sum() / nd
    volume = float((phi[d] >= 0.0).sum()) / nd
    G = volume - vmax
    lap = laplacian(phi, kinds, sg)
    Jn = dJ / scale if scale > 0 else np.zeros_like(dJ)
    lam = np.exp(G) * np.abs(Jn[d] - lap[d]).sum() / nd
    rhs = phi[d] - K * (Jn[d] + lam)
    if max(sg) > 0.0:
        A = implicit_matrix(kinds, K, sg)
        sol = scipy.sparse.linalg.spsolve(A.tocsc(), rhs)
    else:
        sol = rhs
    phi_new = phi.copy()
    phi_new[d] = np.clip(sol, -1.0, 1.0)
    alpha = np.zeros_like(phi)
    alpha[d] = (phi_new[d] >= 0.0).astype(float)
    return phi_new, alpha, {"lambda": lam, "volume": volume, "G": G, "scale": scale}
