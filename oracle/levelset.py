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
  design nodes; a neighbour outside the design domain enters with the fixed
  phase of its node: +1 for fluid nodes and ports, -1 for walls; a
  neighbour outside the box or on a mirror layer counts as the node itself
  (no flux);
* lambda uses lap of the current phi;
* G is the fluid fraction of the design domain (phi >= 0) minus V_max.
The node kinds are those of the mask: DESIGN 0, FLUID 1, INLET 2, OUTLET 3,
WALL 4, HEATED 5, SYM 6.
"""
import numpy as np
import scipy.sparse
import scipy.sparse.linalg

_DESIGN, _SYM = 0, 6
_FLUID_LIKE = (1, 2, 3)    # fixed phase +1
_SOLID_LIKE = (4, 5)       # fixed phase -1
_OFFSETS = ((0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0))


def _neighbours(kinds, z, y, x):
    """(kind, index) of the 6 axis neighbours of a node that lie inside the
    box and are not mirror-layer nodes."""
    nz, ny, nx = kinds.shape
    out = []
    for dz, dy, dx in _OFFSETS:
        zz, yy, xx = z + dz, y + dy, x + dx
        if not (0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx):
            continue
        k = int(kinds[zz, yy, xx])
        if k == _SYM:
            continue
        out.append((k, (zz, yy, xx)))
    return out


def fixed_phase(kind):
    return 1.0 if kind in _FLUID_LIKE else -1.0


def laplacian(phi, kinds):
    """Laplacian of phi [nz, ny, nx] on the design nodes (0 elsewhere)."""
    phi = np.asarray(phi, dtype=np.float64)
    out = np.zeros_like(phi)
    nz, ny, nx = phi.shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if kinds[z, y, x] != _DESIGN:
                    continue
                c = phi[z, y, x]
                s = 0.0
                for k, idx in _neighbours(kinds, z, y, x):
                    v = phi[idx] if k == _DESIGN else fixed_phase(k)
                    s += v - c
                out[z, y, x] = s
    return out


def implicit_matrix(kinds, a):
    """The system of the semi-implicit step over the design nodes:
    A = I - a lap restricted to design unknowns (CSR, in the order of
    np.flatnonzero(kinds == DESIGN)) and b, the fixed-phase neighbours'
    contribution a * sum v, so that A phi_new = rhs + b."""
    d = np.asarray(kinds) == _DESIGN
    ids = -np.ones(kinds.shape, dtype=np.int64)
    nodes = np.argwhere(d)
    ids[d] = np.arange(len(nodes))
    rows, cols, vals = [], [], []
    b = np.zeros(len(nodes))
    for r, (z, y, x) in enumerate(nodes):
        diag = 1.0
        for k, idx in _neighbours(kinds, z, y, x):
            diag += a
            if k == _DESIGN:
                rows.append(r)
                cols.append(ids[idx])
                vals.append(-a)
            else:
                b[r] += a * fixed_phase(k)
        rows.append(r)
        cols.append(r)
        vals.append(diag)
    A = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(len(nodes), len(nodes)))
    return A, b


def levelset_update(phi, dJ, kinds, K, sigma, vmax):
    """One design update: returns (phi_new, alpha, info) with info the
    lambda of Eq. (67), the fluid fraction before the step, G and the scale
    of J'.  sigma is in lattice units.  Non-design entries of phi_new copy
    phi; alpha is returned on the design nodes only (others 0)."""
    phi = np.asarray(phi, dtype=np.float64)
    dJ = np.asarray(dJ, dtype=np.float64)
    kinds = np.asarray(kinds)
    d = kinds == _DESIGN
    nd = int(d.sum())
    scale = np.abs(dJ[d]).sum() / nd
    volume = float((phi[d] >= 0.0).sum()) / nd
    G = volume - vmax
    lap = laplacian(phi, kinds)
    Jn = dJ / scale if scale > 0 else np.zeros_like(dJ)
    lam = np.exp(G) * np.abs(Jn[d] - sigma * lap[d]).sum() / nd
    rhs = phi[d] - K * (Jn[d] + lam)
    if sigma > 0.0:
        A, b = implicit_matrix(kinds, K * sigma)
        sol = scipy.sparse.linalg.spsolve(A.tocsc(), rhs + b)
    else:
        sol = rhs
    phi_new = phi.copy()
    phi_new[d] = np.clip(sol, -1.0, 1.0)
    alpha = np.zeros_like(phi)
    alpha[d] = (phi_new[d] >= 0.0).astype(float)
    return phi_new, alpha, {"lambda": lam, "volume": volume, "G": G, "scale": scale}
