"""Level-set design update of the topology-optimisation loop, plain numpy.

TEST INFRASTRUCTURE ONLY: used by the test suite to check the library's
update; the library never calls it.

Sec. 2.2 of the paper: the design is a level set phi in [-1, 1] (Eq. 13),
moved by the reaction-diffusion equation d phi / d xi = -K (J' - sigma lap phi)
(Eq. 14) with J' = J'_W + lambda, lambda = exp(G) mean |J'_W - sigma lap phi|
(Eq. 67), G the volume-constraint value of Eq. (10); the binary design is
alpha = 1 where phi >= 0, else 0 (Eq. 15).  Readings taken here (the text
leaves them open): one explicit Euler step per optimisation iteration;
J'_W is divided by its mean absolute value over the design domain so that K
is scale free; phi is clamped to [-1, 1] (the range of Eq. 13); lap is the
7-point Laplacian on the design nodes with no flux to other nodes; G is the
fluid fraction of the design domain minus V_max.
"""
import numpy as np


def laplacian(phi, design):
    """7-point Laplacian of phi [nz, ny, nx] over design nodes; a neighbour
    outside the box or not a design node counts as the node itself."""
    out = np.zeros_like(phi)
    nz, ny, nx = phi.shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if not design[z, y, x]:
                    continue
                c = phi[z, y, x]
                s = 0.0
                for dz, dy, dx in ((0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)):
                    zz, yy, xx = z + dz, y + dy, x + dx
                    inside = 0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx
                    s += phi[zz, yy, xx] if inside and design[zz, yy, xx] else c
                out[z, y, x] = s - 6.0 * c
    return out


def levelset_update(phi, dJ, design, K, sigma, vmax):
    """One design update: returns (phi_new, alpha, info) with info the
    lambda of Eq. (67), the fluid fraction before the step, G and the scale
    of J'.  Non-design entries of phi_new copy phi; alpha is returned on the
    design nodes only (others 0)."""
    phi = np.asarray(phi, dtype=np.float64)
    dJ = np.asarray(dJ, dtype=np.float64)
    d = np.asarray(design, dtype=bool)
    nd = int(d.sum())
    scale = np.abs(dJ[d]).sum() / nd
    volume = float((phi[d] >= 0.0).sum()) / nd
    G = volume - vmax
    lap = laplacian(phi, d)
    Jn = dJ / scale if scale > 0 else np.zeros_like(dJ)
    lam = np.exp(G) * np.abs(Jn[d] - sigma * lap[d]).sum() / nd
    phi_new = phi.copy()
    phi_new[d] = np.clip(phi[d] - K * (Jn[d] + lam - sigma * lap[d]), -1.0, 1.0)
    alpha = np.zeros_like(phi)
    alpha[d] = (phi_new[d] >= 0.0).astype(float)
    return phi_new, alpha, {"lambda": lam, "volume": volume, "G": G, "scale": scale}
