"""Helpers shared by the GPU parity tests: run the GPU library through the C
ABI, convert its states to the oracle's layout, and compare."""
import numpy as np
import torch

import oracle
import workloads as W
from paper_2501_02161_amd import lbm


def kinds(w):
    return w.mask.reshape(-1) & 7


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def perm_to_oracle(o, which, two_d=False):
    """perm[i_oracle] = i_gpu for the flow (0) or thermal (1) lattice, matched by
    velocity vectors (the two sides keep their own tables); a 2D problem has
    D2Q9 and D2Q5."""
    eg, wg = lbm.lbm_lattice((2 if which == 0 else 3) if two_d else which)
    eo, wo = o.lattice(which)
    perm = np.zeros(len(wo), dtype=np.int64)
    for i, e in enumerate(eo):
        j = [k for k in range(len(wg)) if np.array_equal(eg[k], e)]
        assert len(j) == 1
        perm[i] = j[0]
        assert wg[j[0]] == wo[i]
    return perm


def gpu_pops(prob, which, o):
    """A workspace state as node-major float64 [N, Q] in oracle order (still
    shifted as stored)."""
    st = prob.state(which)
    s = st.reshape(st.shape[0], -1).T.cpu().numpy().astype(np.float64)
    lat = 0 if which in (lbm.STATE_FLOW, lbm.STATE_ADJ_FLOW) else 1
    return s[:, perm_to_oracle(o, lat, prob.spec.nz == 1)]


def gpu_fields(prob):
    drho = prob.drho.reshape(-1).cpu().numpy().astype(np.float64)
    u = prob.u.reshape(3, -1).T.cpu().numpy().astype(np.float64)
    T = prob.T.reshape(-1).cpu().numpy().astype(np.float64) if prob.thermal else None
    dJ = prob.dJ.reshape(-1).cpu().numpy().astype(np.float64)
    return drho, u, T, dJ


def compare_solution(w, prob, ref, tol_field=1e-5, tol_grad=1e-4):
    """Norm-wise relative errors of (p - p_out, u, T - T_in) over non-wall
    nodes and of dJ/dgamma over design nodes; returns the dict of errors and
    asserts the tolerances."""
    k = kinds(w)
    live = k < W.WALL
    design = k == W.DESIGN
    drho, u, T, dJ = gpu_fields(prob)
    err = {
        "p": rel(drho[live], ref["rho"][live] - w.rho0),
        "u": rel(u[live], ref["u"][live]),
        "dJ": rel(dJ[design], ref["dJ"][design]),
    }
    if w.thermal:
        err["T"] = rel(T[live] - w.T_in, ref["T"][live] - w.T_in)
    for key in ("p", "u", "T"):
        if key in err:
            assert err[key] < tol_field, (key, err)
    assert err["dJ"] < tol_grad, ("dJ", err)
    assert np.all(dJ[~design] == 0.0)
    return err


def run_gpu(w, steps=None, tol=None, check_every=None):
    kw = {}
    if steps is not None:
        kw["max_steps"] = steps
    if tol is not None:
        kw["tol"] = tol
    if check_every is not None:
        kw["check_every"] = check_every
    prob = lbm.Problem(w.replace(**kw) if kw else w, device="cuda:0")
    res = prob.solve(w.gamma)
    torch.cuda.synchronize()
    return prob, res


def run_oracle(w, steps=None, tol=None, check_every=None):
    o = oracle.Oracle(w)
    ref = o.solve(fwd_steps=steps, adj_steps=steps, tol=tol, check_every=check_every)
    return o, ref
