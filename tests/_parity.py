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


def node_classes(w):
    """Boolean node masks for the pointwise report: ports (inlet, outlet),
    non-wall nodes with a wall among their lattice neighbours, non-wall nodes
    next to a mirror plane, nodes of the heat-sink objective layer (next to a
    heated wall), design nodes, and the remaining interior."""
    k = kinds(w).reshape(w.nz, w.ny, w.nx)
    live = k < W.WALL
    two_d = w.nz == 1
    per = getattr(w, "periodic", (False, False, False))
    offs = [(dx, dy, dz) for dz in ((0,) if two_d else (-1, 0, 1)) for dy in (-1, 0, 1)
            for dx in (-1, 0, 1) if (dx, dy, dz) != (0, 0, 0) and abs(dx) + abs(dy) + abs(dz) <= 2]

    def shifted(a, d, fill):
        # value of a at node + d; `fill` beyond a non-periodic face
        out = a
        for ax, dd, p in ((2, d[0], per[0]), (1, d[1], per[1]), (0, d[2], per[2])):
            if dd == 0:
                continue
            out = np.roll(out, -dd, axis=ax)
            if not p:
                sl = [slice(None)] * 3
                sl[ax] = slice(-1, None) if dd > 0 else slice(0, 1)
                out = out.copy()
                out[tuple(sl)] = fill
        return out

    wallish = (k == W.WALL) | (k == W.HEATED)
    heated = k == W.HEATED
    wall_adj = np.zeros_like(live)
    layer = np.zeros_like(live)
    for d in offs:
        wall_adj |= shifted(wallish, d, False)
        if abs(d[0]) + abs(d[1]) + abs(d[2]) == 1:
            layer |= shifted(heated, d, False)
    sym = getattr(w, "symmetric", (False, False, False))
    mirror_adj = np.zeros_like(live)
    if sym[0]:
        mirror_adj[:, :, w.nx - 2] = True
    if sym[1]:
        mirror_adj[:, w.ny - 2, :] = True
    if sym[2]:
        mirror_adj[w.nz - 2, :, :] = True
    cls = {
        "inlet": k == W.INLET,
        "outlet": k == W.OUTLET,
        "wall_adj": live & wall_adj,
        "mirror_adj": live & mirror_adj,
        "layer": live & layer,
        "design": k == W.DESIGN,
    }
    other = live.copy()
    for v in cls.values():
        other &= ~v
    cls["interior"] = other
    return {n: v.reshape(-1) for n, v in cls.items() if v.any()}


def pointwise(w, got, want, live, design, classes=None):
    """Pointwise errors.  got / want: dicts of node fields (p, u [N,3], T,
    population states [N,Q], dJ) on the GPU and the reference.  A field's
    error at a node is |got - want| (the vector norm over a row for u and the
    populations) over the field's scale, max |want| over non-wall nodes; the report holds its maximum per node class.  For
    dJ/dgamma (design nodes): the maximum over max |want|, and the maximum
    relative error |got - want| / |want| over the nodes where
    |want| > 1e-3 max |want|."""
    classes = node_classes(w) if classes is None else classes
    out = {}
    for key in want:
        if key == "dJ" or want[key] is None:
            continue
        g, r = np.asarray(got[key], np.float64), np.asarray(want[key], np.float64)
        d = np.abs(g - r) if g.ndim == 1 else np.linalg.norm(g - r, axis=1)
        mag = np.abs(r) if r.ndim == 1 else np.linalg.norm(r, axis=1)
        scale = max(float(mag[live].max()), 1e-300)
        per = {n: float(d[m & live].max() / scale) for n, m in classes.items() if (m & live).any()}
        per["all"] = float(d[live].max() / scale)
        out[key] = per
    if "dJ" in want:
        g, r = np.asarray(got["dJ"], np.float64)[design], np.asarray(want["dJ"], np.float64)[design]
        if g.size:
            top = max(float(np.abs(r).max()), 1e-300)
            sig = np.abs(r) > 1e-3 * top
            out["dJ"] = {"all": float(np.abs(g - r).max() / top),
                         "sig_rel": float((np.abs(g - r)[sig] / np.abs(r)[sig]).max()) if sig.any() else 0.0,
                         "sig_frac": float(sig.mean())}
    return out


def check_pointwise(pw, tol_point=1e-4, tol_grad_point=1e-3, tol_grad_sig=None):
    """Asserts the pointwise bounds on a report of `pointwise`."""
    for key in pw:
        if key != "dJ":
            assert pw[key]["all"] < tol_point, (key, pw[key])
    if "dJ" in pw:
        assert pw["dJ"]["all"] < tol_grad_point, ("dJ", pw["dJ"])
        if tol_grad_sig is not None:
            assert pw["dJ"]["sig_rel"] < tol_grad_sig, ("dJ", pw["dJ"])


def fmt_pointwise(pw):
    parts = []
    for key, per in pw.items():
        parts.append(key + "[" + " ".join(f"{n} {v:.1e}" for n, v in per.items()) + "]")
    return "pointwise " + " ".join(parts)


def compare_solution(w, prob, ref, tol_field=1e-5, tol_grad=1e-4, tol_point=1e-4,
                     tol_grad_point=1e-3, tol_grad_sig=None):
    """Norm-wise relative errors of (p - p_out, u, T - T_in) over non-wall
    nodes and of dJ/dgamma over design nodes, plus the pointwise report of
    `pointwise` (printed); returns the dict of errors and asserts the
    tolerances (norm-wise, and pointwise as in `check_pointwise`)."""
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
    got = {"p": drho, "u": u, "dJ": dJ}
    want = {"p": ref["rho"] - w.rho0, "u": ref["u"], "dJ": ref["dJ"]}
    if w.thermal:
        got["T"], want["T"] = T - w.T_in, ref["T"] - w.T_in
    pw = pointwise(w, got, want, live, design)
    print(f"[pointwise] {w.name}: {fmt_pointwise(pw)}", flush=True)
    for key in ("p", "u", "T"):
        if key in err:
            assert err[key] < tol_field, (key, err)
    assert err["dJ"] < tol_grad, ("dJ", err)
    check_pointwise(pw, tol_point, tol_grad_point, tol_grad_sig)
    assert np.all(dJ[~design] == 0.0)
    err["pointwise"] = pw
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
