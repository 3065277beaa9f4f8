"""Writes the stored FP64 reference solutions of the full-size configurations.

For each configuration the FP64 oracle (oracle/) solves the forward problem
and the discrete adjoint from rest to a residual far below the GPU's own
criterion, then takes the sensitivity; the script stores the converged
density deviation, velocity, temperature and dJ/dgamma over every node
(float32: the 1e-5 and 1e-4 tolerances they are checked against are far
above that rounding), J, the step counts and residuals, and what identifies
the inputs (the workload's name, grid, parameters and seed, and a digest of
its mask and design field).  With --fd it also stores central differences
of J (h = 1e-4) at seeded design cells: each from two forward solves warm
started at the converged state with the cell's design value moved by +-h,
run the same fixed number of steps (the base state's residue cancels in the
difference).

Only the oracle and the workload generators are used here.  Run from the
repository root:

    python tests/golden/make_converged_fixtures.py heat_sink_160x80x40_Re200
    python tests/golden/make_converged_fixtures.py heat_sink_128x64x32_Re200
    python tests/golden/make_converged_fixtures.py heat_sink_128x64x32_Re200 --fd 32 \
        --fd-steps 12000 --fd-only
    python tests/golden/make_converged_fixtures.py pipe_bend_96 --sample 65536 --tol 1e-9

With --sample K the fields are stored at K seeded non-wall nodes and dJ/dgamma
at K seeded design nodes (their indices beside them) instead of at every
node, which keeps the 96^3 pipe bend's fixture small.

The warm-started solves of some cells excite the slow thermal modes and
need about 10000 steps to settle; once settled, the two FP64 iterations only
exchange rounding noise (a few 1e-15 in J), which limits the differences'
own accuracy at h = 1e-4.  The value at half the steps is stored beside the
final one (fd_half).
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CONFIGS = {
    "heat_sink_160x80x40_Re200": lambda: W.heat_sink(Re=200.0),
    "heat_sink_128x64x32_Re200": W.differentiable_case,
    "pipe_bend_96": W.pipe_bend_3d,
}
TOL = 1e-10          # relative change of the monitors over 1000 steps
MAX_STEPS = 400000
FD_H = 1e-4


def digest(w) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(w.mask, dtype=np.uint8).tobytes())
    h.update(np.ascontiguousarray(w.gamma, dtype=np.float64).tobytes())
    return h.hexdigest()


def fixture_path(name: str) -> str:
    return os.path.join(HERE, f"converged_{name}.npz")


def fd_cells(w, n: int) -> np.ndarray:
    design = np.flatnonzero((w.mask.reshape(-1) & 7) == W.DESIGN)
    rng = np.random.default_rng(W.SEED_BASE + 32)
    return np.sort(rng.choice(design, size=n, replace=False))


def sample_nodes(w, k: int):
    """K seeded non-wall nodes and K seeded design nodes (sorted)."""
    kinds = w.mask.reshape(-1) & 7
    rng = np.random.default_rng(W.SEED_BASE + 96)
    live = np.flatnonzero(kinds < W.WALL)
    design = np.flatnonzero(kinds == W.DESIGN)
    return (np.sort(rng.choice(live, size=min(k, live.size), replace=False)),
            np.sort(rng.choice(design, size=min(k, design.size), replace=False)))


def log(msg):
    print(f"[fixture] {msg}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=sorted(CONFIGS))
    ap.add_argument("--fd", type=int, default=0, help="design cells checked by central differences")
    ap.add_argument("--fd-steps", type=int, default=0,
                    help="steps of each warm-started difference solve (0: twice the forward's)")
    ap.add_argument("--tol", type=float, default=TOL,
                    help="relative change of the monitors over 1000 steps that ends each sweep")
    ap.add_argument("--sample", type=int, default=0,
                    help="store the fields and dJ/dgamma at this many seeded nodes only")
    ap.add_argument("--fd-only", action="store_true",
                    help="add the differences to the stored fixture (the forward is re-solved "
                         "for the warm start, the adjoint is not)")
    args = ap.parse_args()
    w = CONFIGS[args.config]()
    o = oracle.Oracle(w)
    t0 = time.time()
    fw = o.forward(max_steps=MAX_STEPS, tol=args.tol, check_every=1000)
    log(f"{args.config}: forward {fw['steps']} steps, status {fw['status']}, residuals {fw['res']}, "
        f"{time.time() - t0:.0f} s")
    assert fw["status"] == 0, "forward did not converge"
    f, g = fw["f"], fw["g"]
    J = o.objective(f, g)
    if args.fd_only:
        ref = np.load(fixture_path(args.config))
        assert str(ref["inputs_sha256"]) == digest(w), "stored fixture is for other inputs"
        assert int(ref["fwd_steps"]) == fw["steps"] and float(ref["J"]) == J, \
            "re-solved forward differs from the stored one"
        out = {k: ref[k] for k in ref.files if not k.startswith("fd")}
        dJ = ref["dJ"].astype(np.float64)
    else:
        rho, u, T = o.macro(f, g)
        t1 = time.time()
        ad = o.adjoint(f, g, max_steps=MAX_STEPS, tol=args.tol, check_every=1000)
        log(f"adjoint {ad['steps']} steps, status {ad['status']}, residuals {ad['res']}, "
            f"{time.time() - t1:.0f} s")
        assert ad["status"] == 0, "adjoint did not converge"
        dJ = o.sensitivity(f, g, ad["fsC"], ad["gsC"])
        out = dict(drho=(rho - w.rho0).astype(np.float32), u=u.T.astype(np.float32).copy(),
                   T=(T if T is not None else np.zeros(0)).astype(np.float32),
                   dJ=dJ.astype(np.float32), J=np.float64(J),
                   fwd_steps=np.int64(fw["steps"]), adj_steps=np.int64(ad["steps"]),
                   fwd_res=np.asarray(fw["res"], dtype=np.float64),
                   adj_res=np.asarray(ad["res"], dtype=np.float64), tol=np.float64(args.tol),
                   name=np.str_(w.name), grid=np.array([w.nx, w.ny, w.nz], dtype=np.int64),
                   tau=np.float64(w.tau), Re=np.float64(w.Re), seed=np.int64(w.seed),
                   inputs_sha256=np.str_(digest(w)))
        if args.sample > 0:
            live, design = sample_nodes(w, args.sample)
            out.update(sample=live.astype(np.int64), drho=out["drho"][live],
                       u=out["u"][:, live].copy(),
                       T=out["T"][live] if out["T"].size else out["T"],
                       dJ_sample=design.astype(np.int64), dJ=out["dJ"][design])
    if args.fd > 0:
        cells = fd_cells(w, args.fd)
        steps = args.fd_steps or 2 * fw["steps"]
        vals, half = [], []
        for i, k in enumerate(cells):
            Jpm, Jh = [], []
            for s in (+1.0, -1.0):
                gm = o.gamma.copy()
                gm[k] += s * FD_H
                # in two halves: the difference at half the steps shows how
                # far the warm-started solves still were from settling
                r = o.forward(gamma=gm, max_steps=steps // 2, tol=0.0, check_every=0, state=(f, g))
                Jh.append(o.objective(r["f"], r["g"], gamma=gm))
                r = o.forward(gamma=gm, max_steps=steps - steps // 2, tol=0.0, check_every=0,
                              state=(r["f"], r["g"]))
                Jpm.append(o.objective(r["f"], r["g"], gamma=gm))
            vals.append((Jpm[0] - Jpm[1]) / (2.0 * FD_H))
            half.append((Jh[0] - Jh[1]) / (2.0 * FD_H))
            log(f"fd cell {i + 1}/{len(cells)} node {k}: {vals[-1]:.9e} (at half the steps "
                f"{half[-1]:.9e}; adjoint {dJ[k]:.9e}), {time.time() - t0:.0f} s")
        out.update(fd_cells=cells.astype(np.int64), fd=np.asarray(vals, dtype=np.float64),
                   fd_half=np.asarray(half, dtype=np.float64),
                   fd_h=np.float64(FD_H), fd_steps=np.int64(steps))
    np.savez_compressed(fixture_path(args.config), **out)
    log(f"wrote {fixture_path(args.config)} ({os.path.getsize(fixture_path(args.config)) / 1e6:.1f} MB), "
        f"J {J:.12g}, {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
