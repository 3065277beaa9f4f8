"""Stability test of the adjoint solves (Sec. 3.1): for a relaxation time,
the largest inlet speed at which a solve stays stable for a given number of
iterations, for the primal (forward) solve, the discrete adjoint and the
continuous adjoint.  Every (tau, speed, adjoint kind) point is one request to
the continuous-batching engine, so the whole sweep advances in shared
ragged-batch launches; all arithmetic runs in the gfx950 library.

A point is
  "diverged"  in the forward sweep if the forward solve blew up,
  "adjoint diverged" if the forward solve stayed finite and the adjoint blew up,
  "stable"    if both stayed finite for their step caps (converged or not).
"""
from __future__ import annotations

import time

import numpy as np

from . import lbm, serving


def run_points(cases, budget_bytes=16 << 30, quantum=250, log=None):
    """Solve every workload in `cases` through one batch engine (policy ALL:
    all resident points advance together); returns a list of result dicts
    in the same order."""
    eng = serving.BatchEngine(False, lbm.LBM_OBJ_PRESSURE_DROP, budget_bytes=budget_bytes,
                              max_slots=max(1, len(cases)), quantum=quantum,
                              policy=lbm.LBM_BATCH_POLICY_ALL)
    tickets = {eng.submit(w): i for i, w in enumerate(cases)}
    out = [None] * len(cases)
    t0 = time.perf_counter()
    last = t0
    while tickets:
        eng.step()
        for t, i in list(tickets.items()):
            r = eng.collect(t, cases[i].N)
            if r is not None:
                out[i] = r
                del tickets[t]
        now = time.perf_counter()
        if log and now - last > 20.0:
            log(f"{len(cases) - len(tickets)}/{len(cases)} points done after {now - t0:.0f} s")
            last = now
    eng.close()
    return out


def classify(r) -> str:
    if r["state"] == lbm.LBM_BATCH_DONE:
        return "stable"
    if r["adj_steps"] > 0:
        return "adjoint diverged"
    return "diverged"


def sweep(taus, speeds, n=32, max_steps=1000000, log=None, dim=3):
    """Run the grid taus x speeds x {discrete, continuous}; returns
    (points, limits): points[(tau, u, kind)] = (class, fwd_steps, adj_steps),
    limits[tau] = {"primal": u, "discrete": u, "continuous": u} with the
    largest tested speed below which every point is stable (0 if none)."""
    import workloads as W

    keys, cases = [], []
    for tau in taus:
        for u in speeds:
            for kind in (lbm.LBM_ADJOINT_DISCRETE, lbm.LBM_ADJOINT_CONTINUOUS):
                keys.append((tau, u, kind))
                cases.append(W.stability_case(n, tau, u, kind, max_steps=max_steps, dim=dim))
    res = run_points(cases, log=log)
    points = {k: (classify(r), r["fwd_steps"], r["adj_steps"]) for k, r in zip(keys, res)}
    limits = {}
    for tau in taus:
        lim = {"primal": 0.0, "discrete": 0.0, "continuous": 0.0}
        ok = {"primal": True, "discrete": True, "continuous": True}
        for u in sorted(speeds):
            cd = points[(tau, u, lbm.LBM_ADJOINT_DISCRETE)][0]
            cc = points[(tau, u, lbm.LBM_ADJOINT_CONTINUOUS)][0]
            primal_ok = cd != "diverged" and cc != "diverged"
            ok["primal"] = ok["primal"] and primal_ok
            ok["discrete"] = ok["discrete"] and cd == "stable"
            ok["continuous"] = ok["continuous"] and cc == "stable"
            for key in lim:
                if ok[key]:
                    lim[key] = u
        limits[tau] = lim
    return points, limits
