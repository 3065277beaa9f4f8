"""Serving many sensitivity requests on one GPU with continuous batching.

`BatchEngine` wraps the library's batch engine (lbm_batch_*): requests are
queued, admitted by an HBM budget as slots and memory free up, and advanced
together by the ragged-batch kernel on the engine's concurrent lanes: one
launch per lattice step, or, for run sets of up to `persistent_tiles` tiles,
one persistent launch per quantum (off by default: slower on MI355X).  `serve` replays
an arrival trace against it in wall-clock time; `serve_back_to_back` replays
the same trace with one plain solve at a time (lbm_forward_solve,
lbm_adjoint_solve, lbm_sensitivity), which is the comparison the serving
numbers are quoted against.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import lbm


class BatchEngine:
    def __init__(self, thermal: bool, objective: int, budget_bytes: int, max_slots: int = 256,
                 quantum: int = 250, device="cuda:0", policy: int = lbm.LBM_BATCH_POLICY_OVERLAP,
                 fill_tiles: int = 512, persistent_tiles: int = 0):
        self.device = torch.device(device)
        self.h = lbm.lbm_batch_create(thermal, objective, max_slots, quantum)
        lbm.lbm_batch_set_policy(self.h, policy, fill_tiles)
        lbm.lbm_batch_set_persistent(self.h, persistent_tiles)
        self.quantum = quantum
        with torch.cuda.device(self.device):
            total = int(budget_bytes) + lbm.lbm_batch_table_bytes(self.h, int(budget_bytes)) + 512
            self.arena = torch.empty(total, dtype=torch.uint8, device=self.device)
            lbm.lbm_batch_bind_arena(self.h, self.arena)

    def submit(self, spec) -> int:
        d = lbm.make_desc(spec)
        return lbm.lbm_batch_submit(self.h, d, spec.mask, spec.gamma)

    def step(self):
        with torch.cuda.device(self.device):
            return lbm.lbm_batch_step(self.h)

    def collect(self, ticket: int, nodes: int):
        """Result dict (with dJ/dgamma as a numpy array) if the ticket is
        finished, else None.  A finished ticket is released."""
        dJ = np.empty(nodes, dtype=np.float32)
        r = lbm.lbm_batch_poll(self.h, ticket, dJ)
        if r.state in (lbm.LBM_BATCH_QUEUED, lbm.LBM_BATCH_RUNNING):
            return None
        return {"ticket": ticket, "state": int(r.state), "status": int(r.status), "J": float(r.J),
                "fwd_steps": int(r.fwd_steps), "adj_steps": int(r.adj_steps), "dJ": dJ}

    def stats(self) -> dict:
        return lbm.lbm_batch_stats(self.h)

    def close(self):
        if getattr(self, "h", None):
            lbm.lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve(engine: BatchEngine, requests, arrivals, time_scale: float = 1.0, log=None):
    """Replay `requests` arriving at `arrivals` (seconds from start) against
    the engine in wall-clock time.  Returns per-request dicts with arrival,
    completion and latency (seconds), plus the makespan.  `log`, if given, is
    called with a progress line every 16 completed requests."""
    order = np.argsort(arrivals)
    pending = [(float(arrivals[i]) * time_scale, int(i)) for i in order]
    tickets = {}
    results = {}
    t0 = time.perf_counter()
    while len(results) < len(requests):
        now = time.perf_counter() - t0
        while pending and pending[0][0] <= now:
            a, i = pending.pop(0)
            tickets[engine.submit(requests[i])] = (i, a)
        active, queued = engine.step()
        finished = engine.stats()["finished"]
        for t, (i, a) in (list(tickets.items()) if finished else []):
            w = requests[i]
            r = engine.collect(t, w.N)
            if r is None:
                continue
            done = time.perf_counter() - t0
            r.update(arrival=a, completion=done, latency=done - a, index=i)
            results[i] = r
            del tickets[t]
            if log and len(results) % 16 == 0:
                log(f"batched: {len(results)}/{len(requests)} done at {done:.1f} s")
        if active == 0 and queued == 0 and not tickets and pending:
            wait = pending[0][0] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
    makespan = max(r["completion"] for r in results.values())
    return [results[i] for i in range(len(requests))], makespan


def serve_back_to_back(requests, arrivals, device="cuda:0", time_scale: float = 1.0, log=None):
    """The same trace served by one plain solve at a time, in arrival order."""
    order = np.argsort(arrivals)
    results = {}
    t0 = time.perf_counter()
    for i in order:
        a = float(arrivals[i]) * time_scale
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
        w = requests[i]
        prob = lbm.Problem(w, device=device)
        try:
            res = prob.solve(w.gamma)
            dJ = prob.dJ.reshape(-1).cpu().numpy()
            ok = res["forward"]["status"] == lbm.LBM_OK and res["adjoint"]["status"] == lbm.LBM_OK
            r = {"state": lbm.LBM_BATCH_DONE,
                 "status": lbm.LBM_OK if ok else lbm.LBM_NOT_CONVERGED, "J": res["J"],
                 "fwd_steps": res["forward"]["steps"], "adj_steps": res["adjoint"]["steps"],
                 "dJ": dJ}
        except lbm.LBMError as e:
            torch.cuda.synchronize(device)
            r = {"state": lbm.LBM_BATCH_FAILED, "status": e.code, "J": float("nan"),
                 "fwd_steps": 0, "adj_steps": 0, "dJ": np.zeros(0, np.float32)}
        done = time.perf_counter() - t0
        r.update(index=int(i), arrival=a, completion=done, latency=done - a)
        results[int(i)] = r
        prob.close()
        if log and len(results) % 16 == 0:
            log(f"back-to-back: {len(results)}/{len(requests)} done at {done:.1f} s")
    makespan = max(r["completion"] for r in results.values())
    return [results[i] for i in range(len(requests))], makespan


def summarize(results, makespan) -> dict:
    """Latency percentiles over every request (a failed request's latency is
    the time until its failure was reported); MLUPS counts the node updates
    of the completed requests only, over the makespan."""
    lat = np.array([r["latency"] for r in results])
    done = [r for r in results if r["state"] == lbm.LBM_BATCH_DONE]
    updates = sum((r["fwd_steps"] + r["adj_steps"]) * r["dJ"].size for r in done)
    return {"requests": len(results), "completed": len(done),
            "failed": len(results) - len(done),
            "p50_s": round(float(np.percentile(lat, 50)), 4),
            "p99_s": round(float(np.percentile(lat, 99)), 4),
            "mean_s": round(float(lat.mean()), 4), "makespan_s": round(makespan, 3),
            "MLUPS": round(updates / makespan / 1e6, 1)}


def same_results(a, b) -> bool:
    """True if two runs of one trace gave the same outcome for every request:
    the same state, and for completed requests the same step counts, the same
    J and the same dJ/dgamma bit for bit."""
    for ra, rb in zip(a, b):
        if ra["state"] != rb["state"]:
            return False
        if ra["state"] != lbm.LBM_BATCH_DONE:
            continue
        if (ra["fwd_steps"], ra["adj_steps"], ra["J"]) != (rb["fwd_steps"], rb["adj_steps"],
                                                           rb["J"]):
            return False
        if not np.array_equal(ra["dJ"], rb["dJ"]):
            return False
    return True
