"""Continuous batching: requests of different sizes, Re, tau and design
fields, admitted while others run, give bit for bit the results of the same
requests solved alone; the HBM budget bounds what is resident; a diverging
request fails alone."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2501_02161_amd import lbm, serving

pytestmark = pytest.mark.gpu

Q = 250


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


def small_requests():
    shapes = [(24, 14, 10), (32, 16, 10), (20, 12, 8), (40, 16, 12), (24, 12, 10)]
    out = []
    rng = np.random.default_rng(5)
    for i, (nx, ny, nz) in enumerate(shapes):
        tau = float(rng.uniform(0.55, 0.8))
        L = nz - 2
        Re = 0.08 * L / ((tau - 0.5) / 3.0)
        w = W.heat_sink(nx, ny, nz, Re=Re, tau=tau, sigma=1.5, seed=900 + i,
                        name=f"req{i}").replace(max_steps=3000, check_every=250, tol=1e-6)
        out.append(w)
    return out


def alone(w):
    prob = lbm.Problem(w, device="cuda:0")
    res = prob.solve(w.gamma)
    torch.cuda.synchronize()
    dJ = prob.dJ.reshape(-1).cpu().numpy()
    return res, dJ


def _check_same(w, r, ref, dJ_ref):
    res, _ = ref
    assert r["state"] == lbm.LBM_BATCH_DONE
    assert r["fwd_steps"] == res["forward"]["steps"]
    assert r["adj_steps"] == res["adjoint"]["steps"]
    assert r["J"] == res["J"]
    assert np.array_equal(r["dJ"], dJ_ref)


def _drain(eng, tickets, reqs, limit=1000):
    results = {}
    for _ in range(limit):
        a, q = eng.step()
        for t, i in list(tickets.items()):
            r = eng.collect(t, reqs[i].N)
            if r is not None:
                results[i] = r
                del tickets[t]
        if not tickets:
            break
    return results


@pytest.mark.parametrize("persistent_tiles", [1024, 0], ids=["persistent", "per_step"])
def test_batch_results_equal_single_solves(persistent_tiles):
    """Each quantum as one persistent launch (its blocks step the run set with
    a device-wide barrier between steps) or as one launch per step: either
    way every result is the single solve's, bit for bit."""
    reqs = small_requests()
    refs = [alone(w) for w in reqs]
    eng = serving.BatchEngine(True, W.OBJ_HEATSINK, budget_bytes=2 << 30, max_slots=8, quantum=Q,
                              persistent_tiles=persistent_tiles)
    tickets = {eng.submit(reqs[0]): 0, eng.submit(reqs[1]): 1}
    eng.step()
    eng.step()
    tickets[eng.submit(reqs[2])] = 2       # arrives while two are running
    eng.step()
    tickets[eng.submit(reqs[3])] = 3
    tickets[eng.submit(reqs[4])] = 4
    results = _drain(eng, tickets, reqs)
    assert len(results) == len(reqs)
    for i, w in enumerate(reqs):
        _check_same(w, results[i], refs[i], refs[i][1])
    st = eng.stats()
    assert st["running"] == 0 and st["queued"] == 0 and st["bytes_in_use"] == 0
    print(f"[serving] batched results identical to single solves; stats {st}", flush=True)


@pytest.mark.parametrize("policy,fill", [(lbm.LBM_BATCH_POLICY_ALL, 512),
                                         (lbm.LBM_BATCH_POLICY_SRW, 1),
                                         (lbm.LBM_BATCH_POLICY_SRW, 150),
                                         (lbm.LBM_BATCH_POLICY_OVERLAP, 1),
                                         (lbm.LBM_BATCH_POLICY_OVERLAP, 20),
                                         (lbm.LBM_BATCH_POLICY_OVERLAP_FIFO, 20)])
def test_policy_changes_no_result(policy, fill):
    """Whatever the run set of each quantum (all resident requests; one at a
    time; a few by shortest remaining work; two concurrent lanes, requests
    moving between them), paused requests resume where they stopped and
    every result equals the single solve bit for bit."""
    reqs = small_requests()
    refs = [alone(w) for w in reqs]
    eng = serving.BatchEngine(True, W.OBJ_HEATSINK, budget_bytes=2 << 30, max_slots=8, quantum=Q,
                              policy=policy, fill_tiles=fill)
    tickets = {eng.submit(reqs[0]): 0, eng.submit(reqs[1]): 1, eng.submit(reqs[2]): 2}
    eng.step()
    tickets[eng.submit(reqs[3])] = 3
    eng.step()
    tickets[eng.submit(reqs[4])] = 4
    results = _drain(eng, tickets, reqs)
    assert len(results) == len(reqs)
    for i, w in enumerate(reqs):
        _check_same(w, results[i], refs[i], refs[i][1])
    st = eng.stats()
    assert st["running"] == 0 and st["bytes_in_use"] == 0
    # node updates counted = the work of the requests
    want = sum((results[i]["fwd_steps"] + results[i]["adj_steps"]) * w.N
               for i, w in enumerate(reqs))
    assert st["node_updates"] >= want


def test_budget_bounds_residency():
    reqs = small_requests()[:3]
    refs = [alone(w) for w in reqs]
    # room for about one request at a time
    per = max(lbm.lbm_workspace_bytes(lbm.lbm_problem_create(lbm.make_desc(w), w.mask))
              for w in reqs) + 8 * 4 * max(w.N for w in reqs)
    eng = serving.BatchEngine(True, W.OBJ_HEATSINK, budget_bytes=int(per * 1.3), max_slots=8,
                              quantum=Q)
    tickets = {eng.submit(w): i for i, w in enumerate(reqs)}
    results = {}
    max_running = 0
    for _ in range(1000):
        eng.step()
        st = eng.stats()
        assert st["bytes_in_use"] <= st["arena_bytes"]
        max_running = max(max_running, st["running"])
        for t, i in list(tickets.items()):
            r = eng.collect(t, reqs[i].N)
            if r is not None:
                results[i] = r
                del tickets[t]
        if not tickets:
            break
    assert max_running == 1
    for i, w in enumerate(reqs):
        _check_same(w, results[i], refs[i], refs[i][1])


def test_diverging_request_fails_alone():
    reqs = small_requests()[:2]
    refs = [alone(w) for w in reqs]
    bad = W.heat_sink(24, 14, 10, Re=0.6 * 8 / ((0.501 - 0.5) / 3), tau=0.501, sigma=1.5,
                      seed=77).replace(max_steps=3000, check_every=250, tol=1e-6)
    eng = serving.BatchEngine(True, W.OBJ_HEATSINK, budget_bytes=1 << 30, max_slots=4, quantum=Q)
    tickets = {eng.submit(reqs[0]): 0, eng.submit(bad): 2, eng.submit(reqs[1]): 1}
    allreq = {0: reqs[0], 1: reqs[1], 2: bad}
    results = _drain(eng, tickets, allreq)
    assert results[2]["state"] == lbm.LBM_BATCH_FAILED
    assert results[2]["status"] == lbm.LBM_EDIVERGED
    for i in (0, 1):
        _check_same(reqs[i], results[i], refs[i], refs[i][1])


def test_serving_trace_small():
    """A short Poisson trace of mixed requests: every request completes, its
    result equals the back-to-back plain solve, and latencies are recorded."""
    reqs = small_requests()
    arrivals = W.poisson_arrivals(len(reqs), rate=50.0)
    eng = serving.BatchEngine(True, W.OBJ_HEATSINK, budget_bytes=2 << 30, max_slots=8, quantum=Q)
    res_b, mk_b = serving.serve(eng, reqs, arrivals)
    res_s, mk_s = serving.serve_back_to_back(reqs, arrivals)
    for rb, rs in zip(res_b, res_s):
        assert rb["J"] == rs["J"] and np.array_equal(rb["dJ"], rs["dJ"])
    print(f"[serving] batched {serving.summarize(res_b, mk_b)} back-to-back "
          f"{serving.summarize(res_s, mk_s)}", flush=True)


def test_long_solo_quanta_equal_single_solves():
    """Under OVERLAP a lone request too large for the latency lane runs on the
    bandwidth lane up to its next residual check per host visit (here checks
    every 1000 steps, cap 2750: quanta of 1000, 1000 and 750 steps) while a
    small request moves on the latency lane: both results equal their single
    solves bit for bit."""
    big = W.heat_sink(64, 64, 64, Re=0.08 * 62 / ((0.6 - 0.5) / 3.0), tau=0.6, sigma=2.0,
                      seed=931, name="big").replace(max_steps=2750, check_every=1000, tol=1e-7)
    assert big.N // 256 >= 1024
    small = small_requests()[0].replace(max_steps=2750, check_every=250, tol=1e-6)
    reqs = [big, small]
    refs = [alone(w) for w in reqs]
    eng = serving.BatchEngine(True, W.OBJ_HEATSINK, budget_bytes=4 << 30, max_slots=4, quantum=Q,
                              policy=lbm.LBM_BATCH_POLICY_OVERLAP, fill_tiles=512)
    tickets = {eng.submit(big): 0, eng.submit(small): 1}
    results = _drain(eng, tickets, reqs)
    assert len(results) == 2
    for i, w in enumerate(reqs):
        _check_same(w, results[i], refs[i], refs[i][1])
    st = eng.stats()
    assert st["node_updates"] >= sum((results[i]["fwd_steps"] + results[i]["adj_steps"]) * w.N
                                     for i, w in enumerate(reqs))


def test_serving_requests_match_the_oracle():
    """Requests of the serving stream itself (its 64x32x16 and 128x64x32
    grids, with their drawn Re, tau and design fields), served together by
    the batch engine for one 250-step quantum per sweep, give the FP64
    oracle's J (1e-5) and dJ/dgamma over the design nodes (1e-4) after the
    same steps."""
    import oracle
    from _parity import rel

    picks = {}
    for i in range(64):
        w = W.serving_request(i)
        key = (w.nx, w.ny, w.nz)
        if key in ((64, 32, 16), (128, 64, 32)) and key not in picks:
            picks[key] = w.replace(max_steps=Q, check_every=Q, tol=0.0)
        if len(picks) == 2:
            break
    reqs = [picks[(64, 32, 16)], picks[(128, 64, 32)]]
    eng = serving.BatchEngine(True, W.OBJ_HEATSINK, budget_bytes=4 << 30, max_slots=4, quantum=Q)
    tickets = {eng.submit(w): i for i, w in enumerate(reqs)}
    results = _drain(eng, tickets, reqs)
    assert len(results) == 2
    for i, w in enumerate(reqs):
        r = results[i]
        assert r["state"] == lbm.LBM_BATCH_DONE
        assert (r["fwd_steps"], r["adj_steps"]) == (Q, Q)
        ref = oracle.Oracle(w).solve(fwd_steps=Q, adj_steps=Q, tol=0.0, check_every=Q)
        design = (w.mask.reshape(-1) & 7) == W.DESIGN
        e_dJ = rel(r["dJ"][design], ref["dJ"][design])
        e_J = abs(r["J"] - ref["J"]) / abs(ref["J"])
        print(f"[serving] {w.name} tau {w.tau:.4f} Re {w.Re:.1f}: J {e_J:.2e}  dJ/dgamma {e_dJ:.2e}",
              flush=True)
        assert e_J <= 1e-5
        assert e_dJ < 1e-4
