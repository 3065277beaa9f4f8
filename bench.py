"""Benchmark of the steady forward + adjoint + sensitivity hot path on one GPU.

One step = one full sensitivity solve of the coupled heat-sink workload
(D3Q19 flow + D3Q7 heat on 160 x 80 x 40, Re 200): forward sweep to the
residual criterion (1e-7, checks every 1000 steps, at most 20000 steps),
adjoint sweep the same way, then dJ/dgamma.  Inputs are resident in HBM before
the timed region.  value = node updates of both sweeps per second (MLUPS, one
update = both lattices at one node).

The roofline entry is for the step kernel that takes most of the time: its
algorithmic bytes per node-update times the node count, over its average
launch duration.  That duration is measured during the timed region with a
pair of HIP events on the solve's stream around every forward and adjoint
sweep: the step kernels of a sweep run back to back (rocprofv3 shows no gap
between them), so sweep time over launches is the average launch duration.
The CPU baseline times the FP64 oracle on the host cores on a bounded sample
of the same workload.

The serving object replays the first --serving-requests requests of the
serving stream (heat-sink solves on 64x32x16, 128x64x32 or 192x96x48 grids,
Re in [50, 400], tau in [0.52, 0.8], seeded designs, Poisson arrivals) through
the continuous-batching engine under a 200 GB HBM budget, then as plain
back-to-back solves, and reports p50/p99 latency and aggregate MLUPS of both.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+adj MLUPS & % HBM peak (D3Q19+D3Q7 FP32); p50/p99 sensitivity latency"
HBM_PEAK_GBS = 8000.0
MALL_BYTES = 256 * 1024 * 1024      # Infinity Cache of the device
STATUS = {0: "converged", 1: "step cap reached"}

def bytes_per_node(kernel, w):
    """Algorithmic bytes per node-update of a step kernel for workload w:
    every population read once and written once (4 B each), plus the
    per-node inputs each kernel reads once (forward: gamma, flags and, with
    the thermal lattice, the reference temperature its populations are
    stored against; adjoint: u, T, gamma, flags, and the dissipation source
    G)."""
    q = 9 if w.nz == 1 else 19          # D2Q9 on a 2D lattice, else D3Q19
    dim = 2 if w.nz == 1 else 3
    qt = (5 if w.nz == 1 else 7) if w.thermal else 0   # D2Q5 / D3Q7
    if kernel == "forward":
        return (q + qt) * 4 * 2 + 4 + 1 + (4 if w.thermal else 0)
    b = (q + qt) * 4 * 2 + dim * 4 + (4 if w.thermal else 0) + 4 + 1
    if w.objective == 1:                # dissipation: source G (3 floats)
        b += 12
    return b


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heat_sink_Re200",
                    choices=["heat_sink_Re50", "heat_sink_Re200", "heat_sink_Re400",
                             "heat_sink_320x160x80_Re200", "pipe_bend_96", "pipe_bend_96_dp",
                             "paper_heat_sink_Re60", "paper_heat_sink_Re120",
                             "paper_heat_sink_Re240", "pipe_bend_2d_512", "pipe_bend_2d_2048",
                             "paper_heat_sink_2d_Re60", "paper_heat_sink_2d_Re240",
                             "paper_heat_sink_2d_2048x513_Re60"])
    ap.add_argument("--re", type=float, default=0.0,
                    help="Reynolds number of a pipe-bend workload (0: the workload's own)")
    ap.add_argument("--adjoint", default="discrete", choices=["discrete", "continuous"],
                    help="adjoint kind (the continuous variant is for the flow-only pipe bend)")
    ap.add_argument("--u-peak", type=float, default=0.0,
                    help="peak inlet speed of the 160x80x40 heat sink (0: 0.1); tau follows "
                         "from Re at that speed")
    ap.add_argument("--max-steps", type=int, default=0,
                    help="step cap of each forward and adjoint sweep (0: the workload's own, "
                         "20000 for the heat sinks)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-fwd-steps", type=int, default=0,
                    help="oracle sample size in forward (and as many adjoint) steps (0: 300)")
    ap.add_argument("--out-of-cache-steps", type=int, default=1000,
                    help="fixed forward and adjoint steps of the out-of-cache heat sink "
                         "320x160x80 timed for its roofline object (0: skip)")
    ap.add_argument("--profile", action="store_true",
                    help="profiling run for rocprofv3: a plain device copy of known size, then "
                         "one forward + adjoint + sensitivity solve of --fixed-steps steps each")
    ap.add_argument("--fixed-steps", type=int, default=200)
    ap.add_argument("--copy-bw", action="store_true",
                    help="measure device-to-device copy bandwidth (1 GiB, out of cache) and exit")
    ap.add_argument("--no-stream-probe", action="store_true",
                    help="skip timing the forward step's traffic without its arithmetic")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="do not bracket the sweeps with HIP events")
    ap.add_argument("--serving-requests", type=int, default=128,
                    help="requests of the serving stream replayed batched and back to back "
                         "(0: skip the serving leg; the full stream is 256, about 3 minutes "
                         "per mode, so the default replays its first 128)")
    ap.add_argument("--serving-rate", type=float, default=0.0,
                    help="Poisson arrival rate in requests/s (0: the stream's default)")
    ap.add_argument("--serving-policy", default="overlap",
                    choices=["overlap", "overlap_fifo", "srw", "all"],
                    help="batch scheduling: two concurrent lanes, small requests beside the "
                         "oldest one (overlap); the same lanes, small requests only beside "
                         "larger ones that arrived after them (overlap_fifo); shortest "
                         "remaining work first (srw); every resident request every quantum (all)")
    ap.add_argument("--serving-fill", type=int, default=512,
                    help="tiles of 256 nodes per launch that the latency lane (overlap, "
                         "overlap_fifo) or the srw policy fills up to")
    ap.add_argument("--stability", action="store_true",
                    help="run the adjoint stability sweep (3D pipe bend, discrete vs continuous "
                         "adjoint) and print its JSON object")
    ap.add_argument("--stability-dim", type=int, default=3, choices=[2, 3],
                    help="pipe bend of the stability sweep: 3D on 32^3 or 2D (D2Q9) on 64^2")
    ap.add_argument("--stability-steps", type=int, default=1000000,
                    help="step cap of each forward and adjoint solve in the stability sweep")
    ap.add_argument("--accuracy", action="store_true",
                    help="sensitivity accuracy against finite differences: discrete and "
                         "continuous adjoint on the 2D pipe bend 64^2 over --accuracy-re, "
                         "printed as one JSON object")
    ap.add_argument("--accuracy-re", default="1,5,10,20,40",
                    help="comma-separated Reynolds numbers of the accuracy study")
    ap.add_argument("--accuracy-cells", type=int, default=8,
                    help="design cells checked by central differences per Reynolds number")
    ap.add_argument("--accuracy-dim", type=int, default=2, choices=[2, 3],
                    help="pipe bend of the accuracy study: 2D on 64^2 or 3D on 32^3")
    ap.add_argument("--optimize", type=int, default=0,
                    help="run this many level-set optimisation iterations on --workload "
                         "(Sec. 2.2) and print their JSON object")
    ap.add_argument("--opt-k", type=float, default=0.1, help="level-set step size K (Eq. 14)")
    ap.add_argument("--opt-sigma", type=float, default=5e-3,
                    help="level-set regularisation coefficient sigma (Eq. 14)")
    ap.add_argument("--opt-sigma-z", type=float, default=0.0,
                    help="sigma along z if > 0 (anisotropic regularisation, Sec. 3.3.4)")
    ap.add_argument("--opt-max-steps", type=int, default=0,
                    help="step cap of each solve in the optimisation (0: the workload's)")
    ap.add_argument("--opt-vmax", type=float, default=0.5,
                    help="upper limit of the design domain's fluid fraction (Eq. 10)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving leg and print its JSON object")
    return ap.parse_args()


def profile_run(args):
    """Short fixed workload for kernel traces and HBM counters: two copies of a
    256 MiB buffer (torch's copy kernel, whose FETCH_SIZE / WRITE_SIZE per
    dispatch calibrate the counters), then one solve of exactly
    --fixed-steps forward and adjoint steps and as many launches of the
    streaming probe."""
    import torch
    from paper_2501_02161_amd import lbm
    torch.cuda.set_device(0)
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    # and the library's own 16-byte copy kernel (3 untimed + 2 timed launches)
    lbm.lbm_copy_probe(src, dst, 2)
    torch.cuda.synchronize()
    w = make_workload(args.workload, args.adjoint, args.re).replace(max_steps=args.fixed_steps, tol=0.0,
                                             check_every=1000)
    prob = lbm.Problem(w, device="cuda:0")
    res = prob.solve(w.gamma)
    torch.cuda.synchronize()
    # then the same number of launches of the streaming probe (after its 10 untimed ones)
    us = prob.stream_probe(prob.gamma_tensor(w.gamma), args.fixed_steps)
    torch.cuda.synchronize()
    print(json.dumps({"profile": w.name, "nodes": w.N, "copy_bytes": src.numel() * 4,
                      "fwd_steps": res["forward"]["steps"], "adj_steps": res["adjoint"]["steps"],
                      "J": res["J"], "stream_probe_us": us}), flush=True)


def copy_bandwidth(quiet=False):
    """Best read+write bandwidth of a device copy of 1 GiB (out of the 256 MB
    Infinity Cache): torch's copy kernel and the library's own 16-byte
    streaming copy (lbm_copy_probe), the measured HBM ceiling of a plain
    stream beside the vendor peak."""
    import torch
    from paper_2501_02161_amd import lbm
    torch.cuda.set_device(0)
    n = 256 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    best = 0.0
    for _ in range(3):
        b.copy_(a)
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = max(best, 2 * n * 4 / (e0.elapsed_time(e1) / 1e3) / 1e9)
    us = min(lbm.lbm_copy_probe(a, b, 10) for _ in range(3))
    own = 2 * n * 4 / (us * 1e-6) / 1e9
    out = {"copy_GBps_read_plus_write": round(best, 1), "bytes": 2 * n * 4,
           "dwordx4_copy_GBps": round(own, 1),
           "best_GBps": round(max(best, own), 1)}
    del a, b
    torch.cuda.empty_cache()
    if not quiet:
        print(json.dumps(out), flush=True)
    return out


KERNEL_SRC = os.path.join(ROOT, "paper_2501_02161_amd", "csrc", "lbm_kernels.hip")


def counters_path(workload):
    return os.path.join(ROOT, "profiles", f"hbm_counters_{workload}.json")


def counter_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of `workload` (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel
    calibration), or None if there is none for this workload or the kernels
    changed since."""
    import hashlib
    try:
        with open(counters_path(workload)) as fh:
            c = json.load(fh)
        with open(KERNEL_SRC, "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    if c.get("workload") != workload or c.get("kernel_source_sha256") != sha:
        return None
    k = c["kernels"].get(kernel)
    if not k:
        return None
    return int((k["fetch_kib"] * c["fetch_scale"] + k["write_kib"] * c["write_scale"]) * 1024)


def make_workload(name, adjoint="discrete", Re=0.0, u_peak=0.0):
    import workloads as W
    kind = 1 if adjoint == "continuous" else 0
    if name.startswith("pipe_bend_96"):
        obj = W.OBJ_PRESSURE_DROP if name.endswith("_dp") else W.OBJ_DISSIPATION
        w = W.pipe_bend_3d(objective=obj, **({"Re": Re} if Re > 0 else {}))
        return w.replace(adjoint_kind=kind, name=w.name + ("_dp" if name.endswith("_dp") else "")
                         + (f"_Re{Re:g}" if Re > 0 else "") + ("_continuous" if kind else ""))
    if name.startswith("paper_heat_sink_2d"):
        Re = float(name.split("Re")[1])
        if "2048x513" in name:
            return W.paper_heat_sink_2d(2048, 513, Re=Re)
        return W.paper_heat_sink_2d(Re=Re)
    if name.startswith("pipe_bend_2d_"):
        n = int(name.split("_")[3])
        w = W.pipe_bend_2d(n=n, inlet=(n // 8, (23 * n) // 64), outlet=((5 * n) // 8, (55 * n) // 64))
        return w.replace(adjoint_kind=kind, name=w.name + ("_continuous" if kind else ""))
    if name.startswith("paper_heat_sink"):
        return W.paper_heat_sink(Re=float(name.split("Re")[1]))
    if name == "heat_sink_320x160x80_Re200":
        return out_of_cache_workload()
    Re = float(name.split("Re")[1])
    if u_peak > 0:
        return W.heat_sink(Re=Re, u_peak=u_peak,
                           name=f"heat_sink_160x80x40_Re{Re:g}_u{u_peak:g}")
    return W.heat_sink(Re=Re)


def out_of_cache_workload():
    """The heat sink at twice the benchmark grid in every axis (4.1 M nodes,
    0.87 GB of populations per forward step): its working set does not fit
    the 256 MB Infinity Cache, so its step kernels stream from HBM."""
    import workloads as W
    return W.heat_sink(320, 160, 80, Re=200.0, name="heat_sink_320x160x80_Re200")


def working_set_bytes(kernel, w):
    """Bytes a step kernel touches per launch: both population buffers and
    the per-node inputs."""
    return bytes_per_node(kernel, w) * w.N


def out_of_cache_leg(fixed_steps, copy_best_gbps):
    """Step kernels of the out-of-cache heat sink at a fixed number of forward
    and adjoint steps (their average launch duration from the sweep events),
    against the vendor HBM peak and the measured device copy."""
    import torch
    from paper_2501_02161_amd import lbm
    w = out_of_cache_workload().replace(max_steps=fixed_steps, tol=0.0, check_every=1000)
    prob = lbm.Problem(w, device="cuda:0")
    gamma = prob.gamma_tensor(w.gamma)
    warm = lbm.Problem(w.replace(max_steps=200), device="cuda:0")
    warm.solve(gamma)
    warm.close()
    del warm
    torch.cuda.synchronize()
    lbm.lbm_set_kernel_timing(prob.h, True)
    lbm.lbm_kernel_timing(prob.h, reset=True)
    res = prob.solve(gamma)
    torch.cuda.synchronize()
    (ms_f, ms_a), (n_f, n_a) = lbm.lbm_kernel_timing(prob.h, reset=True)
    prob.close()
    out = {"workload": w.name, "nodes": w.N, "fwd_steps": res["forward"]["steps"],
           "adj_steps": res["adjoint"]["steps"], "bound": "hbm", "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "device_copy_GBps": copy_best_gbps, "kernels": {}}
    for k, ms, n in (("forward", ms_f, n_f), ("adjoint", ms_a, n_a)):
        bpl = bytes_per_node(k, w) * w.N
        ach = bpl / (ms / 1e3 / n) / 1e9
        out["kernels"][k] = {"avg_us": round(ms * 1e3 / n, 3), "launches": n,
                             "algorithmic_bytes_per_launch": bpl, "achieved": round(ach, 1),
                             "frac": round(ach / HBM_PEAK_GBS, 4),
                             "frac_of_device_copy": round(ach / copy_best_gbps, 4)
                             if copy_best_gbps else None,
                             "traffic": counter_traffic(w.name, k)}
    dom = max(out["kernels"], key=lambda k: out["kernels"][k]["avg_us"] * out["kernels"][k]["launches"])
    out.update({"kernel": dom, "achieved": out["kernels"][dom]["achieved"],
                "frac": out["kernels"][dom]["frac"], "traffic": out["kernels"][dom]["traffic"]})
    return out


def _oracle_rate(o, w, fwd_steps, adj_steps):
    """Seconds per forward and per adjoint step of the oracle, from rest."""
    t0 = time.perf_counter()
    fw = o.forward(max_steps=fwd_steps, tol=0.0, check_every=0)
    t1 = time.perf_counter()
    if getattr(w, "adjoint_kind", 0) == 1:
        o.cont_adjoint(fw["f"], max_steps=adj_steps, tol=0.0, check_every=0)
    else:
        o.adjoint(fw["f"], fw["g"], max_steps=adj_steps, tol=0.0, check_every=0)
    t2 = time.perf_counter()
    return (t1 - t0) / fwd_steps, (t2 - t1) / adj_steps


def cpu_baseline(w, fwd_steps):
    """The oracle (as it is) on the host cores: a bounded sample of equal
    numbers of forward and adjoint steps of the same workload from rest;
    beside it a shorter sample on one core."""
    import oracle
    o = oracle.Oracle(w)
    adj_steps = fwd_steps
    tf, ta = _oracle_rate(o, w, fwd_steps, adj_steps)
    # the GPU solve takes about as many adjoint as forward steps
    mlups = 2 * w.N / (tf + ta) / 1e6
    cores = oracle.threads_used()
    out = {"value": round(mlups, 4), "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"{fwd_steps} forward + {adj_steps} adjoint steps of {w.name} from rest "
                     f"(FP64, {tf * 1e3:.0f} ms/forward step, {ta * 1e3:.0f} ms/adjoint step; "
                     f"rate for equal forward and adjoint step counts)"}
    if cores > 1:
        f1, a1 = max(1, fwd_steps // 30), max(1, adj_steps // 30)
        oracle.set_threads(1)
        try:
            tf1, ta1 = _oracle_rate(o, w, f1, a1)
        finally:
            oracle.set_threads(cores)
        out["one_core"] = {"value": round(2 * w.N / (tf1 + ta1) / 1e6, 4), "unit": "MLUPS",
                           "sample": f"{f1} forward + {a1} adjoint steps on 1 thread "
                                     f"({tf1 * 1e3:.0f} ms/forward step, "
                                     f"{ta1 * 1e3:.0f} ms/adjoint step)"}
    return out


def serving_leg(n, rate, policy="overlap", fill=512):
    """Replay the first n requests of the serving stream (seeded Poisson
    arrivals) once through the continuous-batching engine and once as plain
    back-to-back solves; report latency percentiles and aggregate MLUPS of
    both and whether every request got the same result both ways."""
    import torch
    import workloads as W
    from paper_2501_02161_amd import lbm, serving

    def log(msg):
        print(f"[serving] {msg}", file=sys.stderr, flush=True)

    rate = rate or W.SERVING_RATE
    reqs = [W.serving_request(i) for i in range(n)]
    arrivals = W.poisson_arrivals(n, rate)
    warm = W.heat_sink(24, 14, 10, Re=20.0, tau=0.6, sigma=1.5,
                       name="warmup").replace(max_steps=500, check_every=250, tol=0.0)
    pol = {"srw": lbm.LBM_BATCH_POLICY_SRW, "all": lbm.LBM_BATCH_POLICY_ALL,
           "overlap": lbm.LBM_BATCH_POLICY_OVERLAP,
           "overlap_fifo": lbm.LBM_BATCH_POLICY_OVERLAP_FIFO}[policy]
    eng = serving.BatchEngine(True, W.OBJ_HEATSINK, budget_bytes=W.SERVING_BUDGET_BYTES,
                              quantum=250, policy=pol, fill_tiles=fill)
    serving.serve(eng, [warm], [0.0])
    log(f"batched replay of {n} requests at {rate} /s")
    res_b, mk_b = serving.serve(eng, reqs, arrivals, log=log)
    st = eng.stats()
    eng.close()
    del eng
    torch.cuda.empty_cache()
    serving.serve_back_to_back([warm], [0.0])
    log(f"back-to-back replay of {n} requests")
    res_s, mk_s = serving.serve_back_to_back(reqs, arrivals, log=log)
    sizes = {}
    for w in reqs:
        key = f"{w.nx}x{w.ny}x{w.nz}"
        sizes[key] = sizes.get(key, 0) + 1
    return {"requests": n, "arrivals": f"Poisson {rate} /s, seeded", "grids": sizes,
            "budget_GB": W.SERVING_BUDGET_BYTES / 1e9, "quantum_steps": 250,
            "policy": policy if policy == "all" else f"{policy}, fill {fill} tiles",
            "tol": reqs[0].tol, "max_steps": reqs[0].max_steps,
            "batched": serving.summarize(res_b, mk_b),
            "back_to_back": serving.summarize(res_s, mk_s),
            "identical_results": serving.same_results(res_b, res_s),
            "batch_launches": st["launches"]}


def stability_leg(steps, dim=3):
    """Largest stable inlet speed per relaxation time for the primal, discrete
    adjoint and continuous adjoint solves (Sec. 3.1) on the pipe bend (3D on
    32^3 or 2D on 64^2), every point a request of the batch engine."""
    import torch
    from paper_2501_02161_amd import stability

    torch.cuda.set_device(0)
    taus = (0.52, 0.55, 0.6, 0.7, 0.8, 1.0)
    speeds = (0.02, 0.04, 0.06, 0.08, 0.1, 0.12, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4, 0.5)
    n = 32 if dim == 3 else 64
    t0 = time.perf_counter()
    points, limits = stability.sweep(
        taus, speeds, n=n, max_steps=steps, dim=dim,
        log=lambda m: print(f"[stability] {m}", file=sys.stderr, flush=True))
    el = time.perf_counter() - t0
    table = {f"{tau:g}": {k: v for k, v in lim.items()} for tau, lim in limits.items()}
    pts = {f"tau {t:g} u {u:g} {'cont' if k else 'disc'}": list(v) for (t, u, k), v in points.items()}
    wl = "pipe_bend_3d_32^3 (port 5, pressure drop)" if dim == 3 else \
        "pipe_bend_2d_64x64 (D2Q9, inlet rows 8-23, outlet columns 40-55, pressure drop)"
    return {"workload": wl, "steps_cap": steps,
            "taus": list(taus), "speeds": list(speeds), "max_stable_speed": table,
            "seconds": round(el, 1), "points": pts}


def accuracy_case(dim, Re):
    """The pipe bend of the accuracy study: 2D on 64^2 (the small
    configuration) or 3D on 32^3 (port 5, pressure drop, tau 0.6)."""
    import workloads as W
    if dim == 2:
        return W.pipe_bend_2d(Re=Re).replace(max_steps=400000, tol=1e-9, check_every=1000)
    w = W.pipe_bend_3d(n=32, tau=0.6, Re=Re, sigma=32 / 24.0, port=5,
                       objective=W.OBJ_PRESSURE_DROP)
    return w.replace(max_steps=400000, tol=1e-9, check_every=1000)


def accuracy_leg(res, ncells, h=1e-2, settle=10000, dim=2):
    """Sensitivity accuracy of the discrete and the continuous adjoint
    (Sec. 3.1; Figs. 7 and 13 compare them with finite differences): on the
    pipe bend (2D 64^2 or 3D 32^3) at each Reynolds number, both adjoint
    dJ/dgamma fields against central differences of converged GPU forward
    solves at the design cells of largest discrete |dJ/dgamma| and at seeded
    random ones (central differences with steps h and h/2, combined by
    Richardson extrapolation), plus the continuous field's scale and
    direction against the discrete one."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2501_02161_amd import lbm

    torch.cuda.set_device(0)
    rows = []
    t0 = time.perf_counter()
    for Re in res:
        w = accuracy_case(dim, Re)
        design = np.flatnonzero((w.mask.reshape(-1) & 7) == W.DESIGN)
        pd = lbm.Problem(w, device="cuda:0")
        rd = pd.solve(w.gamma)
        dJd = pd.dJ.reshape(-1).cpu().numpy().astype(np.float64)
        row = {"Re": Re, "u_peak": Re * (w.tau - 0.5) / 3.0 / w.L_ref, "J": rd["J"],
               "fwd_steps": rd["forward"]["steps"], "fwd_status": rd["forward"]["status"],
               "disc_adj_steps": rd["adjoint"]["steps"], "disc_status": rd["adjoint"]["status"]}
        order = design[np.argsort(-np.abs(dJd[design]))]
        rng = np.random.default_rng(W.SEED_BASE + 9)
        rest = order[ncells // 2:]
        cells = list(order[:ncells // 2]) + list(rng.choice(rest, ncells - ncells // 2,
                                                            replace=False))
        # central differences from warm-started forward solves
        pf = lbm.Problem(w, device="cuda:0")
        pf.forward(w.gamma)
        def central(k, step):
            Jpm = []
            for sgn in (1.0, -1.0):
                g = w.gamma.reshape(-1).copy()
                g[k] += sgn * step
                pf.forward_resume(g)
                # settle the slow modes beyond the residual criterion
                Jpm.append(pf.forward_continue(settle)["J"])
            return (Jpm[0] - Jpm[1]) / (2.0 * step)

        fd_h = np.array([central(k, h) for k in cells])
        fd_h2 = np.array([central(k, h / 2) for k in cells])
        # Richardson extrapolation removes the h^2 term of the central difference
        fd = (4.0 * fd_h2 - fd_h) / 3.0
        scale = np.abs(fd).max()
        row["cells"] = [int(k) for k in cells]
        row["fd"] = fd.tolist()
        row["disc"] = dJd[cells].tolist()
        row["disc_vs_fd"] = float(np.abs(dJd[cells] - fd).max() / scale)
        row["disc_vs_fd_h"] = float(np.abs(dJd[cells] - fd_h).max() / scale)
        try:
            pc = lbm.Problem(w, device="cuda:0", adjoint_kind=1)
            rc = pc.solve(w.gamma)
            dJc = pc.dJ.reshape(-1).cpu().numpy().astype(np.float64)
            a, b = dJc[design], dJd[design]
            row.update({"cont_adj_steps": rc["adjoint"]["steps"],
                        "cont_status": rc["adjoint"]["status"], "cont": dJc[cells].tolist(),
                        "cont_vs_fd": float(np.abs(dJc[cells] - fd).max() / scale),
                        "cont_rescaled_vs_fd": float(np.abs(dJc[cells] * (dJc[cells] @ fd)
                                                            / (dJc[cells] @ dJc[cells]) - fd).max()
                                                     / scale),
                        "cont_scale": float(np.linalg.norm(a) / np.linalg.norm(b)),
                        "cont_one_minus_cos": float(1.0 - a @ b / np.linalg.norm(a)
                                                    / np.linalg.norm(b))})
            pc.close()
        except lbm.LBMError as e:
            row.update({"cont_status": "diverged", "cont_error": str(e)})
        pd.close()
        pf.close()
        print(f"[accuracy] {json.dumps({k: v for k, v in row.items() if k not in ('fd', 'disc', 'cont', 'cells')})}",
              file=sys.stderr, flush=True)
        rows.append(row)
    wl = ("pipe_bend_2d_64x64 (D2Q9, tau 0.6, inlet rows 8-23, outlet columns 40-55, "
          "pressure drop)") if dim == 2 else \
        "pipe_bend_3d_32^3 (D3Q19, tau 0.6, port 5, pressure drop)"
    return {"workload": wl, "h": h, "tol": 1e-9, "settle_steps": settle,
            "seconds": round(time.perf_counter() - t0, 1), "rows": rows}


def optimize_leg(args):
    """Level-set topology optimisation (Sec. 2.2) on --workload from the
    empty chamber: per iteration a warm-started forward solve, adjoint solve,
    sensitivity and level-set update, all on the GPU."""
    import torch
    from paper_2501_02161_amd import optimize

    torch.cuda.set_device(0)
    w = make_workload(args.workload, args.adjoint, args.re)
    if args.opt_max_steps > 0:
        w = w.replace(max_steps=args.opt_max_steps)
    sigma = (args.opt_sigma, args.opt_sigma, args.opt_sigma_z or args.opt_sigma)
    opt = optimize.LevelSetOptimizer(w, K=args.opt_k, sigma=sigma, vmax=args.opt_vmax)
    t0 = time.perf_counter()
    hist = opt.run(args.optimize, log=lambda r: print(f"[optimize] {json.dumps(r)}",
                                                      file=sys.stderr, flush=True))
    el = time.perf_counter() - t0
    return {"workload": w.name, "lattice": [w.nx, w.ny, w.nz], "K": args.opt_k,
            "sigma": list(opt.sigma), "sigma_lattice": list(opt.sigma_lattice), "vmax": args.opt_vmax,
            "max_steps": w.max_steps, "tol": w.tol, "iterations": len(hist),
            "seconds": round(el, 3), "seconds_per_iteration": round(el / max(1, len(hist)), 4),
            "node_updates_per_s": opt.updates / el,
            "J": [h["J"] for h in hist], "volume": [h["volume"] for h in hist],
            "fwd_steps": [h["fwd_steps"] for h in hist], "adj_steps": [h["adj_steps"] for h in hist]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (--gpus {args.gpus} requested); "
              "it has no multi-GPU slab decomposition.",
              file=sys.stderr)
        sys.exit(2)
    if args.profile:
        profile_run(args)
        return
    if args.copy_bw:
        copy_bandwidth()
        return
    if args.stability:
        print(json.dumps({"stability": stability_leg(args.stability_steps, args.stability_dim)}),
              flush=True)
        return
    if args.accuracy:
        res = [float(v) for v in args.accuracy_re.split(",") if v]
        print(json.dumps({"accuracy": accuracy_leg(res, args.accuracy_cells,
                                                   dim=args.accuracy_dim)}), flush=True)
        return
    if args.optimize > 0:
        print(json.dumps({"optimize": optimize_leg(args)}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_leg(args.serving_requests or 256,
                                                 args.serving_rate, args.serving_policy,
                                                 args.serving_fill)}), flush=True)
        return
    import numpy as np
    import torch
    from paper_2501_02161_amd import lbm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = make_workload(args.workload, args.adjoint, args.re, args.u_peak)
    if args.max_steps > 0:
        w = w.replace(max_steps=args.max_steps)
    prob = lbm.Problem(w, device="cuda:0")
    gamma = prob.gamma_tensor(w.gamma)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def one():
        fi = prob.forward(gamma, stream)
        ai = prob.adjoint(stream=stream)
        J = prob.sensitivity(stream=stream)
        return fi, ai, J

    try:
        for _ in range(args.warmup):
            one()
        torch.cuda.synchronize()
        lbm.lbm_set_kernel_timing(prob.h, not args.no_kernel_timing)
        lbm.lbm_kernel_timing(prob.h, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [one() for _ in range(args.steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    except lbm.LBMError as e:
        if e.code != lbm.LBM_EDIVERGED:
            raise
        # no steady state to differentiate about: the line says so and
        # carries no rate
        torch.cuda.synchronize()
        prob.close()
        print(json.dumps({
            "metric": METRIC, "value": None, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": w.name, "nodes": w.N, "tau": round(w.tau, 6), "Re": w.Re,
                       "tol": w.tol, "max_steps": w.max_steps, "fwd_status": "diverged",
                       "error": str(e)}}), flush=True)
        return
    (ms_f, ms_a), (n_f, n_a) = lbm.lbm_kernel_timing(prob.h, reset=True)
    lbm.lbm_set_kernel_timing(prob.h, False)
    elapsed = t1 - t0
    updates = sum(w.N * (fi["steps"] + ai["steps"]) for fi, ai, _ in infos)
    mlups = updates / elapsed / 1e6
    fi, ai, J = infos[-1]

    kernels = {"forward": (ms_f, n_f), "adjoint": (ms_a, n_a)}
    dom = max(kernels, key=lambda k: kernels[k][0])
    ms_tot, n_launch = kernels[dom]
    bpn = bytes_per_node(dom, w)
    achieved = bpn * w.N / (ms_tot / 1e3 / n_launch) / 1e9 if n_launch else None
    per_kernel = {}
    for k, (ms, n) in kernels.items():
        b = bytes_per_node(k, w)
        per_kernel[k] = {"avg_us": round(ms * 1e3 / n, 3) if n else None, "launches": n,
                         "bytes_per_node": b,
                         "GBps": round(b * w.N / (ms / 1e3 / n) / 1e9, 1) if n else None}
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "nodes": w.N,
                   "lattice": ("D2Q9+D2Q5" if w.thermal else "D2Q9") if w.nz == 1 else
                              ("D3Q19+D3Q7" if w.thermal else "D3Q19"),
                   "objective": {0: "pressure drop", 1: "viscous dissipation",
                                 2: "mean floor-layer T + 0.1 pressure drop",
                                 3: "heat generated, -sum beta (1 - T)"}[w.objective],
                   "adjoint": "continuous" if w.adjoint_kind else "discrete",
                   "tau": round(w.tau, 6),
                   "tol": w.tol, "max_steps": w.max_steps, "fwd_steps": fi["steps"],
                   "adj_steps": ai["steps"], "J": J,
                   "fwd_status": STATUS.get(fi["status"], fi["status"]),
                   "adj_status": STATUS.get(ai["status"], ai["status"]),
                   "fwd_residual": [float(v) for v in fi["residual"]],
                   "adj_residual": [float(v) for v in ai["residual"]]},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": counter_traffic(w.name, dom),
                     "algorithmic_bytes_per_launch": bpn * w.N,
                     # the populations a sweep keeps touching fit the Infinity
                     # Cache, so the kernel may stream faster than HBM alone
                     "working_set_bytes": working_set_bytes(dom, w),
                     "residency": "infinity_cache" if working_set_bytes(dom, w) < MALL_BYTES
                                  else "hbm"},
        "kernels": per_kernel,
        "hbm_frac_whole_job": round(
            (bytes_per_node("forward", w) * w.N * fi["steps"] +
             bytes_per_node("adjoint", w) * w.N * ai["steps"]) * args.steps /
            elapsed / 1e9 / HBM_PEAK_GBS, 4),
    }
    if not args.no_stream_probe:
        # the forward step's traffic in its own pattern with none of its
        # arithmetic: the ceiling the pull pattern leaves the step kernel
        us = prob.stream_probe(gamma, 2000)
        fwd_us = per_kernel["forward"]["avg_us"]
        out["stream_ceiling"] = {
            "probe": "forward step traffic and pull pattern, no arithmetic (lbm_stream_probe)",
            "avg_us": round(us, 3),
            "GBps": round(bytes_per_node("forward", w) * w.N / (us * 1e-6) / 1e9, 1),
            "forward_frac": round(us / fwd_us, 4) if fwd_us else None}
    prob.close()
    # the best measured device copy beside the vendor peak
    out["copy_bandwidth"] = copy_bandwidth(quiet=True)
    best = out["copy_bandwidth"]["best_GBps"]
    if achieved:
        out["roofline"]["frac_of_device_copy"] = round(achieved / best, 4)
    if args.out_of_cache_steps > 0 and w.name != out_of_cache_workload().name:
        out["roofline_out_of_cache"] = out_of_cache_leg(args.out_of_cache_steps, best)
    if args.serving_requests > 0:
        out["serving"] = serving_leg(args.serving_requests, args.serving_rate,
                                     args.serving_policy, args.serving_fill)
    if not args.no_cpu_baseline:
        steps = args.cpu_fwd_steps or 300
        out["cpu_baseline"] = cpu_baseline(w, steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
