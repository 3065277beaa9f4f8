"""GPU parity of the paper's own heat-sink formulation (Sec. 3.3): mirror
planes (quarter domain), pressure inlet, heat generation beta(gamma)(1 - T)
and J = -sum Q, against the FP64 oracle:

* fixed step counts on a small quarter domain (fields 1e-5, dJ/dgamma 1e-4);
* converged forward and adjoint on a 32 x 12 x 10 quarter domain;
* the quarter domain against the unfolded full domain on the GPU itself;
* one forward and one adjoint step on the full 128 x 33 x 25 quarter domain.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from _parity import compare_solution, gpu_fields, kinds, rel, run_gpu, run_oracle
from test_gpu_parity import _step_check
from paper_2501_02161_amd import lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield


def test_heatgen_fixed_steps_parity():
    w = W.tiny_paper_heat_sink(16, 8, 7)
    print(f"[heatgen] fixed steps {w.nx}x{w.ny}x{w.nz}", flush=True)
    prob, res = run_gpu(w, steps=800, tol=0.0, check_every=200)
    o, ref = run_oracle(w, steps=800, tol=0.0, check_every=200)
    err = compare_solution(w, prob, ref)
    print(f"[heatgen] errors {err} J {res['J']:.9g} vs {ref['J']:.9g}", flush=True)
    assert abs(res["J"] - ref["J"]) <= 1e-5 * abs(ref["J"])


def test_heatgen_converged_parity():
    w = W.paper_heat_sink(32, 12, 10, Re=10.0, tau=0.8, Pr=1.0, beta_max=2e-3, alpha_max=0.2,
                          buffer=2, sigma=1.5).replace(max_steps=60000, tol=1e-7, check_every=500)
    print(f"[heatgen] converged {w.nx}x{w.ny}x{w.nz}", flush=True)
    prob, res = run_gpu(w)
    assert res["forward"]["status"] == 0 and res["adjoint"]["status"] == 0
    o = oracle.Oracle(w)
    ref = o.solve(tol=1e-11, check_every=500, fwd_steps=400000, adj_steps=400000)
    assert ref["fwd_status"] == 0 and ref["adj_status"] == 0
    err = compare_solution(w, prob, ref)
    print(f"[heatgen] steps {res['forward']['steps']}/{res['adjoint']['steps']} errors {err}",
          flush=True)


def test_quarter_equals_full_domain_on_gpu():
    w = W.tiny_paper_heat_sink(20, 8, 7).replace(max_steps=1000, tol=0.0, check_every=500)
    wf = W.mirror_full(w)
    pq, rq = run_gpu(w)
    pf, rf = run_gpu(wf)
    dq, uq, Tq, gq = gpu_fields(pq)
    df, uf, Tf, gf = gpu_fields(pf)

    def fold(a, ww):
        a = a.reshape((ww.nz, ww.ny, ww.nx) + a.shape[1:])
        return a[:w.nz - 1, :w.ny - 1]

    errs = {k: rel(fold(a, w), fold(b, wf)) for k, a, b in
            (("p", dq, df), ("u", uq, uf), ("T", Tq, Tf), ("dJ", gq, gf))}
    print(f"[heatgen] quarter vs full {errs}; J {rq['J']:.9g} x 4 vs {rf['J']:.9g}", flush=True)
    assert all(v < 1e-6 for v in errs.values()), errs
    assert abs(4.0 * rq["J"] - rf["J"]) <= 1e-5 * abs(rf["J"])


def test_heatgen_full_size_step_parity():
    w = W.paper_heat_sink()
    print(f"[heatgen] full {w.nx}x{w.ny}x{w.nz} one-step check", flush=True)
    err, J = _step_check(w)
    print(f"[heatgen] full errors {err}", flush=True)
    for key, v in err.items():
        assert v < (1e-4 if key == "sens" else 1e-5), (key, err)
