"""Host-side checks of bench.py (no GPU): the one-GPU contract, the
workload table and the algorithmic byte counts the roofline uses."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("name,q,thermal", [("heat_sink_Re200", 19, True), ("pipe_bend_96", 19, False),
                                            ("pipe_bend_2d_512", 9, False),
                                            ("paper_heat_sink_Re60", 19, True),
                                            ("paper_heat_sink_2d_Re60", 9, True)])
def test_bytes_per_node(bench, name, q, thermal):
    w = bench.make_workload(name)
    assert bool(w.thermal) == thermal and (w.nz == 1) == (q == 9)
    qt = (5 if q == 9 else 7) if thermal else 0
    dim = 2 if q == 9 else 3
    # every population read and written once, gamma and flags once, and the
    # thermal lattice's reference temperature
    assert bench.bytes_per_node("forward", w) == (q + qt) * 8 + 4 + 1 + (4 if thermal else 0)
    extra = 12 if w.objective == 1 else 0      # dissipation source
    assert bench.bytes_per_node("adjoint", w) == (q + qt) * 8 + 4 * dim + (4 if thermal else 0) + 5 + extra


def test_headline_workload_is_the_heat_sink(bench):
    w = bench.make_workload("heat_sink_Re200")
    assert (w.nx, w.ny, w.nz) == (160, 80, 40) and w.Re == 200.0 and w.thermal


def test_cpu_baseline_fields(bench):
    """The CPU baseline times the oracle as it is, on every host core and on
    one core, and says what the sample was."""
    import oracle
    import workloads as W
    w = W.tiny_heat_sink()
    out = bench.cpu_baseline(w, 12)
    assert out["kind"] == "oracle" and out["unit"] == "MLUPS" and out["value"] > 0
    assert out["cores"] == oracle.threads_used()
    assert "12 forward + 12 adjoint steps" in out["sample"]
    if out["cores"] > 1:
        assert out["one_core"]["value"] > 0 and "on 1 thread" in out["one_core"]["sample"]


def test_out_of_cache_workload_does_not_fit_the_infinity_cache(bench):
    """The added out-of-cache configuration streams from HBM; the headline's
    forward working set fits the 256 MB Infinity Cache, which the line says."""
    big = bench.out_of_cache_workload()
    assert (big.nx, big.ny, big.nz) == (320, 160, 80)
    for k in ("forward", "adjoint"):
        assert bench.working_set_bytes(k, big) > 3 * bench.MALL_BYTES
    head = bench.make_workload("heat_sink_Re200")
    assert bench.working_set_bytes("forward", head) < bench.MALL_BYTES
