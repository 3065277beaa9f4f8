"""Host-side bookkeeping of the serving replay (no GPU): the summary's
percentiles, failure counts and MLUPS accounting, and the same-result check."""
import numpy as np

from paper_2501_02161_amd import lbm, serving


def _res(i, lat, state=lbm.LBM_BATCH_DONE, steps=(100, 50), n=10, J=1.0):
    return {"index": i, "latency": lat, "completion": lat, "state": state,
            "fwd_steps": steps[0], "adj_steps": steps[1], "J": J,
            "dJ": np.arange(n, dtype=np.float32) if state == lbm.LBM_BATCH_DONE
            else np.zeros(0, np.float32)}


def test_summary_counts_completed_updates_only():
    rs = [_res(i, 0.1 * (i + 1)) for i in range(9)] + [_res(9, 5.0, lbm.LBM_BATCH_FAILED)]
    s = serving.summarize(rs, makespan=2.0)
    assert s["requests"] == 10 and s["completed"] == 9 and s["failed"] == 1
    assert s["MLUPS"] == round(9 * 150 * 10 / 2.0 / 1e6, 1)
    lat = [0.1 * (i + 1) for i in range(9)] + [5.0]
    assert s["p50_s"] == round(float(np.percentile(lat, 50)), 4)
    assert s["p99_s"] == round(float(np.percentile(lat, 99)), 4)


def test_same_results():
    a = [_res(0, 1.0), _res(1, 1.0, lbm.LBM_BATCH_FAILED)]
    b = [_res(0, 2.0), _res(1, 3.0, lbm.LBM_BATCH_FAILED)]
    assert serving.same_results(a, b)
    c = [_res(0, 1.0, J=1.0 + 2**-40), b[1]]
    assert not serving.same_results(a, c)
    d = [_res(0, 1.0), _res(1, 1.0)]
    assert not serving.same_results(a, d)
    e = [_res(0, 1.0, steps=(100, 51)), b[1]]
    assert not serving.same_results(a, e)
    f = [_res(0, 1.0), b[1]]
    f[0]["dJ"] = f[0]["dJ"].copy()
    f[0]["dJ"][3] = np.nextafter(f[0]["dJ"][3], np.float32(10))
    assert not serving.same_results(a, f)
