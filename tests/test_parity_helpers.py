"""Host logic of the pointwise parity report (no GPU)."""
import numpy as np

import workloads as W
from _parity import check_pointwise, node_classes, pointwise


def test_node_classes_heat_sink():
    w = W.heat_sink(12, 7, 6, Re=20.0, sigma=1.0, seed=1)
    c = node_classes(w)
    k = (w.mask & 7).reshape(-1)
    assert c["inlet"].sum() == (k == W.INLET).sum() == 5 * 4
    assert c["outlet"].sum() == (k == W.OUTLET).sum()
    # the layer above the heated floor, and nothing else
    layer = np.zeros((w.nz, w.ny, w.nx), bool)
    layer[1, 1:-1, 1:-1] = True
    assert np.array_equal(c["layer"], layer.reshape(-1))
    # the ports span the x faces, so only the y and z walls (and the heated
    # floor) have neighbours: a non-wall node is wall-adjacent unless it is
    # at least 2 layers from them along y and z
    live = k < W.WALL
    inner = np.zeros((w.nz, w.ny, w.nx), bool)
    inner[2:-2, 2:-2, :] = True
    assert np.array_equal(c["wall_adj"], live & ~inner.reshape(-1))
    assert "mirror_adj" not in c


def test_node_classes_mirror_and_periodic():
    w = W.paper_heat_sink(10, 6, 6, buffer=1, sigma=1.0)
    c = node_classes(w)
    m = c["mirror_adj"].reshape(w.nz, w.ny, w.nx)
    k = w.mask & 7
    assert m[:, w.ny - 2, :][k[:, w.ny - 2, :] < W.WALL].all()
    # the layers before both mirror planes (y and z), nothing else
    expect = np.zeros_like(m)
    expect[:, w.ny - 2, :] = True
    expect[w.nz - 2, :, :] = True
    assert np.array_equal(m, expect & (k < W.WALL))
    # a periodic axis has no faces: nothing is wall-adjacent across it
    p = W.periodic_box(6, 3, 0.5)
    assert "wall_adj" not in node_classes(p)


def test_pointwise_catches_a_local_error():
    w = W.heat_sink(12, 7, 6, Re=20.0, sigma=1.0, seed=1)
    k = (w.mask & 7).reshape(-1)
    live, design = k < W.WALL, k == W.DESIGN
    rng = np.random.default_rng(0)
    T = rng.random(w.N)
    dJ = np.where(design, rng.standard_normal(w.N), 0.0)
    want = {"T": T, "dJ": dJ}
    got = {"T": T * (1 + 1e-7), "dJ": dJ * (1 + 1e-7)}
    pw = pointwise(w, got, want, live, design)
    check_pointwise(pw, 1e-5, 1e-5, 1e-5)
    # one outlet node off by 1e-3 of the scale: invisible in a norm-wise
    # 1e-5 ratio over many nodes, caught pointwise and attributed to its class
    bad = dict(got)
    bad["T"] = got["T"].copy()
    n = int(np.flatnonzero(k == W.OUTLET)[3])
    bad["T"][n] += 1e-3 * T[live].max()
    pw = pointwise(w, bad, want, live, design)
    assert pw["T"]["outlet"] > 5e-4 and pw["T"]["interior" if "interior" in pw["T"] else "design"] < 1e-6
    try:
        check_pointwise(pw, 1e-5, 1e-5)
    except AssertionError:
        pass
    else:
        raise AssertionError("pointwise check missed a local error")
