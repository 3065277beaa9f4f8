"""Pins of the oracle on the degenerate designs of the method (no GPU).

* The empty chamber (gamma = 1 on every design node), the initial geometry of
  the paper's optimisations (Secs. 3.2, 3.3), in the heat-generation
  formulation (Eqs. 68-72): no solid means no heat source, so T stays at the
  inlet value 0 exactly, J = 0, the thermal adjoint source dJ/dg = beta
  vanishes, both adjoint fields stay zero, and dJ/dgamma reduces to the
  explicit term beta_max (1 - T) = beta_max on every design node.
* A binary design (gamma in {0, 1}, the paper's own alpha of Eq. 11): the
  converged discrete adjoint still gives the exact gradient at both ends of
  the interpolation (complex step at solid and at fluid cells), so neither
  alpha_B nor the conductivity interpolation is clipped there.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_adjoint import _complex_step_cell, _converged


def _design(w):
    return (w.mask.reshape(-1) & 7) == W.DESIGN


@pytest.mark.parametrize("make", [W.tiny_paper_heat_sink, W.tiny_paper_heat_sink_2d],
                         ids=["3d_quarter", "2d_half"])
def test_empty_chamber_heatgen_closed_form(make):
    w = make()
    w = w.replace(gamma=np.ones_like(w.gamma))
    o = oracle.Oracle(w)
    d = _design(w)
    for steps, tol in ((300, 0.0), (20000, 1e-12)):
        ref = o.solve(fwd_steps=steps, adj_steps=steps, tol=tol, check_every=100)
        if tol > 0.0:
            assert ref["fwd_status"] == 0 and ref["adj_status"] == 0
        assert np.all(ref["T"] == 0.0)
        assert ref["J"] == 0.0
        assert np.all(ref["gsC"] == 0.0) and np.all(ref["fsC"] == 0.0)
        assert np.all(ref["dJ"][d] == w.beta_max), np.unique(ref["dJ"][d])
        assert np.all(ref["dJ"][~d] == 0.0)
        # the flow is not trivial: the pressure inlet drives it
        assert np.abs(ref["u"]).max() > 1e-4


def test_binary_design_gradient_matches_complex_step():
    w = W.tiny_heat_sink()
    w = w.replace(gamma=(w.gamma >= 0.5).astype(w.gamma.dtype))
    o = oracle.Oracle(w)
    fw, ad, dJ = _converged(o)
    d = np.nonzero(_design(w))[0]
    g = w.gamma.reshape(-1)
    solid, fluid = d[g[d] == 0.0], d[g[d] == 1.0]
    assert len(solid) >= 2 and len(fluid) >= 2
    rng = np.random.default_rng(17)
    cells = list(rng.choice(solid, 2, replace=False)) + list(rng.choice(fluid, 2, replace=False))
    steps = max(int(2.5 * fw["steps"]), 3000)
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        ref = list(ex.map(lambda k: _complex_step_cell(o, fw, k, steps), cells))
    scale = np.abs(dJ[d]).max()
    for k, r in zip(cells, ref):
        assert abs(dJ[k] - r) <= 1e-8 * scale, (k, g[k], dJ[k], r)
