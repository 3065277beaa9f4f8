"""Pins of the oracle's level-set update (Eqs. 13-15, 67), independent of the
update's own arithmetic: the stencil on fields whose Laplacian is known,
the multiplier on inputs where it has a closed form, and the step on
uniform inputs."""
import numpy as np

from oracle.levelset import laplacian, levelset_update


def _box(n=6):
    d = np.ones((n, n, n), dtype=bool)
    d[0], d[-1], d[:, 0], d[:, -1], d[:, :, 0], d[:, :, -1] = (False,) * 6
    return d


def test_laplacian_of_quadratic_is_exact():
    z, y, x = np.meshgrid(np.arange(7.), np.arange(7.), np.arange(7.), indexing="ij")
    phi = 0.5 * x ** 2 - 0.25 * y ** 2 + 0.125 * z ** 2 + 3 * x * y
    d = np.ones(phi.shape, dtype=bool)
    lap = laplacian(phi, d)
    inner = (slice(1, -1),) * 3
    assert np.allclose(lap[inner], 1.0 - 0.5 + 0.25, atol=1e-12)


def test_laplacian_no_flux_and_constant():
    d = _box()
    phi = np.full(d.shape, 0.3)
    assert np.allclose(laplacian(phi, d), 0.0, atol=1e-15)
    # a non-design neighbour counts as the node itself
    phi2 = np.zeros(d.shape)
    phi2[~d] = 5.0
    assert np.all(laplacian(phi2, d) == 0.0)


def test_lambda_closed_form_and_uniform_step():
    d = _box()
    rng = np.random.default_rng(0)
    phi = rng.uniform(-0.5, 0.5, d.shape)
    dJ = np.where(d, 2.0, 0.0)                       # uniform sensitivity
    K, vmax = 0.05, 0.3
    new, alpha, info = levelset_update(phi, dJ, d, K, 0.0, vmax)
    v = (phi[d] >= 0).mean()
    assert info["volume"] == v and np.isclose(info["G"], v - vmax)
    # sigma = 0, |J'/mean|J'|| = 1 everywhere: lambda = exp(G)
    assert np.isclose(info["lambda"], np.exp(v - vmax), rtol=1e-15)
    assert np.allclose(new[d], np.clip(phi[d] - K * (1.0 + np.exp(v - vmax)), -1, 1), rtol=1e-15)
    assert np.array_equal(alpha[d], (new[d] >= 0).astype(float))
    assert np.array_equal(new[~d], phi[~d])


def test_clamp_and_direction():
    d = _box()
    phi = np.full(d.shape, 0.99)
    dJ = np.where(d, -1.0, 0.0)                      # J decreases with more fluid
    new, _, info = levelset_update(phi, dJ, d, 1.0, 0.0, 1.0)
    # volume 1 = vmax: G = 0, lambda = 1, step -K(-1 + 1) = 0
    assert np.isclose(info["lambda"], 1.0) and np.allclose(new[d], 0.99)
    new2, _, _ = levelset_update(np.full(d.shape, -0.99), dJ, d, 10.0, 0.0, 1.0)
    assert np.all(new2[d] <= 1.0) and np.all(new2[d] >= -1.0)
