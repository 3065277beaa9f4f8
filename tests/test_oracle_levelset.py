"""Pins of the oracle's level-set update (Eqs. 13-15, 67), independent of the
update's own arithmetic: the stencil on fields whose Laplacian is known and
next to non-design nodes (no flux), the implicit system against the loop stencil
applied to unit vectors, the step against Eq. (14) evaluated with the loop
stencil, and closed forms on uniform inputs."""
import numpy as np

from oracle.levelset import implicit_matrix, laplacian, levelset_update

D, F, I, O, W_, H, S = 0, 1, 2, 3, 4, 5, 6


def _box(n=6):
    k = np.full((n, n, n), D, dtype=np.uint8)
    k[0], k[-1], k[:, 0], k[:, -1], k[:, :, 0], k[:, :, -1] = (W_,) * 6
    return k


def test_laplacian_of_quadratic_is_exact():
    z, y, x = np.meshgrid(np.arange(7.), np.arange(7.), np.arange(7.), indexing="ij")
    phi = 0.5 * x ** 2 - 0.25 * y ** 2 + 0.125 * z ** 2 + 3 * x * y
    k = np.zeros(phi.shape, dtype=np.uint8)
    lap = laplacian(phi, k)
    inner = (slice(1, -1),) * 3
    assert np.allclose(lap[inner], 1.0 - 0.5 + 0.25, atol=1e-12)
    # sum_a sigma_a d_aa phi with phi_xx = 1, phi_yy = -0.5, phi_zz = 0.25
    lap3 = laplacian(phi, k, (2.0, 3.0, 4.0))
    assert np.allclose(lap3[inner], 2.0 * 1.0 - 3.0 * 0.5 + 4.0 * 0.25, atol=1e-12)
    # a box face counts as the node itself: a constant field has no Laplacian
    assert np.all(laplacian(np.full(phi.shape, 0.3), k) == 0.0)


def test_no_flux_to_non_design_nodes():
    k = np.full((3, 3, 5), D, dtype=np.uint8)
    k[:, :, 0] = W_
    k[:, :, 4] = F
    k[2] = S
    phi = np.where(k == D, 0.25, 0.0)
    phi[1, 1, 2] = 1.0
    lap = laplacian(phi, k)
    # non-design neighbours (whatever their phase) and box faces count as
    # the node itself
    assert np.isclose(lap[1, 1, 1], 0.75) and np.isclose(lap[1, 1, 3], 0.75)
    assert np.isclose(lap[1, 1, 2], -3.75)           # 5 design neighbours at 0.25
    assert np.all(lap[k != D] == 0.0)
    for kind in (I, O, H, W_, F, S):
        k2 = k.copy()
        k2[:, :, 0] = kind
        assert np.isclose(laplacian(phi, k2)[1, 1, 1], 0.75)


def test_implicit_matrix_is_the_loop_stencil():
    k = _box(5)
    k[2, 2, 0] = I
    k[1, 4, 2] = F
    k[3, 3, 3] = W_
    d = k == D
    nodes = np.argwhere(d)
    K, sig = 0.7, (0.5, 1.5, 4.0)
    A = implicit_matrix(k, K, sig)
    zero = np.zeros(k.shape)
    assert np.all(laplacian(zero, k, sig) == 0.0)      # lap is linear
    for j, idx in enumerate(nodes):
        e = zero.copy()
        e[tuple(idx)] = 1.0
        col = e[d] - K * laplacian(e, k, sig)[d]
        assert np.allclose(A[:, j].toarray().ravel(), col, atol=1e-15)
    assert np.allclose(A.toarray(), A.toarray().T)


def test_step_satisfies_eq14():
    rng = np.random.default_rng(0)
    k = _box(7)
    k[3, 3, 0] = I
    k[3, 0, 3] = O
    k[2, 2, 2] = W_
    d = k == D
    phi = np.where(d, rng.uniform(-0.5, 0.5, k.shape), 0.0)
    dJ = np.where(d, rng.normal(size=k.shape), 0.0)
    K, sigma, vmax = 0.05, 0.8, 0.4
    new, alpha, info = levelset_update(phi, dJ, k, K, sigma, vmax)
    assert np.all(np.abs(new[d]) < 1.0)           # no clamp active
    s = np.abs(dJ[d]).mean()
    lam_ref = np.exp(info["G"]) * np.abs(dJ[d] / s - sigma * laplacian(phi, k)[d]).mean()
    assert np.isclose(info["lambda"], lam_ref, rtol=1e-14)
    lhs = (new[d] - phi[d]) / K
    rhs = -(dJ[d] / s + info["lambda"]) + sigma * laplacian(new, k)[d]
    assert np.allclose(lhs, rhs, atol=1e-10)
    # anisotropic: sigma_z = 10 sigma_x as in Sec. 3.3.4
    sig = (sigma, sigma, 10 * sigma)
    new3, _, info3 = levelset_update(phi, dJ, k, K, sig, vmax)
    lam3 = np.exp(info3["G"]) * np.abs(dJ[d] / s - laplacian(phi, k, sig)[d]).mean()
    assert np.isclose(info3["lambda"], lam3, rtol=1e-14)
    lhs3 = (new3[d] - phi[d]) / K
    rhs3 = -(dJ[d] / s + info3["lambda"]) + laplacian(new3, k, sig)[d]
    assert np.allclose(lhs3, rhs3, atol=1e-10)
    assert np.array_equal(alpha[d], (new[d] >= 0).astype(float))
    assert np.array_equal(new[~d], phi[~d])


def test_lambda_closed_form_and_uniform_step():
    k = np.zeros((6, 6, 6), dtype=np.uint8)       # all design
    d = k == D
    phi = np.full(k.shape, 0.2)
    dJ = np.full(k.shape, 2.0)                     # uniform sensitivity
    K, vmax = 0.05, 0.3
    for sigma in (0.0, 0.5):
        new, alpha, info = levelset_update(phi, dJ, k, K, sigma, vmax)
        assert info["volume"] == 1.0 and np.isclose(info["G"], 1.0 - vmax)
        # |J'/mean|J'|| = 1 and lap phi = 0: lambda = exp(G), uniform step
        assert np.isclose(info["lambda"], np.exp(1.0 - vmax), rtol=1e-15)
        assert np.allclose(new, 0.2 - K * (1.0 + np.exp(1.0 - vmax)), rtol=1e-13)


def test_clamp_and_direction():
    k = _box()
    d = k == D
    phi = np.where(d, 0.99, 0.0)
    dJ = np.where(d, -1.0, 0.0)                      # J decreases with more fluid
    new, _, info = levelset_update(phi, dJ, k, 1.0, 0.0, 1.0)
    # volume 1 = vmax: G = 0, lambda = 1, step -K(-1 + 1) = 0
    assert np.isclose(info["lambda"], 1.0) and np.allclose(new[d], 0.99)
    new2, _, _ = levelset_update(np.where(d, -0.99, 0.0), dJ, k, 10.0, 0.3, 1.0)
    assert np.all(new2[d] <= 1.0) and np.all(new2[d] >= -1.0)
