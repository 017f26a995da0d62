"""Pins of the surrogate oracle (oracle/mlp.py): closed forms, central
differences and exactly representable BF16 values. No GPU."""
import numpy as np
import pytest

from oracle import mlp

WIDTHS = [3, 5, 5, 5, 5, 2]  # the surrogate's shape (4 hidden SiLU layers), small


def _net(seed=0, widths=WIDTHS):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(widths, rng)
    # larger weights than the init so that the SiLU curvature matters
    return [(2.0 * W, b) for W, b in p]


def test_silu_derivatives_and_values():
    z = np.linspace(-6, 6, 49)
    h = 1e-5
    np.testing.assert_allclose(mlp.dsilu(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(mlp.d2silu(z), (mlp.dsilu(z + h) - mlp.dsilu(z - h)) / (2 * h), rtol=1e-7, atol=1e-9)
    assert mlp.silu(0.0) == 0.0 and mlp.dsilu(0.0) == 0.5 and mlp.d2silu(0.0) == 0.5
    # silu(z) -> z and silu'(z) -> 1 for large z; silu(-z) = silu(z) - z
    np.testing.assert_allclose(mlp.silu(-z), mlp.silu(z) - z, atol=1e-12)


def test_jacobian_matches_central_differences():
    p = _net(1)
    rng = np.random.default_rng(2)
    u = rng.normal(size=(4, WIDTHS[0]))
    o, J, _ = mlp.forward(p, u)
    h = 1e-6
    for t in range(WIDTHS[0]):
        du = np.zeros_like(u)
        du[:, t] = h
        fd = (mlp.forward(p, u + du)[0] - mlp.forward(p, u - du)[0]) / (2 * h)
        np.testing.assert_allclose(J[:, :, t], fd, rtol=1e-7, atol=1e-9)


def test_loss_gradient_matches_central_differences_for_every_parameter():
    p = _net(3)
    rng = np.random.default_rng(4)
    n = 6
    u = rng.normal(size=(n, WIDTHS[0]))
    y = rng.normal(size=(n, WIDTHS[-1]))
    G = rng.normal(size=(n, WIDTHS[-1], WIDTHS[0]))
    wv, wj = 0.7, 1.3
    loss, grads = mlp.loss_and_grad(p, u, y, G, wv, wj)
    o, J, _ = mlp.forward(p, u)
    assert loss == pytest.approx(mlp.sobolev_loss(o, J, y, G, wv, wj), rel=1e-14)
    vec = mlp.flatten(p)
    g = mlp.flatten(grads)
    h = 1e-6
    fd = np.empty_like(vec)
    for i in range(vec.size):
        up, dn = vec.copy(), vec.copy()
        up[i] += h
        dn[i] -= h
        lu, _ = mlp.loss_and_grad(mlp.unflatten(up, WIDTHS), u, y, G, wv, wj)
        ld, _ = mlp.loss_and_grad(mlp.unflatten(dn, WIDTHS), u, y, G, wv, wj)
        fd[i] = (lu - ld) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8 * np.abs(fd).max())


def test_one_hidden_unit_closed_form():
    # o = w2 silu(w1 u + b1) + b2, J = w2 silu'(z) w1
    w1, b1, w2, b2 = 0.8, -0.3, 1.7, 0.2
    p = [(np.array([[w1]]), np.array([b1])), (np.array([[w2]]), np.array([b2]))]
    u, y, G = 0.45, 0.1, -0.4
    wv, wj = 0.6, 1.1
    z = w1 * u + b1
    o = w2 * mlp.silu(z) + b2
    J = w2 * mlp.dsilu(z) * w1
    ro, rJ = 2 * wv * (o - y), 2 * wj * (J - G)
    want = {
        "w2": ro * mlp.silu(z) + rJ * mlp.dsilu(z) * w1,
        "b2": ro,
        "w1": ro * w2 * mlp.dsilu(z) * u + rJ * w2 * (mlp.d2silu(z) * u * w1 + mlp.dsilu(z)),
        "b1": ro * w2 * mlp.dsilu(z) + rJ * w2 * mlp.d2silu(z) * w1,
    }
    loss, g = mlp.loss_and_grad(p, np.array([[u]]), np.array([[y]]), np.array([[[G]]]), wv, wj)
    assert loss == pytest.approx(wv * (o - y) ** 2 + wj * (J - G) ** 2, rel=1e-14)
    assert g[1][0][0, 0] == pytest.approx(want["w2"], rel=1e-13)
    assert g[1][1][0] == pytest.approx(want["b2"], rel=1e-13)
    assert g[0][0][0, 0] == pytest.approx(want["w1"], rel=1e-13)
    assert g[0][1][0] == pytest.approx(want["b1"], rel=1e-13)


def test_bf16_rounding():
    exact = np.array([1.0, 0.5, 3.0, -2.25, 0.0, 2.0 ** -20, 1.0 + 2.0 ** -7])
    np.testing.assert_array_equal(mlp.round_bf16(exact), exact)
    # ties go to the even significand; the spacing at 1 is 2^-7
    assert mlp.round_bf16(1.0 + 2.0 ** -8) == 1.0
    assert mlp.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert mlp.round_bf16(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    assert mlp.round_bf16(-(1.0 + 2.0 ** -8 + 2.0 ** -12)) == -(1.0 + 2.0 ** -7)
    x = np.random.default_rng(0).normal(size=1000)
    assert np.all(np.abs(mlp.round_bf16(x) - x) <= 2.0 ** -8 * np.abs(x))


def test_bf16_mode_stays_within_bf16_accuracy():
    p = _net(5)
    p = [(mlp.round_bf16(W), mlp.round_bf16(b)) for W, b in p]
    rng = np.random.default_rng(6)
    u = rng.normal(size=(8, WIDTHS[0]))
    o, J, _ = mlp.forward(p, u)
    ob, Jb, _ = mlp.forward(p, u, bf16=True)
    assert np.abs(ob - o).max() <= 3e-2 * np.abs(o).max()
    assert np.abs(Jb - J).max() <= 3e-2 * np.abs(J).max()
