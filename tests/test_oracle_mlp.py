"""Pins of the FP64 MLP oracle: finite differences, closed forms, Adam by hand."""
import numpy as np

from oracle import mlp as O
from paper_1305_1183_amd import inputs as I


def rand_params(d, h, L, seed, scale=0.5):
    _, n = O.layout(d, h, L)
    return I.uniform_pm1(seed, 0, n).astype(np.float64) * scale


def test_layout_counts():
    lay, n = O.layout(32, 128, 3)
    assert n == 32 * 128 + 128 + 2 * (128 * 128 + 128) + 128 + 1
    assert lay[-1][2:] == (128, 1)


def test_gradient_matches_central_differences():
    d, h, L, n = 5, 7, 3, 11
    p = rand_params(d, h, L, 1)
    X = I.uniform_pm1(1, 1, n * d).reshape(n, d).astype(np.float64)
    y = I.uniform_pm1(1, 2, n).astype(np.float64)
    loss, g = O.loss_grad(p, X, y, d, h, L)
    step = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = step
        num[i] = (O.loss_grad(p + e, X, y, d, h, L)[0] - O.loss_grad(p - e, X, y, d, h, L)[0]) / (2 * step)
    rel = np.linalg.norm(num - g) / np.linalg.norm(g)
    assert rel <= 1e-6, rel


def test_bias_only_network():
    """Zero weights: the output is the output bias, only it has a gradient."""
    d, h, L = 4, 6, 3
    lay, ntot = O.layout(d, h, L)
    p = np.zeros(ntot)
    p[lay[-1][1]] = 0.75
    X = np.ones((3, d))
    y = np.array([0.25, 0.5, 1.0])
    pred, _ = O.forward(p, X, d, h, L)
    assert np.all(pred == 0.75)
    loss, g = O.loss_grad(p, X, y, d, h, L)
    assert loss == np.mean((0.75 - y) ** 2)
    ob = lay[-1][1]
    assert abs(g[ob] - 2 * np.mean(0.75 - y)) <= 1e-15
    assert np.all(np.delete(g, ob) == 0.0)


def test_positive_network_is_linear():
    """All-positive inputs and weights keep every ReLU active, so the network
    equals the product of its affine maps."""
    d, h, L, n = 3, 5, 3, 4
    p = np.abs(rand_params(d, h, L, 2)) + 0.01
    X = np.abs(I.uniform_pm1(2, 1, n * d).reshape(n, d).astype(np.float64)) + 0.1
    layers = O.unpack(p, d, h, L)
    z = X
    for W, b in layers:
        z = z @ W + b
    np.testing.assert_allclose(O.forward(p, X, d, h, L)[0], z[:, 0], rtol=1e-14)


def test_adam_first_step_by_hand():
    """Step 1 with bias correction: mhat = g, vhat = g^2, so the update is
    lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3])
    p = np.array([1.0, 1.0, 1.0])
    lr, eps = 0.01, 1e-8
    p1, m, v = O.adam(p, g, np.zeros(3), np.zeros(3), 1, lr, eps=eps)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=1e-12)
    # second step with the same gradient keeps mhat = g and vhat = g^2
    p2, m2, v2 = O.adam(p1, g, m, v, 2, lr, eps=eps)
    np.testing.assert_allclose(p2, p1 - lr * g / (np.abs(g) + eps), rtol=1e-12)
