"""Pins of the FP64 surrogate-MLP reference: its analytic backpropagation
against central finite differences of the loss, and its building blocks
against closed forms."""
import numpy as np
from scipy.special import erf

from oracle import mlp


def test_gelu_and_derivative():
    x = np.linspace(-6, 6, 241)
    assert np.allclose(mlp.gelu(x), x * 0.5 * (1 + erf(x / np.sqrt(2))), atol=0, rtol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(x)).max() < 1e-8
    assert mlp.gelu(0.0) == 0.0 and abs(mlp.gelu_grad(0.0) - 0.5) < 1e-15


def test_bce_stable_form():
    z = np.linspace(-30, 30, 121)
    for y in (0.0, 1.0):
        naive = -(y * np.log(1 / (1 + np.exp(-z))) + (1 - y) * np.log(1 - 1 / (1 + np.exp(-z))))
        ok = np.abs(z) < 8  # where 1 - sigmoid(z) keeps its digits
        assert np.allclose(mlp.bce(z[ok], y), naive[ok], rtol=1e-12, atol=1e-14)
    # asymptotes: BCE(z, 0) -> z and BCE(-z, 1) -> z for large z, without overflow
    big = np.array([25.0, 100.0, 1000.0])
    assert np.allclose(mlp.bce(big, 0.0), big, rtol=1e-10)
    assert np.allclose(mlp.bce(-big, 1.0), big, rtol=1e-10)
    assert mlp.bce(np.array([1000.0]), 1.0)[0] == 0.0


def test_backprop_matches_finite_differences():
    H = 8
    rng = np.random.default_rng(3)
    p = mlp.init(H, 11)
    for k in p:  # non-zero biases exercise every term
        p[k] = p[k] + 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((16, 4))
    y = (rng.random(16) < 0.4).astype(np.float64)
    t = rng.standard_normal(16)
    g = mlp.flatten(mlp.gradients(p, x, y, t), H)
    flat = mlp.flatten(p, H)
    fd = np.empty_like(flat)
    h = 1e-6
    for i in range(flat.size):
        a, b = flat.copy(), flat.copy()
        a[i] += h
        b[i] -= h
        fd[i] = (mlp.loss(mlp.unflatten(a, H), x, y, t) - mlp.loss(mlp.unflatten(b, H), x, y, t)) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-6 * max(1.0, np.abs(g).max())


def test_no_blowup_in_batch_drops_the_time_term():
    H = 4
    p = mlp.init(H, 1)
    x = np.random.default_rng(0).standard_normal((5, 4))
    y = np.zeros(5)
    g = mlp.gradients(p, x, y, np.full(5, 123.0))
    out, _ = mlp.forward(p, x)
    assert abs(mlp.loss(p, x, y, np.zeros(5)) - mlp.bce(out[:, 0], 0.0).mean()) < 1e-15
    assert np.all(mlp.gradients(p, x, y, np.zeros(5))["W3"] == g["W3"])


def test_adam_first_step():
    """With zero moments, the bias-corrected first step is -lr * g / (|g| + eps)."""
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -4.0, 0.0])}
    z = {"w": np.zeros(3)}
    pn, m, v = mlp.adam(p, g, z, z, 1, 1e-3)
    expect = p["w"] - 1e-3 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(pn["w"], expect, rtol=0, atol=1e-15)
    assert np.allclose(m["w"], 0.1 * g["w"]) and np.allclose(v["w"], 0.001 * g["w"] ** 2)
