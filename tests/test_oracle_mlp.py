"""Pins of the float64 network oracle (O5): back-propagation against central
finite differences, a linear special case with a closed-form gradient, and the
first Adam step."""
import numpy as np

from oracle import mlp


def _case(din=5, h=7, dout=3, N=11, seed=0):
    rng = np.random.default_rng(seed)
    theta = mlp.init(din, h, dout, rng)
    theta += 0.1 * rng.standard_normal(theta.shape)  # nonzero biases too
    X = rng.standard_normal((N, din))
    T = rng.standard_normal((N, dout))
    return theta, X, T, din, h, dout


def test_gradient_matches_central_differences():
    theta, X, T, din, h, dout = _case()
    L, g = mlp.grad(theta, X, T, din, h, dout)
    assert np.isclose(L, mlp.loss(theta, X, T, din, h, dout))
    eps = 1e-6
    num = np.empty_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        num[i] = (mlp.loss(tp, X, T, din, h, dout) - mlp.loss(tm, X, T, din, h, dout)) / (2 * eps)
    assert np.max(np.abs(num - g)) <= 1e-8 * max(1.0, np.max(np.abs(g)))


def test_linear_special_case_has_the_least_squares_gradient():
    """With W3 = 0 the output is the constant b3, and dL/db3 = mean(b3 - T);
    the gradient of W3 is (Y - T)^T a2 / N with a2 the hidden activations, and
    no gradient reaches the hidden layers."""
    theta, X, T, din, h, dout = _case(seed=3)
    parts = mlp.unpack(theta, din, h, dout)
    W1, b1, W2, b2, W3, b3 = parts
    W3[:] = 0.0
    theta = np.concatenate([p.ravel() for p in parts])
    L, g = mlp.grad(theta, X, T, din, h, dout)
    gparts = mlp.unpack(g, din, h, dout)
    assert np.allclose(gparts[5], np.mean(b3 - T, axis=0))
    a2 = np.tanh(np.tanh(X @ W1.T + b1) @ W2.T + b2)
    assert np.allclose(gparts[4], (b3 - T).T @ a2 / X.shape[0])
    for k in range(4):
        assert np.all(gparts[k] == 0.0)
    assert np.isclose(L, 0.5 * np.sum((b3 - T) ** 2) / X.shape[0])


def test_first_adam_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(20)
    g = rng.standard_normal(20)
    new, m, v = mlp.adam_step(theta, g, np.zeros(20), np.zeros(20), 1, lr=1e-2)
    assert np.allclose(new - theta, -1e-2 * np.sign(g), atol=1e-9)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_the_loss_on_a_smooth_target():
    """Sanity of the definition as a trainer: a few hundred Adam steps fit a
    smooth map much better than the initial network."""
    rng = np.random.default_rng(7)
    din, h, dout = 2, 16, 1
    X = rng.uniform(-1, 1, size=(64, din))
    T = np.sin(2 * X[:, :1]) * np.cos(X[:, 1:])
    theta = mlp.init(din, h, dout, rng)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    L0 = mlp.loss(theta, X, T, din, h, dout)
    for t in range(1, 401):
        _, g = mlp.grad(theta, X, T, din, h, dout)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, lr=1e-2)
    assert mlp.loss(theta, X, T, din, h, dout) < 0.05 * L0
