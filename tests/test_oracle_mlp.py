"""Pins of the float64 MLP oracle (the paper has no MLP: pinned by FD and Adam's first step)."""
import numpy as np

from oracle import mlp


def test_backward_matches_central_fd():
    rng = np.random.default_rng(0)
    layers = mlp.init([5, 7, 6, 1], rng)
    X = rng.normal(size=(9, 5))
    y = rng.normal(size=9)
    L, grads = mlp.backward(layers, X, y)
    h = 1e-6
    for li in range(3):
        for k in range(2):
            P = layers[li][k]
            it = np.nditer(P, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = P[idx]
                P[idx] = old + h
                lp = mlp.loss(layers, X, y)
                P[idx] = old - h
                lm = mlp.loss(layers, X, y)
                P[idx] = old
                assert abs((lp - lm) / (2 * h) - grads[li][k][idx]) < 1e-8


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(1)
    layers = mlp.init([3, 4, 4, 1], rng)
    X = rng.normal(size=(6, 3))
    y = rng.normal(size=6)
    _, grads = mlp.backward(layers, X, y)
    before = [[W.copy(), b.copy()] for W, b in layers]
    st = mlp.adam_init(layers)
    lr = 0.01
    mlp.adam_step(layers, grads, st, lr=lr)
    for li in range(3):
        for k in range(2):
            g = grads[li][k]
            want = before[li][k] - lr * g / (np.abs(g) + 1e-8)
            assert np.allclose(layers[li][k], want, atol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    layers = mlp.init([4, 16, 16, 1], rng)
    X = rng.normal(size=(64, 4))
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1]
    st = mlp.adam_init(layers)
    l0 = mlp.loss(layers, X, y)
    for _ in range(300):
        _, g = mlp.backward(layers, X, y)
        mlp.adam_step(layers, g, st, lr=1e-2)
    assert mlp.loss(layers, X, y) < 0.1 * l0
