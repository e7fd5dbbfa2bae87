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


def _scaled(layers, s):
    return [[W * s, b * s] for W, b in layers]


def test_forward_is_odd_without_biases():
    # tanh is odd, so with every bias at zero the whole network is odd: f(-x) = -f(x). A bias
    # that leaked in, or an activation that is not odd, breaks this.
    rng = np.random.default_rng(3)
    layers = mlp.init([5, 7, 6, 1], rng)
    X = rng.normal(size=(11, 5))
    f, _ = mlp.forward(layers, X)
    g, _ = mlp.forward(layers, -X)
    assert np.abs(f).max() > 1e-2
    np.testing.assert_allclose(g, -f, rtol=0, atol=1e-15)


def test_small_weights_reduce_to_the_linear_map():
    # tanh(z) = z - z^3/3 + ..., so for weights of size eps the network is the plain matrix
    # product W3 W2 W1 x up to a relative O(eps^2): pins the order of the layers and the
    # orientation of every (non-square) weight matrix.
    rng = np.random.default_rng(4)
    base = [[rng.normal(size=(7, 5)), np.zeros(7)], [rng.normal(size=(6, 7)), np.zeros(6)],
            [rng.normal(size=(1, 6)), np.zeros(1)]]
    X = rng.normal(size=(8, 5))
    lin = X @ (base[2][0] @ base[1][0] @ base[0][0]).T  # [8, 1]
    for eps in (1e-2, 1e-3):
        f, _ = mlp.forward(_scaled(base, eps), X)
        want = lin[:, 0] * eps ** 3
        rel = np.abs(f - want).max() / np.abs(want).max()
        assert rel < 50 * eps ** 2, (eps, rel)


def test_output_layer_is_affine():
    # The last layer has no activation: scaling W3 and b3 by s scales the output by s, and a
    # bias b3 alone (all weights zero) is returned for every input.
    rng = np.random.default_rng(5)
    layers = mlp.init([4, 6, 5, 1], rng)
    for W, b in layers:
        b[:] = rng.normal(size=b.shape)
    X = rng.normal(size=(7, 4))
    f, _ = mlp.forward(layers, X)
    two = [list(l) for l in layers]
    two[2] = [2.5 * layers[2][0], 2.5 * layers[2][1]]
    g, _ = mlp.forward(two, X)
    np.testing.assert_allclose(g, 2.5 * f, rtol=1e-14, atol=1e-15)
    zero = [[np.zeros_like(W), np.zeros_like(b)] for W, b in layers]
    zero[2][1] = np.array([1.75])
    h, _ = mlp.forward(zero, X)
    assert np.all(h == 1.75)


def test_rows_are_independent():
    # Each sample's output depends on its own row only (batch and feature axes not swapped).
    rng = np.random.default_rng(6)
    layers = mlp.init([5, 7, 6, 1], rng)
    X = rng.normal(size=(6, 5))
    f, _ = mlp.forward(layers, X)
    for i in range(6):
        fi, _ = mlp.forward(layers, X[i:i + 1])
        np.testing.assert_allclose(fi, f[i:i + 1], rtol=1e-15, atol=0)


def test_biases_act_as_weights_on_a_constant_unit():
    # A bias is a weight on a unit that always outputs 1. Moving b1 into an extra input column
    # fixed at 1, and b2 into an extra first-layer unit saturated at tanh(40) = 1 (exact in
    # float64), must give the same outputs: a dropped or misplaced hidden bias fails.
    rng = np.random.default_rng(7)
    layers = mlp.init([4, 6, 5, 1], rng)
    for W, b in layers:
        b[:] = rng.normal(size=b.shape)
    (W1, b1), (W2, b2), (W3, b3) = layers
    X = rng.normal(size=(9, 4))
    f, _ = mlp.forward(layers, X)
    X1 = np.concatenate([X, np.ones((9, 1))], 1)
    W1e = np.concatenate([np.concatenate([W1, b1[:, None]], 1), np.zeros((1, 5))], 0)  # [7, 5]
    b1e = np.zeros(7)
    b1e[6] = 40.0  # the constant unit
    W2e = np.concatenate([W2, b2[:, None]], 1)  # [5, 7]
    g, _ = mlp.forward([[W1e, b1e], [W2e, np.zeros(5)], [W3, b3]], X1)
    np.testing.assert_allclose(g, f, rtol=1e-14, atol=1e-15)
