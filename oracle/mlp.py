"""Float64 multilayer perceptron: forward, manual backward, Adam (test infrastructure only).

The paper has no learned component: this is the reference for the runtime cost model
that ranks contraction trees. PARITY UNPINNED by the paper. Pinned instead by central
finite differences of the loss (backward), by Adam's closed-form first step
(bias-corrected, the first update is lr * g / (|g| + eps) elementwise), and by properties of
the forward: with zero biases the network is odd; for small weights it tends to the plain
product of the weight matrices; a bias equals a weight on a constant unit; the output layer
is affine; each sample's output depends on its own row only.

Network: x -> tanh(W1 x + b1) -> tanh(W2 h1 + b2) -> W3 h2 + b3 (scalar output).
Loss: mean squared error over the batch, L = mean_b (yhat_b - y_b)^2.
Weights are stored as W[out, in], biases as b[out].
"""
from __future__ import annotations

import numpy as np


def init(sizes, rng):
    layers = []
    for i in range(len(sizes) - 1):
        fan_in = sizes[i]
        W = rng.uniform(-1.0, 1.0, size=(sizes[i + 1], fan_in)) / np.sqrt(fan_in)
        b = np.zeros(sizes[i + 1])
        layers.append([W, b])
    return layers


def forward(layers, X):
    """X [B, in] -> (yhat [B], activations list)."""
    acts = [np.asarray(X, dtype=np.float64)]
    h = acts[0]
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        h = np.tanh(z) if li < len(layers) - 1 else z
        acts.append(h)
    return h[:, 0], acts


def loss(layers, X, y):
    yhat, _ = forward(layers, X)
    return float(np.mean((yhat - y) ** 2))


def backward(layers, X, y):
    """Returns (loss, grads) with grads shaped like layers."""
    yhat, acts = forward(layers, X)
    B = X.shape[0]
    r = yhat - y
    L = float(np.mean(r**2))
    d = (2.0 / B) * r[:, None]  # dL/d(output pre-activation)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        h_in = acts[li]
        grads[li] = [d.T @ h_in, d.sum(axis=0)]
        if li > 0:
            dh = d @ W
            d = dh * (1.0 - acts[li] ** 2)  # tanh' at the previous layer's output
    return L, grads


def adam_init(layers):
    return {"t": 0, "m": [[np.zeros_like(W), np.zeros_like(b)] for W, b in layers],
            "v": [[np.zeros_like(W), np.zeros_like(b)] for W, b in layers]}


def adam_step(layers, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015) with bias correction, in place."""
    state["t"] += 1
    t = state["t"]
    for li in range(len(layers)):
        for k in range(2):
            g = grads[li][k]
            m = state["m"][li][k] = b1 * state["m"][li][k] + (1 - b1) * g
            v = state["v"][li][k] = b2 * state["v"][li][k] + (1 - b2) * g * g
            mh = m / (1 - b1**t)
            vh = v / (1 - b2**t)
            layers[li][k] = layers[li][k] - lr * mh / (np.sqrt(vh) + eps)
    return layers
