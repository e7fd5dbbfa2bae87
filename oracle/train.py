"""Training-loop oracle in float64 (test infrastructure only; never on the product path).

The variational loop of Sec. 4: the cost f(theta) = <0|U^dag(theta) O U(theta)|0> is
minimised by gradient steps, the gradient of each step taken by the oracle's parameter-shift
rule (Sec. 4.2). Used for the multiple-qubit-rotation benchmark of Sec. 6.1 (cost =
sum_i <Z_i>). Updates: plain gradient descent theta <- theta - lr g, or Adam (Kingma and Ba)
with bias correction, written out here from its definition.
"""
from __future__ import annotations

import math

import numpy as np

from . import sv


def trajectory(c, lr, iters, adam=False, b1=0.9, b2=0.999, eps=1e-8):
    """(costs before each update, parameters after the last update)."""
    theta = np.asarray(c.params, dtype=np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    costs = []
    for t in range(1, iters + 1):
        costs.append(float(sv.circuit_f(c, theta)[0]))
        g = sv.param_shift_grad(c, params=theta)
        if adam:
            m = b1 * m + (1 - b1) * g
            v = b2 * v + (1 - b2) * g * g
            theta = theta - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        else:
            theta = theta - lr * g
    return np.array(costs), theta
