"""Pins of the training-loop oracle: the descent recursion of a single rotation in closed
form, Adam's first step (a step of size lr against the gradient's sign), and convergence of
the multiple-qubit rotation to |1..1> (cost -n)."""
import math

import numpy as np

from oracle import train
from paper_2301_05451_amd import mqr
from paper_2301_05451_amd import workloads as W


def test_descent_on_one_rotation_closed_form():
    # f(theta) = <Z> after RY(theta) = cos(theta), so theta <- theta + lr sin(theta)
    c = W.Circuit(1, W.GateList().add(W.RY, [0], [0]).array(), np.array([0.7]), 1, W.zterms([([0], 1.0, 0)]))
    costs, theta = train.trajectory(c, 0.2, 5)
    t = 0.7
    for k in range(5):
        assert abs(costs[k] - math.cos(t)) < 1e-14
        t = t + 0.2 * math.sin(t)
    assert abs(theta[0] - t) < 1e-13


def test_adam_first_step_is_lr_against_gradient_sign():
    c = W.Circuit(1, W.GateList().add(W.RY, [0], [0]).array(), np.array([0.7]), 1, W.zterms([([0], 1.0, 0)]))
    _, theta = train.trajectory(c, 0.05, 1, adam=True)
    assert abs(theta[0] - (0.7 + 0.05 * (1 - 1e-8 / (math.sin(0.7) + 1e-8)))) < 1e-9


def test_mqr_converges_to_all_ones():
    c = mqr.mqr_circuit(3, layers=2)
    costs, _ = train.trajectory(c, 0.2, 150)
    assert costs[0] > -2.5 and costs[-1] < -3 + 1e-3
