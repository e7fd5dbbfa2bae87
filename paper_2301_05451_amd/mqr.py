"""Multiple-qubit rotation (MQR), the paper's small end-to-end training benchmark (Sec. 6.1):
a hardware-efficient network on |0..0> is trained by gradient steps to minimise the sum of
the Pauli-Z expectations of every qubit, which drives the register towards |1..1>
(sum = -n). One training step = compiled forward (state + expectation values) + adjoint
backward + the parameter update, all libtq calls on the device.

The network (the paper's figure is not readable; this build's reading): ``layers`` layers of
RY(theta) on every qubit, RZ(phi) on every qubit, then a CNOT chain q -> q + 1. Parameters
are [layer][gate type][qubit], drawn U[0, 2 pi) from a seed and rounded to float32.
"""
from __future__ import annotations

import math

import numpy as np

from . import workloads as W


def mqr_circuit(n, layers=4, seed=2301):
    rng = np.random.default_rng(seed)
    params = W.f32_angles(rng, layers * 2 * n, 0.0, 2 * math.pi)
    g = W.GateList()
    for l in range(layers):
        for k, op in enumerate((W.RY, W.RZ)):
            for q in range(n):
                g.add(op, [q], [(l * 2 + k) * n + q])
        for q in range(n - 1):
            g.add(W.CNOT, [q, q + 1])
    return W.Circuit(n, g.array(), params, 1, W.zterms([([q], 1.0, 0) for q in range(n)]))


class MQRTrainer:
    """Gradient-descent (or Adam) training of one MQR circuit on the GPU."""

    def __init__(self, circuit: W.Circuit, lr=0.1, adam=False, c128=False, graph=True, eps=1e-8):
        import torch

        from . import lib

        self.c = circuit
        self.lr, self.adam, self.eps = lr, adam, eps
        rdt = torch.float64 if c128 else torch.float32
        self.spec = lib.BatchSpec.from_circuits([circuit])
        self.svb = lib.SVBatch(self.spec, circuit.terms, 1, c128=c128, graph=graph)
        self.params = torch.tensor(circuit.params, dtype=rdt, device="cuda")
        self.states = self.svb.new_states()
        self.cost = torch.empty(1, 1, dtype=rdt, device="cuda")
        self.w = torch.ones(1, 1, dtype=rdt, device="cuda")
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0

    def step(self):
        from . import lib

        self.svb.forward(self.params, self.states, self.cost)
        self.svb.backward(self.params, self.states, self.w, self.grad)
        self.t += 1
        lib.optimizer_step(self.params, self.grad, self.lr, self.t, self.m, self.v, adam=self.adam, eps=self.eps)
        return self.cost

    def run(self, iters):
        """Costs before each of the ``iters`` updates (a device tensor)."""
        import torch
        hist = torch.empty(iters, dtype=self.cost.dtype, device="cuda")
        for i in range(iters):
            hist[i:i + 1] = self.step()[0]
        return hist
