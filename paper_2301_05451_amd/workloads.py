"""Seeded synthetic circuit generators and the shared gate-list record.

This module is the only code that both the oracle and the HIP path import. It holds
circuit *structure* and random draws, nothing of the simulation arithmetic: no gate
matrices, no contraction, no expectation values.

Conventions (TeD-Q paper, Sec. 5.1 "Fast simulation": qubits are counted from 0 with
qubit 0 on the left):

* qubit ``q`` of an ``n``-qubit register sits at bit position ``n-1-q`` of the
  amplitude index (qubit 0 is the most significant bit);
* a gate's rotation angle in slot ``j`` is ``pscale[j] * params[pidx[j]]`` when
  ``pidx[j] >= 0``, otherwise the constant ``pscale[j]``; parameters are listed in
  gate order (Sec. 2, circuit compilation);
* two-qubit gates list ``[control, target]`` (CNOT, CRX, CRY, CRZ) or an unordered pair
  (CZ, RZZ).

Angles are drawn in float64 and rounded to float32, so that the complex64 GPU path
and the complex128 oracle see the very same parameter values.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ---- gate codes (must match include/tq.h) ------------------------------------------
H, X, Y, Z, RX, RY, RZ, U3, ROT, CNOT, CZ, RZZ, CRX, CRY, CRZ = range(15)
OP_NAMES = ["H", "X", "Y", "Z", "RX", "RY", "RZ", "U3", "ROT", "CNOT", "CZ", "RZZ", "CRX", "CRY", "CRZ"]
N_ANGLES = {H: 0, X: 0, Y: 0, Z: 0, RX: 1, RY: 1, RZ: 1, U3: 3, ROT: 3, CNOT: 0, CZ: 0, RZZ: 1,
            CRX: 1, CRY: 1, CRZ: 1}
N_QUBITS = {H: 1, X: 1, Y: 1, Z: 1, RX: 1, RY: 1, RZ: 1, U3: 1, ROT: 1, CNOT: 2, CZ: 2, RZZ: 2,
            CRX: 2, CRY: 2, CRZ: 2}

# C layout of ``tq_gate``: int32 op, int32 q[2], int32 pidx[3], double pscale[3]  (48 bytes)
GATE_DTYPE = np.dtype(
    [("op", "<i4"), ("q", "<i4", (2,)), ("pidx", "<i4", (3,)), ("pscale", "<f8", (3,))],
    align=True,
)
assert GATE_DTYPE.itemsize == 48

# C layout of ``tq_zterm``: uint64 mask (bit q = Z on qubit q), double coeff, int32 obs, pad
ZTERM_DTYPE = np.dtype([("mask", "<u8"), ("coeff", "<f8"), ("obs", "<i4"), ("_pad", "<i4")], align=True)
assert ZTERM_DTYPE.itemsize == 24


@dataclasses.dataclass
class Circuit:
    """One parameterised circuit: structure plus its parameter vector."""

    n: int
    gates: np.ndarray  # GATE_DTYPE records in application order
    params: np.ndarray  # float64 values, each exactly representable in float32
    n_obs: int = 1
    terms: np.ndarray = None  # ZTERM_DTYPE records

    @property
    def n_params(self) -> int:
        return int(self.params.shape[0])


class GateList:
    """Small builder used by the generators and the tests."""

    def __init__(self):
        self.rows = []

    def add(self, op, qubits, pidx=(), pscale=None):
        na = N_ANGLES[op]
        q = list(qubits) + [-1] * (2 - len(qubits))
        pi = list(pidx) + [-1] * (3 - len(pidx))
        if pscale is None:
            pscale = [1.0] * len(pidx)
        ps = list(pscale) + [0.0] * (3 - len(pscale))
        assert len(qubits) == N_QUBITS[op], (op, qubits)
        assert len(pidx) <= na and len(pscale) <= max(na, len(pidx))
        self.rows.append((op, q, pi, ps))
        return self

    def const(self, op, qubits, angles=()):
        """A gate with constant angles (pidx = -1, pscale holds the angle)."""
        return self.add(op, qubits, pidx=[-1] * len(angles), pscale=list(angles))

    def array(self) -> np.ndarray:
        a = np.zeros(len(self.rows), dtype=GATE_DTYPE)
        for i, (op, q, pi, ps) in enumerate(self.rows):
            a[i]["op"] = op
            a[i]["q"] = q
            a[i]["pidx"] = pi
            a[i]["pscale"] = ps
        return a


# C layout of ``tq_pauli_term``: uint64 x_mask, uint64 z_mask (bit q: qubit q carries X when
# only x is set, Z when only z is set, Y when both are), double coeff, int32 obs, pad
PAULI_DTYPE = np.dtype([("x", "<u8"), ("z", "<u8"), ("coeff", "<f8"), ("obs", "<i4"), ("_pad", "<i4")],
                       align=True)
assert PAULI_DTYPE.itemsize == 32


def pauli_terms(rows):
    """``rows`` = list of (Pauli string over qubits as {qubit: 'X'|'Y'|'Z'}, coeff, obs)."""
    a = np.zeros(len(rows), dtype=PAULI_DTYPE)
    for i, (ps, c, o) in enumerate(rows):
        x = z = 0
        for q, p in ps.items():
            if p in ("X", "Y"):
                x |= 1 << int(q)
            if p in ("Z", "Y"):
                z |= 1 << int(q)
        a[i]["x"], a[i]["z"], a[i]["coeff"], a[i]["obs"] = x, z, c, o
    return a


def zterms(pairs):
    """``pairs`` = list of (qubit list, coeff, obs index) -> ZTERM_DTYPE array."""
    a = np.zeros(len(pairs), dtype=ZTERM_DTYPE)
    for i, (qs, c, o) in enumerate(pairs):
        m = 0
        for q in qs:
            m |= 1 << int(q)
        a[i]["mask"] = m
        a[i]["coeff"] = c
        a[i]["obs"] = o
    return a


def f32_angles(rng, size, lo, hi):
    """Uniform angles drawn in float64 then rounded to float32 values (held as float64)."""
    return rng.uniform(lo, hi, size=size).astype(np.float32).astype(np.float64)


# ---- workloads ---------------------------------------------------------------------

def hea_ring(n=10, layers=4, seed=1001):
    """Hardware-efficient ansatz: per layer RY on every qubit, RZ on every qubit, then
    a CNOT ring q -> (q+1) mod n. Parameters are [layer][gate type][qubit]."""
    rng = np.random.default_rng(seed)
    params = f32_angles(rng, layers * 2 * n, 0.0, 2 * math.pi)
    g = GateList()
    for l in range(layers):
        for k, op in enumerate((RY, RZ)):
            for q in range(n):
                g.add(op, [q], [(l * 2 + k) * n + q])
        for q in range(n):
            g.add(CNOT, [q, (q + 1) % n])
    return Circuit(n, g.array(), params, 1, zterms([([0], 1.0, 0)]))


def brickwork(n=24, layers=20, seed=1002):
    """Per layer: RX, RY, RZ on every qubit, then CZ on (0,1),(2,3).. for even layers and
    (1,2),(3,4).. for odd layers (no wrap). Observable sum_i Z_i as one output."""
    rng = np.random.default_rng(seed)
    params = f32_angles(rng, layers * 3 * n, 0.0, 2 * math.pi)
    g = GateList()
    for l in range(layers):
        for k, op in enumerate((RX, RY, RZ)):
            for q in range(n):
                g.add(op, [q], [(l * 3 + k) * n + q])
        for a in range(l % 2, n - 1, 2):
            g.add(CZ, [a, a + 1])
    terms = zterms([([q], 1.0, 0) for q in range(n)])
    return Circuit(n, g.array(), params, 1, terms)


def qnn_structure(n=16, layers=8):
    """Angle encoding RY(x_q) on every qubit, then per layer RY all, RZ all and a CNOT
    chain q -> q+1. Parameter vector per sample: [x_0..x_{n-1}, theta (layers*2*n)]."""
    g = GateList()
    for q in range(n):
        g.add(RY, [q], [q])
    for l in range(layers):
        for k, op in enumerate((RY, RZ)):
            for q in range(n):
                g.add(op, [q], [n + (l * 2 + k) * n + q])
        for q in range(n - 1):
            g.add(CNOT, [q, q + 1])
    return g.array()


def qnn_batch(n=16, layers=8, batch=512, seed=1003):
    """Batched QML step: inputs x ~ U[0, pi], shared weights ~ U[0, 2pi), targets ~ U[-1, 1].
    Returns (gates, x[batch, n], theta[layers*2*n], y[batch])."""
    rng = np.random.default_rng(seed)
    x = f32_angles(rng, (batch, n), 0.0, math.pi)
    theta = f32_angles(rng, layers * 2 * n, 0.0, 2 * math.pi)
    y = rng.uniform(-1.0, 1.0, size=batch).astype(np.float32).astype(np.float64)
    return qnn_structure(n, layers), x, theta, y


def random_u3_cnot(n, rng):
    """2n layers of U3 on every qubit, then floor(n/2) disjoint CNOT pairs drawn from a
    seeded permutation (control = first element of each pair)."""
    layers = 2 * n
    params = f32_angles(rng, layers * n * 3, 0.0, 2 * math.pi)
    g = GateList()
    for l in range(layers):
        for q in range(n):
            b = (l * n + q) * 3
            g.add(U3, [q], [b, b + 1, b + 2])
        perm = rng.permutation(n)
        for k in range(n // 2):
            g.add(CNOT, [int(perm[2 * k]), int(perm[2 * k + 1])])
    return Circuit(n, g.array(), params, 1, zterms([([0], 1.0, 0)]))


def uneven_batch(count=1024, nmin=8, nmax=20, seed=1004):
    """``count`` random circuits with qubit counts uniform in [nmin, nmax]."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    return [random_u3_cnot(int(n), rng) for n in ns]


def random_regular_graph(d, n, rng, max_tries=10000):
    """Uniform-ish random d-regular simple graph by the pairing model with rejection."""
    assert (n * d) % 2 == 0
    for _ in range(max_tries):
        stubs = np.repeat(np.arange(n), d)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        e = {tuple(sorted(map(int, p))) for p in pairs}
        if len(e) != len(pairs):
            continue
        return sorted(e)
    raise RuntimeError("no simple regular graph found")


@dataclasses.dataclass
class QAOAProblem:
    n: int
    edges: list  # sorted (i, j) with i < j
    p: int
    gammas: np.ndarray  # [p] float64 (float32 values)
    betas: np.ndarray  # [p]


def qaoa_maxcut(n=50, p=4, seed=1005):
    """QAOA MaxCut on a seeded random 3-regular graph; gamma, beta ~ U[0, pi]."""
    rng = np.random.default_rng(seed)
    edges = random_regular_graph(3, n, rng)
    gam = f32_angles(rng, p, 0.0, math.pi)
    bet = f32_angles(rng, p, 0.0, math.pi)
    return QAOAProblem(n, edges, p, gam, bet)


def qaoa_circuit(prob: QAOAProblem):
    """QAOA circuit on the whole register: H on every qubit, then for each layer l
    RZZ(gamma_l) on every edge and RX(2 beta_l) on every qubit. Parameter vector:
    [gamma_0..gamma_{p-1}, beta_0..beta_{p-1}]."""
    g = GateList()
    for v in range(prob.n):
        g.const(H, [v])
    for l in range(prob.p):
        for (a, b) in prob.edges:
            g.add(RZZ, [a, b], [l])
        for v in range(prob.n):
            g.add(RX, [v], [prob.p + l], [2.0])
    params = np.concatenate([prob.gammas, prob.betas])
    return Circuit(prob.n, g.array(), params)


def random_circuit(n, n_gates, rng, ops=None, n_params=None):
    """Random gate list over all gate types, for parity tests. Each parameterised slot
    draws a parameter index (parameters may be shared) and a scale in {1, 2, -0.5}."""
    if ops is None:
        ops = list(range(12)) if n >= 2 else [H, X, Y, Z, RX, RY, RZ, U3, ROT]
    # (the controlled rotations CRX, CRY, CRZ are drawn only when ``ops`` lists them)
    if n_params is None:
        n_params = max(1, n_gates)
    g = GateList()
    for _ in range(n_gates):
        op = int(rng.choice(ops))
        nq = N_QUBITS[op]
        qs = [int(v) for v in rng.choice(n, size=nq, replace=False)]
        na = N_ANGLES[op]
        pidx = [int(rng.integers(n_params)) for _ in range(na)]
        ps = [float(rng.choice([1.0, 2.0, -0.5])) for _ in range(na)]
        g.add(op, qs, pidx, ps)
    params = f32_angles(rng, n_params, 0.0, 2 * math.pi)
    return Circuit(n, g.array(), params, 1, zterms([([0], 1.0, 0)]))
