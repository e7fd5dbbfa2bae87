"""Tensor-network oracle in complex128 (test infrastructure only; never on the product path).

Follows the paper's tensor-network mode (Sec. 3.2):

* Sec. 3.2.1: a circuit becomes a network whose vertices are the state, gate and
  observable tensors and whose edges are the indices; an expectation value needs the
  circuit followed by its complex-conjugate copy (the worked two-qubit example whose
  contraction gives sin^2(theta/2) - cos^2(theta/2)). Here the network is the plain
  line graph: every gate is one tensor with its output legs first, then input legs.
* Sec. 3.2.1 also notes that the value does not depend on the order of summation; the
  oracle contracts pairwise with ``np.einsum`` in its own greedy order (smallest
  result first).
* Sec. 3.2.3, slicing: fixing the sliced indices to every assignment, contracting each
  identical sub-network and summing the partial results gives the original value.

For QAOA the network is restricted to the reverse light cone of the measured edge
(gates outside it cancel against their conjugates); :func:`qaoa_edge_zz_sv` evaluates
the same quantity by plain state-vector evolution of the cone qubits as a second route.
"""
from __future__ import annotations

import itertools

import numpy as np

from paper_2301_05451_amd import workloads as W

from . import sv


class Net:
    """A list of (array, labels) pairs; labels are ints, every dimension is 2 (or 2**n
    for a user initial state split into n legs)."""

    def __init__(self):
        self.tensors = []
        self._next = 0

    def label(self):
        self._next += 1
        return self._next - 1

    def add(self, arr, labels):
        arr = np.asarray(arr, dtype=np.complex128)
        assert arr.ndim == len(labels), (arr.shape, labels)
        self.tensors.append((arr, list(labels)))


def expectation_network(n, gates, params, zqubits, init=None):
    """Doubled network for <psi|prod_{q in zqubits} Z_q|psi>, psi = U|init>."""
    net = Net()
    ket = [net.label() for _ in range(n)]
    bra = [net.label() for _ in range(n)]
    if init is None:
        e0 = np.array([1.0, 0.0])
        for q in range(n):
            net.add(e0, [ket[q]])
            net.add(e0, [bra[q]])
    else:
        v = sv.initial_state(n, init).reshape((2,) * n)
        net.add(v, list(ket))
        net.add(np.conj(v), list(bra))
    for g in gates:
        qs = sv.gate_qubits(g)
        U = sv.gate_matrix(int(g["op"]), sv.gate_angles(g, params))
        k = len(qs)
        T = U.reshape((2,) * (2 * k))
        kin = [ket[q] for q in qs]
        bin_ = [bra[q] for q in qs]
        kout = [net.label() for _ in qs]
        bout = [net.label() for _ in qs]
        net.add(T, kout + kin)
        net.add(np.conj(T), bout + bin_)
        for i, q in enumerate(qs):
            ket[q] = kout[i]
            bra[q] = bout[i]
    zq = set(zqubits)
    for q in range(n):
        if q in zq:
            net.add(np.array([[1.0, 0.0], [0.0, -1.0]]), [bra[q], ket[q]])
        else:
            net.add(np.eye(2), [bra[q], ket[q]])
    return net


def _pair_out(la, lb, others):
    keep = set()
    for l in others:
        keep |= set(l)
    out = []
    for l in la + lb:
        if l in keep and l not in out:
            out.append(l)
    return out


def contract(tensors, sliced=()):
    """Contract a closed network to a scalar by greedy pairwise einsum. ``sliced`` lists
    labels to fix: the value is the sum over every assignment (paper Sec. 3.2.3)."""
    if sliced:
        total = 0.0 + 0.0j
        for vals in itertools.product((0, 1), repeat=len(sliced)):
            fix = dict(zip(sliced, vals))
            sub = []
            for arr, labels in tensors:
                a, ls = arr, list(labels)
                for lab, v in fix.items():
                    while lab in ls:
                        ax = ls.index(lab)
                        a = np.take(a, v, axis=ax)
                        ls.pop(ax)
                sub.append((a, ls))
            total += contract(sub)
        return total
    ts = [(a, list(l)) for a, l in tensors]
    while len(ts) > 1:
        best = None
        for i in range(len(ts)):
            for j in range(i + 1, len(ts)):
                if not set(ts[i][1]) & set(ts[j][1]):
                    continue
                others = [ts[k][1] for k in range(len(ts)) if k != i and k != j]
                out = _pair_out(ts[i][1], ts[j][1], others)
                size = len(out)
                if best is None or size < best[0]:
                    best = (size, i, j, out)
        if best is None:  # disconnected pieces: outer product of the first two
            i, j = 0, 1
            others = [ts[k][1] for k in range(2, len(ts))]
            out = _pair_out(ts[0][1], ts[1][1], others)
        else:
            _, i, j, out = best
        a, la = ts[i]
        b, lb = ts[j]
        local = {l: i for i, l in enumerate(dict.fromkeys(la + lb))}  # einsum wants labels < 52
        c = np.einsum(a, [local[l] for l in la], b, [local[l] for l in lb], [local[l] for l in out])
        ts = [t for k, t in enumerate(ts) if k not in (i, j)] + [(c, out)]
    a, l = ts[0]
    if l:  # leftover self-traced labels cannot occur in a closed network
        raise ValueError("open labels left in a closed network")
    return complex(a)


def circuit_zexp_tn(c: W.Circuit, zqubits, sliced=(), init=None):
    net = expectation_network(c.n, c.gates, c.params, zqubits, init)
    return contract(net.tensors, sliced)


# ---- QAOA --------------------------------------------------------------------------
#
# The value <Z_i Z_j> only depends on the gates in the reverse causal cone of {i, j}: walking
# the circuit backwards, a gate belongs to the cone iff it touches a qubit already in it, and
# then its qubits join. Every other gate commutes past the observable and meets its own
# inverse in <psi| ... |psi> (the light-cone reduction the paper lists as the first step of
# its tensor-network mode, Sec. 3.2). For a QAOA circuit this cone holds the graph nodes
# within distance p of the edge (each cost layer widens it by one graph step).


def _is_diagonal(g):
    """Whether a gate's matrix (the oracle's own, at a generic angle) is diagonal."""
    U = sv.gate_matrix(int(g["op"]), [0.731, 1.913, 2.377])
    return bool(np.all(U[~np.eye(U.shape[0], dtype=bool)] == 0))


def cone_circuit(c: W.Circuit, qubits):
    """Sub-circuit of the reverse causal cone of ``qubits``, relabelled onto the cone's
    qubits in increasing order. Returns (circuit, cone qubit list).

    Walking backwards, a gate is kept iff it touches the cone, and its qubits join the
    cone. Diagonal gates commute with each other and with a Z-string observable, so a
    maximal run of consecutive diagonal gates is one commuting block: each gate of the
    block is tested against the cone as it stood after the block, and the qubits of the
    kept ones join afterwards (a gate that misses that cone can be moved past the whole
    block and then cancels against its conjugate)."""
    cone = set(int(q) for q in qubits)
    keep = []
    k = len(c.gates) - 1
    while k >= 0:
        if not _is_diagonal(c.gates[k]):
            qs = sv.gate_qubits(c.gates[k])
            if cone.intersection(qs):
                keep.append(k)
                cone.update(qs)
            k -= 1
            continue
        block = []
        while k >= 0 and _is_diagonal(c.gates[k]):
            block.append(k)
            k -= 1
        joined = set()
        for b in block:
            qs = sv.gate_qubits(c.gates[b])
            if cone.intersection(qs):
                keep.append(b)
                joined.update(qs)
        cone |= joined
    order = sorted(cone)
    pos = {q: i for i, q in enumerate(order)}
    keep.sort()
    gates = c.gates[np.array(keep, dtype=np.int64)].copy() if keep else c.gates[:0].copy()
    for k in range(len(gates)):
        nq = W.N_QUBITS[int(gates[k]["op"])]
        gates["q"][k, :nq] = [pos[int(q)] for q in gates["q"][k, :nq]]
    return W.Circuit(len(order), gates, c.params.copy()), order


def graph_ball(n, edges, centre, radius):
    """Graph nodes within ``radius`` steps of any node of ``centre`` (breadth-first)."""
    nbr = [[] for _ in range(n)]
    for a, b in edges:
        nbr[a].append(b)
        nbr[b].append(a)
    dist = {int(v): 0 for v in centre}
    frontier = list(dist)
    for d in range(1, radius + 1):
        nxt = []
        for v in frontier:
            for w in nbr[v]:
                if w not in dist:
                    dist[w] = d
                    nxt.append(w)
        frontier = nxt
    return sorted(dist)


def qaoa_cone(prob: W.QAOAProblem, edge, gammas=None, betas=None):
    """(cone circuit, position of edge[0], position of edge[1], cone qubits)."""
    pr = prob if gammas is None else W.QAOAProblem(prob.n, prob.edges, prob.p, np.asarray(gammas),
                                                    np.asarray(betas))
    c, order = cone_circuit(W.qaoa_circuit(pr), edge)
    return c, order.index(edge[0]), order.index(edge[1]), order


def qaoa_edge_zz_sv(prob: W.QAOAProblem, edge, gammas=None, betas=None):
    """<Z_i Z_j> for one edge by state-vector evolution of its light-cone qubits."""
    c, i, j, _ = qaoa_cone(prob, edge, gammas, betas)
    psi = sv.run(c.n, c.gates, c.params)
    return float(np.dot(np.abs(psi) ** 2, sv.zstring_diag(c.n, [i, j])))


def qaoa_edge_zz_tn(prob: W.QAOAProblem, edge, sliced_count=0):
    """<Z_i Z_j> for one edge by contracting the light-cone doubled network; optionally
    slicing the first ``sliced_count`` labels of the initial ket legs."""
    c, i, j, _ = qaoa_cone(prob, edge)
    net = expectation_network(c.n, c.gates, c.params, [i, j])
    sliced = list(range(sliced_count))
    return contract(net.tensors, sliced)


def qaoa_full_zz_sv(prob: W.QAOAProblem, edge):
    """<Z_i Z_j> from the whole register (no light cone): only for small graphs."""
    c = W.qaoa_circuit(prob)
    psi = sv.run(c.n, c.gates, c.params)
    return float(np.dot(np.abs(psi) ** 2, sv.zstring_diag(c.n, list(edge))))
