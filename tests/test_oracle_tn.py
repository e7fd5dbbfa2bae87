"""Pins of the tensor-network oracle: paper's worked example, SV route, slicing identity."""
import math

import numpy as np
import pytest

from oracle import sv, tn
from paper_2301_05451_amd import workloads as W


@pytest.mark.parametrize("theta", [0.3, 1.7, 2.9])
def test_worked_example_as_network(theta):
    g = W.GateList().const(W.X, [0]).const(W.RY, [1], [theta]).add(W.CNOT, [0, 1])
    c = W.Circuit(2, g.array(), np.zeros(1))
    T = tn.circuit_zexp_tn(c, [1])
    assert abs(T.real - (math.sin(theta / 2) ** 2 - math.cos(theta / 2) ** 2)) < 1e-14
    assert abs(T.imag) < 1e-14


@pytest.mark.parametrize("seed", range(4))
def test_tn_equals_sv_random(seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(2, 6))
    c = W.random_circuit(n, 18, rng)
    zq = [0, n - 1] if n > 1 else [0]
    psi = sv.run(n, c.gates, c.params)
    want = float(np.dot(np.abs(psi) ** 2, sv.zstring_diag(n, zq)))
    T = tn.circuit_zexp_tn(c, zq)
    assert abs(T.real - want) < 1e-12 and abs(T.imag) < 1e-12


def test_sliced_equals_unsliced():
    rng = np.random.default_rng(7)
    c = W.random_circuit(4, 16, rng)
    net = tn.expectation_network(c.n, c.gates, c.params, [1, 2])
    full = tn.contract(net.tensors)
    # slice three internal labels (any labels work: the sum over assignments is exact)
    labels = sorted({l for _, ls in net.tensors for l in ls})
    for sl in ([labels[5]], [labels[3], labels[9]], labels[10:13]):
        assert abs(tn.contract(net.tensors, sliced=sl) - full) < 1e-12


def test_user_initial_state_network():
    rng = np.random.default_rng(8)
    c = W.random_circuit(3, 10, rng)
    v = rng.normal(size=8) + 1j * rng.normal(size=8)
    psi = sv.run(3, c.gates, c.params, init=v)
    want = float(np.dot(np.abs(psi) ** 2, sv.zstring_diag(3, [2])))
    assert abs(tn.circuit_zexp_tn(c, [2], init=v) - want) < 1e-12


def _small_qaoa(n=10, p=2, seed=11):
    rng = np.random.default_rng(seed)
    edges = W.random_regular_graph(3, n, rng)
    gam = W.f32_angles(rng, p, 0, math.pi)
    bet = W.f32_angles(rng, p, 0, math.pi)
    return W.QAOAProblem(n, edges, p, gam, bet)


def test_qaoa_light_cone_equals_full_register():
    prob = _small_qaoa()
    for e in prob.edges[:5]:
        full = tn.qaoa_full_zz_sv(prob, e)
        cone = tn.qaoa_edge_zz_sv(prob, e)
        assert abs(full - cone) < 1e-12


def test_qaoa_tn_equals_cone_sv():
    prob = _small_qaoa(n=8, p=1, seed=12)
    for e in prob.edges[:3]:
        a = tn.qaoa_edge_zz_tn(prob, e, sliced_count=2)
        b = tn.qaoa_edge_zz_sv(prob, e)
        assert abs(a.real - b) < 1e-12 and abs(a.imag) < 1e-12


def test_qaoa_zero_angle_cases():
    prob = _small_qaoa(n=8, p=2, seed=13)
    e = prob.edges[0]
    z = np.zeros(prob.p)
    assert abs(tn.qaoa_edge_zz_sv(prob, e, gammas=z, betas=prob.betas)) < 1e-14
    assert abs(tn.qaoa_edge_zz_sv(prob, e, gammas=prob.gammas, betas=z)) < 1e-14


def test_qaoa_p1_closed_form():
    # p = 1 with RZZ(g) = exp(-i g ZZ/2) and RX(2b) (the textbook analytic p = 1 result,
    # rewritten for this sign convention):
    # <Z_u Z_v> = (1/2) sin(4b) sin(g) (cos^du g + cos^dv g)
    #           + (1/2) sin^2(2b) cos^(du+dv-2t) g (1 - cos^t 2g)
    # du, dv = neighbours of u, v other than each other; t = triangles through (u, v).
    rng = np.random.default_rng(21)
    n = 8
    edges = W.random_regular_graph(3, n, rng)
    adj = {v: set() for v in range(n)}
    for a, b in edges:
        adj[a].add(b); adj[b].add(a)
    for g, b in ((0.61, 0.37), (2.3, 1.1)):
        prob = W.QAOAProblem(n, edges, 1, np.array([g]), np.array([b]))
        for (u, v) in edges:
            du, dv = len(adj[u]) - 1, len(adj[v]) - 1
            t = len(adj[u] & adj[v])
            want = (0.5 * math.sin(4 * b) * math.sin(g) * (math.cos(g) ** du + math.cos(g) ** dv)
                    + 0.5 * math.sin(2 * b) ** 2 * math.cos(g) ** (du + dv - 2 * t) * (1 - math.cos(2 * g) ** t))
            assert abs(tn.qaoa_edge_zz_sv(prob, (u, v)) - want) < 1e-12, (u, v)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_qaoa_cone_is_graph_ball(p):
    # the reverse causal cone of an edge holds exactly the nodes within distance p
    prob = W.qaoa_maxcut(p=p)
    for e in prob.edges[::7]:
        _, i, j, order = tn.qaoa_cone(prob, e)
        assert order == tn.graph_ball(prob.n, prob.edges, e, p)
        assert (order[i], order[j]) == tuple(e)


def test_qaoa_p3_cone_equals_full_register():
    rng = np.random.default_rng(31)
    n = 12
    edges = W.random_regular_graph(3, n, rng)
    prob = W.QAOAProblem(n, edges, 3, W.f32_angles(rng, 3, 0, math.pi), W.f32_angles(rng, 3, 0, math.pi))
    for e in edges[:6]:
        assert abs(tn.qaoa_full_zz_sv(prob, e) - tn.qaoa_edge_zz_sv(prob, e)) < 1e-12


@pytest.mark.parametrize("seed", range(5))
def test_cone_circuit_keeps_value_random(seed):
    # random circuits over all gate types (with runs of diagonal gates): the value of a
    # Z-string on one or two qubits is the same from the cone and from the whole register
    rng = np.random.default_rng(400 + seed)
    n = 7
    c = W.random_circuit(n, 12, rng)
    for zq in ([0], [2, 5], [6]):
        full = sv.run(n, c.gates, c.params)
        want = float(np.dot(np.abs(full) ** 2, sv.zstring_diag(n, zq)))
        cc, order = tn.cone_circuit(c, zq)
        psi = sv.run(cc.n, cc.gates, cc.params)
        got = float(np.dot(np.abs(psi) ** 2, sv.zstring_diag(cc.n, [order.index(q) for q in zq])))
        assert abs(got - want) < 1e-12
