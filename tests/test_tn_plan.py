"""CPU tests of the tensor-network planner (network construction with hyperedges, trees,
slicing, FLOP count) against the oracle. The planner's network is contracted here with
numpy along the planner's own tree; the oracle computes the same value by its own route."""
import math

import numpy as np
import pytest

from oracle import sv as osv
from oracle import tn as otn
from paper_2301_05451_amd import tn
from paper_2301_05451_amd import workloads as W


def _leaf_value(net, lf):
    """Leaf tensor of the planner's network (built here with the oracle's gate matrices;
    element e holds entry e ^ flip)."""
    if lf.kind == tn.LEAF_CONST:
        v = np.asarray(lf.value, dtype=np.complex128)
    else:
        g = net.gates[lf.gate]
        U = osv.gate_matrix(int(g["op"]), osv.gate_angles(g, net.params))
        if lf.kind in (tn.LEAF_DIAG1, tn.LEAF_DIAG2):
            v = np.diag(U).copy()
        else:
            v = U.reshape(-1)
        v = np.conj(v) if lf.conj else v
    return v[np.arange(v.size) ^ lf.flip]


def _numpy_contract(net, tree):
    ts = [(_leaf_value(net, lf).reshape((2,) * len(lf.inds)), list(lf.inds)) for lf in net.leaves]
    for (a, b), (ia, ib, io) in zip(tree.pairs, tn.tree_steps(net, tree, sliced=[])):
        A, la = ts[a]
        B, lb = ts[b]
        loc = {l: i for i, l in enumerate(dict.fromkeys(la + lb))}
        C = np.einsum(A, [loc[l] for l in la], B, [loc[l] for l in lb], [loc[l] for l in io])
        ts.append((C, list(io)))
    return complex(ts[-1][0])


def test_flops_formula_two_tensor_cases():
    # Sec. 3.2.2: FLOPs = p(2q - 1); A_ab B_bc -> C_ac: p = 4, q = 2 -> 12; outer product: q = 1 -> p
    assert tn.step_flops(("a", "b"), ("b", "c"), ("a", "c")) == 4 * (2 * 2 - 1)
    assert tn.step_flops(("a",), ("c",), ("a", "c")) == 4
    assert tn.step_flops(("a", "b"), ("a", "b"), ()) == 1 * (2 * 4 - 1)


@pytest.mark.parametrize("seed", range(4))
def test_network_and_trees_match_oracle(seed):
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(2, 6))
    c = W.random_circuit(n, 20, rng)
    zq = [0] if n == 1 else [0, n - 1]
    net = tn.circuit_network(c, zq)
    psi = osv.run(n, c.gates, c.params)
    want = float(np.dot(np.abs(psi) ** 2, osv.zstring_diag(n, zq)))
    for tree in (tn.greedy_tree(net), tn.elimination_tree(net, tn.elimination_order(net)[0]),
                 tn.elimination_tree(net, tn.elimination_order(net, np.random.default_rng(1), "degree")[0])):
        assert sorted(i for p in tree.pairs for i in p) == list(range(2 * len(net.leaves) - 2))
        v = _numpy_contract(net, tree)
        assert abs(v.real - want) < 1e-12 and abs(v.imag) < 1e-12


def test_qaoa_light_cone_network():
    rng = np.random.default_rng(3)
    edges = W.random_regular_graph(3, 12, rng)
    prob = W.QAOAProblem(12, edges, 2, W.f32_angles(rng, 2, 0, math.pi), W.f32_angles(rng, 2, 0, math.pi))
    for e in edges[:4]:
        net, cone = tn.qaoa_edge_network(prob, e)
        assert cone == otn.qaoa_cone(prob, e)[3]
        v = _numpy_contract(net, tn.elimination_tree(net, tn.elimination_order(net)[0]))
        assert abs(v.real - otn.qaoa_edge_zz_sv(prob, e)) < 1e-12


def test_slicing_reaches_target_and_keeps_tree():
    prob = W.qaoa_maxcut(p=3)
    net, _ = tn.qaoa_edge_network(prob, prob.edges[0])
    t = tn.elimination_tree(net, tn.elimination_order(net)[0])
    target = max(4, t.max_rank - 4)
    s = tn.slice_tree(net, t, target)
    assert s.pairs == t.pairs and len(s.sliced) >= 1
    ranks = [len(o) for _, _, o in tn.tree_steps(net, s)]
    assert max(ranks) <= target
    assert s.flops == pytest.approx(sum(tn.step_flops(*st) for st in tn.tree_steps(net, s)) * 2 ** len(s.sliced))


def test_candidate_trees_are_valid():
    prob = W.qaoa_maxcut(p=2)
    net, _ = tn.qaoa_edge_network(prob, prob.edges[3])
    cands = tn.candidate_trees(net, n_random=5, seed=2, target_rank=10)
    assert len(cands) == 8
    for t in cands:
        assert sorted(i for p in t.pairs for i in p) == list(range(2 * len(net.leaves) - 2))
        assert t.max_rank >= 0 and t.flops > 0


def test_bisection_trees_are_valid_and_exact():
    """Recursive-bisection trees (after rank simplification) use every tensor once and give
    the oracle's value when contracted along them."""
    rng = np.random.default_rng(5)
    edges = W.random_regular_graph(3, 10, rng)
    prob = W.QAOAProblem(10, edges, 2, W.f32_angles(rng, 2, 0, math.pi), W.f32_angles(rng, 2, 0, math.pi))
    for e in edges[:3]:
        net, _ = tn.qaoa_edge_network(prob, e)
        for seed, imb, leaf in ((0, 0.1, 4), (1, 0.3, 8), (2, 0.2, 3)):
            t = tn.bisection_tree(net, np.random.default_rng(seed), imbalance=imb, leaf_size=leaf)
            assert sorted(i for p in t.pairs for i in p) == list(range(2 * len(net.leaves) - 2))
            v = _numpy_contract(net, t)
            assert abs(v.real - otn.qaoa_edge_zz_sv(prob, e)) < 1e-12 and abs(v.imag) < 1e-12


def test_rank_simplification_never_grows_a_tensor():
    prob = W.qaoa_maxcut(p=2)
    net, _ = tn.qaoa_edge_network(prob, prob.edges[4])
    pairs, live = tn.rank_simplify(net)
    assert len(live) + len(pairs) == len(net.leaves) and len(live) < len(net.leaves) // 2
    t = tn.bisection_tree(net)
    steps = tn.tree_steps(net, t)
    for a, b, o in steps[:len(pairs)]:
        assert len(o) <= max(len(a), len(b))


def test_path_search_pool_and_slicing_search():
    prob = W.qaoa_maxcut(p=3)
    net, _ = tn.qaoa_edge_network(prob, prob.edges[2])
    pool = tn.tree_pool(net, seed=1, n_bisect=2)
    best = tn.best_tree(net, seed=1, n_bisect=2)
    assert best.flops == min(t.flops for t in pool)
    target = max(4, best.max_rank - 3)
    s = tn.slice_search(net, best, target, trials=3, rng=np.random.default_rng(0))
    assert s.pairs == best.pairs and max(len(o) for _, _, o in tn.tree_steps(net, s)) <= target
    assert s.flops <= tn.slice_tree(net, best, target).flops
