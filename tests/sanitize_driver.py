"""Drives the library's host-side planners through the C ABI for the sanitizer test: it is
run in a child process on the host-only build with AddressSanitizer and
UndefinedBehaviorSanitizer (see test_host_sanitize.py), so any out-of-bounds access, use
after free or undefined behaviour in the host C++ aborts it. Needs no GPU: every call here
is host-only (gate lowering, Pauli decomposition, schedule construction without a context,
tensor-network plans without a context).

Usage: TQ_LIBRARY=<sanitized library> LD_PRELOAD=<ASan runtime> python tests/sanitize_driver.py
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2301_05451_amd import lib  # noqa: E402
from paper_2301_05451_amd import tn  # noqa: E402
from paper_2301_05451_amd import workloads as W  # noqa: E402

ALL_OPS = list(range(15))


def schedules(rng):
    count = 0
    circuits = [W.brickwork(), W.hea_ring(), W.Circuit(16, W.qnn_structure(), None, 1, None)]
    circuits += W.uneven_batch(count=12, seed=77)
    for _ in range(60):
        n = int(rng.integers(1, 23))
        ops = ALL_OPS if n >= 2 else [W.H, W.X, W.Y, W.Z, W.RX, W.RY, W.RZ, W.U3, W.ROT]
        circuits.append(W.random_circuit(n, int(rng.integers(0, 160)), rng, ops=ops))
    for c in circuits:
        gates = c.gates
        low = lib.lower_gates(gates)
        assert len(low) >= len(gates)
        for c128 in (False, True):
            for mode in (0, 1, 2):
                lib.plan_info(c.n, gates, c128, mode, host=True)
                count += 1
            # a few explicit shapes, valid or not (invalid ones must fail cleanly)
            for _ in range(3):
                t = int(rng.integers(1, 15))
                r = int(rng.integers(1, 6))
                cb = int(rng.integers(0, 11))
                for mode in (0, 2):
                    try:
                        lib.plan_info(c.n, gates, c128, mode, t, r, cb, host=True)
                        count += 1
                    except lib.TQError:
                        pass
    # malformed gate lists are rejected
    bad = W.random_circuit(4, 10, rng).gates.copy()
    bad[3]["q"][0] = 9
    for g in (bad,):
        try:
            lib.plan_info(4, g, host=True)
            raise AssertionError("an out-of-range qubit was accepted")
        except lib.TQError:
            pass
    return count


def decompositions(rng):
    for k in range(1, 6):
        a = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
        qs = [int(q) for q in rng.choice(40, size=k, replace=False)]
        t = lib.pauli_decompose(a + a.conj().T, qs)
        assert len(t) <= 4 ** k
    return 5


def plans(rng):
    count = 0
    nets = []
    for _ in range(8):
        n = int(rng.integers(3, 10))
        c = W.random_circuit(n, int(rng.integers(10, 50)), rng, ops=ALL_OPS)
        net = tn.circuit_network(c, [int(rng.integers(n))])
        nets.append(net)
    prob = W.qaoa_maxcut(p=3)
    for e in prob.edges[:3]:
        nets.append(tn.qaoa_edge_network(prob, e)[0])
    prob4 = W.qaoa_maxcut(p=4)
    nets.append(tn.qaoa_edge_network(prob4, prob4.edges[0])[0])
    for k, net in enumerate(nets):
        trees = tn.tree_pool(net, seed=k, n_bisect=2)
        wide = max(trees, key=lambda t: t.max_rank)
        trees.append(tn.slice_search(net, wide, max(4, wide.max_rank - 4), 2, np.random.default_rng(k)))
        for tree in trees:
            leaf_inds = [lf.inds for lf in net.leaves]
            for c128 in (False, True):
                for group, policy in ((0, lib.TN_RECOMPUTE), (1, lib.TN_AUTO), (0, lib.TN_STORE)):
                    try:
                        p = lib.TnPlan(leaf_inds, tree.pairs, tree.sliced, net.output, c128, group,
                                       mem_budget=int(rng.choice([0, 1 << 20])), store_policy=policy,
                                       host_only=True)
                    except lib.TQError:
                        continue  # e.g. STORE over a budget that cannot hold every slice
                    p.workspace_bytes(False)
                    p.workspace_bytes(True)
                    count += 1
    # a tree (of the required n_leaves - 1 steps) that uses one tensor twice is rejected
    net = nets[0]
    tree = tn.tree_pool(net, 0, 0)[0]
    bad = [tuple(p) for p in tree.pairs]
    bad[-1] = bad[0]
    try:
        lib.TnPlan([lf.inds for lf in net.leaves], bad, (), net.output, host_only=True)
        raise AssertionError("a tree that consumes a tensor twice was accepted")
    except lib.TQError:
        pass
    return count


def main():
    rng = np.random.default_rng(2301)
    s = schedules(rng)
    print(f"sanitize driver: {s} schedules", flush=True)
    d = decompositions(rng)
    print(f"sanitize driver: {d} decompositions", flush=True)
    p = plans(rng)
    print(f"sanitize driver: {p} network plans", flush=True)
    print("sanitize driver: done", flush=True)


if __name__ == "__main__":
    main()
