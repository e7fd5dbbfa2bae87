"""CPU checks of the library's host-only entry points against the oracle: the Pauli
decomposition of a Hermitian observable (its terms rebuild the observable's expectation value
on random states) and the lowering of controlled rotations."""
import numpy as np
import pytest

from oracle import sv as osv
from paper_2301_05451_amd import workloads as W


def _hermitian(rng, k):
    a = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
    return a + a.conj().T


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_pauli_decomposition_rebuilds_the_observable(k):
    from paper_2301_05451_amd import lib

    rng = np.random.default_rng(900 + k)
    n = 6
    for _ in range(3):
        h = _hermitian(rng, k)
        qs = [int(q) for q in rng.choice(n, size=k, replace=False)]
        terms = lib.pauli_decompose(h, qs, obs=2)
        assert len(terms) <= 4 ** k and (terms["obs"] == 2).all()
        big = osv.embed(n, h, qs)
        for _ in range(3):
            psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
            psi /= np.linalg.norm(psi)
            want = osv.expval_hermitian(psi, big)
            got = osv.pauli_expvals(psi, n, terms, 3)[2]
            assert abs(got - want) <= 1e-12 * max(1.0, np.abs(h).sum())


def test_pauli_decomposition_of_known_matrices():
    from paper_2301_05451_amd import lib

    x = np.array([[0, 1], [1, 0]], dtype=complex)
    z = np.diag([1.0, -1.0]).astype(complex)
    t = lib.pauli_decompose(np.kron(x, z) * 0.5 + np.eye(4), [4, 1])
    got = {(int(r["x"]), int(r["z"])): float(r["coeff"]) for r in t}
    # X on qubit 4 (first listed), Z on qubit 1, and the identity
    assert got == {(1 << 4, 1 << 1): 0.5, (0, 0): 1.0}
    assert len(lib.pauli_decompose(np.zeros((2, 2)), [0])) == 0
    with pytest.raises(lib.TQError):
        lib.pauli_decompose(np.eye(4), [1, 1])


def test_schedule_shape_without_a_device():
    # the headline circuit's fused schedule as the bench reports it, built with no context
    from paper_2301_05451_amd import lib

    c = W.brickwork()
    info = lib.plan_info(c.n, c.gates, host=True)
    assert (info["sweeps"], info["tile_bits"], info["reg_bits"]) == (14, 12, 4)
    assert info["flops_per_amp"] == 6468
    plain = lib.plan_info(c.n, c.gates, mode=1, host=True)
    assert plain["sweeps"] == len(c.gates)
    rev = lib.plan_info(c.n, c.gates, mode=2, host=True)
    assert rev["sweeps"] >= 1 and rev["tile_bits"] == 12
    with pytest.raises(lib.TQError):
        lib.plan_info(c.n, c.gates, mode=3, host=True)


def test_network_plan_without_a_device():
    from paper_2301_05451_amd import lib
    from paper_2301_05451_amd import tn

    prob = W.qaoa_maxcut(p=3)
    net, _ = tn.qaoa_edge_network(prob, prob.edges[0])
    tree = tn.best_tree(net, seed=0, n_bisect=2)
    p = lib.TnPlan([lf.inds for lf in net.leaves], tree.pairs, tree.sliced, net.output, host_only=True)
    assert p.ctx is None and p.info["flops"] > 0
    assert p.workspace_bytes(True) >= p.workspace_bytes(False) > 0


def test_peak_probe_rejects_bad_arguments_on_the_host():
    """Argument checks of tq_peak_probe run before any launch (the pointer is never used)."""
    import ctypes as ct

    from paper_2301_05451_amd import lib

    w = ct.c_double(0.0)
    dummy = ct.c_void_p(0x1000)
    assert lib._lib.tq_peak_probe(7, dummy, ct.c_uint64(1 << 20), 1, ct.byref(w), None) == 1       # unknown kind
    assert lib._lib.tq_peak_probe(0, dummy, ct.c_uint64(3 << 14), 1, ct.byref(w), None) == 2       # not 32 KiB
    assert lib._lib.tq_peak_probe(0, dummy, ct.c_uint64(0), 1, ct.byref(w), None) == 2
    assert lib._lib.tq_peak_probe(1, dummy, ct.c_uint64(1 << 20), 1, ct.byref(w), None) == 2       # < 2 MiB
    assert lib._lib.tq_peak_probe(3, dummy, ct.c_uint64(1 << 21), 1, ct.byref(w), None) == 2       # < 4 MiB
    assert lib._lib.tq_peak_probe(2, dummy, ct.c_uint64(1 << 21), 0, ct.byref(w), None) == 1       # iters < 1
    assert lib._lib.tq_peak_probe(0, None, ct.c_uint64(1 << 20), 1, ct.byref(w), None) == 1        # null buffer
    assert w.value == 0.0


def test_batched_leaf_calls_reject_bad_arguments_on_the_host():
    """Argument checks of tq_tn_build_leaves_batch / tq_tn_param_grad_batch run before any
    launch: a null context or arrays, a negative count, and a plan that cannot run (planned
    without a device) are refused, the last with the failing network named; an empty batch
    is a no-op. The context pointer below is never dereferenced on these paths."""
    import ctypes as ct

    from paper_2301_05451_amd import lib
    from paper_2301_05451_amd import tn

    dummy = ct.c_void_p(0x1000)
    for f, nargs in ((lib._lib.tq_tn_build_leaves_batch, 9), (lib._lib.tq_tn_param_grad_batch, 9)):
        assert f(None, 0, *([None] * nargs)) == 1           # null context
        assert f(dummy, -1, *([None] * nargs)) == 1         # negative count
        assert f(dummy, 2, *([None] * nargs)) == 1          # null arrays
        assert f(dummy, 0, *([None] * nargs)) == 0          # empty batch
    prob = W.qaoa_maxcut(p=1)
    net, _ = tn.qaoa_edge_network(prob, prob.edges[0])
    tree = tn.elimination_tree(net, tn.elimination_order(net)[0])
    p = lib.TnPlan([lf.inds for lf in net.leaves], tree.pairs, tree.sliced, net.output, host_only=True)
    specs, consts = tn.leaf_specs(net)
    g = np.ascontiguousarray(net.gates, dtype=W.GATE_DTYPE)
    ls = np.ascontiguousarray(specs, dtype=lib.TN_LEAF_DTYPE)
    cv = np.ascontiguousarray(np.asarray(consts, dtype=np.complex128).view(np.float64))
    one = lambda x: lib._ptrs([x])  # noqa: E731
    buf = ct.c_void_p(0x2000)
    st = lib._lib.tq_tn_build_leaves_batch(dummy, 1, one(p.h.value), one(g.ctypes.data), lib._i32s([g.shape[0]]),
                                           one(ls.ctypes.data), one(cv.ctypes.data), lib._i32s([cv.shape[0] // 2]),
                                           one(buf.value), one(buf.value), None)
    assert st != 0 and lib.last_error().startswith("network 0: ")
