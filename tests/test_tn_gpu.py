"""GPU parity of the tensor-network path (tq_tn_build_leaves, tq_tn_contract,
tq_tn_backward, tq_tn_param_grad) against the oracle: the paper's worked example, random
circuits vs state-vector values and parameter-shift gradients, QAOA light cones (sliced
and unsliced, several slice groups), and a dense step on the FP32-MFMA GEMM path vs einsum."""
import math

import numpy as np
import pytest

from oracle import sv as osv
from oracle import tn as otn
from paper_2301_05451_amd import tn
from paper_2301_05451_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _params(net, c128):
    return torch.tensor(net.params, dtype=torch.float64 if c128 else torch.float32, device="cuda")


@pytest.mark.parametrize("theta", [0.3, 1.7, 2.9])
def test_worked_example_tn_gpu(theta):
    g = W.GateList().const(W.X, [0]).const(W.RY, [1], [theta]).add(W.CNOT, [0, 1])
    c = W.Circuit(2, g.array(), np.zeros(1))
    net = tn.circuit_network(c, [1])
    prog = tn.TNProgram(net, tn.elimination_tree(net, tn.elimination_order(net)[0]), c128=True)
    v = prog.value(_params(net, True)).cpu().numpy()[0]
    assert abs(v.real - (math.sin(theta / 2) ** 2 - math.cos(theta / 2) ** 2)) < 1e-14 and abs(v.imag) < 1e-14


@pytest.mark.parametrize("c128", [False, True])
def test_random_circuits_value_and_grad(c128):
    tol = 1e-12 if c128 else 1e-5
    rng = np.random.default_rng(60)
    for n in (3, 5, 7):
        c = W.random_circuit(n, 30, rng, n_params=10)
        zq = [0, n - 1]
        net = tn.circuit_network(c, zq)
        print(f"tn random n={n} c128={c128}", flush=True)
        prog = tn.TNProgram(net, tn.greedy_tree(net), c128=c128)
        p = _params(net, c128)
        v = prog.value(p).cpu().numpy()[0]
        psi = osv.run(n, c.gates, c.params)
        want = float(np.dot(np.abs(psi) ** 2, osv.zstring_diag(n, zq)))
        assert abs(v.real - want) <= tol and abs(v.imag) <= tol
        g = prog.grad(p).cpu().numpy()
        c.terms, c.n_obs = W.zterms([(zq, 1.0, 0)]), 1
        assert np.abs(g - osv.param_shift_grad(c)).max() <= tol


@pytest.mark.parametrize("c128", [False, True])
def test_anti_diagonal_reduction_value_and_grad(c128):
    """Circuits rich in X and Y: those gates become wire flips (no tensors), and the later
    tensors on a flipped wire, including parameterised ones and the Z observable, are built
    with that index complemented; values and gradients against the oracle."""
    tol = 1e-12 if c128 else 1e-5
    rng = np.random.default_rng(61)
    ops = [W.X, W.Y, W.X, W.Y, W.RX, W.RY, W.RZ, W.U3, W.CNOT, W.CZ, W.RZZ, W.H]
    for n in (2, 4, 6):
        c = W.random_circuit(n, 36, rng, ops=ops, n_params=8)
        zq = [n - 1] if n == 2 else [0, n // 2]
        net = tn.circuit_network(c, zq)
        assert any(lf.flip for lf in net.leaves)
        n_xy = int(np.isin(c.gates["op"], [W.X, W.Y]).sum())
        assert len(net.leaves) < 2 * (len(c.gates) - n_xy) + 2 * n + len(zq) + 2 * n_xy
        print(f"tn flips n={n} c128={c128}", flush=True)
        prog = tn.TNProgram(net, tn.greedy_tree(net), c128=c128)
        p = _params(net, c128)
        v = prog.value(p).cpu().numpy()[0]
        psi = osv.run(n, c.gates, c.params)
        want = float(np.dot(np.abs(psi) ** 2, osv.zstring_diag(n, zq)))
        assert abs(v.real - want) <= tol and abs(v.imag) <= tol
        g = prog.grad(p).cpu().numpy()
        c.terms, c.n_obs = W.zterms([(zq, 1.0, 0)]), 1
        assert np.abs(g - osv.param_shift_grad(c)).max() <= 2 * tol


def _qaoa10():
    r = np.random.default_rng(11)
    edges = W.random_regular_graph(3, 10, r)
    return W.QAOAProblem(10, edges, 2, W.f32_angles(r, 2, 0, math.pi), W.f32_angles(r, 2, 0, math.pi))


def test_qaoa_sliced_unsliced_groups_and_grad():
    prob = _qaoa10()
    for e in prob.edges[:3]:
        net, cone = tn.qaoa_edge_network(prob, e)
        t0 = tn.elimination_tree(net, tn.elimination_order(net)[0])
        ts = tn.slice_tree(net, t0, max(2, t0.max_rank - 3))
        want = otn.qaoa_edge_zz_sv(prob, e)
        c, i, j, _ = otn.qaoa_cone(prob, e)
        c.terms, c.n_obs = W.zterms([([i, j], 1.0, 0)]), 1
        gw = osv.param_shift_grad(c)
        for tree, G in ((t0, 0), (ts, 0), (ts, 2), (ts, 1)):
            print(f"qaoa {e} sliced={len(tree.sliced)} G={G}", flush=True)
            prog = tn.TNProgram(net, tree, slice_group=G)
            p = _params(net, False)
            v = prog.value(p).cpu().numpy()[0]
            assert abs(v.real - want) <= 1e-5 and abs(v.imag) <= 1e-5
            assert np.abs(prog.grad(p).cpu().numpy() - gw).max() <= 1e-5


def test_autograd_tn_expval():
    prob = _qaoa10()
    e = prob.edges[5]
    net, cone = tn.qaoa_edge_network(prob, e)
    prog = tn.TNProgram(net, tn.elimination_tree(net, tn.elimination_order(net)[0]))
    p = _params(net, False).requires_grad_(True)
    f = tn.tn_expval(prog, p)
    (3.0 * f).backward()
    c, i, j, _ = otn.qaoa_cone(prob, e)
    c.terms, c.n_obs = W.zterms([([i, j], 1.0, 0)]), 1
    assert abs(f.item() - otn.qaoa_edge_zz_sv(prob, e)) <= 1e-5
    assert np.abs(p.grad.cpu().numpy() - 3.0 * osv.param_shift_grad(c)).max() <= 3e-5


def test_qaoa50_p3_edges_vs_cone_state_vector():
    """50-node 3-regular graph, p = 3: edges whose light cone has <= 20 qubits, against the
    oracle's state-vector evolution of the cone."""
    prob = W.qaoa_maxcut(p=3)
    done = 0
    for e in prob.edges:
        net, cone = tn.qaoa_edge_network(prob, e)
        if len(cone) > 20:
            continue
        prog = tn.TNProgram(net, tn.elimination_tree(net, tn.elimination_order(net)[0]))
        v = prog.value(_params(net, False)).cpu().numpy()[0]
        assert abs(v.real - otn.qaoa_edge_zz_sv(prob, e)) <= 1e-5, e
        done += 1
        if done == 4:
            break
    assert done >= 1


def _gemm_network(rs, permuted, mb=7, kb=5, nb=6):
    b = [0]
    m = list(range(1, 1 + mb))
    k = list(range(1 + mb, 1 + mb + kb))
    nn = list(range(1 + mb + kb, 1 + mb + kb + nb))
    ra, rb, rc = 1 + mb + kb, 1 + kb + nb, 1 + mb + nb
    A = (rs.normal(size=2 ** ra) + 1j * rs.normal(size=2 ** ra))
    B = (rs.normal(size=2 ** rb) + 1j * rs.normal(size=2 ** rb))
    Cc = (rs.normal(size=2 ** rc) + 1j * rs.normal(size=2 ** rc))
    if permuted:
        inds = [k[::-1] + m + b, nn + b + k, m[::-1] + nn + b]
    else:
        inds = [b + m + k, b + k + nn, b + m + nn]
    return (A, B, Cc), inds


@pytest.mark.parametrize("shape", [(7, 5, 6), (6, 7, 5)])
@pytest.mark.parametrize("c128", [False, True])
@pytest.mark.parametrize("permuted", [False, True])
def test_dense_step_on_mfma_gemm_path(permuted, c128, shape):
    """A dense step on the MFMA complex GEMM (FP32 for complex64, FP64 for complex128). Shape
    = (bits of M, K, N) with a batch of 2: M = 128, N = 64 runs the FP32 product's 128 x 128
    tile, M = 64, N = 32 its 64 x 64 tile."""
    from paper_2301_05451_amd import lib

    mb, kb, nb = shape
    rs = np.random.default_rng(3)
    (A, B, Cc), inds = _gemm_network(rs, permuted, mb, kb, nb)
    plan = lib.TnPlan(inds, [(0, 1), (2, 3)], c128=c128)
    assert plan.info["gemm_steps"] == 1
    cdt = torch.complex128 if c128 else torch.complex64
    tol = 1e-12 if c128 else 1e-5
    leaves = torch.tensor(np.concatenate([A, B, Cc]), dtype=cdt, device="cuda")
    v = lib.tn_contract(plan, leaves).cpu().numpy()[0]
    At, Bt, Ct = (t.reshape((2,) * len(i)) for t, i in zip((A, B, Cc), inds))
    want = np.einsum(At, inds[0], Bt, inds[1], Ct, inds[2], [])
    assert abs(v - want) / abs(want) <= tol
    env = lib.tn_backward(plan, leaves, torch.ones(1, dtype=cdt, device="cuda")).cpu().numpy()
    envA = np.einsum(Bt, inds[1], Ct, inds[2], inds[0]).reshape(-1)
    assert np.abs(env[: A.size] - envA).max() / np.abs(envA).max() <= tol


def test_plan_validation():
    from paper_2301_05451_amd import lib

    with pytest.raises(lib.TQError):
        lib.TnPlan([[0, 1], [1, 0]], [(0, 0)])  # a tree step reusing an id
    with pytest.raises(lib.TQError):
        lib.TnPlan([[0, 1], [1, 2]], [(0, 1)], sliced=[7])  # sliced index in no leaf
    with pytest.raises(lib.TQError):
        lib.TnPlan([[0, 1], [1, 2]], [(0, 1)], out_inds=[5])  # no tensor carries index 5
    # a plan built without a context has the same shape as a device plan and cannot run
    host = lib.TnPlan([[0, 1], [1, 2]], [(0, 1)], out_inds=[0, 2], host_only=True)
    dev = lib.TnPlan([[0, 1], [1, 2]], [(0, 1)], out_inds=[0, 2])
    assert host.info == dev.info and host.workspace_bytes(True) == dev.workspace_bytes(True)
    leaves = torch.ones(8, dtype=torch.complex64, device="cuda")
    assert torch.allclose(lib.tn_contract(dev, leaves).cpu(), torch.full((4,), 2, dtype=torch.complex64))
    with pytest.raises(lib.TQError):
        lib.tn_contract(host, leaves)


@pytest.mark.parametrize("c128", [False, True])
@pytest.mark.parametrize("case", ["scalar18", "out14"])
def test_wide_direct_steps(case, c128):
    """Large steps on the generic kernel: a scalar from 18 summed indices (256 lanes per
    output, reduced through LDS) and a 14-index output with 4 summed indices; values and
    the reverse pass against einsum."""
    from paper_2301_05451_amd import lib

    if case == "scalar18":
        inds, outi = [list(range(18)), list(range(18))], []
    else:
        inds, outi = [list(range(16)), list(range(12, 18))], list(range(12)) + [16, 17]
    rs = np.random.default_rng(8)
    ra, rb = len(inds[0]), len(inds[1])
    A = rs.normal(size=2 ** ra) + 1j * rs.normal(size=2 ** ra)
    B = rs.normal(size=2 ** rb) + 1j * rs.normal(size=2 ** rb)
    cdt = torch.complex128 if c128 else torch.complex64
    plan = lib.TnPlan(inds, [(0, 1)], out_inds=outi, c128=c128)
    assert plan.info["gemm_steps"] == 0
    leaves = torch.tensor(np.concatenate([A, B]), dtype=cdt, device="cuda")
    v = lib.tn_contract(plan, leaves).cpu().numpy()
    want = np.einsum(A.reshape((2,) * ra), inds[0], B.reshape((2,) * rb), inds[1], outi).reshape(-1)
    tol = 1e-12 if c128 else 1e-5
    assert np.abs(v - want).max() <= tol * np.abs(want).max()
    g = np.ones(1) if not outi else rs.normal(size=v.size)
    env = lib.tn_backward(plan, leaves, torch.tensor(g, dtype=cdt, device="cuda")).cpu().numpy()
    envA = np.einsum(g.reshape((2,) * len(outi)) if outi else np.array(1.0), outi, B.reshape((2,) * rb), inds[1],
                     inds[0]).reshape(-1)
    assert np.abs(env[:2 ** ra] - envA).max() <= tol * np.abs(envA).max()


def test_qaoa50_p4_narrowest_edge_sliced_vs_unsliced():
    """p = 4 on the 50-node graph: the edge whose min-fill tree is narrowest (a 33-qubit
    light cone, width 20 at this seed; too large for the oracle's state vector): the value
    unsliced and with the same tree sliced (Sec. 3.2.3: the sum over slices is the value),
    real to float32 precision and within [-1, 1]."""
    prob = W.qaoa_maxcut(p=4)
    best = None
    for e in prob.edges:
        net, cone = tn.qaoa_edge_network(prob, e)
        tr = tn.elimination_tree(net, tn.elimination_order(net, None, "fill")[0])
        if best is None or tr.max_rank < best[2].max_rank:
            best = (e, net, tr, cone)
    e, net, tr, cone = best
    print(f"p4 edge {e} cone {len(cone)} width {tr.max_rank}", flush=True)
    p = _params(net, False)
    v1 = tn.TNProgram(net, tr).value(p).cpu().numpy()[0]
    tr2 = tn.slice_tree(net, tr, tr.max_rank - 3)
    assert len(tr2.sliced) >= 1
    v2 = tn.TNProgram(net, tr2).value(p).cpu().numpy()[0]
    assert abs(v1.imag) <= 1e-5 and abs(v1 - v2) <= 2e-5
    assert abs(v1.real) <= 1.0 + 1e-5


@pytest.mark.parametrize("c128", [False, True])
def test_batched_networks_match_single_calls_and_oracle(c128):
    """tq_tn_contract_batch / tq_tn_backward_batch over the 75 light-cone networks of the
    p = 2 QAOA problem on a 50-node graph plus six sliced networks (which take the one-by-one
    route, on several streams): values and gradients equal the single-network calls, and
    values match the cone state vector of the oracle on sampled edges."""
    prob = W.qaoa_maxcut(p=2)
    progs, pars = [], []
    for e in prob.edges:
        net, _ = tn.qaoa_edge_network(prob, e)
        progs.append(tn.TNProgram(net, tn.elimination_tree(net, tn.elimination_order(net)[0]), c128=c128))
        pars.append(_params(net, c128))
    for e in prob.edges[:6]:  # sliced copies: the one-by-one route, spread over the stream pool
        net0, _ = tn.qaoa_edge_network(prob, e)
        t0 = tn.elimination_tree(net0, tn.elimination_order(net0)[0])
        progs.append(tn.TNProgram(net0, tn.slice_tree(net0, t0, max(2, t0.max_rank - 2)), c128=c128))
        pars.append(_params(net0, c128))
    batch = tn.TNBatch(progs)
    vals = [v.cpu().numpy() for v in batch.values(pars)]
    grads = [g.cpu().numpy() for g in batch.grads(pars)]
    for rep in range(2):  # one leaf build for both passes, the shared unit upstream reused
        v2, g2 = batch.value_and_grads(pars)
        for k in range(len(progs)):
            assert np.array_equal(v2[k].cpu().numpy(), vals[k]), (rep, k)
            assert np.array_equal(g2[k].cpu().numpy(), grads[k]), (rep, k)
    tol = 1e-12 if c128 else 1e-5
    for k, (pg, pt) in enumerate(zip(progs, pars)):
        assert np.abs(vals[k] - pg.value(pt).cpu().numpy()).max() <= tol, k
        assert np.abs(grads[k] - pg.grad(pt).cpu().numpy()).max() <= tol, k
    for k in (0, 17, 41, 74):
        want = otn.qaoa_edge_zz_sv(prob, prob.edges[k])
        assert abs(vals[k][0].real - want) <= max(tol, 1e-5), k
    for k in range(6):
        assert abs(vals[75 + k][0] - vals[k][0]) <= 2 * tol, k


@pytest.mark.parametrize("c128", [False, True])
def test_batched_leaves_and_param_grads_equal_single_calls(c128):
    """tq_tn_build_leaves_batch / tq_tn_param_grad_batch (one launch for all networks) give
    the single calls' results bit for bit, on the 75 p = 2 light-cone networks, with random
    leaf environments for the chain rule; a batch of mixed dtypes is refused."""
    from paper_2301_05451_amd import lib

    prob = W.qaoa_maxcut(p=2)
    progs, pars = [], []
    for e in prob.edges:
        net, _ = tn.qaoa_edge_network(prob, e)
        progs.append(tn.TNProgram(net, tn.elimination_tree(net, tn.elimination_order(net)[0]), c128=c128))
        pars.append(_params(net, c128))
    plans = [p.plan for p in progs]
    gates = [p.net.gates for p in progs]
    specs = [p.specs for p in progs]
    Lb = lib.tn_build_leaves_batch(plans, gates, specs, [p.consts for p in progs], pars)
    gen = torch.Generator(device="cpu").manual_seed(5)
    rdt = torch.float64 if c128 else torch.float32
    envs = [torch.complex(torch.randn(p.plan.leaf_elems, generator=gen, dtype=rdt),
                          torch.randn(p.plan.leaf_elems, generator=gen, dtype=rdt)).cuda() for p in progs]
    Gb = lib.tn_param_grad_batch(plans, gates, specs, pars, envs)
    for k, (pg, pt) in enumerate(zip(progs, pars)):
        assert torch.equal(Lb[k], pg.leaves(pt)), k
        gs = lib.tn_param_grad(pg.plan, pg.net.gates, pg.specs, pt, envs[k])
        assert torch.equal(Gb[k], gs), k
        assert bool(torch.isfinite(gs).all()) and float(gs.abs().max()) > 0, k
    # 300 networks: two launch chunks of the batched calls
    L4 = lib.tn_build_leaves_batch(plans * 4, gates * 4, specs * 4, [p.consts for p in progs] * 4, pars * 4)
    G4 = lib.tn_param_grad_batch(plans * 4, gates * 4, specs * 4, pars * 4, envs * 4)
    for k in range(300):
        assert torch.equal(L4[k], Lb[k % 75]) and torch.equal(G4[k], Gb[k % 75]), k
    other = tn.TNProgram(progs[0].net, progs[0].tree, c128=not c128)
    with pytest.raises(RuntimeError, match="same dtype"):
        lib.tn_build_leaves_batch([plans[0], other.plan], gates[:1] * 2, specs[:1] * 2,
                                  [progs[0].consts] * 2, [pars[0], _params(progs[0].net, not c128)])


def _p4_graph(n=16, seed=41):
    r = np.random.default_rng(seed)
    edges = W.random_regular_graph(3, n, r)
    return W.QAOAProblem(n, edges, 4, W.f32_angles(r, 4, 0, math.pi), W.f32_angles(r, 4, 0, math.pi))


@pytest.mark.timeout(600)
def test_qaoa_p4_small_graph_vs_oracle_full_register():
    """QAOA p = 4 on a 16-node 3-regular graph (every light cone is the whole register):
    the tensor-network value of every edge against the oracle's whole-register state vector,
    and the gamma/beta gradients of four edges against the oracle's central differences on
    the cone circuit (8 parameters, each shared by every edge or node of its layer)."""
    prob = _p4_graph()
    psi = osv.run(prob.n, W.qaoa_circuit(prob).gates, np.concatenate([prob.gammas, prob.betas]))
    prob_sq = np.abs(psi) ** 2
    for k, e in enumerate(prob.edges):
        net, cone = tn.qaoa_edge_network(prob, e)
        tr = tn.elimination_tree(net, tn.elimination_order(net)[0])
        prog = tn.TNProgram(net, tr)
        p = _params(net, False)
        v = prog.value(p).cpu().numpy()[0]
        want = float(np.dot(prob_sq, osv.zstring_diag(prob.n, list(e))))
        assert abs(v.real - want) <= 1e-5 and abs(v.imag) <= 1e-5, (e, v, want)
        if k % 6 == 0:
            c, i, j, _ = otn.qaoa_cone(prob, e)
            c.terms, c.n_obs = W.zterms([([i, j], 1.0, 0)]), 1
            gw = osv.fd_grad(c)
            got = prog.grad(p).cpu().numpy()
            print(f"p4 edge {e}: width {tr.max_rank}, max|d grad| = {np.abs(got - gw).max():.2e}", flush=True)
            assert np.abs(got - gw).max() <= 1e-5, (e, got, gw)


def test_qaoa50_p1_closed_form_all_edges():
    """p = 1 on the 50-node graph: all 75 light-cone networks in one batched launch against
    the analytic p = 1 value (in this build's RZZ(g) = exp(-i g ZZ/2), RX(2b) convention):
    <Z_u Z_v> = 1/2 sin(4b) sin(g) (cos^du g + cos^dv g)
              + 1/2 sin^2(2b) cos^(du+dv-2t) g (1 - cos^t 2g),
    du, dv the other neighbours of u and v, t the triangles through (u, v)."""
    prob = W.qaoa_maxcut(p=1)
    adj = {v: set() for v in range(prob.n)}
    for a, b in prob.edges:
        adj[a].add(b)
        adj[b].add(a)
    g, b = float(prob.gammas[0]), float(prob.betas[0])
    progs, pars = [], []
    for e in prob.edges:
        net, _ = tn.qaoa_edge_network(prob, e)
        progs.append(tn.TNProgram(net, tn.elimination_tree(net, tn.elimination_order(net)[0])))
        pars.append(_params(net, False))
    vals = [v.cpu().numpy()[0] for v in tn.TNBatch(progs).values(pars)]
    for (u, v), val in zip(prob.edges, vals):
        du, dv = len(adj[u]) - 1, len(adj[v]) - 1
        t = len(adj[u] & adj[v])
        want = (0.5 * math.sin(4 * b) * math.sin(g) * (math.cos(g) ** du + math.cos(g) ** dv)
                + 0.5 * math.sin(2 * b) ** 2 * math.cos(g) ** (du + dv - 2 * t) * (1 - math.cos(2 * g) ** t))
        assert abs(val.real - want) <= 1e-5 and abs(val.imag) <= 1e-5, ((u, v), val, want)


def test_store_and_recompute_policies():
    """Store policy (the forward's intermediates kept in the workspace, Sec. 4.1) and
    recompute policy give the same environments and gradients; auto picks store when every
    slice fits the budget at once and recompute otherwise; store under a budget too small for
    all slices is refused; a too-small workspace is TQ_EWORKSPACE."""
    from paper_2301_05451_amd import lib

    prob = _qaoa10()
    e = prob.edges[2]
    net, _ = tn.qaoa_edge_network(prob, e)
    t0 = tn.elimination_tree(net, tn.elimination_order(net)[0])
    ts = tn.slice_tree(net, t0, max(2, t0.max_rank - 3))
    p = _params(net, False)
    want = otn.qaoa_edge_zz_sv(prob, e)
    rec = tn.TNProgram(net, ts, store_policy=lib.TN_RECOMPUTE)
    sto = tn.TNProgram(net, ts, store_policy=lib.TN_STORE)
    assert not rec.plan.stores and sto.plan.stores
    v1, g1 = rec.value_and_grad(p)
    v2, g2 = sto.value_and_grad(p)
    assert abs(v2.cpu().numpy()[0].real - want) <= 1e-5
    assert torch.equal(v1, v2) and torch.equal(g1, g2)
    auto_small = tn.TNProgram(net, ts, slice_group=1, store_policy=lib.TN_AUTO)
    assert not auto_small.plan.stores and auto_small.plan.info["slice_group"] == 1
    v3, g3 = auto_small.value_and_grad(p)
    assert abs(v3.cpu().numpy()[0] - v1.cpu().numpy()[0]) <= 1e-6
    assert (g3 - g1).abs().max().item() <= 1e-6
    with pytest.raises(lib.TQError) as ei:
        tn.TNProgram(net, ts, slice_group=1, store_policy=lib.TN_STORE)
    assert ei.value.status == 3  # TQ_ENOTSUP
    L = sto.leaves(p)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    g = torch.ones(1, dtype=torch.complex64, device="cuda")
    st = lib.raw().tq_tn_backward(sto.plan.ctx.h, sto.plan.h, L.data_ptr(), g.data_ptr(), L.data_ptr(),
                                  small.data_ptr(), 16, None)
    assert st == 5  # TQ_EWORKSPACE
