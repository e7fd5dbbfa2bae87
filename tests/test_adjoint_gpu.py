"""GPU parity of the adjoint backward (tq_sv_backward, SVExpval.backward) against the
oracle's parameter-shift gradients (exact) and central finite differences.
Tolerances: complex64 |d grad| <= 1e-5, complex128 <= 1e-12, times the weight scale
sum_o |w_o| sum_{terms of o} |coeff| of the differentiated sum (1 for a unit weight on one
unit-coefficient Z-string)."""
import math

import numpy as np
import pytest

from oracle import sv as osv
from paper_2301_05451_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}


def _types(name):
    return (torch.complex64, torch.float32) if name == "c64" else (torch.complex128, torch.float64)


def _wscale(terms, weights):
    w = np.abs(np.asarray(weights, dtype=np.float64)).reshape(-1)
    return float(sum(abs(float(t["coeff"])) * w[int(t["obs"])] for t in terms))


def _adjoint(circs, name, terms, n_obs, weights, **kw):
    from paper_2301_05451_amd import lib

    cdt, rdt = _types(name)
    spec = lib.BatchSpec.from_circuits(circs)
    params = torch.tensor(np.concatenate([c.params for c in circs]), dtype=rdt, device="cuda")
    psi = lib.zero_states(spec, cdt)
    lib.sv_apply(psi, params, spec)
    w = torch.tensor(np.asarray(weights), dtype=rdt, device="cuda").reshape(len(circs), n_obs)
    g = lib.sv_backward(psi, params, spec, terms, n_obs, w, **kw)
    torch.cuda.synchronize()
    return spec, g.cpu().numpy()


@pytest.mark.parametrize("name", ["c64", "c128"])
def test_random_circuits_vs_param_shift(name):
    rng = np.random.default_rng(31)
    terms = W.zterms([([0], 1.0, 0), ([1], -0.5, 0), ([0, 1], 0.7, 1)])
    for n in [2, 3, 5, 8, 11, 13]:
        c = W.random_circuit(n, 50, rng, n_params=12)
        print(f"adjoint n={n} {name}", flush=True)
        w = [[0.8, -1.1]]
        _, g = _adjoint([c], name, terms, 2, w)
        c.terms, c.n_obs = terms, 2
        want = osv.param_shift_grad(c, weights=np.array(w[0]))
        err = np.abs(g - want).max()
        print(f"  max|d grad| = {err:.2e}", flush=True)
        assert err <= TOL[name] * _wscale(terms, w), (n, err)


@pytest.mark.parametrize("tile", [(5, 2), (6, 3), (8, 4), (10, 4)])
def test_adjoint_tile_shapes_multi_stage(tile):
    t, R = tile
    rng = np.random.default_rng(40 + t)
    terms = W.zterms([([0], 1.0, 0)])
    for n in [t + 1, t + 3]:
        c = W.random_circuit(n, 70, rng, n_params=20)
        print(f"adjoint tile={tile} n={n}", flush=True)
        _, g = _adjoint([c], "c64", terms, 1, [[1.0]], tile_bits=t, reg_bits=R)
        c.terms, c.n_obs = terms, 1
        want = osv.param_shift_grad(c)
        err = np.abs(g - want).max()
        print(f"  max|d grad| = {err:.2e}", flush=True)
        assert err <= 1e-5


def test_hea_ring_adjoint_matches_param_shift_and_fd():
    c = W.hea_ring()
    _, g = _adjoint([c], "c64", c.terms, 1, [[1.0]])
    ps = osv.param_shift_grad(c)
    fd = osv.fd_grad(c)
    assert np.abs(g - ps).max() <= 1e-5
    assert np.abs(ps - fd).max() <= 1e-8


def test_single_rotation_closed_form_on_gpu():
    for theta in (0.3, 2.0, 4.4):
        c = W.Circuit(1, W.GateList().add(W.RY, [0], [0]).array(), np.array([theta]), 1, W.zterms([([0], 1.0, 0)]))
        _, g = _adjoint([c], "c128", c.terms, 1, [[1.0]])
        assert abs(g[0] + math.sin(theta)) < 1e-13


def test_autograd_function_mse_loss():
    """SVExpval inside a torch graph: MSE on <Z0> over a batch, gradient vs oracle."""
    from paper_2301_05451_amd import lib, sv

    n, B = 6, 5
    gates, x, theta, y = W.qnn_batch(n=n, layers=2, batch=B, seed=77)
    P = n + theta.shape[0]
    spec = lib.BatchSpec.uniform(n, gates, B, P)
    terms = W.zterms([([0], 1.0, 0)])
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    th = torch.tensor(theta, dtype=torch.float32, device="cuda", requires_grad=True)
    params = torch.cat([xt, th[None, :].expand(B, -1)], 1).reshape(-1)
    f = sv.expval(params, spec, terms, 1)[:, 0]
    yt = torch.tensor(y, dtype=torch.float32, device="cuda")
    loss = torch.mean((f - yt) ** 2)
    loss.backward()
    # oracle: dL/dtheta = (2/B) sum_b (f_b - y_b) df_b/dtheta
    want = np.zeros(theta.shape[0])
    fo = np.zeros(B)
    for b in range(B):
        cb = W.Circuit(n, gates, np.concatenate([x[b], theta]), 1, terms)
        fo[b] = osv.circuit_f(cb)[0]
        gb = osv.param_shift_grad(cb)
        want += 2.0 / B * (fo[b] - y[b]) * gb[n:]
    assert np.abs(f.detach().cpu().numpy() - fo).max() <= 1e-5
    assert np.abs(th.grad.cpu().numpy() - want).max() <= 1e-5


def test_qnn16_batch_adjoint_vs_gpu_param_shift_and_oracle():
    """16-qubit QNN, 64 samples: adjoint vs the GPU parameter-shift baseline on every sample
    and every parameter; oracle parameter shift on one sample for 12 parameters."""
    from paper_2301_05451_amd import lib, sv

    n, B = 16, 64
    gates, x, theta, y = W.qnn_batch(n=n, layers=8, batch=B, seed=1003)
    P = n + theta.shape[0]
    assert sv.single_occurrence(gates, P)
    pb = np.concatenate([x, np.broadcast_to(theta, (B, theta.shape[0]))], 1)
    params = torch.tensor(pb.reshape(-1), dtype=torch.float32, device="cuda")
    spec = lib.BatchSpec.uniform(n, gates, B, P)
    terms = W.zterms([([0], 1.0, 0)])
    psi = lib.zero_states(spec, torch.complex64)
    lib.sv_apply(psi, params, spec)
    w = torch.ones(B, 1, device="cuda")
    g_adj = lib.sv_backward(psi, params, spec, terms, 1, w).reshape(B, P)
    g_ps = sv.param_shift_grad_gpu(params.reshape(B, P), gates, n, terms, 1, w)
    torch.cuda.synchronize()
    assert (g_adj - g_ps).abs().max().item() <= 1e-5
    cb = W.Circuit(n, gates, pb[3], 1, terms)
    sel = list(range(0, P, P // 12))[:12]
    for p in sel:
        # oracle shift of parameter p (single occurrence, scale 1)
        pp, pm = pb[3].copy(), pb[3].copy()
        pp[p] += math.pi / 2
        pm[p] -= math.pi / 2
        want = 0.5 * (osv.circuit_f(cb, pp)[0] - osv.circuit_f(cb, pm)[0])
        assert abs(g_adj[3, p].item() - want) <= 1e-5, p


def test_backward_validation():
    from paper_2301_05451_amd import lib

    c = W.hea_ring()
    spec = lib.BatchSpec.uniform(c.n, c.gates, 1, c.n_params)
    params = torch.tensor(c.params, dtype=torch.float32, device="cuda")
    psi = lib.zero_states(spec, torch.complex64)
    with pytest.raises(lib.TQError):
        lib.sv_backward(psi, params, spec, W.zterms([([0], 1.0, 3)]), 1, torch.ones(1, 1, device="cuda"))
    with pytest.raises(lib.TQError):
        lib.sv_backward(psi, params, spec, c.terms, 1, torch.ones(1, 1, device="cuda"), reg_bits=7)


@pytest.mark.parametrize("name", ["c64", "c128"])
def test_one_qubit_runs_vs_param_shift(name):
    """Long runs of one-qubit gates on each qubit (diagonal, fixed and parameterised gates,
    one to three angles each) separated by two-qubit gates: the reverse sweep takes up to
    three angles' worth of a run as one op, so runs are split at every angle count."""
    rng = np.random.default_rng(77)
    one_q = [W.H, W.X, W.Y, W.Z, W.RX, W.RY, W.RZ, W.U3, W.ROT]
    terms = W.zterms([([0], 1.0, 0), ([1, 2], 0.6, 0)])
    for n in [3, 6, 9]:
        g = W.GateList()
        n_params = 10
        for layer in range(4):
            for q in range(n):
                for _ in range(int(rng.integers(1, 9))):
                    op = int(rng.choice(one_q))
                    na = W.N_ANGLES[op]
                    g.add(op, [q], [int(rng.integers(n_params)) for _ in range(na)],
                          [float(rng.choice([1.0, -0.5, 2.0])) for _ in range(na)])
            for q in range(layer % 2, n - 1, 2):
                op2 = int(rng.choice([W.CNOT, W.CZ, W.RZZ]))
                na2 = W.N_ANGLES[op2]
                g.add(op2, [q, q + 1], [int(rng.integers(n_params))] * na2, [1.0] * na2)
        c = W.Circuit(n, g.array(), W.f32_angles(rng, n_params, 0.0, 2 * math.pi), 1, terms)
        print(f"adjoint runs n={n} {name} gates={len(c.gates)}", flush=True)
        _, got = _adjoint([c], name, terms, 1, [[1.0]])
        want = osv.param_shift_grad(c)
        err = np.abs(got - want).max()
        print(f"  max|d grad| = {err:.2e}", flush=True)
        assert err <= TOL[name] * _wscale(terms, [1.0]), (n, err)


def test_backward_workspace_query_and_errors():
    """tq_sv_backward runs in the caller's workspace: the size query's bytes suffice, a NULL or
    smaller workspace is TQ_EWORKSPACE, and a reused larger workspace gives the same result."""
    import ctypes as ct

    from paper_2301_05451_amd import lib

    rng = np.random.default_rng(90)
    circs = [W.random_circuit(n, 30, rng, n_params=8) for n in (5, 9, 5)]
    spec = lib.BatchSpec.from_circuits(circs)
    params = torch.tensor(np.concatenate([c.params for c in circs]), dtype=torch.float32, device="cuda")
    terms = W.zterms([([0], 1.0, 0)])
    psi = lib.zero_states(spec, torch.complex64)
    lib.sv_apply(psi, params, spec)
    need = lib.sv_backward_workspace(psi, spec, terms, 1)
    assert need > 2 * (1 << 9) * 8
    w = torch.ones(3, 1, device="cuda")
    big = torch.empty(need + 4096, dtype=torch.uint8, device="cuda")
    g1 = lib.sv_backward(psi, params, spec, terms, 1, w, work=big)
    g2 = lib.sv_backward(psi, params, spec, terms, 1, w)
    assert torch.equal(g1, g2)
    for i, c in enumerate(circs):
        c.terms, c.n_obs = terms, 1
        p0 = int(spec.param_off[i])
        assert np.abs(g1[p0:p0 + c.n_params].cpu().numpy() - osv.param_shift_grad(c)).max() <= 1e-5
    grad = torch.empty_like(params)
    tt = np.ascontiguousarray(terms)
    o = lib.SvOpts(0, 0, 0, 0)
    for buf, nbytes in ((None, 0), (big, need - 1)):
        st = lib.raw().tq_sv_backward(lib.context().h, 0, ct.byref(spec.c), spec.gates.ctypes.data,
                                      spec.n_params.ctypes.data, params.data_ptr(), psi.data_ptr(), tt.ctypes.data, 1,
                                      1, w.data_ptr(), grad.data_ptr(), ct.byref(o),
                                      None if buf is None else buf.data_ptr(), nbytes, None)
        assert st == 5, lib.last_error()  # TQ_EWORKSPACE
