"""The allocation-free expectation entry point (tq_expval_noalloc) against tq_expval: two
calls in a row through the C ABI, the second on a smaller input, each compared with
tq_expval on the same states (same kernels: equal bitwise) and with the oracle."""
import ctypes as ct

import numpy as np
import pytest

from oracle import sv as osv
from paper_2301_05451_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _states(n, count, rng, cdt):
    v = rng.normal(size=(count, 1 << n)) + 1j * rng.normal(size=(count, 1 << n))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return torch.tensor(v.reshape(-1), dtype=cdt, device="cuda"), v


def _terms(n, rng, k, n_obs):
    rows = []
    for i in range(k):
        qs = sorted(int(q) for q in rng.choice(n, size=int(rng.integers(1, min(n, 4) + 1)), replace=False))
        rows.append((qs, float(rng.uniform(-1, 1)), i % n_obs))
    return W.zterms(rows)


@pytest.mark.parametrize("c128", [False, True])
def test_noalloc_matches_expval_two_calls(c128):
    from paper_2301_05451_amd import lib

    cdt, rdt = (torch.complex128, torch.float64) if c128 else (torch.complex64, torch.float32)
    rng = np.random.default_rng(71)
    for n, count, k, n_obs in ((20, 3, 40, 3), (11, 2, 5, 2)):
        print(f"noalloc c128={c128} n={n} count={count} terms={k}", flush=True)
        psi, host = _states(n, count, rng, cdt)
        terms = _terms(n, rng, k, n_obs)
        spec = lib.BatchSpec.uniform(n, W.GateList().array(), count, 1)
        want = lib.expval(psi, spec, terms, n_obs)
        out = torch.full((count, n_obs), float("nan"), dtype=rdt, device="cuda")
        tt = np.ascontiguousarray(terms)
        st = lib.raw().tq_expval_noalloc(1 if c128 else 0, n, count, ct.c_int64(1 << n), psi.data_ptr(),
                                         tt.ctypes.data, int(tt.shape[0]), n_obs, out.data_ptr(), None)
        assert st == 0, lib.last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, want)
        hv = psi.cpu().numpy().astype(np.complex128).reshape(count, -1)
        tol = 1e-12 if c128 else 1e-5
        for i in range(count):
            o = osv.expvals(hv[i], n, terms, n_obs)
            assert np.abs(out[i].cpu().numpy() - o).max() <= tol


def test_noalloc_limits():
    from paper_2301_05451_amd import lib

    psi = torch.zeros(1 << 10, dtype=torch.complex64, device="cuda")
    out = torch.empty(1, 1, device="cuda")
    with pytest.raises(lib.TQError) as e:
        lib.expval_noalloc(psi, 10, 1, W.zterms([([0], 1.0, 0)] * 65), 1, out)
    assert e.value.status == 1
    big = torch.zeros(1 << 20, dtype=torch.complex64, device="cuda")
    with pytest.raises(lib.TQError) as e:  # 65535 circuits of 4 qubits: over the static limit
        lib.expval_noalloc(big, 4, 65535, W.zterms([([0], 1.0, 0)]), 1, torch.empty(65535, 1, device="cuda"))
    assert e.value.status == 5
