"""The attainable-peak probes (tq_peak_probe) do the work they report: the copy probe copies,
the FMA chains and the matrix-core accumulations produce their closed-form values, and the
reported work follows the launch shape (2048 blocks of 256 threads, 8 chains)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

THREADS = 2048 * 256


def test_copy_probe_copies_and_reports_bytes():
    from paper_2301_05451_amd import lib

    buf = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    g = torch.Generator(device="cpu").manual_seed(5)
    buf[: 1 << 19] = torch.randint(0, 256, (1 << 19,), dtype=torch.uint8, generator=g).cuda()
    buf[1 << 19:] = 0
    w = lib.peak_probe(lib.PEAK_COPY, buf)
    torch.cuda.synchronize()
    assert w == float(1 << 20)
    assert torch.equal(buf[1 << 19:], buf[: 1 << 19])
    before = buf.clone()
    assert lib.peak_probe(lib.PEAK_READ, buf) == float(1 << 20)
    torch.cuda.synchronize()
    assert torch.equal(buf[4:], before[4:])  # the read probe may write only the first float


def test_fma_probe_matches_the_recurrence():
    from paper_2301_05451_amd import lib

    out = torch.zeros(THREADS, dtype=torch.float32, device="cuda")
    iters = 40
    w = lib.peak_probe(lib.PEAK_FP32_FMA, out, iters)
    assert w == THREADS * iters * 8 * 2.0
    got = out.cpu().numpy().astype(np.float64)
    x, y = np.float64(np.float32(0.999)), np.float64(np.float32(1e-3))
    t = np.arange(THREADS)
    want = np.zeros(THREADS)
    for c in range(8):
        a0 = (t & 7) + 0.25 * c
        want += a0 * x ** iters + y * (1 - x ** iters) / (1 - x)  # a <- a x + y, iters times
    np.testing.assert_allclose(got, want, rtol=2e-5)


@pytest.mark.parametrize("kind,dt", [("f32", torch.float32), ("f64", torch.float64)])
def test_mfma_probe_matches_the_product(kind, dt):
    from paper_2301_05451_amd import lib

    out = torch.zeros(THREADS, dtype=dt, device="cuda")
    iters = 3
    w = lib.peak_probe(lib.PEAK_FP32_MFMA if kind == "f32" else lib.PEAK_FP64_MFMA, out, iters)
    assert w == (THREADS // 64) * iters * 8 * 2048.0
    # A[r][k] = x r and B[k][c] = x k (lane l supplies row/column l mod 16 and k = l div 16), so
    # D = A B has D[r][c] = 6 x^2 r; a wave's 64 outputs together hold 8 chains x iters x sum(D).
    x = 1e-3
    per_wave = out.cpu().numpy().astype(np.float64).reshape(-1, 64).sum(axis=1)
    want = 8 * iters * 6 * x * x * 16 * sum(range(16))
    np.testing.assert_allclose(per_wave, want, rtol=1e-5 if kind == "f32" else 1e-12)
