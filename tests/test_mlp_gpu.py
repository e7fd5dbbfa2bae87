"""GPU parity of the cost-model MLP kernels (tq_mlp_forward, tq_mlp_train_step) against the
float64 oracle: outputs, loss, gradients, one Adam step, a 100-step trajectory,
repeatability, and the cost model fitting a known function."""
import numpy as np
import pytest

from oracle import mlp as om

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = [16, 64, 64, 1]


def _setup(seed, B):
    rng = np.random.default_rng(seed)
    layers = om.init(SIZES, rng)
    for W, b in layers:
        b[:] = rng.normal(size=b.shape) * 0.1
    # the device works in float32: hand the oracle the same float32-representable values
    layers = [[W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)] for W, b in layers]
    X = rng.normal(size=(B, SIZES[0])).astype(np.float32)
    Y = rng.normal(size=B).astype(np.float32)
    return layers, X, Y


def _flat(layers):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


@pytest.mark.parametrize("B", [1, 37, 1000])
def test_forward_matches_oracle(B):
    from paper_2301_05451_amd import lib

    layers, X, _ = _setup(1, B)
    y = lib.mlp_forward(SIZES, _dev(_flat(layers)), _dev(X)).cpu().numpy()
    yo, _ = om.forward(layers, X.astype(np.float64))
    assert np.abs(y - yo).max() <= 1e-5 * max(1.0, np.abs(yo).max())


def test_train_step_loss_grad_and_adam_match_oracle():
    from paper_2301_05451_amd import lib

    layers, X, Y = _setup(2, 200)
    p = _dev(_flat(layers))
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    loss, g = lib.mlp_train_step(SIZES, p, m, v, 1, _dev(X), _dev(Y), lr=1e-3, want_grad=True)
    lo, go = om.backward(layers, X.astype(np.float64), Y.astype(np.float64))
    assert abs(loss.item() - lo) <= 1e-5 * max(1.0, lo)
    gf = _flat(go)
    assert np.abs(g.cpu().numpy() - gf).max() <= 1e-5 * max(1.0, np.abs(gf).max())
    st = om.adam_init(layers)
    om.adam_step(layers, go, st, lr=1e-3)
    assert np.abs(p.cpu().numpy() - _flat(layers)).max() <= 1e-6


def test_hundred_steps_track_oracle_and_repeat_bitwise():
    from paper_2301_05451_amd import lib

    layers0, X, Y = _setup(3, 128)
    runs = []
    for _ in range(2):
        p = _dev(_flat(layers0))
        m, v = torch.zeros_like(p), torch.zeros_like(p)
        losses = []
        for t in range(1, 101):
            loss, _ = lib.mlp_train_step(SIZES, p, m, v, t, _dev(X), _dev(Y), lr=3e-3)
            losses.append(loss.item())
        runs.append((p.cpu().numpy(), losses))
    assert np.array_equal(runs[0][0], runs[1][0])
    layers = [[W.copy(), b.copy()] for W, b in layers0]
    st = om.adam_init(layers)
    ol = []
    for t in range(100):
        lo, go = om.backward(layers, X.astype(np.float64), Y.astype(np.float64))
        ol.append(lo)
        om.adam_step(layers, go, st, lr=3e-3)
    assert np.abs(np.array(runs[0][1]) - np.array(ol)).max() <= 1e-4 * max(ol)
    assert ol[-1] < 0.5 * ol[0]
    assert np.abs(runs[0][0] - _flat(layers)).max() <= 1e-4


def test_cost_model_fits_a_known_function():
    from paper_2301_05451_amd import costmodel

    rng = np.random.default_rng(4)
    F = rng.normal(size=(512, costmodel.N_FEATURES))
    y = 0.7 * F[:, 0] - 0.3 * F[:, 5] + 0.2 * np.sin(F[:, 3])
    cm = costmodel.CostModel(seed=0)
    hist = cm.fit(F[:400], y[:400], epochs=600, lr=3e-3)
    assert hist[-1] < 0.05 * hist[0]
    pred = cm.predict_log_ms(F[400:])
    assert np.sqrt(np.mean((pred - y[400:]) ** 2)) < 0.15 * np.std(y)


def test_mlp_validation():
    from paper_2301_05451_amd import lib

    with pytest.raises(lib.TQError):
        lib.mlp_param_count([16, 64, 2])  # last layer must have one output
    p = torch.zeros(lib.mlp_param_count(SIZES), device="cuda")
    with pytest.raises(lib.TQError):
        lib.mlp_train_step(SIZES, p, p.clone(), p.clone(), 0, torch.zeros(4, 16, device="cuda"),
                           torch.zeros(4, device="cuda"))  # Adam step count is 1-based
