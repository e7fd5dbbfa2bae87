"""What the trained cost model gains over the paper's FLOP ranking (Sec. 3.2.2; Sec. 6.6 notes
that small pairwise steps make GPU runtime and FLOPs disagree), measured on the GPU: the MLP
(trained by the libtq kernels on timings of the same executor) picks one candidate (tree x
slicing) per held-out network; the total measured time of its picks is compared with that
of the fewest-FLOP picks, at equal accuracy (every candidate gives the same value), and with
the fastest measured candidate (the bound on any ranking's gain)."""
import pytest

from paper_2301_05451_amd import costmodel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_learned_ranking_gain_on_heldout_graph():
    train = []
    for seed in (2001, 2002, 2003):
        g = costmodel.qaoa_graph(seed)
        train += costmodel.plan_candidates(g, g.edges[::7][:10])
    held = costmodel.qaoa_graph(4004)
    test = costmodel.plan_candidates(held, held.edges[::4][:15])
    r = costmodel.ranking_experiment(train, test, reps=5)
    print(f"learned gain {r['learned_gain']:.3f} (bound {r['max_possible_gain']:.3f}), "
          f"flop {r['ms_flop_ranked']:.1f} ms, mlp {r['ms_mlp_ranked']:.1f} ms, best {r['ms_fastest_measured']:.1f} ms, "
          f"rms log error {r['heldout_rms_log_time_error']:.3f}", flush=True)
    assert r["max_value_spread_between_candidates"] <= 1e-5  # equal accuracy
    assert r["learned_gain"] <= r["max_possible_gain"] + 1e-9
    # The fewest-FLOP candidate of this path search is already within a few per cent of the
    # fastest measured one, which bounds what any learned ranking can gain; the model's
    # held-out error is of the same size. Over repeated runs the measured gain spread over
    # 0.97-1.06 (its picks and the FLOP picks are timed separately, each with that much
    # noise): the model may not lose more than that noise.
    assert r["max_possible_gain"] < 1.2
    assert r["learned_gain"] > 0.95
