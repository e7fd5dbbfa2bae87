"""CPU tests of the contraction-tree features that the cost model ranks on."""
import math

import numpy as np

from paper_2301_05451_amd import costmodel, tn
from paper_2301_05451_amd import workloads as W


def test_features_match_tree_statistics():
    prob = W.qaoa_maxcut(p=2)
    net, _ = tn.qaoa_edge_network(prob, prob.edges[0])
    for tree in (tn.greedy_tree(net), tn.elimination_tree(net, tn.elimination_order(net)[0])):
        t = tn.slice_tree(net, tree, max(3, tree.max_rank - 2))
        f = costmodel.tree_features(net, t)
        steps = tn.tree_steps(net, t)
        assert f.shape == (costmodel.N_FEATURES,) and np.all(np.isfinite(f))
        assert f[0] == math.log2(t.flops + 1)
        assert f[3] == len(steps) / 100.0 == (len(net.leaves) - 1) / 100.0
        assert f[4] == len(t.sliced)
        assert f[5] == max(len(o) for _, _, o in steps)
        assert abs(sum(2 ** f[8:14] - 1) - len(steps)) < 1e-9
        assert 0.0 < f[15] <= 1.0


def test_flop_pick_is_the_fewest_flops():
    prob = W.qaoa_maxcut(p=2)
    net, _ = tn.qaoa_edge_network(prob, prob.edges[1])
    trees = tn.candidate_trees(net, n_random=4, seed=0, target_rank=12)
    cands = [(t, None, costmodel.tree_features(net, t)) for t in trees]
    k = costmodel.pick(cands)
    assert trees[k].flops == min(t.flops for t in trees)
