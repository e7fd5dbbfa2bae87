"""Learned runtime model for ranking contraction trees.

The paper picks a contraction tree (and its slicing) by the FLOP count p(2q-1) summed over
the pairwise steps (Sec. 3.2.2) and observes that on a GPU many small pairwise steps cost
far more than their FLOPs suggest (Sec. 6.6). Here candidate trees are ranked instead by
the runtime a small MLP predicts from features of the tree and of its execution plan. The
MLP is trained on the GPU, by libtq's tq_mlp_* kernels, on measured times of the same
executor (tq_tn_contract + tq_tn_backward), and ranks new networks' candidates.

Features (16 per tree, all computed on the host):
  0  log2 FLOPs (paper count, all slices)        8-13 log2(1 + number of steps) whose output
  1  log2 elements written (all slices)                rank is in 0-4, 5-8, 9-12, 13-16,
  2  log2 elements read (all slices)                   17-20, >20
  3  steps / 100                                  14  log2 largest intermediate
  4  log2 slices                                  15  share of FLOPs in the largest step
  5  largest rank (width)
  6  steps on the MFMA GEMM path (plan)
  7  log2(1 + FLOPs on the GEMM path)
Target: natural log of the measured time in milliseconds, centred per network (the model
ranks the candidates of one network), and only candidates within a small factor of the
fewest FLOPs are re-ranked.
"""
from __future__ import annotations

import math

import numpy as np

from . import tn

N_FEATURES = 16
SIZES = (N_FEATURES, 64, 64, 1)


def tree_features(net, tree, plan_info=None):
    steps = tn.tree_steps(net, tree)
    S = 2 ** len(tree.sliced)
    fl = [tn.step_flops(*s) for s in steps]
    tot = float(sum(fl)) * S
    wr = float(sum(2 ** len(o) for _, _, o in steps)) * S
    rd = float(sum(2 ** len(a) + 2 ** len(b) for a, b, _ in steps)) * S
    ranks = [len(o) for _, _, o in steps]
    hist = np.zeros(6)
    for r in ranks:
        hist[min(5, max(0, (r - 1) // 4))] += 1
    f = np.zeros(N_FEATURES)
    f[0] = math.log2(tot + 1)
    f[1] = math.log2(wr + 1)
    f[2] = math.log2(rd + 1)
    f[3] = len(steps) / 100.0
    f[4] = len(tree.sliced)
    f[5] = max(ranks + [0])
    if plan_info is not None:
        f[6] = plan_info["gemm_steps"]
        f[7] = math.log2(1 + plan_info["gemm_flops"])
    f[8:14] = np.log2(1 + hist)
    f[14] = math.log2(max([2 ** r for r in ranks] + [1]))
    f[15] = (max(fl) / sum(fl)) if fl else 0.0
    return f


def time_program(prog, params, reps=3, grad=True):
    """Median milliseconds of value (+ gradient) of a TNProgram (HIP events)."""
    import torch

    prog.value(params)
    if grad:
        prog.grad(params)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        prog.value(params)
        if grad:
            prog.grad(params)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


class CostModel:
    """MLP 16-64-64-1 trained with Adam on (features, log ms) pairs; inputs are
    standardised with the training set's mean and spread."""

    def __init__(self, seed=0, device="cuda"):
        import torch

        from . import lib

        self.lib = lib
        rng = np.random.default_rng(seed)
        parts = []
        for i in range(len(SIZES) - 1):
            fan_in = SIZES[i]
            parts.append(rng.uniform(-1.0, 1.0, size=(SIZES[i + 1], fan_in)).reshape(-1) / math.sqrt(fan_in))
            parts.append(np.zeros(SIZES[i + 1]))
        self.params = torch.tensor(np.concatenate(parts), dtype=torch.float32, device=device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.mu = np.zeros(N_FEATURES)
        self.sd = np.ones(N_FEATURES)
        self.y_mu = 0.0
        self.device = device

    def _x(self, feats):
        import torch
        x = (np.asarray(feats, dtype=np.float64) - self.mu) / self.sd
        return torch.tensor(x, dtype=torch.float32, device=self.device).contiguous()

    def fit(self, feats, log_ms, epochs=400, lr=3e-3, batch=None):
        """Full-batch (or mini-batch) Adam on the standardised data; returns the loss history."""
        import torch

        feats = np.asarray(feats, dtype=np.float64)
        self.mu = feats.mean(0)
        self.sd = feats.std(0) + 1e-6
        self.y_mu = float(np.mean(log_ms))
        X = self._x(feats)
        Y = torch.tensor(np.asarray(log_ms) - self.y_mu, dtype=torch.float32, device=self.device)
        n = X.shape[0]
        bs = n if batch is None else min(batch, n)
        hist = []
        rng = np.random.default_rng(1)
        for _ in range(epochs):
            order = np.arange(n) if bs == n else rng.permutation(n)
            for s in range(0, n - bs + 1, bs):
                idx = torch.tensor(order[s:s + bs], device=self.device)
                self.t += 1
                loss, _ = self.lib.mlp_train_step(SIZES, self.params, self.m, self.v, self.t,
                                                  X[idx].contiguous(), Y[idx].contiguous(), lr=lr)
            hist.append(loss)
        return [float(h.item()) for h in hist]

    def predict_log_ms(self, feats):
        y = self.lib.mlp_forward(SIZES, self.params, self._x(feats))
        return y.cpu().numpy().astype(np.float64) + self.y_mu

    def fit_groups(self, groups, epochs=800, lr=3e-3):
        """Ranking within a network is what matters: ``groups`` is a list of (features [k, F],
        log ms [k]) per network, and the model learns the differences from each network's
        mean (features and targets both centred per network)."""
        F = np.concatenate([np.asarray(f) - np.mean(f, 0) for f, _ in groups])
        y = np.concatenate([np.asarray(t) - np.mean(t) for _, t in groups])
        return self.fit(F, y, epochs=epochs, lr=lr)

    def predict_relative(self, feats):
        """Predicted log-time differences from the mean of these candidates (one network)."""
        f = np.asarray(feats, dtype=np.float64)
        return self.predict_log_ms(f - f.mean(0))


def candidates_with_plans(net, n_random=5, seed=0, target_rank=26):
    """Candidate trees of a network with their libtq plans and features."""
    out = []
    for tree in tn.candidate_trees(net, n_random=n_random, seed=seed, target_rank=target_rank):
        prog = tn.TNProgram(net, tree)
        out.append((tree, prog, tree_features(net, tree, prog.plan.info)))
    return out


def pick(cands, model=None, trust=4.0):
    """Index of the candidate with the fewest FLOPs (model None), or of the lowest predicted
    time among the candidates within ``trust`` times the fewest FLOPs (the model re-ranks
    near-optimal trees; it is not asked to extrapolate to far costlier ones)."""
    fl = np.array([t.flops for t, _, _ in cands], dtype=np.float64)
    if model is None:
        return int(np.argmin(fl))
    ok = np.nonzero(fl <= trust * fl.min())[0]
    score = model.predict_relative([cands[i][2] for i in range(len(cands))])
    return int(ok[np.argmin(score[ok])])
