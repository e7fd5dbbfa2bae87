"""Learned runtime model for ranking contraction trees.

The paper picks a contraction tree (and its slicing) by the FLOP count p(2q-1) summed over
the pairwise steps (Sec. 3.2.2) and observes that on a GPU many small pairwise steps cost
far more than their FLOPs suggest (Sec. 6.6). Here candidate trees are ranked instead by
the runtime a small MLP predicts from features of the tree and of its execution plan. The
MLP is trained on the GPU, by libtq's tq_mlp_* kernels, on measured times of the same
executor (tq_tn_contract + tq_tn_backward), and ranks new networks' candidates.

Features (16 per candidate, all computed on the host):
  0  log2 FLOPs (paper count, all slices)        8-13 log2(1 + number of steps) whose output
  1  log2 elements written (all slices)                rank is in 0-4, 5-8, 9-12, 13-16,
  2  log2 elements read (all slices)                   17-20, >20
  3  steps / 100                                  14  log2 elements moved by the steps too
  4  log2 slices                                      large to run in a fused launch
  5  largest rank (width)                         15  share of FLOPs in the largest step
  6  log2(1 + forward launch segments) (plan)
  7  log2(1 + forward segments that are single large steps) (plan)
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
        f[6] = math.log2(1 + plan_info.get("fwd_segments", 0))
        f[7] = math.log2(1 + plan_info.get("fwd_segments", 0) - plan_info.get("fwd_fused", 0))
    f[8:14] = np.log2(1 + hist)
    big = 0.0
    for (a, b, o), w in zip(steps, fl):
        if len(o) > 12 or w > 2 ** 17:  # outside the fused small-step runs
            big += 2.0 ** len(a) + 2.0 ** len(b) + 2.0 ** len(o)
    f[14] = math.log2(1 + big * S)
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


def slicings(net, tree, deltas=(0, 2, 4), seed=0):
    """A tree and its slicings to ``width - d`` for each d > 0 (Sec. 3.2.3 two-phase search):
    the candidates differ in run time (more slices, more parallel copies, more FLOPs)."""
    out = []
    for d in deltas:
        if d == 0:
            out.append(tree)
        elif tree.max_rank - d >= 4:
            out.append(tn.slice_search(net, tree, tree.max_rank - d, 2, np.random.default_rng(seed + d)))
    return out


def edge_candidates(args):
    """(network, candidate trees x slicings) of one QAOA edge (host only; usable in workers)."""
    prob, edge, seed, n_bisect, deltas = args
    net, _ = tn.qaoa_edge_network(prob, edge)
    out = []
    for tree in tn.tree_pool(net, seed, n_bisect):
        out += slicings(net, tree, deltas, seed)
    return net, out


def plan_candidates(prob, edges, n_bisect=3, deltas=(0, 2, 4), workers=1):
    jobs = [(prob, e, k, n_bisect, deltas) for k, e in enumerate(edges)]
    if workers <= 1:
        return [edge_candidates(j) for j in jobs]
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(edge_candidates, jobs))


def qaoa_graph(seed, p=4, n=50):
    """A seeded random 3-regular graph with QAOA angles (training and held-out graphs)."""
    from . import workloads as W
    r = np.random.default_rng(seed)
    edges = W.random_regular_graph(3, n, r)
    return W.QAOAProblem(n, edges, p, W.f32_angles(r, p, 0, math.pi), W.f32_angles(r, p, 0, math.pi))


def measure_candidates(net, trees, reps=3, spread=8.0):
    """(tree, features, median ms of value + gradient, value) of each candidate within
    ``spread`` times the fewest FLOPs (costlier ones are never picked, so not run)."""
    import torch
    fmin = min(t.flops for t in trees)
    pt = torch.tensor(net.params, dtype=torch.float32, device="cuda")
    rows = []
    for t in trees:
        if t.flops > spread * fmin:
            continue
        prog = tn.TNProgram(net, t)
        rows.append((t, tree_features(net, t, prog.plan.info), time_program(prog, pt, reps=reps),
                     prog.value(pt).cpu().numpy()[0]))
        del prog
    return rows


def ranking_experiment(train, test, seed=0, trust=4.0, reps=3, margin=0.05, log=None):
    """Trains a CostModel on the measured candidates of the ``train`` networks and compares,
    on the ``test`` networks, the measured time of its picks with the fewest-FLOP picks and
    with the fastest measured candidate. ``train``/``test``: lists of (network, trees). The
    model leaves the fewest-FLOP pick only when it predicts the other candidate faster by
    more than ``margin`` in log time (its held-out error is of that order)."""
    import torch
    groups = []
    for k, (net, trees) in enumerate(train):
        rows = measure_candidates(net, trees, reps)
        groups.append((np.array([r[1] for r in rows]), np.log(np.array([r[2] for r in rows]))))
        if log:
            log(f"ranking: train network {k}, {len(rows)} candidates")
    cm = CostModel(seed=seed)
    hist = cm.fit_groups(groups, epochs=800, lr=3e-3)
    torch.cuda.synchronize()
    t_flop = t_mlp = t_best = 0.0
    same, spread, err = 0, 0.0, []
    for k, (net, trees) in enumerate(test):
        rows = measure_candidates(net, trees, reps)
        fl = np.array([r[0].flops for r in rows])
        ms = np.array([r[2] for r in rows])
        vals = np.array([r[3] for r in rows])
        spread = max(spread, float(np.abs(vals - vals[0]).max()))
        pred = cm.predict_relative(np.array([r[1] for r in rows]))
        kf = int(np.argmin(fl))
        ok = np.nonzero(fl <= trust * fl.min())[0]
        km = int(ok[np.argmin(pred[ok])])
        if pred[kf] - pred[km] <= margin:
            km = kf
        same += km == kf
        t_flop += ms[kf]
        t_mlp += ms[km]
        t_best += ms.min()
        lm = np.log(ms)
        err.append(float(np.sqrt(np.mean(((lm - lm.mean()) - pred) ** 2))))
        if log:
            log(f"ranking: held-out network {k}, {len(rows)} candidates")
    return {"train_samples": int(sum(len(t) for _, t in groups)), "train_mse_first_last": [hist[0], hist[-1]],
            "heldout_rms_log_time_error": float(np.mean(err)), "ms_flop_ranked": t_flop, "ms_mlp_ranked": t_mlp,
            "ms_fastest_measured": t_best, "learned_gain": t_flop / t_mlp, "max_possible_gain": t_flop / t_best,
            "same_pick": same, "networks": len(test), "max_value_spread_between_candidates": spread}


def candidates_with_plans(net, trees=None, seed=0, deltas=(0, 2, 4), n_bisect=3):
    """Candidates (tree x slicing) of a network with their libtq plans and features."""
    trees = tn.tree_pool(net, seed, n_bisect) if trees is None else trees
    out = []
    for tree in trees:
        for t in slicings(net, tree, deltas, seed):
            prog = tn.TNProgram(net, t)
            out.append((t, prog, tree_features(net, t, prog.plan.info)))
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
