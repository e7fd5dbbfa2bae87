"""Host planner of the tensor-network mode (paper Sec. 3.2).

Steps (a)-(d) of the paper's TN workflow run here, once per circuit structure; step (e),
the contraction, runs in libtq kernels (tq_tn_contract / tq_tn_backward):

(a) circuit -> network: the expectation value <psi|O|psi> needs the circuit followed by
    its complex-conjugate copy (Sec. 3.2.1). Gates outside the reverse light cone of the
    measured qubits cancel against their conjugates and are dropped.
(b) structural simplification (Sec. 3.2.1): a diagonal gate (RZ, Z, CZ, RZZ) does not
    start a new index on its qubits; it becomes a tensor on the existing wire indices, so
    a wire index may join many tensors (a hyperedge, Sec. 3.2.1 and its figure). An
    anti-diagonal gate (X; Y as a diagonal then X) becomes no tensor at all: it flips its
    wire, and the wire's later tensors are built with that index complemented. Rank
    simplification then absorbs every tensor whose contraction with a neighbour does not
    raise the rank (|0> vectors, one-qubit gates, diagonals).
(c) contraction trees: the path search's pool (min-fill and min-degree elimination,
    pairwise greedy, and the own recursive balanced bisection of the tensor hypergraph,
    Sec. 3.2.2), ranked by the paper's FLOP count p(2q-1) per pairwise step.
(d) slicing (Sec. 3.2.3): the two-phase search fixes indices until every intermediate fits
    the target size; the value is the sum of the identical sub-network contractions.

Every index has dimension 2. A tensor with index list [i_0, .., i_{r-1}] is stored as 2^r
complex numbers with i_0 the most significant bit.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

from . import workloads as W

# leaf kinds: how the device builds a leaf from the circuit parameters (tq_tn_leaves)
LEAF_CONST = 0   # constant tensor given by value
LEAF_GATE1 = 1   # one-qubit gate matrix [out, in] (conj on the bra side)
LEAF_DIAG1 = 2   # one-qubit diagonal gate as a vector over the wire index
LEAF_DIAG2 = 3   # two-qubit diagonal gate as a 2x2 over the two wire indices
LEAF_GATE2 = 4   # two-qubit gate [out_a, out_b, in_a, in_b]


@dataclasses.dataclass
class Leaf:
    inds: List[int]
    kind: int
    gate: int = -1         # index into the circuit's gate list
    conj: bool = False     # bra-side copy
    value: np.ndarray = None  # LEAF_CONST data (complex128, 2^rank)
    flip: int = 0          # element e holds entry e ^ flip (bit 0 = last index): flipped wires


@dataclasses.dataclass
class Network:
    leaves: List[Leaf]
    n_index: int
    output: List[int]
    gates: np.ndarray      # the circuit's gate records (the leaves refer to them)
    params: np.ndarray     # parameter vector
    qubits: List[int] = dataclasses.field(default_factory=list)  # register qubits the network keeps


_DIAG = {W.Z, W.RZ, W.CZ, W.RZZ}


def light_cone(gates, qubits):
    """Indices of the gates in the reverse causal cone of ``qubits`` (program order), and
    the cone's qubits. Diagonal gates commute with one another and with the Z observable:
    within a run of consecutive diagonal gates, membership is decided against the cone as
    it stands after the run, so a cost layer of RZZ gates widens a QAOA cone by one graph
    step (nodes within distance p of the measured edge)."""
    cone = set(qubits)
    keep = []
    pending, grow = False, set()
    for k in range(len(gates) - 1, -1, -1):
        g = gates[k]
        op = int(g["op"])
        qs = [int(q) for q in g["q"][: W.N_QUBITS[op]]]
        if op in _DIAG:
            pending = True
            if cone & set(qs):
                keep.append(k)
                grow |= set(qs)
            continue
        if pending:
            cone |= grow
            pending, grow = False, set()
        if cone & set(qs):
            keep.append(k)
            cone |= set(qs)
    cone |= grow
    return keep[::-1], cone


def circuit_network(c: W.Circuit, zqubits, use_light_cone=True):
    """Doubled network of <psi| prod Z |psi> for psi = U|0..0>, with diagonal gates as
    hyperedge tensors. Controlled rotations are first lowered to the gates the kernels build
    (tq_lower_gates). Returns a Network whose leaves reference its ``gates``."""
    gates = c.gates
    if np.isin(gates["op"], [W.CRX, W.CRY, W.CRZ]).any():
        from . import lib
        gates = lib.lower_gates(gates)
    if use_light_cone:
        keep, used = light_cone(gates, zqubits)
    else:
        keep, used = list(range(len(gates))), set(range(c.n))
    used = sorted(set(used) | set(zqubits))
    nidx = [0]

    def new():
        nidx[0] += 1
        return nidx[0] - 1

    leaves = []
    ket = {q: new() for q in used}
    bra = {q: new() for q in used}
    # anti-diagonal reduction (Sec. 3.2.1): X is no tensor, it flips its wire, and Y is the
    # diagonal diag(i, -i) then a flip; every later tensor on a flipped wire reads that index
    # complemented (the ket and bra halves flip alike, so their final identity is unchanged)
    flipped = {q: 0 for q in used}

    def fmask(qs):
        m = 0
        for k, q in enumerate(qs):
            m |= flipped[q] << (len(qs) - 1 - k)
        return m

    e0 = np.array([1.0, 0.0], dtype=np.complex128)
    ydiag = np.array([1j, -1j], dtype=np.complex128)
    for q in used:
        leaves.append(Leaf([ket[q]], LEAF_CONST, value=e0))
        leaves.append(Leaf([bra[q]], LEAF_CONST, value=e0))
    for k in keep:
        g = gates[k]
        op = int(g["op"])
        qs = [int(q) for q in g["q"][: W.N_QUBITS[op]]]
        if op in (W.X, W.Y):
            q = qs[0]
            if op == W.Y:
                leaves.append(Leaf([ket[q]], LEAF_CONST, value=ydiag, flip=flipped[q]))
                leaves.append(Leaf([bra[q]], LEAF_CONST, value=ydiag.conj(), flip=flipped[q]))
            flipped[q] ^= 1
            continue
        if op in _DIAG:
            kind = LEAF_DIAG1 if len(qs) == 1 else LEAF_DIAG2
            leaves.append(Leaf([ket[q] for q in qs], kind, k, False, flip=fmask(qs)))
            leaves.append(Leaf([bra[q] for q in qs], kind, k, True, flip=fmask(qs)))
            continue
        kout = [new() for _ in qs]
        bout = [new() for _ in qs]
        kind = LEAF_GATE1 if len(qs) == 1 else LEAF_GATE2
        leaves.append(Leaf(kout + [ket[q] for q in qs], kind, k, False, flip=fmask(qs)))
        leaves.append(Leaf(bout + [bra[q] for q in qs], kind, k, True, flip=fmask(qs)))
        for i, q in enumerate(qs):
            ket[q] = kout[i]
            bra[q] = bout[i]
            flipped[q] = 0
    # observable: identity merges the ket and bra wire; Z adds a [1, -1] vector on it
    merged = {}
    for q in used:
        merged[bra[q]] = ket[q]
    for lf in leaves:
        lf.inds = [merged.get(i, i) for i in lf.inds]
    zv = np.array([1.0, -1.0], dtype=np.complex128)
    for q in zqubits:
        leaves.append(Leaf([ket[q]], LEAF_CONST, value=zv, flip=flipped[q]))
    # renumber indices densely
    ren = {}
    for lf in leaves:
        for i in lf.inds:
            if i not in ren:
                ren[i] = len(ren)
    for lf in leaves:
        lf.inds = [ren[i] for i in lf.inds]
    return Network(leaves, len(ren), [], gates, c.params, used)


def qaoa_edge_network(prob: W.QAOAProblem, edge):
    """<Z_i Z_j> network of one edge of a QAOA graph: the whole-register circuit reduced to
    the reverse light cone of the edge's two qubits, then doubled. The cone's qubits are
    the graph nodes within distance p of the edge. Returns (network, cone qubits)."""
    net = circuit_network(W.qaoa_circuit(prob), list(edge), use_light_cone=True)
    return net, list(net.qubits)


# ---- contraction trees -----------------------------------------------------------------

@dataclasses.dataclass
class Tree:
    """SSA pairwise order: step s contracts tensors pairs[s] = (a, b) (ids < n_leaves are
    leaves, id n_leaves + s is the result of step s). The last step yields the output."""
    pairs: List[tuple]
    n_leaves: int
    flops: float = 0.0         # paper's count: sum p(2q-1)
    max_rank: int = 0
    sliced: List[int] = dataclasses.field(default_factory=list)
    step_ranks: List[tuple] = dataclasses.field(default_factory=list)


def _index_counts(tensors):
    cnt = {}
    for t in tensors:
        for i in t:
            cnt[i] = cnt.get(i, 0) + 1
    return cnt


def _out_inds(a, b, cnt, output):
    """Indices kept after contracting index sets a, b: those appearing in other tensors or
    in the output (count over all live tensors, minus the two being merged)."""
    sa, sb = set(a), set(b)
    keep = []
    for i in list(dict.fromkeys(list(a) + list(b))):
        inside = (i in sa) + (i in sb)
        if cnt[i] > inside or i in output:
            keep.append(i)
    return keep


def greedy_tree(net: Network, rng=None, temperature=0.0, sliced=()):
    """Greedy pairwise order: repeatedly contract the connected pair with the smallest
    cost = size(out) - size(a) - size(b) (random-greedy: Boltzmann-perturbed choice)."""
    sl = set(sliced)
    tensors = {i: tuple(x for x in lf.inds if x not in sl) for i, lf in enumerate(net.leaves)}
    cnt = _index_counts(tensors.values())
    output = set(net.output)
    nid = len(net.leaves)
    # index -> live tensor ids
    holders = {}
    for tid, t in tensors.items():
        for i in t:
            holders.setdefault(i, set()).add(tid)
    pairs = []

    def cost(a, b):
        o = _out_inds(tensors[a], tensors[b], cnt, output)
        return 2.0 ** len(o) - 2.0 ** len(tensors[a]) - 2.0 ** len(tensors[b]), o

    while len(tensors) > 1:
        cands = set()
        for i, hs in holders.items():
            if len(hs) >= 2:
                hl = sorted(hs)
                for x in range(len(hl)):
                    for y in range(x + 1, len(hl)):
                        cands.add((hl[x], hl[y]))
        if not cands:  # disconnected: join the two smallest
            ids = sorted(tensors, key=lambda t: len(tensors[t]))[:2]
            cands = {(min(ids), max(ids))}
        scored = []
        for a, b in cands:
            c, o = cost(a, b)
            scored.append((c, a, b, o))
        if rng is not None and temperature > 0:
            cs = np.array([s[0] for s in scored])
            w = np.exp(-(cs - cs.min()) / (temperature * max(1.0, abs(cs.min())) + 1e-12))
            k = int(rng.choice(len(scored), p=w / w.sum()))
            _, a, b, o = scored[k]
        else:
            _, a, b, o = min(scored)
        pairs.append((a, b))
        for i in tensors[a]:
            cnt[i] -= 1
            holders[i].discard(a)
        for i in tensors[b]:
            cnt[i] -= 1
            holders[i].discard(b)
        del tensors[a], tensors[b]
        tensors[nid] = tuple(o)
        for i in o:
            cnt[i] = cnt.get(i, 0) + 1
            holders.setdefault(i, set()).add(nid)
        nid += 1
    tree = Tree(pairs, len(net.leaves))
    score_tree(net, tree)
    return tree


def tree_steps(net: Network, tree: Tree, sliced=None):
    """Index lists of every step: list of (a_inds, b_inds, out_inds)."""
    sl = set(tree.sliced if sliced is None else sliced)
    ts = [tuple(x for x in lf.inds if x not in sl) for lf in net.leaves]
    cnt = _index_counts(ts)
    output = set(net.output)
    steps = []
    for a, b in tree.pairs:
        o = _out_inds(ts[a], ts[b], cnt, output)
        for i in ts[a]:
            cnt[i] -= 1
        for i in ts[b]:
            cnt[i] -= 1
        for i in o:
            cnt[i] = cnt.get(i, 0) + 1
        steps.append((ts[a], ts[b], tuple(o)))
        ts.append(tuple(o))
    return steps


def step_flops(a, b, o):
    """Paper Sec. 3.2.2: FLOPs = p(2q - 1), p = product of outer dims, q = contracted."""
    sa, sb, so = set(a), set(b), set(o)
    q = 2 ** len((sa & sb) - so)
    p = 2 ** len(so)
    return p * (2 * q - 1)


def score_tree(net: Network, tree: Tree):
    steps = tree_steps(net, tree)
    tree.flops = float(sum(step_flops(*s) for s in steps)) * 2 ** len(tree.sliced)
    tree.max_rank = max([len(s[2]) for s in steps] + [len(s[0]) for s in steps] + [len(s[1]) for s in steps] + [0])
    tree.step_ranks = [(len(a), len(b), len(o)) for a, b, o in steps]
    return tree


def slice_tree(net: Network, tree: Tree, target_rank, rng=None):
    """Greedy slicing (Sec. 3.2.3): while some intermediate has more than target_rank
    indices, fix the index that appears in the most over-size intermediates (ties: the
    one that lowers the largest rank most, then the lowest id; random repeats pick among
    ties with ``rng``)."""
    sliced = list(tree.sliced)
    while True:
        steps = tree_steps(net, tree, sliced)
        big = [s[2] for s in steps if len(s[2]) > target_rank] + [s[0] for s in steps if len(s[0]) > target_rank]
        if not big:
            break
        freq = {}
        for t in big:
            for i in t:
                freq[i] = freq.get(i, 0) + 1
        best = max(freq.values())
        ties = sorted(i for i, f in freq.items() if f == best)
        pick = ties[0] if rng is None else int(rng.choice(ties))
        sliced.append(pick)
    t2 = Tree(list(tree.pairs), tree.n_leaves, sliced=sliced)
    score_tree(net, t2)
    return t2


def elimination_order(net: Network, rng=None, mode="fill", sliced=()):
    """Index elimination order on the interaction graph (vertices = indices, every tensor
    a clique): repeatedly remove the index with the fewest fill-in edges (``fill``) or the
    smallest degree (``degree``); ``rng`` breaks near-ties at random. Returns (order,
    width) where width = largest neighbourhood met (rank of the biggest intermediate)."""
    sl = set(sliced)
    adj = {}
    for lf in net.leaves:
        t = set(lf.inds) - sl
        for i in t:
            adj.setdefault(i, set()).update(t - {i})
    for i in net.output:
        adj.pop(i, None)
        for x in adj.values():
            x.discard(i)
    order, width = [], 0
    while adj:
        cand = []
        for i, nb in adj.items():
            if mode == "fill":
                nbl = list(nb)
                f = sum(1 for x in range(len(nbl)) for y in range(x + 1, len(nbl)) if nbl[y] not in adj[nbl[x]])
                cand.append(((f, len(nb)), i))
            else:
                cand.append(((len(nb), 0), i))
        cand.sort()
        if rng is not None:
            k0 = cand[0][0][0]
            ties = [c for c in cand[:6] if c[0][0] <= k0 + (1 if mode == "degree" else max(1, k0 // 4))]
            _, i = ties[int(rng.integers(len(ties)))]
        else:
            _, i = cand[0]
        nb = adj.pop(i)
        width = max(width, len(nb))
        for x in nb:
            adj[x] |= nb - {x}
            adj[x].discard(i)
        order.append(i)
    return order, width


def elimination_tree(net: Network, order):
    """Pairwise tree from an elimination order: for each index in turn, the live tensors
    holding it are merged (smallest first); the index is summed at the last merge."""
    live = {i: tuple(lf.inds) for i, lf in enumerate(net.leaves)}
    nid = len(net.leaves)
    pairs = []
    for idx in order:
        hold = sorted([t for t, inds in live.items() if idx in inds], key=lambda t: (len(live[t]), t))
        while len(hold) > 1:
            a, b = hold[0], hold[1]
            merged = tuple(dict.fromkeys(live[a] + live[b]))
            pairs.append((a, b))
            del live[a], live[b]
            live[nid] = merged
            hold = sorted([nid] + hold[2:], key=lambda t: (len(live[t]), t))
            nid += 1
    rest = sorted(live, key=lambda t: (len(live[t]), t))
    while len(rest) > 1:  # disconnected parts (scalars): outer products
        a, b = rest[0], rest[1]
        pairs.append((a, b))
        live[nid] = tuple(dict.fromkeys(live[a] + live[b]))
        del live[a], live[b]
        rest = sorted([nid] + rest[2:], key=lambda t: (len(live[t]), t))
        nid += 1
    tree = Tree(pairs, len(net.leaves))
    score_tree(net, tree)
    return tree


def candidate_trees(net: Network, n_random=31, seed=0, target_rank=28):
    """Candidate contraction trees for ranking (flop model or learned cost model): the
    min-fill and min-degree elimination trees, the pairwise greedy tree, then random
    restarts of all three heuristics; each sliced to ``target_rank``."""
    rng = np.random.default_rng(seed)
    out = []
    for mode in ("fill", "degree"):
        out.append(slice_tree(net, elimination_tree(net, elimination_order(net, None, mode)[0]), target_rank))
    out.append(slice_tree(net, greedy_tree(net), target_rank))
    for r in range(n_random):
        kind = r % 3
        if kind == 2:
            t = greedy_tree(net, rng, temperature=0.3 + 0.7 * rng.random())
        else:
            t = elimination_tree(net, elimination_order(net, rng, "fill" if kind == 0 else "degree")[0])
        out.append(slice_tree(net, t, target_rank, rng))
    return out


# ---- structural simplification and recursive bisection (Sec. 3.2.1, 3.2.2) --------------------

def rank_simplify(net: Network, sliced=()):
    """Rank simplification (Sec. 3.2.1): repeatedly contract a pair of tensors sharing an
    index whenever the result has no more indices than the larger of the two (absorbing the
    |0> vectors, one-qubit gates and diagonal tensors into their neighbours). Returns the SSA
    pairs and the remaining tensors as {id: index tuple}."""
    sl = set(sliced)
    live = {i: tuple(x for x in lf.inds if x not in sl) for i, lf in enumerate(net.leaves)}
    cnt = _index_counts(live.values())
    output = set(net.output)
    holders = {}
    for tid, t in live.items():
        for i in t:
            holders.setdefault(i, set()).add(tid)
    pairs = []
    nid = len(net.leaves)
    changed = True
    while changed:
        changed = False
        for tid in sorted(live, key=lambda t: (len(live[t]), t)):
            if tid not in live:
                continue
            best = None
            for i in live[tid]:
                for other in holders.get(i, ()):
                    if other == tid or other not in live:
                        continue
                    o = _out_inds(live[tid], live[other], cnt, output)
                    if len(o) <= max(len(live[tid]), len(live[other])):
                        key = (len(o), len(live[other]), other)
                        if best is None or key < best[0]:
                            best = (key, other, o)
            if best is None:
                continue
            _, other, o = best
            a, b = min(tid, other), max(tid, other)
            pairs.append((a, b))
            for j in live[a]:
                cnt[j] -= 1
                holders[j].discard(a)
            for j in live[b]:
                cnt[j] -= 1
                holders[j].discard(b)
            del live[a], live[b]
            live[nid] = tuple(o)
            for j in o:
                cnt[j] = cnt.get(j, 0) + 1
                holders.setdefault(j, set()).add(nid)
            nid += 1
            changed = True
    return pairs, live


def _bisect(verts, tens, rng, imbalance, kept_outside):
    """Balanced two-way split of ``verts`` (tensor ids with index tuples ``tens``) that cuts
    few indices: region growing from a random seed to half the vertices, then passes of
    single-vertex moves (Fiduccia-Mattheyses style: best gain first, each vertex moved once
    per pass, the best prefix kept) within the balance bound. An index counts as cut when
    tensors on both sides hold it; indices also held outside ``verts`` are cut whatever the
    split and do not count."""
    verts = list(verts)
    n = len(verts)
    edges = {}
    for v in verts:
        for i in tens[v]:
            if i not in kept_outside:
                edges.setdefault(i, []).append(v)
    nbr = {v: set() for v in verts}
    for i, hs in edges.items():
        for v in hs:
            nbr[v].update(hs)
    for v in verts:
        nbr[v].discard(v)
    lo = int(math.floor(n * (0.5 - imbalance / 2)))
    hi = n - lo
    seed = verts[int(rng.integers(n))]
    side = {v: 1 for v in verts}
    side[seed] = 0
    frontier = [seed]
    size0 = 1
    order = list(verts)
    while size0 < n // 2:
        if not frontier:  # disconnected: restart from any unassigned vertex
            rest = [v for v in order if side[v] == 1]
            frontier = [rest[int(rng.integers(len(rest)))]]
            side[frontier[0]] = 0
            size0 += 1
            continue
        v = frontier.pop(0)
        cand = [w for w in nbr[v] if side[w] == 1]
        rng.shuffle(cand)
        for w in cand:
            if size0 >= n // 2:
                break
            side[w] = 0
            size0 += 1
            frontier.append(w)

    def counts():
        c = {}
        for i, hs in edges.items():
            a = sum(1 for v in hs if side[v] == 0)
            c[i] = [a, len(hs) - a]
        return c

    def cut(c):
        return sum(1 for a, b in c.values() if a and b)

    for _ in range(6):
        c = counts()
        best_cut, cur = cut(c), cut(c)
        locked, moves, best_k = set(), [], 0
        size = [sum(1 for v in verts if side[v] == 0), 0]
        size[1] = n - size[0]
        for _step in range(n):
            best = None
            for v in verts:
                if v in locked:
                    continue
                s0 = side[v]
                if size[s0] - 1 < lo:
                    continue
                g = 0
                for i in tens[v]:
                    if i in c:
                        a, b = c[i][s0], c[i][1 - s0]
                        if a == 1 and b > 0:
                            g += 1
                        elif b == 0 and a > 1:
                            g -= 1
                if best is None or g > best[0]:
                    best = (g, v)
            if best is None:
                break
            g, v = best
            s0 = side[v]
            side[v] = 1 - s0
            size[s0] -= 1
            size[1 - s0] += 1
            for i in tens[v]:
                if i in c:
                    c[i][s0] -= 1
                    c[i][1 - s0] += 1
            cur -= g
            locked.add(v)
            moves.append(v)
            if cur < best_cut:
                best_cut, best_k = cur, len(moves)
        for v in moves[best_k:][::-1]:  # undo the moves after the best prefix
            side[v] = 1 - side[v]
        if best_k == 0:
            break
    A = [v for v in verts if side[v] == 0]
    B = [v for v in verts if side[v] == 1]
    return A, B


def bisection_tree(net: Network, rng=None, imbalance=0.2, leaf_size=8, simplify=True, sliced=()):
    """Contraction tree by recursive balanced bisection of the tensor hypergraph (Sec. 3.2.2:
    the tensors are split in two parts sharing few indices, each part is split again, and the
    parts are contracted bottom up), after rank simplification. Parts of at most
    ``leaf_size`` tensors are ordered greedily."""
    rng = np.random.default_rng(0) if rng is None else rng
    pairs, live = rank_simplify(net, sliced) if simplify else ([], {
        i: tuple(x for x in lf.inds if x not in set(sliced)) for i, lf in enumerate(net.leaves)})
    tens = dict(live)
    nid = [len(net.leaves) + len(pairs)]
    output = set(net.output)
    holder = {}
    for t, inds in tens.items():
        for i in inds:
            holder.setdefault(i, set()).add(t)

    def contract(a, b, outside):
        o = [i for i in dict.fromkeys(tens[a] + tens[b])
             if i in output or i in outside or (holder[i] - {a, b})]
        pairs.append((a, b))
        c = nid[0]
        nid[0] += 1
        for i in tens[a]:
            holder[i].discard(a)
        for i in tens[b]:
            holder[i].discard(b)
        tens[c] = tuple(o)
        for i in o:
            holder.setdefault(i, set()).add(c)
        return c

    def solve(verts):
        verts = list(verts)
        if len(verts) == 1:
            return verts[0]
        vs = set(verts)
        outside = {i for v in verts for i in tens[v] if i in output or (holder[i] - vs)}
        if len(verts) <= leaf_size:
            cur = list(verts)
            while len(cur) > 1:
                best = None
                for x in range(len(cur)):
                    for y in range(x + 1, len(cur)):
                        a, b = cur[x], cur[y]
                        shared = set(tens[a]) & set(tens[b])
                        o = [i for i in dict.fromkeys(tens[a] + tens[b])
                             if i in output or i in outside or (holder[i] - {a, b})]
                        key = (0 if shared else 1, 2.0 ** len(o) - 2.0 ** len(tens[a]) - 2.0 ** len(tens[b]), x, y)
                        if best is None or key < best[0]:
                            best = (key, a, b)
                _, a, b = best
                c = contract(a, b, outside)
                cur = [v for v in cur if v not in (a, b)] + [c]
            return cur[0]
        A, B = _bisect(verts, tens, rng, imbalance, outside)
        if not A or not B:
            half = len(verts) // 2
            A, B = verts[:half], verts[half:]
        ra, rb = solve(A), solve(B)
        return contract(ra, rb, outside)

    solve(sorted(tens))
    tree = Tree(pairs, len(net.leaves))
    score_tree(net, tree)
    return tree


def slice_search(net: Network, tree: Tree, target_rank, trials=8, rng=None):
    """Two-phase slicing (Sec. 3.2.3): the greedy slicing first (pseudo-slicing: fix the
    index met in the most over-size intermediates), then randomised trials that break ties
    at random; the slicing with the fewest total FLOPs (all slices) is kept."""
    rng = np.random.default_rng(0) if rng is None else rng
    best = slice_tree(net, tree, target_rank)
    for _ in range(trials):
        t = slice_tree(net, tree, target_rank, rng)
        if (t.flops, len(t.sliced)) < (best.flops, len(best.sliced)):
            best = t
    return best


def tree_pool(net: Network, seed=0, n_bisect=4):
    """The path search's candidate trees of one network (unsliced): min-fill and min-degree
    elimination, pairwise greedy, and ``n_bisect`` recursive-bisection trees with different
    seeds, balance bounds and leaf-part sizes."""
    out = [elimination_tree(net, elimination_order(net, None, "fill")[0]),
           elimination_tree(net, elimination_order(net, None, "degree")[0]),
           greedy_tree(net)]
    shapes = [(0.1, 8), (0.3, 14), (0.2, 10), (0.3, 8), (0.1, 14), (0.2, 16)]
    for k in range(n_bisect):
        imb, leaf = shapes[k % len(shapes)]
        out.append(bisection_tree(net, np.random.default_rng(seed * 1000 + k), imbalance=imb, leaf_size=leaf))
    return out


def best_tree(net: Network, seed=0, n_bisect=4, target_rank=None, slice_trials=4):
    """The fewest-FLOP tree of the pool (the paper's FLOP ranking, Sec. 3.2.2), sliced to
    ``target_rank`` by the two-phase slicing search when it is wider (Sec. 3.2.3)."""
    t = min(tree_pool(net, seed, n_bisect), key=lambda x: (x.flops, x.max_rank))
    if target_rank is not None and t.max_rank > target_rank:
        t = slice_search(net, t, target_rank, slice_trials, np.random.default_rng(seed))
    return t


def _plan_edge(args):
    prob, edge, seed, n_bisect, target_rank = args
    net, _ = qaoa_edge_network(prob, edge)
    return net, best_tree(net, seed, n_bisect, target_rank)


def plan_qaoa(prob: W.QAOAProblem, edges=None, n_bisect=4, target_rank=None, workers=1):
    """(network, fewest-FLOP tree of the pool, sliced to ``target_rank``) for every edge; the
    host search runs in ``workers`` spawned processes (it holds no GPU state)."""
    edges = list(prob.edges) if edges is None else list(edges)
    jobs = [(prob, e, k, n_bisect, target_rank) for k, e in enumerate(edges)]
    if workers <= 1:
        return [_plan_edge(j) for j in jobs]
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_plan_edge, jobs, chunksize=2))


# ---- device execution (steps (e) and its reverse) -------------------------------------------

def leaf_specs(net: Network):
    """tq_tn_leaf records and the constant values of a circuit network."""
    from . import lib

    specs = np.zeros(len(net.leaves), dtype=lib.TN_LEAF_DTYPE)
    consts = []
    for i, lf in enumerate(net.leaves):
        specs[i]["kind"] = lf.kind
        specs[i]["gate"] = lf.gate
        specs[i]["conj"] = 1 if lf.conj else 0
        specs[i]["flip"] = lf.flip
        if lf.kind == LEAF_CONST:
            specs[i]["const_off"] = sum(len(c) for c in consts)
            consts.append(np.asarray(lf.value, dtype=np.complex128).reshape(-1))
    cv = np.concatenate(consts) if consts else np.zeros(1, dtype=np.complex128)
    return specs, cv


class TNProgram:
    """A planned circuit network: builds leaves from parameters, contracts, differentiates."""

    def __init__(self, net: Network, tree: Tree, c128=False, slice_group=0, mem_budget=0, store_policy=0):
        from . import lib

        self.net, self.tree = net, tree
        self.plan = lib.TnPlan([lf.inds for lf in net.leaves], tree.pairs, tree.sliced, net.output, c128,
                               slice_group, mem_budget, store_policy=store_policy)
        self.specs, self.consts = leaf_specs(net)
        self.c128 = c128

    def leaves(self, params):
        from . import lib
        return lib.tn_build_leaves(self.plan, self.net.gates, self.specs, self.consts, params)

    def value(self, params):
        from . import lib
        return lib.tn_contract(self.plan, self.leaves(params))

    def grad(self, params, grad_out=None):
        """d Re(T) / d params (times grad_out) through the reverse pass and the chain rule."""
        import torch
        from . import lib

        L = self.leaves(params)
        g = torch.ones(1 << self.plan.n_out, dtype=L.dtype, device=L.device) if grad_out is None else grad_out
        env = lib.tn_backward(self.plan, L, g)
        return lib.tn_param_grad(self.plan, self.net.gates, self.specs, params, env)

    def value_and_grad(self, params, grad_out=None, work=None):
        """Value and d Re(T)/d params in one pass pair: tq_tn_contract then tq_tn_backward on
        one workspace (under the store policy the reverse pass reuses the intermediates)."""
        import torch
        from . import lib

        L = self.leaves(params)
        need = self.plan.workspace_bytes(True)
        if work is None or work.numel() < need:
            work = torch.empty(max(need, 16), dtype=torch.uint8, device=L.device)
        v = lib.tn_contract(self.plan, L, work)
        g = torch.ones(1 << self.plan.n_out, dtype=L.dtype, device=L.device) if grad_out is None else grad_out
        env = lib.tn_backward(self.plan, L, g, work)
        return v, lib.tn_param_grad(self.plan, self.net.gates, self.specs, params, env)


class TNBatch:
    """Many planned networks evaluated together (tq_tn_contract_batch / tq_tn_backward_batch):
    the 75 light-cone networks of a QAOA graph run as one launch, one work-group each."""

    def __init__(self, programs):
        self.programs = list(programs)
        self.plans = [p.plan for p in self.programs]

    def values(self, params_list):
        from . import lib
        return lib.tn_contract_batch(self.plans, self._leaves(params_list))

    def _unit_grad_outs(self, leaves):
        """Upstream values of all ones, one shared read-only tensor per output size and dtype."""
        import torch

        cache = self.__dict__.setdefault("_ones", {})
        outs = []
        for p, L in zip(self.programs, leaves):
            key = (1 << p.plan.n_out, L.dtype, L.device)
            if key not in cache:
                cache[key] = torch.ones(key[0], dtype=L.dtype, device=L.device)
            outs.append(cache[key])
        return outs

    def grads(self, params_list, grad_outs=None):
        """d Re(T_k) / d params_k (times grad_outs[k]) for every network k."""
        return self.value_and_grads(params_list, grad_outs, values=False)[1]

    def _same_dtype(self):
        return len({p.plan.c128 for p in self.programs}) <= 1

    def _leaves(self, params_list):
        from . import lib

        if not self._same_dtype():
            return [p.leaves(q) for p, q in zip(self.programs, params_list)]
        P = self.programs
        return lib.tn_build_leaves_batch(self.plans, [p.net.gates for p in P], [p.specs for p in P],
                                         [p.consts for p in P], params_list)

    def value_and_grads(self, params_list, grad_outs=None, values=True):
        """Values and d Re(T_k) / d params_k of every network from one build of the leaves:
        the leaves of all networks in one launch, the batched forward, the batched reverse
        pass on the same leaves, and the chain rule of all networks in one launch."""
        from . import lib

        leaves = self._leaves(params_list)
        if grad_outs is None:
            grad_outs = self._unit_grad_outs(leaves)
        vals = lib.tn_contract_batch(self.plans, leaves) if values else None
        envs = lib.tn_backward_batch(self.plans, leaves, grad_outs)
        P = self.programs
        if not self._same_dtype():
            return vals, [lib.tn_param_grad(p.plan, p.net.gates, p.specs, q, e) for p, q, e in zip(P, params_list, envs)]
        return vals, lib.tn_param_grad_batch(self.plans, [p.net.gates for p in P], [p.specs for p in P], params_list,
                                             envs)


def tn_expval(program: TNProgram, params):
    """Differentiable Re(T) of a scalar network (torch.autograd.Function)."""
    import torch

    class _F(torch.autograd.Function):
        @staticmethod
        def forward(ctx, p):
            ctx.save_for_backward(p)
            return program.value(p).real.to(p.dtype)

        @staticmethod
        def backward(ctx, g):
            (p,) = ctx.saved_tensors
            cdt = torch.complex128 if program.c128 else torch.complex64
            return program.grad(p, g.to(cdt)).to(p.dtype)

    return _F.apply(params)
