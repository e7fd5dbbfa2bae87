// Host lowering of a gate list into scheduled operations and fused LDS-tile stages.
//
// The state-vector mode of the paper (Sec. 3.1) applies the gate matrices one after
// another. The lowering keeps that product exactly and only regroups it:
//   * consecutive one-qubit gates on the same qubit are multiplied into one 2x2
//     (gates on other qubits commute with them);
//   * diagonal gates (Z, RZ, CZ, RZZ) never need their qubits to be tile-local: the
//     value of every index bit is known inside a tile, so they are applied in place;
//   * a stage is one read and one write of the state: a tile holds 2^t amplitudes whose
//     index varies over t "local" qubits (the lowest index bits always among them so that
//     HBM accesses are contiguous), and every operation whose non-diagonal target is
//     local and whose earlier dependencies are done is applied in LDS/registers;
//   * inside a stage, phases hold R target bits per thread in registers; moving between
//     phases is one LDS exchange.
// The schedule depends only on the circuit structure, so it is built once and reused for
// new parameter values (the paper's reuse of compiled circuits and contraction paths).
#include <algorithm>
#include <set>

#include "tq_internal.h"

namespace tq {

int gate_n_angles(int op) {
  switch (op) {
    case TQ_RX: case TQ_RY: case TQ_RZ: case TQ_RZZ: case TQ_CRX: case TQ_CRY: case TQ_CRZ: return 1;
    case TQ_U3: case TQ_ROT: return 3;
    default: return 0;
  }
}
static bool is_controlled_rotation(int op) { return op == TQ_CRX || op == TQ_CRY || op == TQ_CRZ; }
static int n_qubits_of(int op) {
  return (op == TQ_CNOT || op == TQ_CZ || op == TQ_RZZ || is_controlled_rotation(op)) ? 2 : 1;
}

bool has_controlled(const tq_gate* g, int64_t n_gates) {
  for (int64_t k = 0; k < n_gates; ++k)
    if (is_controlled_rotation(g[k].op)) return true;
  return false;
}

// Controlled rotations become gates the kernels apply directly, by exact identities (no
// global phase is introduced, so amplitudes are unchanged), on (control c, target t):
//   CRZ(a) = RZ_t(a/2) RZZ_ct(-a/2)    (both diagonal: diag(1, 1, e^{-ia/2}, e^{ia/2}))
//   CRX(a) = H_t CRZ(a) H_t            (H Z H = X)
//   CRY(a) = RZ_t(pi/2) CRX(a) RZ_t(-pi/2)   (RZ(pi/2) X RZ(-pi/2) = Y)
// An angle a = pscale * params[pidx] keeps its parameter with half (or minus half) the scale,
// so gradients summed over the pieces are those of the original gate.
void lower_controlled(const tq_gate* g, int n_gates, std::vector<tq_gate>& out) {
  const double half_pi = 1.5707963267948966;
  auto one = [](int op, int q, int32_t pidx, double scale) {
    tq_gate x{};
    x.op = op;
    x.q[0] = q;
    x.q[1] = -1;
    x.pidx[0] = pidx;
    x.pidx[1] = x.pidx[2] = -1;
    x.pscale[0] = scale;
    return x;
  };
  for (int k = 0; k < n_gates; ++k) {
    const tq_gate& x = g[k];
    if (!is_controlled_rotation(x.op)) {
      out.push_back(x);
      continue;
    }
    const int c = x.q[0], t = x.q[1];
    const int32_t pi = x.pidx[0];
    const double sc = x.pscale[0];  // the angle's scale, or the constant angle when pi < 0
    if (x.op == TQ_CRY) out.push_back(one(TQ_RZ, t, -1, -half_pi));
    if (x.op != TQ_CRZ) out.push_back(one(TQ_H, t, -1, 0.0));
    out.push_back(one(TQ_RZ, t, pi, 0.5 * sc));
    tq_gate zz = one(TQ_RZZ, c, pi, -0.5 * sc);
    zz.q[1] = t;
    out.push_back(zz);
    if (x.op != TQ_CRZ) out.push_back(one(TQ_H, t, -1, 0.0));
    if (x.op == TQ_CRY) out.push_back(one(TQ_RZ, t, -1, half_pi));
  }
}
static bool diag1(int op) { return op == TQ_Z || op == TQ_RZ; }

tq_status validate_gates(const tq_gate* g, int n_gates, int n, int n_params) {
  if (n_gates < 0) return fail(TQ_EINVAL, "negative gate count");
  if (n_gates > 0 && g == nullptr) return fail(TQ_EINVAL, "null gate array");
  for (int k = 0; k < n_gates; ++k) {
    const tq_gate& x = g[k];
    if (x.op < 0 || x.op >= TQ_NUM_OPS)
      return fail(TQ_EINVAL, "gate " + std::to_string(k) + ": unknown op " + std::to_string(x.op));
    int nq = n_qubits_of(x.op);
    for (int i = 0; i < nq; ++i)
      if (x.q[i] < 0 || x.q[i] >= n)
        return fail(TQ_EINVAL, "gate " + std::to_string(k) + ": qubit " + std::to_string(x.q[i]) +
                                   " outside [0," + std::to_string(n) + ")");
    if (nq == 2 && x.q[0] == x.q[1])
      return fail(TQ_EINVAL, "gate " + std::to_string(k) + ": duplicate qubit");
    for (int j = 0; j < gate_n_angles(x.op); ++j)
      if (x.pidx[j] >= n_params)
        return fail(TQ_EINVAL, "gate " + std::to_string(k) + ": parameter index " +
                                   std::to_string(x.pidx[j]) + " >= n_params " + std::to_string(n_params));
  }
  return TQ_OK;
}

void lower_ops(const tq_gate* g, int n_gates, int n, bool fuse, std::vector<Recipe>& recipes,
               std::vector<HostOp>& ops) {
  recipes.clear();
  ops.clear();
  if (!fuse) {
    for (int k = 0; k < n_gates; ++k) {
      const tq_gate& x = g[k];
      if (x.op == TQ_CNOT) {
        ops.push_back({K_CX, x.q[1], x.q[0], -1, k});
      } else if (x.op == TQ_CZ) {
        ops.push_back({K_CZ, x.q[0], x.q[1], -1, k});
      } else if (x.op == TQ_RZZ) {
        recipes.push_back({R_DIAG2, x.q[0], x.q[1], {k}});
        ops.push_back({K_DIAG2, x.q[0], x.q[1], (int)recipes.size() - 1, -1});
      } else if (diag1(x.op)) {
        recipes.push_back({R_DIAG1, x.q[0], -1, {k}});
        ops.push_back({K_DIAG1, x.q[0], -1, (int)recipes.size() - 1, -1});
      } else {
        recipes.push_back({R_MAT2, x.q[0], -1, {k}});
        ops.push_back({K_MAT1, x.q[0], -1, (int)recipes.size() - 1, -1});
      }
    }
    return;
  }
  std::vector<std::vector<int>> pending(n);
  std::vector<int> last(n, -1);  // last emitted op touching each qubit
  auto flush = [&](int q) {
    if (pending[q].empty()) return;
    bool all_diag = true;
    for (int k : pending[q]) all_diag = all_diag && diag1(g[k].op);
    recipes.push_back({all_diag ? R_DIAG1 : R_MAT2, q, -1, pending[q]});
    ops.push_back({all_diag ? K_DIAG1 : K_MAT1, q, -1, (int)recipes.size() - 1, -1});
    last[q] = (int)ops.size() - 1;
    pending[q].clear();
  };
  auto pending_all_diag = [&](int q) {
    for (int k : pending[q])
      if (!diag1(g[k].op)) return false;
    return true;
  };
  for (int k = 0; k < n_gates; ++k) {
    const tq_gate& x = g[k];
    if (n_qubits_of(x.op) == 1) {
      pending[x.q[0]].push_back(k);
      continue;
    }
    int a = x.q[0], b = x.q[1];
    if (x.op == TQ_CNOT) {
      flush(a);
      flush(b);
      ops.push_back({K_CX, b, a, -1, k});
      last[a] = last[b] = (int)ops.size() - 1;
      continue;
    }
    // CZ / RZZ: diagonal on (a, b). Pending diagonal one-qubit gates merge into it.
    bool pa = pending_all_diag(a), pb = pending_all_diag(b);
    std::vector<int> pre;
    if (pa) { pre.insert(pre.end(), pending[a].begin(), pending[a].end()); pending[a].clear(); } else flush(a);
    if (pb) { pre.insert(pre.end(), pending[b].begin(), pending[b].end()); pending[b].clear(); } else flush(b);
    int lo = last[a];
    bool merge = lo >= 0 && lo == last[b] && (ops[lo].kind == K_DIAG2 || ops[lo].kind == K_CZ);
    if (merge) {
      HostOp& o = ops[lo];
      if (o.kind == K_CZ) {  // the earlier CZ had no recipe: give it one
        recipes.push_back({R_DIAG2, o.qa, o.qb, {o.src}});
        o.kind = K_DIAG2;
        o.mat = (int)recipes.size() - 1;
      }
      Recipe& r = recipes[o.mat];
      r.gates.insert(r.gates.end(), pre.begin(), pre.end());
      r.gates.push_back(k);
    } else if (x.op == TQ_CZ && pre.empty()) {
      ops.push_back({K_CZ, a, b, -1, k});
      last[a] = last[b] = (int)ops.size() - 1;
    } else {
      std::vector<int> gl = pre;
      gl.push_back(k);
      recipes.push_back({R_DIAG2, a, b, gl});
      ops.push_back({K_DIAG2, a, b, (int)recipes.size() - 1, -1});
      last[a] = last[b] = (int)ops.size() - 1;
    }
  }
  for (int q = 0; q < n; ++q) flush(q);
}

static void op_qubits(const HostOp& o, int* qs, int* nq, int* need) {
  *nq = 0;
  qs[(*nq)++] = o.qa;
  if (o.qb >= 0) qs[(*nq)++] = o.qb;
  *need = (o.kind == K_MAT1 || o.kind == K_CX) ? o.qa : -1;
}

// Greedy selection of a set of at most `cap` "need" resources (qubits or tile positions)
// starting from `fixed`; takes every op, in order, that is not blocked by an earlier
// skipped op on a shared qubit and whose need fits. Returns taken ops; the rest stay.
static void greedy_take(const std::vector<HostOp>& all, std::vector<int>& remaining, std::set<int>& S,
                        int cap, const std::vector<int>& res_of_qubit, std::vector<int>& taken) {
  std::set<int> blocked;
  std::vector<int> rest;
  for (int oi : remaining) {
    int qs[2], nq, need;
    op_qubits(all[oi], qs, &nq, &need);
    bool blk = false;
    for (int i = 0; i < nq; ++i) blk = blk || blocked.count(qs[i]);
    int r = need >= 0 ? res_of_qubit[need] : -1;
    bool ok = !blk && (r < 0 || S.count(r) || (int)S.size() < cap);
    if (ok) {
      if (r >= 0) S.insert(r);
      taken.push_back(oi);
    } else {
      for (int i = 0; i < nq; ++i) blocked.insert(qs[i]);
      rest.push_back(oi);
    }
  }
  remaining.swap(rest);
}

// Register bits an op reads or changes, and whether it is diagonal (diagonal ops commute
// with each other).
static uint32_t op_reg_bits(const DevOp& d, bool* diag) {
  *diag = false;
  if (d.kind == K_MAT1) return 1u << d.rbit;
  if (d.kind == K_CX) return (1u << d.rbit) | (d.pb ? 1u << (d.pb - 1) : 0u);
  *diag = true;
  const int ka = (d.rbit & 15) - 1, kb = (d.rbit >> 4) - 1;
  return (ka >= 0 ? 1u << ka : 0u) | (kb >= 0 ? 1u << kb : 0u);
}

// Forward stages: order one phase's ops by layers and merge each layer's one-qubit matrices
// and CZs. Ops in one layer touch disjoint register bits (thread and tile bits are never
// changed inside a phase), so they commute; a layer is the earliest one after every op
// that must precede. One-qubit matrices of a layer become one MATG op (their matrices get
// consecutive table indices through `remap`); register-register CZs become the uniform
// flip mask of a ZG op, which also takes up to two CZs with one register operand. This
// cuts the per-op loop overhead of the stage kernel; the arithmetic is the same.
static void emit_layered(const std::vector<DevOp>& pd, int R, std::vector<int>& remap, int& n_mapped,
                         std::vector<DevOp>& out) {
  const int n = (int)pd.size();
  const size_t first = out.size();  // ops of earlier phases are not touched
  std::vector<int> lay(n);
  int last_any[8] = {0}, last_nd[8] = {0}, top = 0;
  for (int i = 0; i < n; ++i) {
    bool diag;
    const uint32_t b = op_reg_bits(pd[i], &diag);
    int l = 1;
    for (int k = 0; k < R; ++k)
      if ((b >> k) & 1u) l = std::max(l, 1 + (diag ? last_nd[k] : last_any[k]));
    lay[i] = l;
    top = std::max(top, l);
    for (int k = 0; k < R; ++k)
      if ((b >> k) & 1u) {
        last_any[k] = std::max(last_any[k], l);
        if (!diag) last_nd[k] = l;
      }
  }
  auto new_mat = [&](int old) {
    if (remap[old] < 0) remap[old] = n_mapped++;
    return remap[old];
  };
  for (int l = 1; l <= top; ++l) {
    // one-qubit matrices, ascending register bit (a bit holds at most one per layer)
    int mat_of_bit[8];
    uint32_t mask = 0;
    for (int i = 0; i < n; ++i)
      if (lay[i] == l && pd[i].kind == K_MAT1) {
        mask |= 1u << pd[i].rbit;
        mat_of_bit[pd[i].rbit] = pd[i].mat;
      }
    bool fresh = true;  // the group's matrices can take consecutive new indices
    for (int k = 0; k < R; ++k)
      if (((mask >> k) & 1u) && remap[mat_of_bit[k]] >= 0) fresh = false;
    if (mask && !fresh) {
      for (int i = 0; i < n; ++i)
        if (lay[i] == l && pd[i].kind == K_MAT1) {
          DevOp d = pd[i];
          d.mat = new_mat(d.mat);
          out.push_back(d);
        }
    } else if (mask) {
      DevOp g{};
      g.kind = K_MATG;
      g.rbit = (uint8_t)mask;
      g.mat = -1;
      for (int k = 0; k < R; ++k)
        if ((mask >> k) & 1u) {
          const int m = new_mat(mat_of_bit[k]);
          if (g.mat < 0) g.mat = m;
        }
      out.push_back(g);
    }
    // CZs: register-register ones as a flip mask, up to two register-other ones per op
    uint32_t flips = 0;
    std::vector<std::pair<int, int>> half;  // (register index, partner x-position)
    for (int i = 0; i < n; ++i) {
      if (lay[i] != l || pd[i].kind != K_CZ) continue;
      const int ka = (pd[i].rbit & 15) - 1, kb = (pd[i].rbit >> 4) - 1;
      if (ka >= 0 && kb >= 0) {
        for (int j = 0; j < (1 << R); ++j)
          if (((j >> ka) & 1) && ((j >> kb) & 1)) flips ^= 1u << j;
      } else if (ka >= 0) {
        half.push_back({ka, pd[i].pb});
      } else if (kb >= 0) {
        half.push_back({kb, pd[i].pa});
      } else {
        out.push_back(pd[i]);  // no register operand: stays a plain CZ
      }
    }
    // with only register-register CZs, the flips ride on the matrix op emitted just before
    // (pa | pb << 8) if it belongs to this phase: it is this layer's (disjoint bits) or the
    // previous layer's last op, so nothing lies between it and the flips
    if (half.empty() && flips != 0 && out.size() > first && out.back().kind == K_MATG && R <= 4) {
      out.back().pa ^= (uint8_t)(flips & 0xffu);
      out.back().pb ^= (uint8_t)(flips >> 8);
      flips = 0;
    }
    size_t h = 0;
    bool any = flips != 0 || !half.empty();
    while (any) {
      DevOp z{};
      z.kind = K_ZG;
      z.mat = (int32_t)flips;
      flips = 0;
      if (h < half.size()) {
        z.rbit = (uint8_t)(half[h].first + 1);
        z.pa = (uint8_t)half[h].second;
        ++h;
      }
      if (h < half.size()) {
        z.rbit |= (uint8_t)((half[h].first + 1) << 4);
        z.pb = (uint8_t)half[h].second;
        ++h;
      }
      out.push_back(z);
      any = h < half.size();
    }
    // everything else of the layer in program order
    for (int i = 0; i < n; ++i) {
      if (lay[i] != l || pd[i].kind == K_MAT1 || pd[i].kind == K_CZ) continue;
      DevOp d = pd[i];
      if (d.mat >= 0) d.mat = new_mat(d.mat);
      out.push_back(d);
    }
  }
}

void build_stages(Schedule& s) {
  const int n = s.n;
  s.stages.clear();
  s.phases.clear();
  s.dops.clear();
  s.dstages.clear();
  const int t = std::min(s.t, n);
  const int R = std::min(s.R, t);
  // layered grouping: forward schedules whose register index fits a 16-way mask
  const bool group = !s.adjoint && R <= 4;
  std::vector<int> remap(group ? s.recipes.size() : 0, -1);
  int n_mapped = 0;
  const int c = std::min(s.c, std::max(0, t - 1));
  std::vector<int> remaining(s.ops.size());
  for (size_t i = 0; i < s.ops.size(); ++i) remaining[i] = (int)i;
  std::vector<int> pos_of_q(n);
  for (int q = 0; q < n; ++q) pos_of_q[q] = n - 1 - q;
  while (!remaining.empty()) {
    std::set<int> S;  // global positions of local qubits
    if (t == n) {
      for (int p = 0; p < n; ++p) S.insert(p);
    } else {
      for (int p = 0; p < c; ++p) S.insert(p);
    }
    std::vector<int> taken;
    greedy_take(s.ops, remaining, S, t, pos_of_q, taken);
    if (s.adjoint) {
      // cap the gradient slots of one stage (their partial sums live in LDS); the ops cut
      // off are later in program order than every op kept, so they return to `remaining`
      int slots = 0;
      size_t keep = 0;
      while (keep < taken.size() && slots + s.ops[taken[keep]].nang <= kAdjMaxSlotsPerStage)
        slots += s.ops[taken[keep++]].nang;
      if (keep < taken.size()) {
        remaining.insert(remaining.end(), taken.begin() + keep, taken.end());
        std::sort(remaining.begin(), remaining.end());
        taken.resize(keep);
      }
    }
    // fill the local set up to t with the lowest free positions
    for (int p = 0; (int)S.size() < t && p < n; ++p) S.insert(p);
    StageHost st;
    st.t = t;
    st.lpos.assign(S.begin(), S.end());
    for (int p = 0; p < n; ++p)
      if (!S.count(p)) st.npos.push_back(p);
    std::vector<int> loc_of_pos(n, -1);
    for (int i = 0; i < t; ++i) loc_of_pos[st.lpos[i]] = i;
    auto xpos = [&](int q) {
      int p = pos_of_q[q];
      if (loc_of_pos[p] >= 0) return loc_of_pos[p];
      int k = (int)(std::lower_bound(st.npos.begin(), st.npos.end(), p) - st.npos.begin());
      return t + k;
    };
    // phases: register sets over tile-local positions
    std::vector<int> loc_of_q(n);
    for (int q = 0; q < n; ++q) loc_of_q[q] = loc_of_pos[pos_of_q[q]];
    st.phase_begin = (int)s.phases.size();
    std::vector<int> prem = taken;
    std::vector<uint8_t> cur_r, cur_t;  // current layout (starts as the load layout)
    for (int k = 0; k < R; ++k) cur_r.push_back((uint8_t)(t - R + k));
    for (int k = 0; k < t - R; ++k) cur_t.push_back((uint8_t)k);
    while (!prem.empty()) {
      std::set<int> Rs;
      std::vector<int> ptaken;
      greedy_take(s.ops, prem, Rs, R, loc_of_q, ptaken);
      // keep bits of the current layout where possible (fewer changes is not required for
      // correctness; it only makes the register order stable), then fill
      std::vector<int> rv(Rs.begin(), Rs.end());
      for (int k = t - 1; (int)rv.size() < R && k >= 0; --k)
        if (!Rs.count(k)) { rv.push_back(k); Rs.insert(k); }
      std::sort(rv.begin(), rv.end());
      DevPhase ph{};
      ph.op_begin = (int)s.dops.size();
      std::vector<uint8_t> nr, nt;
      for (int k = 0; k < R; ++k) nr.push_back((uint8_t)rv[k]);
      for (int k = 0; k < t; ++k)
        if (!Rs.count(k)) nt.push_back((uint8_t)k);
      ph.xchg = (nr != cur_r) ? 1 : 0;
      cur_r = nr;
      cur_t = nt;
      for (int k = 0; k < R; ++k) ph.rpos[k] = nr[k];
      for (int k = 0; k < t - R; ++k) ph.tpos[k] = nt[k];
      std::vector<DevOp> pd;  // this phase's ops in program order
      for (int oi : ptaken) {
        const HostOp& o = s.ops[oi];
        DevOp d{};
        d.kind = (uint8_t)o.kind;
        d.mat = o.mat;
        // register index of a qubit in this phase, or -1 (thread or tile bit)
        auto reg_of = [&](int q) {
          const int lp = loc_of_q[q];
          if (lp < 0) return -1;
          const auto it = std::find(rv.begin(), rv.end(), lp);
          return it == rv.end() ? -1 : (int)(it - rv.begin());
        };
        if (o.kind == K_MAT1 || o.kind == K_CX) {
          d.rbit = (uint8_t)reg_of(o.qa);
          if (o.kind == K_CX) {
            d.pa = (uint8_t)xpos(o.qb);
            d.pb = (uint8_t)(reg_of(o.qb) + 1);  // control's register index + 1 (0: not a register bit)
          }
        } else {
          d.pa = (uint8_t)xpos(o.qa);
          d.pb = o.qb >= 0 ? (uint8_t)xpos(o.qb) : 0;
          // register indices + 1 of both operands (0: not a register bit), low and high nibble
          const int ka = reg_of(o.qa), kb = o.qb >= 0 ? reg_of(o.qb) : -1;
          d.rbit = (uint8_t)((ka + 1) | ((kb + 1) << 4));
        }
        pd.push_back(d);
      }
      if (group) {
        emit_layered(pd, R, remap, n_mapped, s.dops);
        // the stage kernel takes grouped phases' ops two at a time: pad to an even count
        // with a sign group that flips nothing
        if ((s.dops.size() - (size_t)ph.op_begin) % 2 != 0) {
          DevOp z{};
          z.kind = K_ZG;
          s.dops.push_back(z);
        }
      } else {
        s.dops.insert(s.dops.end(), pd.begin(), pd.end());
      }
      ph.op_end = (int)s.dops.size();
      s.phases.push_back(ph);
      st.n_ops += (int)ptaken.size();
    }
    st.phase_end = (int)s.phases.size();
    DevStage ds{};
    {
      std::vector<uint8_t> load_r;
      for (int k = 0; k < R; ++k) load_r.push_back((uint8_t)(t - R + k));
      ds.store_xchg = (cur_r != load_r) ? 1 : 0;
    }
    ds.t = t;
    ds.phase_begin = st.phase_begin;
    ds.phase_end = st.phase_end;
    ds.n_nonlocal = n - t;
    for (int i = 0; i < t; ++i) ds.lpos[i] = (uint8_t)st.lpos[i];
    for (int i = 0; i < n - t; ++i) ds.npos[i] = (uint8_t)st.npos[i];
    s.dstages.push_back(ds);
    s.stages.push_back(std::move(st));
  }
  if (group) {
    // renumber the matrix table in first-use order (recipes no op uses go last)
    int next = n_mapped;
    for (int& r : remap)
      if (r < 0) r = next++;
    std::vector<Recipe> rec(s.recipes.size());
    for (size_t i = 0; i < s.recipes.size(); ++i) rec[remap[i]] = std::move(s.recipes[i]);
    s.recipes = std::move(rec);
    for (HostOp& o : s.ops)
      if (o.mat >= 0) o.mat = remap[o.mat];
  }
}

}  // namespace tq

namespace tq {

// Reverse-sweep op list. A run of one-qubit gates on one qubit with no other gate on that
// qubit in between (at most three angles, at most kAdjMaxRun gates) is reversed as one op:
// the gates between its members act on other qubits and commute with it, so it sits at the
// position of its last gate. Every other gate is its own op. mat holds the gate index of
// the op's last gate (its matrix-table entry); nang the op's angle count.
static bool adj_one_qubit(int op) { return op != TQ_CNOT && op != TQ_CZ && op != TQ_RZZ; }

void lower_adjoint_ops(const tq_gate* g, int n_gates, std::vector<HostOp>& ops, std::vector<int32_t>& runs) {
  ops.clear();
  // group runs in forward order
  std::vector<std::vector<int>> run_of_last(n_gates);  // run gates, stored at the last one
  std::vector<char> is_member(n_gates, 0);            // inside a run that ends later
  std::vector<std::vector<int>> open(kMaxQ + 1);
  std::vector<int> open_ang(kMaxQ + 1, 0);
  auto close = [&](int q) {
    if (open[q].empty()) return;
    const int last = open[q].back();
    for (size_t i = 0; i + 1 < open[q].size(); ++i) is_member[open[q][i]] = 1;
    run_of_last[last] = open[q];
    open[q].clear();
    open_ang[q] = 0;
  };
  for (int k = 0; k < n_gates; ++k) {
    const tq_gate& x = g[k];
    const int na = gate_n_angles(x.op);
    if (adj_one_qubit(x.op)) {
      const int q = x.q[0];
      if (!open[q].empty() && (open_ang[q] + na > 3 || (int)open[q].size() >= kAdjMaxRun)) close(q);
      open[q].push_back(k);
      open_ang[q] += na;
    } else {
      close(x.q[0]);
      close(x.q[1]);
      run_of_last[k] = {k};
    }
  }
  for (int q = 0; q <= kMaxQ; ++q) close(q);
  runs.assign(n_gates + 1, 0);
  std::vector<int32_t> list;
  for (int k = 0; k < n_gates; ++k) {
    runs[k] = (int32_t)list.size();
    if (!is_member[k]) list.insert(list.end(), run_of_last[k].begin(), run_of_last[k].end());
  }
  runs[n_gates] = (int32_t)list.size();
  runs.insert(runs.end(), list.begin(), list.end());

  for (int k = n_gates - 1; k >= 0; --k) {
    if (is_member[k]) continue;
    const tq_gate& x = g[k];
    const std::vector<int>& rg = run_of_last[k];
    HostOp o{};
    o.mat = k;
    o.src = k;
    o.nang = 0;
    for (int m : rg) o.nang += gate_n_angles(g[m].op);
    if (x.op == TQ_CNOT) { o.kind = K_CX; o.qa = x.q[1]; o.qb = x.q[0]; }
    else if (x.op == TQ_CZ) { o.kind = K_CZ; o.qa = x.q[0]; o.qb = x.q[1]; }
    else if (x.op == TQ_RZZ) { o.kind = K_DIAG2; o.qa = x.q[0]; o.qb = x.q[1]; }
    else if (rg.size() == 1 && diag1(x.op)) { o.kind = K_DIAG1; o.qa = x.q[0]; o.qb = -1; }
    else { o.kind = K_MAT1; o.qa = x.q[0]; o.qb = -1; }
    ops.push_back(o);
  }
}

// Gradient slots: one per (gate, angle), numbered stage by stage in execution order, plus
// the parameter -> slots table used by the final reduction.
void build_adjoint_slots(Schedule& s, const tq_gate* g, int n_gates) {
  s.dslot.assign(s.dops.size(), 0);
  s.stage_slot0.clear();
  s.stage_nslot.clear();
  s.slot_gate.clear();
  s.slot_angle.clear();
  int global = 0;
  for (size_t st = 0; st < s.dstages.size(); ++st) {
    s.stage_slot0.push_back(global);
    int local = 0;
    for (int p = s.dstages[st].phase_begin; p < s.dstages[st].phase_end; ++p)
      for (int o = s.phases[p].op_begin; o < s.phases[p].op_end; ++o) {
        // the op's angles: its run's gates in forward order, each gate's angles in order
        const int k = s.dops[o].mat;
        const int base = n_gates + 1;
        int na = 0;
        for (int r = s.adj_runs[k]; r < s.adj_runs[k + 1]; ++r) {
          const int m = s.adj_runs[base + r];
          for (int j = 0; j < gate_n_angles(g[m].op); ++j) {
            s.slot_gate.push_back(m);
            s.slot_angle.push_back(j);
            ++na;
          }
        }
        s.dslot[o] = (local << 2) | na;
        local += na;
      }
    s.stage_nslot.push_back(local);
    global += local;
  }
  s.n_slots = global;
  int np = 0;
  for (int k = 0; k < n_gates; ++k)
    for (int j = 0; j < gate_n_angles(g[k].op); ++j) np = std::max(np, g[k].pidx[j] + 1);
  s.n_params_used = np;
  std::vector<std::vector<std::pair<int, double>>> by(np);
  for (int sl = 0; sl < global; ++sl) {
    const tq_gate& x = g[s.slot_gate[sl]];
    const int pi = x.pidx[s.slot_angle[sl]];
    if (pi >= 0) by[pi].push_back({sl, x.pscale[s.slot_angle[sl]]});
  }
  s.pslot_ptr.assign(1, 0);
  s.pslot_idx.clear();
  s.pslot_scale.clear();
  for (int p = 0; p < np; ++p) {
    std::sort(by[p].begin(), by[p].end());
    for (auto& e : by[p]) {
      s.pslot_idx.push_back(e.first);
      s.pslot_scale.push_back(e.second);
    }
    s.pslot_ptr.push_back((int)s.pslot_idx.size());
  }
}

}  // namespace tq
