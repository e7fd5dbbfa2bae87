// Compiled batches (tq_svb_*): a batch of circuits of uneven size and structure compiled
// once and evaluated many times (the paper's reusable compiled circuit, Sec. 2, and its
// vmap batches, Sec. 5.3).
//
// Every circuit keeps its own fused schedule. Stage k of all circuits that have a stage k
// forms one "level"; a level is one kernel launch over a work list of (circuit, tile) items,
// longest items first, with the work-group sized for the level's largest tile. Levels are
// ordered by stream order only: no work-group ever waits on another, so there are no
// inter-work-group spins. The whole launch sequence of a call (initial state, gate matrices,
// levels, expectation values; or the reverse sweep) is captured once per set of buffer
// pointers and replayed as a HIP graph. The autotuner times candidate tile shapes on the
// device and keeps the fastest.
#include <algorithm>
#include <array>
#include <map>

#include "sv_device.h"

namespace tq {
namespace {

// Device buffer owned by a compiled batch.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  tq_status ensure(size_t want) {
    if (want == 0) want = 256;
    if (bytes >= want) return TQ_OK;
    release();
    if (hipMalloc(&p, want) != hipSuccess) {
      p = nullptr;
      return fail(TQ_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes for a compiled batch failed");
    }
    bytes = want;
    return TQ_OK;
  }
  template <typename V>
  tq_status upload(const std::vector<V>& v) {
    TQ_TRY(ensure(std::max<size_t>(v.size() * sizeof(V), 16)));
    if (!v.empty()) TQ_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice));
    return TQ_OK;
  }
};

// Circuits with equal n: initial state and expectation-value launches.
struct NGroup {
  int n = 0;
  std::vector<int> members;
  BatchMap smap{}, rows{};
  const unsigned char* terms = nullptr;
  size_t pcap = 0;
};

struct GraphEntry {
  int which = 0;
  std::array<const void*, 4> ptrs{};
  hipGraphExec_t exec = nullptr;
};

struct LevelBufs {
  BatchLaunch L;
  DevBuf circ, pref, ppref, items;
};

}  // namespace
}  // namespace tq

using namespace tq;

struct tq_svb {
  tq_ctx* ctx = nullptr;
  int dt = TQ_C64;
  int count = 0;
  std::vector<int32_t> n, n_gates, n_params;
  std::vector<int64_t> gate_off, param_off, state_off;
  std::vector<tq_gate> gates;
  std::vector<tq_zterm> terms;
  int n_obs = 1;
  tq_svb_opts opts{};
  bool adj_tuned = false;  // the adjoint shape came from a tuning table
  std::string key;
  int64_t grad_elems = 0;  // 1 + largest parameter offset + count
  // forward
  LevelBufs fwd;
  DevBuf mats;
  std::vector<NGroup> ngroups;
  DevBuf exp_partial;
  // reverse sweep (built on first use)
  bool adj_built = false;
  LevelBufs adj;
  DevBuf adj_mats, psi, lam, partial;
  // graphs
  hipStream_t cap = nullptr;
  std::vector<GraphEntry> graphs;
  int64_t captures = 0, replays = 0;

  ~tq_svb() {
    clear_graphs();
    if (cap) (void)hipStreamDestroy(cap);
  }
  void clear_graphs() {
    for (GraphEntry& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  tq_batch view() const {
    return tq_batch{count, n.data(), gate_off.data(), n_gates.data(), param_off.data(), state_off.data()};
  }
};

namespace tq {
namespace {

// Per-level work lists: items of level L are the tiles of stage L of every circuit that has
// one, longest stages first (ties: batch order, then tile).
void make_levels(const std::vector<Schedule*>& sched, const std::vector<int32_t>& n, BatchLaunch& L,
                 std::vector<BatchItem>& items, bool adjoint) {
  size_t levels = 0;
  for (Schedule* s : sched) levels = std::max(levels, s->stages.size());
  L.level_begin.assign(1, 0);
  L.level_t.clear();
  L.level_nslot.clear();
  items.clear();
  for (size_t lv = 0; lv < levels; ++lv) {
    std::vector<std::pair<int, int>> order;  // (-ops, circuit)
    int tmax = 1, smax = 0;
    for (size_t i = 0; i < sched.size(); ++i) {
      const Schedule* s = sched[i];
      if (lv >= s->stages.size()) continue;
      order.push_back({-s->stages[lv].n_ops, (int)i});
      tmax = std::max(tmax, s->stages[lv].t);
      if (adjoint) smax = std::max(smax, s->stage_nslot[lv]);
    }
    std::stable_sort(order.begin(), order.end());
    for (const auto& o : order) {
      const int i = o.second;
      const uint32_t tiles = 1u << (n[i] - sched[i]->stages[lv].t);
      for (uint32_t tl = 0; tl < tiles; ++tl) items.push_back({i, tl});
    }
    L.level_begin.push_back((int64_t)items.size());
    L.level_t.push_back(tmax);
    L.level_nslot.push_back(smax);
  }
}

size_t csize(int dt) { return dt == TQ_C64 ? 8 : 16; }

// Forward schedules, descriptors and work lists for shape (T, R, c).
tq_status build_forward(tq_svb* b, int T, int R, int c) {
  tq_ctx* ctx = b->ctx;
  int min_t = 64;
  for (int i = 0; i < b->count; ++i) min_t = std::min(min_t, std::min(T, b->n[i]));
  const int Reff = std::max(1, std::min(R, min_t));
  const tq_sv_opts so{0, T, Reff, c};
  const tq_batch bv = b->view();
  std::vector<Group> groups;
  TQ_TRY(group_batch(&bv, b->n_params.data(), groups));
  std::vector<Schedule*> sched(b->count, nullptr);
  for (const Group& gr : groups) {
    Schedule* s;
    TQ_TRY(get_schedule(ctx, b->dt, b->gates.data() + gr.gate_off, gr.n_gates, gr.n, 0, &so, &s));
    for (int i : gr.members) sched[i] = s;
  }
  std::vector<DevCirc> hc(b->count);
  std::vector<int64_t> pref(b->count + 1, 0);
  for (int i = 0; i < b->count; ++i) {
    const Schedule* s = sched[i];
    DevCirc& d = hc[i];
    std::memset(&d, 0, sizeof d);
    d.stages = (const DevStage*)s->d_stages;
    d.phases = (const DevPhase*)s->d_phases;
    d.ops = (const DevOp*)s->d_ops;
    d.gates = (const tq_gate*)s->d_gates;
    d.rec = (const int32_t*)s->d_rec;
    d.rec_gates = (const int32_t*)s->d_rec_gates;
    d.mats_off = 4 * pref[i];
    d.state_off = b->state_off[i];
    d.param_off = b->param_off[i];
    d.n = b->n[i];
    d.n_mats = (int32_t)s->recipes.size();
    d.n_stages = (int32_t)s->stages.size();
    d.n_params = b->n_params[i];
    d.row = i;
    pref[i + 1] = pref[i] + d.n_mats;
  }
  std::vector<BatchItem> items;
  BatchLaunch& L = b->fwd.L;
  make_levels(sched, b->n, L, items, false);
  TQ_TRY(b->fwd.circ.upload(hc));
  TQ_TRY(b->fwd.pref.upload(pref));
  TQ_TRY(b->fwd.items.upload(items));
  L.d_circ = (const DevCirc*)b->fwd.circ.p;
  L.d_pref = (const int64_t*)b->fwd.pref.p;
  L.d_items = (const BatchItem*)b->fwd.items.p;
  L.count = b->count;
  L.total_mats = pref[b->count];
  L.T = T;
  L.R = Reff;
  TQ_TRY(b->mats.ensure((size_t)std::max<int64_t>(L.total_mats, 1) * 4 * csize(b->dt)));
  return TQ_OK;
}

tq_status build_adjoint(tq_svb* b, int T, int R, int c) {
  tq_ctx* ctx = b->ctx;
  int min_t = 64;
  for (int i = 0; i < b->count; ++i) min_t = std::min(min_t, std::min(T, b->n[i]));
  const int Reff = std::max(1, std::min(R, min_t));
  const tq_sv_opts so{0, T, Reff, c};
  const tq_batch bv = b->view();
  std::vector<Group> groups;
  TQ_TRY(group_batch(&bv, b->n_params.data(), groups));
  std::vector<Schedule*> sched(b->count, nullptr);
  for (const Group& gr : groups) {
    Schedule* s;
    TQ_TRY(get_adjoint_schedule(ctx, b->dt, b->gates.data() + gr.gate_off, gr.n_gates, gr.n, &so, &s));
    for (int i : gr.members) sched[i] = s;
  }
  std::map<int, const unsigned char*> tt;
  for (int i = 0; i < b->count; ++i)
    if (!tt.count(b->n[i]))
      TQ_TRY(term_table(ctx, b->n[i], b->terms.data(), (int)b->terms.size(), &tt[b->n[i]]));
  std::vector<DevCirc> hc(b->count);
  std::vector<int64_t> pref(b->count + 1, 0), ppref(b->count + 1, 0);
  int64_t work = 0, part = 0, max_amps = 1;
  for (int i = 0; i < b->count; ++i) {
    const Schedule* s = sched[i];
    DevCirc& d = hc[i];
    std::memset(&d, 0, sizeof d);
    d.stages = (const DevStage*)s->d_stages;
    d.phases = (const DevPhase*)s->d_phases;
    d.ops = (const DevOp*)s->d_ops;
    d.gates = (const tq_gate*)s->d_gates;
    d.rec = (const int32_t*)s->d_stage_slot0;
    d.rec_gates = (const int32_t*)s->d_adj_runs;
    d.dslot = (const int32_t*)s->d_dslot;
    d.pslot_ptr = (const int32_t*)s->d_pslot_ptr;
    d.pslot_idx = (const int32_t*)s->d_pslot_idx;
    d.pslot_scale = (const double*)s->d_pslot_scale;
    d.terms = tt[b->n[i]];
    d.mats_off = (int64_t)kAdjMatStride * pref[i];
    d.state_off = b->state_off[i];
    d.param_off = b->param_off[i];
    d.work_off = work;
    d.part_off = part;
    d.n = b->n[i];
    d.n_mats = b->n_gates[i];
    d.n_stages = (int32_t)s->stages.size();
    d.n_slots = s->n_slots;
    d.n_params = b->n_params[i];
    d.n_used = std::min(s->n_params_used, b->n_params[i]);
    d.row = i;
    d.n_terms = (int32_t)b->terms.size();
    const int64_t amps = int64_t(1) << d.n;
    const int64_t ntiles = s->stages.empty() ? 1 : (int64_t(1) << (d.n - s->stages[0].t));
    work += amps;
    part += std::max<int64_t>(1, (int64_t)s->n_slots * ntiles);
    max_amps = std::max(max_amps, amps);
    pref[i + 1] = pref[i] + d.n_mats;
    ppref[i + 1] = ppref[i] + d.n_params;
  }
  std::vector<BatchItem> items;
  BatchLaunch& L = b->adj.L;
  make_levels(sched, b->n, L, items, true);
  TQ_TRY(b->adj.circ.upload(hc));
  TQ_TRY(b->adj.pref.upload(pref));
  TQ_TRY(b->adj.ppref.upload(ppref));
  TQ_TRY(b->adj.items.upload(items));
  L.d_circ = (const DevCirc*)b->adj.circ.p;
  L.d_pref = (const int64_t*)b->adj.pref.p;
  L.d_ppref = (const int64_t*)b->adj.ppref.p;
  L.d_items = (const BatchItem*)b->adj.items.p;
  L.count = b->count;
  L.total_mats = pref[b->count];
  L.total_params = ppref[b->count];
  L.max_amps = max_amps;
  L.T = T;
  L.R = Reff;
  TQ_TRY(b->adj_mats.ensure((size_t)std::max<int64_t>(L.total_mats, 1) * kAdjMatStride * csize(b->dt)));
  TQ_TRY(b->psi.ensure((size_t)work * csize(b->dt)));
  TQ_TRY(b->lam.ensure((size_t)work * csize(b->dt)));
  TQ_TRY(b->partial.ensure((size_t)part * sizeof(double)));
  b->adj_built = true;
  return TQ_OK;
}

// Init / expval groups (by n).
tq_status build_ngroups(tq_svb* b) {
  tq_ctx* ctx = b->ctx;
  std::map<int, std::vector<int>> by_n;
  for (int i = 0; i < b->count; ++i) by_n[b->n[i]].push_back(i);
  b->ngroups.clear();
  size_t pcap = 0;
  for (auto& kv : by_n) {
    NGroup g;
    g.n = kv.first;
    g.members = kv.second;
    TQ_TRY(member_map(ctx, S_MISC, b->state_off.data(), g.members, nullptr, &g.smap));
    std::vector<int64_t> rows(g.members.begin(), g.members.end());
    std::vector<int> ident(g.members.size());
    for (size_t i = 0; i < ident.size(); ++i) ident[i] = (int)i;
    TQ_TRY(member_map(ctx, S_MISC, rows.data(), ident, nullptr, &g.rows));
    TQ_TRY(term_table(ctx, g.n, b->terms.data(), (int)b->terms.size(), &g.terms));
    g.pcap = expval_scratch_doubles(g.n, (int)g.members.size(), b->n_obs);
    pcap = std::max(pcap, g.pcap);
    b->ngroups.push_back(std::move(g));
  }
  TQ_TRY(b->exp_partial.ensure(pcap * sizeof(double)));
  return TQ_OK;
}

void default_fwd(int dt, int* T, int* R, int* c) {
  *T = dt == TQ_C64 ? 13 : 12;
  *R = 4;
  *c = dt == TQ_C64 ? 5 : 4;
}
void default_adj(int dt, int* T, int* R, int* c) {
  *T = dt == TQ_C64 ? 12 : 11;
  *R = dt == TQ_C64 ? 4 : 3;
  *c = dt == TQ_C64 ? 5 : 4;
}

void fwd_shape(const tq_svb* b, int* T, int* R, int* c) {
  default_fwd(b->dt, T, R, c);
  if (b->opts.tile_bits) *T = b->opts.tile_bits;
  if (b->opts.reg_bits) *R = b->opts.reg_bits;
  if (b->opts.coal_bits) *c = b->opts.coal_bits;
}
void adj_shape(const tq_svb* b, int* T, int* R, int* c) {
  default_adj(b->dt, T, R, c);
  if (b->opts.adj_tile_bits) *T = b->opts.adj_tile_bits;
  if (b->opts.adj_reg_bits) *R = b->opts.adj_reg_bits;
  if (b->opts.adj_coal_bits) *c = b->opts.adj_coal_bits;
}

template <typename T>
tq_status enqueue_forward(tq_svb* b, const void* d_params, void* d_states, void* d_out, hipStream_t s) {
  using C = typename Cx<T>::type;
  if (b->opts.init == 0)
    for (const NGroup& g : b->ngroups)
      TQ_TRY(launch_init_basis<T>(d_states, g.smap, g.n, (int)g.members.size(), 0, b->ctx->n_cu, s));
  TQ_TRY(launch_batch_forward<T>(b->fwd.L, d_params, b->mats.p, d_states, s));
  if (d_out) {
    const int nt = (int)b->terms.size();
    for (const NGroup& g : b->ngroups)
      TQ_TRY(launch_expval<T>((const C*)d_states, g.smap, g.n, (int)g.members.size(), (const uint64_t*)g.terms,
                              (const double*)(g.terms + 8 * (size_t)nt), (const int32_t*)(g.terms + 16 * (size_t)nt),
                              nt, b->n_obs, (double*)b->exp_partial.p, b->exp_partial.bytes / sizeof(double),
                              (T*)d_out, g.rows, s));
  }
  return TQ_OK;
}

template <typename T>
tq_status enqueue_backward(tq_svb* b, const void* d_params, const void* d_states, const void* d_grad_out,
                           void* d_grad, hipStream_t s) {
  return launch_batch_adjoint<T>(b->adj.L, d_params, b->adj_mats.p, d_states, b->psi.p, b->lam.p,
                                 (double*)b->partial.p, (const T*)d_grad_out, b->n_obs, (T*)d_grad, s);
}

// Runs `enqueue` directly, or through a HIP graph: the first call with a pointer set runs
// eagerly (warming every cache and allocation), the second captures and replays, later
// calls replay.
template <typename F>
tq_status run_graphed(tq_svb* b, int which, std::array<const void*, 4> ptrs, hipStream_t stream, F&& enqueue) {
  if (!b->opts.graph) return enqueue(stream);
  GraphEntry* e = nullptr;
  for (GraphEntry& g : b->graphs)
    if (g.which == which && g.ptrs == ptrs) e = &g;
  if (!e) {
    if (b->graphs.size() >= 16) {
      if (b->graphs.front().exec) (void)hipGraphExecDestroy(b->graphs.front().exec);
      b->graphs.erase(b->graphs.begin());
    }
    b->graphs.push_back(GraphEntry{which, ptrs, nullptr});
    return enqueue(stream);
  }
  if (!e->exec) {
    TQ_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const tq_status st = enqueue(b->cap);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(b->cap, &g);
    if (st != TQ_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (ee != hipSuccess) return fail(TQ_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) return fail(TQ_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    e->exec = ex;
    ++b->captures;
  }
  TQ_HIP(hipGraphLaunch(e->exec, stream));
  ++b->replays;
  return TQ_OK;
}

// Exact key of a batch structure (dtype, sizes and gate records): autotuned shapes are
// shared only between byte-identical structures.
std::string structure_key(const tq_svb* b) {
  std::string k = "svb:";
  const int32_t head[2] = {(int32_t)b->dt, (int32_t)b->count};
  k.append((const char*)head, sizeof head);
  for (int i = 0; i < b->count; ++i) {
    const int32_t sz[2] = {(int32_t)b->n[i], (int32_t)b->n_gates[i]};
    k.append((const char*)sz, sizeof sz);
    k.append((const char*)(b->gates.data() + b->gate_off[i]), (size_t)b->n_gates[i] * sizeof(tq_gate));
  }
  return k;
}

// Digest of a structure key plus its length and pass, as a map key: two running
// 64-bit hashes (FNV-1a, and a multiply-xorshift), the key's length and the pass letter.
// Imported shapes are matched by it; a collision could only pick a slower valid shape.
std::string tuning_digest(const std::string& key, char pass) {
  uint64_t a = 1469598103934665603ull, c = 0x9e3779b97f4a7c15ull;
  for (unsigned char ch : key) {
    a = (a ^ ch) * 1099511628211ull;
    c = (c + ch) * 0xff51afd7ed558ccdull;
    c ^= c >> 33;
  }
  const uint64_t rec[4] = {a, c, (uint64_t)key.size(), (uint64_t)(unsigned char)pass};
  return std::string((const char*)rec, sizeof rec);
}

// A tuned shape for (structure, pass): this context's own autotune result, else an imported
// one, else none.
bool find_tuned(const tq_ctx* ctx, const std::string& key, char pass, std::pair<int, int>* out) {
  auto it = ctx->tuned.find(key + (pass == 'f' ? ":f" : ":b"));
  if (it != ctx->tuned.end()) {
    *out = it->second;
    return true;
  }
  auto jt = ctx->tuned_digest.find(tuning_digest(key, pass));
  if (jt != ctx->tuned_digest.end()) {
    *out = jt->second;
    return true;
  }
  return false;
}

// Serialised autotune table: header then one record per (structure, pass).
struct TuneFileHead {
  char magic[4];  // "TQTU"
  uint32_t version, count, pad;
};
struct TuneFileRec {
  char digest[32];
  int32_t t, r;
};
static_assert(sizeof(TuneFileRec) == 40, "tuning record layout");

}  // namespace
}  // namespace tq

extern "C" {

int64_t tq_ctx_export_tuning(const tq_ctx* ctx, void* buf, int64_t cap) {
  using namespace tq;
  if (!ctx || cap < 0) {
    fail(TQ_EINVAL, "tq_ctx_export_tuning: null context or negative capacity");
    return -1;
  }
  std::map<std::string, std::pair<int, int>> recs(ctx->tuned_digest.begin(), ctx->tuned_digest.end());
  for (const auto& kv : ctx->tuned) {  // own results replace imported ones of the same digest
    const std::string& k = kv.first;
    recs[tuning_digest(k.substr(0, k.size() - 2), k.back())] = kv.second;
  }
  const int64_t need = (int64_t)sizeof(TuneFileHead) + (int64_t)recs.size() * (int64_t)sizeof(TuneFileRec);
  if (!buf) return need;
  if (cap < need) {
    fail(TQ_ESIZE, "tq_ctx_export_tuning: " + std::to_string(need) + " bytes needed");
    return -1;
  }
  TuneFileHead h{{'T', 'Q', 'T', 'U'}, 1u, (uint32_t)recs.size(), 0u};
  std::memcpy(buf, &h, sizeof h);
  unsigned char* p = (unsigned char*)buf + sizeof h;
  for (const auto& kv : recs) {
    TuneFileRec r{};
    std::memcpy(r.digest, kv.first.data(), sizeof r.digest);
    r.t = kv.second.first;
    r.r = kv.second.second;
    std::memcpy(p, &r, sizeof r);
    p += sizeof r;
  }
  return need;
}

tq_status tq_ctx_import_tuning(tq_ctx* ctx, const void* buf, int64_t len) {
  using namespace tq;
  if (!ctx || (!buf && len > 0)) return fail(TQ_EINVAL, "null argument");
  TuneFileHead h{};
  if (len < (int64_t)sizeof h) return fail(TQ_EINVAL, "tuning buffer shorter than its header");
  std::memcpy(&h, buf, sizeof h);
  if (std::memcmp(h.magic, "TQTU", 4) != 0 || h.version != 1u)
    return fail(TQ_EINVAL, "not a tuning table of this library version");
  if (len != (int64_t)sizeof h + (int64_t)h.count * (int64_t)sizeof(TuneFileRec))
    return fail(TQ_EINVAL, "tuning buffer length does not match its record count");
  std::vector<std::pair<std::string, std::pair<int, int>>> got;
  const unsigned char* p = (const unsigned char*)buf + sizeof h;
  for (uint32_t i = 0; i < h.count; ++i, p += sizeof(TuneFileRec)) {
    TuneFileRec r;
    std::memcpy(&r, p, sizeof r);
    if (r.t < 1 || r.t > 14 || r.r < 1 || r.r > 5) return fail(TQ_EINVAL, "tuning record with an invalid shape");
    got.emplace_back(std::string(r.digest, sizeof r.digest), std::make_pair((int)r.t, (int)r.r));
  }
  for (auto& g : got) ctx->tuned_digest[g.first] = g.second;  // all records valid: apply
  return TQ_OK;
}

tq_status tq_svb_create(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates,
                        const int32_t* n_params, const tq_zterm* terms, int32_t n_terms, int32_t n_obs,
                        const tq_svb_opts* opts, tq_svb** out) {
  if (!ctx || !out) return fail(TQ_EINVAL, "null context or output pointer");
  *out = nullptr;
  if (dt != TQ_C64 && dt != TQ_C128) return fail(TQ_EINVAL, "unknown dtype");
  if (!n_params) return fail(TQ_EINVAL, "n_params is required for a compiled batch");
  if (n_obs < 1) return fail(TQ_EINVAL, "n_obs must be >= 1");
  if (n_terms < 0 || (n_terms > 0 && !terms)) return fail(TQ_EINVAL, "bad terms");
  std::vector<Group> groups;
  TQ_TRY(group_batch(batch, n_params, groups));
  for (int k = 0; k < n_terms; ++k)
    if (terms[k].obs < 0 || terms[k].obs >= n_obs) return fail(TQ_EINVAL, "term obs index out of range");
  int64_t gate_end = 0;
  for (const Group& gr : groups) {
    TQ_TRY(validate_gates(gates + gr.gate_off, gr.n_gates, gr.n, gr.n_params));
    for (int k = 0; k < n_terms; ++k)
      if (gr.n < 64 && (terms[k].mask >> gr.n) != 0) return fail(TQ_EINVAL, "term names a qubit >= n");
    gate_end = std::max(gate_end, gr.gate_off + gr.n_gates);
  }
  TQ_HIP(hipSetDevice(ctx->device));
  auto b = std::make_unique<tq_svb>();
  b->ctx = ctx;
  b->dt = dt;
  b->count = batch->count;
  b->n.assign(batch->n_qubits, batch->n_qubits + batch->count);
  b->n_gates.assign(batch->n_gates, batch->n_gates + batch->count);
  b->n_params.assign(n_params, n_params + batch->count);
  b->gate_off.assign(batch->gate_off, batch->gate_off + batch->count);
  b->param_off.assign(batch->param_off, batch->param_off + batch->count);
  b->state_off.assign(batch->state_off, batch->state_off + batch->count);
  b->gates.assign(gates, gates + gate_end);
  if (has_controlled(gates, gate_end)) {
    // lower the controlled rotations of every distinct gate segment once (circuits sharing a
    // segment keep sharing its lowered copy)
    std::vector<tq_gate> low;
    std::map<std::pair<int64_t, int>, std::pair<int64_t, int>> seg;
    for (int i = 0; i < b->count; ++i) {
      const auto key = std::make_pair(b->gate_off[i], b->n_gates[i]);
      auto it = seg.find(key);
      if (it == seg.end()) {
        const int64_t off = (int64_t)low.size();
        lower_controlled(gates + key.first, key.second, low);
        it = seg.emplace(key, std::make_pair(off, (int)((int64_t)low.size() - off))).first;
      }
      b->gate_off[i] = it->second.first;
      b->n_gates[i] = it->second.second;
    }
    b->gates.swap(low);
  }
  if (n_terms > 0) b->terms.assign(terms, terms + n_terms);
  b->n_obs = n_obs;
  if (opts) b->opts = *opts;
  for (int i = 0; i < b->count; ++i) b->grad_elems = std::max(b->grad_elems, b->param_off[i] + b->n_params[i]);
  b->key = structure_key(b.get());
  // start from a tuned shape for this structure unless the caller fixed one
  std::pair<int, int> tsh;
  bool tuned_fwd = false;
  if (!b->opts.tile_bits && !b->opts.reg_bits && find_tuned(ctx, b->key, 'f', &tsh)) {
    b->opts.tile_bits = tsh.first;
    b->opts.reg_bits = tsh.second;
    tuned_fwd = true;
  }
  if (!b->opts.adj_tile_bits && !b->opts.adj_reg_bits && find_tuned(ctx, b->key, 'b', &tsh)) {
    b->opts.adj_tile_bits = tsh.first;
    b->opts.adj_reg_bits = tsh.second;
    b->adj_tuned = true;
  }
  int T, R, c;
  fwd_shape(b.get(), &T, &R, &c);
  tq_status bst = build_forward(b.get(), T, R, c);
  if (bst == TQ_EINVAL && tuned_fwd) {  // a tuned shape this structure cannot take: defaults
    b->opts.tile_bits = b->opts.reg_bits = 0;
    fwd_shape(b.get(), &T, &R, &c);
    bst = build_forward(b.get(), T, R, c);
  }
  TQ_TRY(bst);
  TQ_TRY(build_ngroups(b.get()));
  TQ_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  *out = b.release();
  return TQ_OK;
}

void tq_svb_destroy(tq_svb* b) { delete b; }

tq_status tq_svb_forward(tq_ctx* ctx, tq_svb* b, const void* d_params, void* d_states, void* d_out,
                         void* stream) {
  if (!ctx || !b || b->ctx != ctx) return fail(TQ_EINVAL, "compiled batch does not belong to this context");
  if (b->count == 0) return TQ_OK;
  if (!d_params || !d_states) return fail(TQ_EINVAL, "null device pointer");
  hipStream_t s = (hipStream_t)stream;
  const std::array<const void*, 4> key{d_params, d_states, d_out, nullptr};
  return run_graphed(b, 0, key, s, [&](hipStream_t q) {
    return b->dt == TQ_C64 ? enqueue_forward<float>(b, d_params, d_states, d_out, q)
                           : enqueue_forward<double>(b, d_params, d_states, d_out, q);
  });
}

tq_status tq_svb_backward(tq_ctx* ctx, tq_svb* b, const void* d_params, const void* d_states,
                          const void* d_grad_out, void* d_grad, void* stream) {
  if (!ctx || !b || b->ctx != ctx) return fail(TQ_EINVAL, "compiled batch does not belong to this context");
  if (b->count == 0) return TQ_OK;
  if (!d_params || !d_states || !d_grad_out || !d_grad) return fail(TQ_EINVAL, "null device pointer");
  if (!b->adj_built) {
    int T, R, c;
    adj_shape(b, &T, &R, &c);
    tq_status bst = build_adjoint(b, T, R, c);
    if (bst == TQ_EINVAL && b->adj_tuned) {  // a tuned shape this structure cannot take: defaults
      b->opts.adj_tile_bits = b->opts.adj_reg_bits = 0;
      b->adj_tuned = false;
      adj_shape(b, &T, &R, &c);
      bst = build_adjoint(b, T, R, c);
    }
    TQ_TRY(bst);
  }
  hipStream_t s = (hipStream_t)stream;
  const std::array<const void*, 4> key{d_params, d_states, d_grad_out, d_grad};
  return run_graphed(b, 1, key, s, [&](hipStream_t q) {
    return b->dt == TQ_C64 ? enqueue_backward<float>(b, d_params, d_states, d_grad_out, d_grad, q)
                           : enqueue_backward<double>(b, d_params, d_states, d_grad_out, d_grad, q);
  });
}

tq_status tq_svb_autotune(tq_ctx* ctx, tq_svb* b, const void* d_params, void* d_states, int32_t which,
                          int32_t reps, void* stream, tq_svb_opts* best, double* best_ms) {
  if (!ctx || !b || b->ctx != ctx) return fail(TQ_EINVAL, "compiled batch does not belong to this context");
  if (which != 0 && which != 1) return fail(TQ_EINVAL, "which must be 0 (forward) or 1 (backward)");
  if (reps < 1) return fail(TQ_EINVAL, "reps must be >= 1");
  if (!d_params || !d_states) return fail(TQ_EINVAL, "null device pointer");
  hipStream_t s = (hipStream_t)stream;
  // rebuilding rewrites the launch tables in place: nothing may still be reading them
  TQ_HIP(hipDeviceSynchronize());
  const size_t rsz = b->dt == TQ_C64 ? 4 : 8;
  DevBuf gout, grad;
  if (which == 1) {
    std::vector<double> ones_d((size_t)b->count * b->n_obs, 1.0);
    std::vector<float> ones_f((size_t)b->count * b->n_obs, 1.0f);
    if (b->dt == TQ_C64) TQ_TRY(gout.upload(ones_f)); else TQ_TRY(gout.upload(ones_d));
    TQ_TRY(grad.ensure((size_t)std::max<int64_t>(b->grad_elems, 1) * rsz));
  }
  std::vector<std::pair<int, int>> cands;
  const int csz = (int)csize(b->dt);
  for (int T = (b->dt == TQ_C64 ? 13 : 12); T >= (b->dt == TQ_C64 ? 10 : 9); --T) {
    if (which == 1 && T > (b->dt == TQ_C64 ? 12 : 11)) continue;
    for (int R = 2; R <= (which == 1 || b->dt == TQ_C128 ? 4 : 5); ++R) {
      if (T - R > 9) continue;  // work-groups of at most 512 threads (the kernels' launch bounds)
      if (((size_t)csz << T) * (which == 1 ? 2 : 1) > b->ctx->lds_max) continue;
      cands.push_back({T, R});
    }
  }
  hipEvent_t e0, e1;
  TQ_HIP(hipEventCreate(&e0));
  TQ_HIP(hipEventCreate(&e1));
  double best_t = 1e300;
  std::pair<int, int> arg{0, 0};
  int T0, R0, c0;
  if (which == 0) fwd_shape(b, &T0, &R0, &c0); else adj_shape(b, &T0, &R0, &c0);
  tq_status st = TQ_OK;
  for (const auto& cd : cands) {
    st = which == 0 ? build_forward(b, cd.first, cd.second, c0) : build_adjoint(b, cd.first, cd.second, c0);
    if (st == TQ_EINVAL) {  // shape rejected by the schedule builder: not a candidate here
      st = TQ_OK;
      continue;
    }
    if (st != TQ_OK) break;
    auto once = [&]() -> tq_status {
      if (which == 0)
        return b->dt == TQ_C64 ? enqueue_forward<float>(b, d_params, d_states, nullptr, s)
                               : enqueue_forward<double>(b, d_params, d_states, nullptr, s);
      return b->dt == TQ_C64 ? enqueue_backward<float>(b, d_params, d_states, gout.p, grad.p, s)
                             : enqueue_backward<double>(b, d_params, d_states, gout.p, grad.p, s);
    };
    if ((st = once()) != TQ_OK) break;
    if (hipEventRecord(e0, s) != hipSuccess) { st = fail(TQ_EHIP, "hipEventRecord failed"); break; }
    for (int r = 0; r < reps && st == TQ_OK; ++r) st = once();
    if (st != TQ_OK) break;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      st = fail(TQ_EHIP, "event timing failed");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double per = (double)ms / reps;
    if (per < best_t) {
      best_t = per;
      arg = cd;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  TQ_HIP(hipStreamSynchronize(s));
  if (st != TQ_OK) return st;
  if (arg.first == 0) return fail(TQ_ENOTSUP, "no candidate shape fits this device");
  b->clear_graphs();
  if (which == 0) {
    b->opts.tile_bits = arg.first;
    b->opts.reg_bits = arg.second;
    TQ_TRY(build_forward(b, arg.first, arg.second, c0));
    ctx->tuned[b->key + ":f"] = arg;
  } else {
    b->opts.adj_tile_bits = arg.first;
    b->opts.adj_reg_bits = arg.second;
    TQ_TRY(build_adjoint(b, arg.first, arg.second, c0));
    ctx->tuned[b->key + ":b"] = arg;
  }
  if (best) *best = b->opts;
  if (best_ms) *best_ms = best_t;
  return TQ_OK;
}

tq_status tq_svb_info(const tq_svb* b, int64_t out[8]) {
  if (!b || !out) return fail(TQ_EINVAL, "null argument");
  const BatchLaunch& F = b->fwd.L;
  out[0] = F.level_begin.empty() ? 0 : (int64_t)F.level_begin.size() - 1;
  out[1] = F.level_begin.empty() ? 0 : F.level_begin.back();
  out[2] = b->adj_built ? (int64_t)b->adj.L.level_begin.size() - 1 : 0;
  out[3] = b->adj_built ? b->adj.L.level_begin.back() : 0;
  out[4] = b->captures;
  out[5] = b->replays;
  out[6] = F.T;
  out[7] = F.R;
  return TQ_OK;
}

}  // extern "C"
