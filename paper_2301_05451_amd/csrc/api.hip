// C ABI entry points of libtq: context, errors, schedule cache, state-vector calls.
#include <algorithm>
#include <cstdio>
#include <map>
#include <tuple>

#include "sv_device.h"

namespace tq {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

tq_status fail(tq_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

Schedule::~Schedule() {
  // every device table of a schedule lives in one allocation (see Packer)
  if (d_blob) (void)hipFree(d_blob);
}

// Packs a schedule's host tables into one device allocation with a single copy: each table
// starts on a 256-byte boundary, and its pointer is set to its place in the block.
struct Packer {
  std::vector<unsigned char> host;
  std::vector<std::pair<size_t, void**>> dst;
  template <typename V>
  void add(const std::vector<V>& v, void** out) {
    const size_t at = (host.size() + 255) & ~size_t(255);
    host.resize(at + std::max<size_t>(v.size() * sizeof(V), 16), 0);
    if (!v.empty()) std::memcpy(host.data() + at, v.data(), v.size() * sizeof(V));
    dst.push_back({at, out});
  }
  tq_status upload(void** blob) {
    void* d = nullptr;
    TQ_HIP(hipMalloc(&d, std::max<size_t>(host.size(), 256)));
    if (!host.empty()) TQ_HIP(hipMemcpy(d, host.data(), host.size(), hipMemcpyHostToDevice));
    *blob = d;
    for (auto& e : dst) *e.second = (unsigned char*)d + e.first;
    return TQ_OK;
  }
};

tq_status scratch(tq_ctx* ctx, int slot, size_t bytes, void** out, bool zero) {
  if (bytes == 0) bytes = 256;
  if (ctx->scratch_bytes[slot] < bytes) {
    // Grow without waiting for the device: work already queued may still use the old
    // buffer, so it is retired (freed when the context is destroyed) rather than freed.
    // Sizes at least double, so retired buffers add up to less than the live one.
    if (ctx->scratch[slot]) ctx->retired.push_back(ctx->scratch[slot]);
    ctx->scratch[slot] = nullptr;
    size_t want = std::max(bytes, std::max((size_t)4096, 2 * ctx->scratch_bytes[slot]));
    ctx->scratch_bytes[slot] = 0;
    if (hipMalloc(&ctx->scratch[slot], want) != hipSuccess)
      return fail(TQ_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes of context scratch failed");
    ctx->scratch_bytes[slot] = want;
    if (zero) TQ_HIP(hipMemset(ctx->scratch[slot], 0, want));
  }
  *out = ctx->scratch[slot];
  return TQ_OK;
}

// Immutable small host tables (offset maps, observable terms) live in device memory cached
// by their full content (the key is the bytes themselves, so equal keys mean equal tables),
// so repeated calls neither re-upload nor synchronise (and can be captured in a hipGraph once
// warmed up). The cache is bounded (kTableCacheBytes / kTableCacheEntries): when a new
// table would exceed it, the device is synchronised once and the least recently used
// tables are freed.
tq_status cached_table(tq_ctx* ctx, const void* host, size_t bytes, void** dev) {
  std::string key((const char*)host, bytes);
  auto it = ctx->tables.find(key);
  ++ctx->table_clock;
  if (it != ctx->tables.end()) {
    it->second.last_use = ctx->table_clock;
    *dev = it->second.dev;
    return TQ_OK;
  }
  if (ctx->table_bytes + bytes > kTableCacheBytes || ctx->tables.size() + 1 > kTableCacheEntries) {
    TQ_HIP(hipDeviceSynchronize());
    std::vector<std::pair<uint64_t, const std::string*>> age;
    for (auto& kv : ctx->tables) age.push_back({kv.second.last_use, &kv.first});
    std::sort(age.begin(), age.end());
    for (auto& a : age) {
      if (ctx->table_bytes + bytes <= kTableCacheBytes / 2 && ctx->tables.size() + 1 <= kTableCacheEntries / 2) break;
      auto jt = ctx->tables.find(*a.second);
      (void)hipFree(jt->second.dev);
      ctx->table_bytes -= jt->second.bytes;
      ctx->tables.erase(jt);
    }
  }
  void* d = nullptr;
  TQ_HIP(hipMalloc(&d, std::max<size_t>(bytes, 16)));
  if (bytes) TQ_HIP(hipMemcpy(d, host, bytes, hipMemcpyHostToDevice));
  ctx->tables.emplace(std::move(key), TableEntry{d, bytes, ctx->table_clock});
  ctx->table_bytes += bytes;
  *dev = d;
  return TQ_OK;
}

tq_status stage_upload(tq_ctx* ctx, int slot, const void* host, size_t bytes, hipStream_t stream, void** dev) {
  TQ_TRY(scratch(ctx, slot, bytes, dev));
  if (ctx->pinned_pending) {  // the previous upload may still read the staging buffer
    TQ_HIP(hipEventSynchronize(ctx->pinned_done));
    ctx->pinned_pending = false;
  }
  if (ctx->pinned_bytes < bytes) {
    if (ctx->pinned) TQ_HIP(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    const size_t want = std::max<size_t>(bytes, 64 * 1024);
    TQ_HIP(hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
    ctx->pinned_bytes = want;
  }
  if (!ctx->pinned_done) TQ_HIP(hipEventCreateWithFlags(&ctx->pinned_done, hipEventDisableTiming));
  std::memcpy(ctx->pinned, host, bytes);
  TQ_HIP(hipMemcpyAsync(*dev, ctx->pinned, bytes, hipMemcpyHostToDevice, stream));
  TQ_HIP(hipEventRecord(ctx->pinned_done, stream));
  ctx->pinned_pending = true;
  return TQ_OK;
}

// Cache key of a schedule: the gate records themselves plus the shape (an exact key: two
// structures share a schedule only if their bytes are equal).
static std::string schedule_key(const tq_gate* g, int n_gates, int n, int mode, int t, int R, int c) {
  const int32_t head[7] = {n, n_gates, mode, t, R, c, (int32_t)sizeof(tq_gate)};
  std::string k((const char*)head, sizeof head);
  k.append((const char*)g, (size_t)n_gates * sizeof(tq_gate));
  return k;
}

static void pack_schedule(Schedule& s, const tq_gate* g, int n_gates, Packer& pk) {
  pk.add(std::vector<tq_gate>(g, g + n_gates), &s.d_gates);
  std::vector<int32_t> rec, rg;
  for (const Recipe& r : s.recipes) {
    rec.push_back(r.kind);
    rec.push_back(r.qa);
    rec.push_back(r.qb);
    rec.push_back((int32_t)rg.size());
    rg.insert(rg.end(), r.gates.begin(), r.gates.end());
  }
  rec.push_back(0); rec.push_back(0); rec.push_back(0); rec.push_back((int32_t)rg.size());  // sentinel
  pk.add(rec, &s.d_rec);
  pk.add(rg, &s.d_rec_gates);
  pk.add(s.dops, &s.d_ops);
  pk.add(s.phases, &s.d_phases);
  pk.add(s.dstages, &s.d_stages);
}

// Default fused shapes (the autotuner may override): 2^12-amplitude tiles (32 KiB of LDS for
// complex64, so several work-groups per CU), 16 amplitudes per thread, the 4 lowest index
// bits always local (runs of 16 contiguous amplitudes per HBM access).
static void default_shape(int dt, int n, int* t, int* R, int* c) {
  *t = 12;  // measured best on the 24-qubit brickwork sweep (tile 12, 4 register bits, 4 coalesced)
  *R = 4;
  *c = 4;
  if (*t > n) *t = n;
}

// Resolved and checked (tile, register, coalesced) bits of a forward schedule.
static tq_status forward_shape(size_t lds_max, int dt, int n, int mode, const tq_sv_opts* opts, int* t, int* R,
                               int* c) {
  default_shape(dt, n, t, R, c);
  if (opts) {
    if (opts->tile_bits) *t = std::min(opts->tile_bits, n);
    if (opts->reg_bits) *R = opts->reg_bits;
    if (opts->coal_bits) *c = opts->coal_bits;
  }
  if (mode != 0) {
    *t = *R = *c = 0;
    return TQ_OK;
  }
  const size_t csz = dt == TQ_C64 ? 8 : 16;
  if (*t < 1 || *t > 14 || (csz << *t) > lds_max)
    return fail(TQ_EINVAL, "tile_bits " + std::to_string(*t) + " does not fit LDS for this dtype");
  if (*R < 1 || *R > 5) return fail(TQ_EINVAL, "reg_bits must be in 1..5");
  if (dt == TQ_C128 && *R > 4) return fail(TQ_EINVAL, "reg_bits must be <= 4 for complex128 (register file)");
  // the stage kernels are compiled for work-groups of at most 512 threads
  if (*t - std::min(*R, *t) > 9) return fail(TQ_EINVAL, "tile_bits - reg_bits must be <= 9 (512 threads)");
  if (*c < 0 || *c > 10) return fail(TQ_EINVAL, "coal_bits must be in 0..10");
  return TQ_OK;
}

// Host construction of a forward schedule of a checked shape (no device copies).
static void build_schedule(const tq_gate* g, int n_gates, int n, int mode, int t, int R, int c, Schedule& s) {
  s.n = n;
  s.mode = mode;
  s.t = t;
  s.R = R;
  s.c = c;
  s.n_gates = n_gates;
  lower_ops(g, n_gates, n, mode == 0, s.recipes, s.ops);
  if (mode == 0) build_stages(s);
}

tq_status get_schedule(tq_ctx* ctx, int dt, const tq_gate* g, int n_gates, int n, int mode, const tq_sv_opts* opts,
                       Schedule** out) {
  int t, R, c;
  TQ_TRY(forward_shape(ctx->lds_max, dt, n, mode, opts, &t, &R, &c));
  std::string key = schedule_key(g, n_gates, n, mode, t, R, c);
  auto it = ctx->schedules.find(key);
  if (it != ctx->schedules.end()) {
    *out = it->second.get();
    return TQ_OK;
  }
  auto s = std::make_unique<Schedule>();
  build_schedule(g, n_gates, n, mode, t, R, c, *s);
  Packer pk;
  pack_schedule(*s, g, n_gates, pk);
  TQ_TRY(pk.upload(&s->d_blob));
  *out = s.get();
  ctx->schedules.emplace(key, std::move(s));
  return TQ_OK;
}

// Resolved and checked shape of a reverse-sweep schedule (two tiles in LDS).
static tq_status adjoint_shape(size_t lds_max, int dt, int n, const tq_sv_opts* opts, int* t, int* R, int* c) {
  *t = dt == TQ_C64 ? 12 : 11;
  *R = dt == TQ_C64 ? 4 : 3;
  *c = dt == TQ_C64 ? 5 : 4;
  if (opts) {
    if (opts->tile_bits) *t = opts->tile_bits;
    if (opts->reg_bits) *R = opts->reg_bits;
    if (opts->coal_bits) *c = opts->coal_bits;
  }
  *t = std::min(*t, n);
  const size_t csz = dt == TQ_C64 ? 8 : 16;
  if (*t < 1 || *t > 13 || 2 * (csz << *t) + 16384 > lds_max)
    return fail(TQ_EINVAL, "adjoint tile_bits " + std::to_string(*t) + " does not fit LDS (two tiles)");
  if (*R < 1 || *R > 4) return fail(TQ_EINVAL, "adjoint reg_bits must be in 1..4");
  if (*t - std::min(*R, *t) > 9) return fail(TQ_EINVAL, "adjoint tile_bits - reg_bits must be <= 9 (512 threads)");
  return TQ_OK;
}

// Host construction of a reverse-sweep schedule of a checked shape (no device copies).
static void build_adjoint_schedule(const tq_gate* g, int n_gates, int n, int t, int R, int c, Schedule& s) {
  s.n = n;
  s.mode = 2;
  s.adjoint = true;
  s.t = t;
  s.R = R;
  s.c = c;
  s.n_gates = n_gates;
  lower_adjoint_ops(g, n_gates, s.ops, s.adj_runs);
  build_stages(s);
  build_adjoint_slots(s, g, n_gates);
}

// Reverse-sweep schedule of a circuit structure (cached; key mode 2).
tq_status get_adjoint_schedule(tq_ctx* ctx, int dt, const tq_gate* g, int n_gates, int n, const tq_sv_opts* opts,
                               Schedule** out) {
  int t, R, c;
  TQ_TRY(adjoint_shape(ctx->lds_max, dt, n, opts, &t, &R, &c));
  std::string key = schedule_key(g, n_gates, n, 2, t, R, c);
  auto it = ctx->schedules.find(key);
  if (it != ctx->schedules.end()) {
    *out = it->second.get();
    return TQ_OK;
  }
  auto s = std::make_unique<Schedule>();
  build_adjoint_schedule(g, n_gates, n, t, R, c, *s);
  Packer pk;
  pack_schedule(*s, g, n_gates, pk);
  pk.add(s->dslot, &s->d_dslot);
  pk.add(s->adj_runs, &s->d_adj_runs);
  std::vector<int32_t> slot_pairs;  // per stage: (first slot, slot count), read by batched launches
  for (size_t k = 0; k < s->stage_slot0.size(); ++k) {
    slot_pairs.push_back(s->stage_slot0[k]);
    slot_pairs.push_back(s->stage_nslot[k]);
  }
  pk.add(slot_pairs, &s->d_stage_slot0);
  pk.add(s->pslot_ptr, &s->d_pslot_ptr);
  pk.add(s->pslot_idx, &s->d_pslot_idx);
  pk.add(s->pslot_scale, &s->d_pslot_scale);
  TQ_TRY(pk.upload(&s->d_blob));
  *out = s.get();
  ctx->schedules.emplace(key, std::move(s));
  return TQ_OK;
}

// Observable terms in device form: [pos masks (u64)] [coeffs (f64)] [obs (i32)], masks over
// bit positions of an n-qubit index.
tq_status term_table(tq_ctx* ctx, int n, const tq_zterm* terms, int n_terms, const unsigned char** dev) {
  std::vector<unsigned char> blob((size_t)n_terms * 20 + 64, 0);
  for (int k = 0; k < n_terms; ++k) {
    uint64_t m = 0;
    for (int q = 0; q < n; ++q)
      if ((terms[k].mask >> q) & 1ull) m |= 1ull << (n - 1 - q);
    std::memcpy(blob.data() + 8 * k, &m, 8);
    std::memcpy(blob.data() + (size_t)n_terms * 8 + 8 * k, &terms[k].coeff, 8);
    std::memcpy(blob.data() + (size_t)n_terms * 16 + 4 * k, &terms[k].obs, 4);
  }
  void* d;
  TQ_TRY(cached_table(ctx, blob.data(), blob.size(), &d));
  *dev = (const unsigned char*)d;
  return TQ_OK;
}

tq_status group_batch(const tq_batch* b, const int32_t* n_params, std::vector<Group>& groups) {
  if (!b) return fail(TQ_EINVAL, "null batch");
  if (b->count < 0) return fail(TQ_EINVAL, "negative batch count");
  if (b->count == 0) return TQ_OK;
  if (!b->n_qubits || !b->gate_off || !b->n_gates || !b->param_off || !b->state_off)
    return fail(TQ_EINVAL, "batch arrays must not be null");
  std::map<std::tuple<int, int64_t, int>, int> idx;
  for (int i = 0; i < b->count; ++i) {
    const int n = b->n_qubits[i];
    if (n < 1 || n > 34) return fail(TQ_ENOTSUP, "circuit " + std::to_string(i) + ": n_qubits must be in 1..34");
    if (b->n_gates[i] < 0 || b->gate_off[i] < 0 || b->param_off[i] < 0 || b->state_off[i] < 0)
      return fail(TQ_EINVAL, "circuit " + std::to_string(i) + ": negative offset or count");
    auto key = std::make_tuple(n, b->gate_off[i], b->n_gates[i]);
    auto it = idx.find(key);
    int np = n_params ? n_params[i] : 0x7fffffff;
    if (it == idx.end()) {
      idx[key] = (int)groups.size();
      groups.push_back({n, b->gate_off[i], b->n_gates[i], np, {i}});
    } else {
      groups[it->second].members.push_back(i);
      groups[it->second].n_params = std::min(groups[it->second].n_params, np);
    }
  }
  return TQ_OK;
}

// Offsets of a group's members: affine (base + i * stride) when possible, else uploaded.
tq_status member_map(tq_ctx* ctx, int slot, const int64_t* all, const std::vector<int>& m, hipStream_t stream,
                     BatchMap* out) {
  out->off = nullptr;
  out->base = all[m[0]];
  out->stride = m.size() > 1 ? all[m[1]] - all[m[0]] : 0;
  bool affine = true;
  for (size_t i = 0; i < m.size() && affine; ++i) affine = all[m[i]] == out->base + out->stride * (int64_t)i;
  if (affine) return TQ_OK;
  std::vector<int64_t> v(m.size());
  for (size_t i = 0; i < m.size(); ++i) v[i] = all[m[i]];
  void* d;
  (void)slot;
  (void)stream;
  TQ_TRY(cached_table(ctx, v.data(), v.size() * sizeof(int64_t), &d));
  out->off = (const int64_t*)d;
  return TQ_OK;
}

// basis < 0: apply to the states as they are (tq_sv_apply); basis >= 0: to |basis>, which the
// first fused stage forms in place of reading the states (tq_sv_run).
template <typename T>
static tq_status sv_apply_t(tq_ctx* ctx, const tq_batch* batch, const tq_gate* gates, const int32_t* n_params,
                            const void* d_params, void* d_states, const tq_sv_opts* opts, hipStream_t stream,
                            int64_t basis = -1) {
  using C = typename Cx<T>::type;
  std::vector<Group> groups;
  TQ_TRY(group_batch(batch, n_params, groups));
  const int mode = opts ? opts->mode : 0;
  if (mode != 0 && mode != 1) return fail(TQ_ENOTSUP, "sv mode must be 0 (fused) or 1 (plain)");
  if (!groups.empty() && (!d_params || !d_states)) return fail(TQ_EINVAL, "null device pointer");
  for (const Group& gr : groups) {
    const tq_gate* g = gates + gr.gate_off;
    TQ_TRY(validate_gates(g, gr.n_gates, gr.n, gr.n_params));
    if (basis >= 0 && gr.n < 63 && basis >= (int64_t(1) << gr.n))
      return fail(TQ_EINVAL, "basis index outside [0, 2^n)");
  }
  for (const Group& gr : groups) {
    const GateView gv(gates + gr.gate_off, gr.n_gates);  // controlled rotations lowered
    Schedule* s;
    TQ_TRY(get_schedule(ctx, sizeof(T) == 4 ? TQ_C64 : TQ_C128, gv.g, gv.n, gr.n, mode, opts, &s));
    const int count = (int)gr.members.size();
    BatchMap pmap, smap;
    TQ_TRY(member_map(ctx, S_OFFS, batch->param_off, gr.members, stream, &pmap));
    TQ_TRY(member_map(ctx, S_MISC, batch->state_off, gr.members, stream, &smap));
    void* mats;
    TQ_TRY(scratch(ctx, S_MATS, (size_t)count * std::max<size_t>(s->recipes.size(), 1) * 4 * sizeof(C), &mats));
    TQ_TRY(launch_gate_build<T>(*s, d_params, pmap, mats, count, stream));
    const bool fused_init = basis >= 0 && mode == 0 && !s->stages.empty();
    if (basis >= 0 && !fused_init)  // no stage to form the basis state in: a preparation pass
      TQ_TRY(launch_init_basis<T>(d_states, smap, gr.n, count, basis, ctx->n_cu, stream));
    if (mode == 1)
      TQ_TRY(launch_plain<T>(*s, d_states, smap, mats, count, ctx->n_cu, stream));
    else
      TQ_TRY(launch_stages<T>(*s, d_states, smap, mats, count, fused_init ? basis : -1, stream));
  }
  return TQ_OK;
}

template <typename T>
static tq_status expval_t(tq_ctx* ctx, const tq_batch* batch, const void* d_states, const tq_zterm* terms,
                          int n_terms, int n_obs, void* d_out, hipStream_t stream) {
  std::vector<Group> groups;
  TQ_TRY(group_batch(batch, nullptr, groups));
  if (n_obs < 1) return fail(TQ_EINVAL, "n_obs must be >= 1");
  if (n_terms < 0 || (n_terms > 0 && !terms)) return fail(TQ_EINVAL, "bad terms");
  if (!groups.empty() && (!d_states || !d_out)) return fail(TQ_EINVAL, "null device pointer");
  for (int k = 0; k < n_terms; ++k)
    if (terms[k].obs < 0 || terms[k].obs >= n_obs) return fail(TQ_EINVAL, "term obs index out of range");
  // output rows follow batch order: out[i * n_obs + o]. Groups are computed per distinct n.
  for (const Group& gr : groups) {
    for (int k = 0; k < n_terms; ++k)
      if (gr.n < 64 && (terms[k].mask >> gr.n) != 0) return fail(TQ_EINVAL, "term names a qubit >= n");
  }
  // group by n only (gates do not matter here)
  std::map<int, std::vector<int>> by_n;
  for (const Group& gr : groups)
    for (int i : gr.members) by_n[gr.n].push_back(i);
  for (auto& kv : by_n) {
    const int n = kv.first;
    std::vector<int>& mem = kv.second;
    std::sort(mem.begin(), mem.end());
    std::vector<uint64_t> pm(n_terms);
    std::vector<double> cf(n_terms);
    std::vector<int32_t> ob(n_terms);
    for (int k = 0; k < n_terms; ++k) {
      uint64_t m = 0;
      for (int q = 0; q < n; ++q)
        if ((terms[k].mask >> q) & 1ull) m |= 1ull << (n - 1 - q);
      pm[k] = m;
      cf[k] = terms[k].coeff;
      ob[k] = terms[k].obs;
    }
    std::vector<unsigned char> blob(n_terms * 20 + 64);
    std::memcpy(blob.data(), pm.data(), n_terms * 8);
    std::memcpy(blob.data() + n_terms * 8, cf.data(), n_terms * 8);
    std::memcpy(blob.data() + n_terms * 16, ob.data(), n_terms * 4);
    void* dterms;
    TQ_TRY(cached_table(ctx, blob.data(), blob.size(), &dterms));
    const unsigned char* db = (const unsigned char*)dterms;
    BatchMap smap, omap;
    TQ_TRY(member_map(ctx, S_MISC, batch->state_off, mem, stream, &smap));
    // output rows: the members' batch indices (affine when consecutive)
    std::vector<int64_t> rows(mem.begin(), mem.end());
    std::vector<int> ident(mem.size());
    for (size_t i = 0; i < mem.size(); ++i) ident[i] = (int)i;
    TQ_TRY(member_map(ctx, S_MISC, rows.data(), ident, stream, &omap));
    const size_t pcap = expval_scratch_doubles(n, (int)mem.size(), n_obs);
    void* partial;
    TQ_TRY(scratch(ctx, S_PARTIAL, pcap * sizeof(double), &partial));
    TQ_TRY(launch_expval<T>((const typename Cx<T>::type*)d_states, smap, n, (int)mem.size(), (const uint64_t*)db,
                            (const double*)(db + n_terms * 8), (const int32_t*)(db + n_terms * 16), n_terms, n_obs,
                            (double*)partial, pcap, (T*)d_out, omap, stream));
  }
  return TQ_OK;
}

// Validation shared by the adjoint size query and the call itself.
static tq_status sv_backward_check(const tq_batch* batch, const tq_gate* gates, const int32_t* n_params,
                                   const tq_zterm* terms, int n_terms, int n_obs, std::vector<Group>& groups) {
  if (!n_params) return fail(TQ_EINVAL, "n_params is required for the backward pass");
  TQ_TRY(group_batch(batch, n_params, groups));
  if (n_obs < 1) return fail(TQ_EINVAL, "n_obs must be >= 1");
  if (n_terms < 0 || (n_terms > 0 && !terms)) return fail(TQ_EINVAL, "bad terms");
  for (int k = 0; k < n_terms; ++k)
    if (terms[k].obs < 0 || terms[k].obs >= n_obs) return fail(TQ_EINVAL, "term obs index out of range");
  for (const Group& gr : groups) {
    TQ_TRY(validate_gates(gates + gr.gate_off, gr.n_gates, gr.n, gr.n_params));
    for (int i : gr.members)
      if (n_params[i] != gr.n_params)
        return fail(TQ_EINVAL, "circuits sharing a gate list must have equal n_params for the backward pass");
    for (int k = 0; k < n_terms; ++k)
      if (gr.n < 64 && (terms[k].mask >> gr.n) != 0) return fail(TQ_EINVAL, "term names a qubit >= n");
  }
  return TQ_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// The adjoint sweep. Circuits sharing a gate list run together in runs of consecutive batch
// indices; the runs execute one after another on the stream and reuse one workspace region:
// psi and lambda copies (one state each per circuit), the adjoint gate matrices and the
// per-tile gradient partial sums. With d_work == nullptr only the schedules and tables are
// prepared (cached in the context) and *need receives the workspace bytes.
// Pauli terms of an observable over bit positions of an n-qubit index.
static tq_status pauli_for_n(int n, const tq_pauli_term* pt, int n_pt, int n_obs, AdjPauli* out) {
  if (n_pt < 0 || n_pt > kAdjPauliTerms || (n_pt > 0 && !pt))
    return fail(TQ_EINVAL, "the backward pass takes 0.." + std::to_string(kAdjPauliTerms) + " Pauli terms");
  *out = AdjPauli{};
  out->n = n_pt;
  for (int k = 0; k < n_pt; ++k) {
    if (pt[k].obs < 0 || pt[k].obs >= n_obs) return fail(TQ_EINVAL, "term obs index out of range");
    if (n < 64 && ((pt[k].x_mask | pt[k].z_mask) >> n) != 0) return fail(TQ_EINVAL, "term names a qubit >= n");
    uint64_t f = 0, m = 0;
    int ny = 0;
    for (int q = 0; q < n; ++q) {
      const bool xb = (pt[k].x_mask >> q) & 1ull, zb = (pt[k].z_mask >> q) & 1ull;
      if (xb) f |= 1ull << (n - 1 - q);
      if (zb) m |= 1ull << (n - 1 - q);
      ny += xb && zb;
    }
    out->f[k] = f;
    out->m[k] = m;
    out->c[k] = pt[k].coeff;
    out->ob[k] = pt[k].obs;
    out->cls[k] = ny & 3;
  }
  return TQ_OK;
}

template <typename T>
static tq_status sv_backward_t(tq_ctx* ctx, const tq_batch* batch, const tq_gate* gates, const int32_t* n_params,
                               const void* d_params, const void* d_states, const tq_zterm* terms, int n_terms,
                               int n_obs, const void* d_grad_out, void* d_grad, const tq_sv_opts* opts,
                               void* d_work, int64_t work_bytes, int64_t* need, hipStream_t stream,
                               const tq_pauli_term* pterms = nullptr, int n_pterms = 0) {
  using C = typename Cx<T>::type;
  const int dt = sizeof(T) == 4 ? TQ_C64 : TQ_C128;
  const bool exec = d_work != nullptr || need == nullptr;
  std::vector<Group> groups;
  TQ_TRY(sv_backward_check(batch, gates, n_params, terms, n_terms, n_obs, groups));
  if (exec && !groups.empty() && (!d_params || !d_states || !d_grad_out || !d_grad))
    return fail(TQ_EINVAL, "null device pointer");
  // first pass: schedules, tables and the workspace size
  struct Run {
    Schedule* s;
    const unsigned char* tt;
    std::vector<int> mem;
    size_t psi, lam, mats, part;
    int n, n_params;
    AdjPauli pauli;
  };
  std::vector<Run> runs;
  size_t ws = 256;
  for (const Group& gr : groups) {
    const GateView gv(gates + gr.gate_off, gr.n_gates);  // controlled rotations lowered
    Schedule* s;
    TQ_TRY(get_adjoint_schedule(ctx, dt, gv.g, gv.n, gr.n, opts, &s));
    const unsigned char* tt;
    TQ_TRY(term_table(ctx, gr.n, terms, n_terms, &tt));
    size_t i0 = 0;
    while (i0 < gr.members.size()) {
      size_t i1 = i0 + 1;
      while (i1 < gr.members.size() && gr.members[i1] == gr.members[i1 - 1] + 1) ++i1;
      Run r{s, tt, std::vector<int>(gr.members.begin() + i0, gr.members.begin() + i1), 0, 0, 0, 0, gr.n,
            gr.n_params, AdjPauli{}};
      if (pterms) TQ_TRY(pauli_for_n(gr.n, pterms, n_pterms, n_obs, &r.pauli));
      const size_t count = r.mem.size();
      const int64_t namps = int64_t(1) << gr.n;
      const int64_t ntiles = s->stages.empty() ? 1 : (int64_t(1) << (gr.n - s->stages[0].t));
      r.psi = 0;
      r.lam = align256(count * namps * sizeof(C));
      r.mats = r.lam + align256(count * namps * sizeof(C));
      r.part = r.mats + align256(count * std::max(gv.n, 1) * kAdjMatEntries * sizeof(C));
      ws = std::max(ws, r.part + align256(count * std::max(s->n_slots, 1) * ntiles * sizeof(double)));
      BatchMap pmap, smap;  // warm the offset tables
      TQ_TRY(member_map(ctx, S_OFFS, batch->param_off, r.mem, stream, &pmap));
      TQ_TRY(member_map(ctx, S_MISC, batch->state_off, r.mem, stream, &smap));
      runs.push_back(std::move(r));
      i0 = i1;
    }
  }
  if (need) *need = (int64_t)ws;
  if (!exec) return TQ_OK;
  if (!d_work || work_bytes < (int64_t)ws)
    return fail(TQ_EWORKSPACE, "adjoint workspace of " + std::to_string(work_bytes) + " bytes is smaller than the " +
                                   std::to_string(ws) + " bytes tq_sv_backward_workspace reports");
  unsigned char* w = (unsigned char*)d_work;
  for (const Run& r : runs) {
    BatchMap pmap, smap;
    TQ_TRY(member_map(ctx, S_OFFS, batch->param_off, r.mem, stream, &pmap));
    TQ_TRY(member_map(ctx, S_MISC, batch->state_off, r.mem, stream, &smap));
    const int64_t namps = int64_t(1) << r.n;
    BatchMap wmap{nullptr, 0, namps};
    TQ_TRY(launch_adjoint<T>(*r.s, d_params, pmap, d_states, smap, w + r.psi, w + r.lam, wmap, w + r.mats,
                             (double*)(w + r.part), (const uint64_t*)r.tt, (const double*)(r.tt + n_terms * 8),
                             (const int32_t*)(r.tt + n_terms * 16), n_terms,
                             (const T*)d_grad_out + (int64_t)r.mem[0] * n_obs, n_obs, (T*)d_grad, r.n_params,
                             (int)r.mem.size(), stream, pterms ? &r.pauli : nullptr));
  }
  return TQ_OK;
}

}  // namespace tq

using namespace tq;

extern "C" {

const char* tq_last_error(void) { return g_last_error.c_str(); }

int32_t tq_lower_gates(const tq_gate* in, int32_t n_in, tq_gate* out, int32_t cap) {
  if (n_in < 0 || (n_in > 0 && !in)) {
    fail(TQ_EINVAL, "tq_lower_gates: bad input");
    return -1;
  }
  std::vector<tq_gate> low;
  lower_controlled(in, n_in, low);
  if (out) {
    if ((int64_t)low.size() > cap) {
      fail(TQ_ESIZE, "tq_lower_gates: capacity " + std::to_string(cap) + " < " + std::to_string(low.size()));
      return -1;
    }
    std::copy(low.begin(), low.end(), out);
  }
  return (int32_t)low.size();
}

int tq_version(void) { return 100; }

int tq_hip_build_version(void) { return HIP_VERSION; }

int tq_hip_runtime_version(void) {
  int v = 0;
  if (hipRuntimeGetVersion(&v) != hipSuccess) return -1;
  return v;
}

tq_status tq_ctx_create(int device, tq_ctx** out) {
  if (!out) return fail(TQ_EINVAL, "null output pointer");
  *out = nullptr;
  int ndev = 0;
  TQ_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(TQ_EINVAL, "device index out of range");
  TQ_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  TQ_HIP(hipGetDeviceProperties(&prop, device));
  auto* c = new tq_ctx();
  c->device = device;
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->lds_max = prop.sharedMemPerBlock > 0 ? prop.sharedMemPerBlock : 64 * 1024;
  *out = c;
  return TQ_OK;
}

void tq_ctx_destroy(tq_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->schedules.clear();
  for (int i = 0; i < 9; ++i)
    if (ctx->scratch[i]) (void)hipFree(ctx->scratch[i]);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->pinned_done) (void)hipEventDestroy(ctx->pinned_done);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  for (int i = 0; i < 4; ++i) {
    if (ctx->pool[i]) (void)hipStreamDestroy(ctx->pool[i]);
    if (ctx->pool_done[i]) (void)hipEventDestroy(ctx->pool_done[i]);
  }
  for (auto& kv : ctx->tables) (void)hipFree(kv.second.dev);
  for (void* p : ctx->retired) (void)hipFree(p);
  delete ctx;
}

tq_status tq_sv_apply(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates, const int32_t* n_params,
                      const void* d_params, void* d_states, const tq_sv_opts* opts, void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null context");
  if (dt == TQ_C64) return sv_apply_t<float>(ctx, batch, gates, n_params, d_params, d_states, opts, (hipStream_t)stream);
  if (dt == TQ_C128)
    return sv_apply_t<double>(ctx, batch, gates, n_params, d_params, d_states, opts, (hipStream_t)stream);
  return fail(TQ_EINVAL, "unknown dtype");
}

tq_status tq_sv_run(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates, const int32_t* n_params,
                    const void* d_params, int64_t basis, void* d_states, const tq_sv_opts* opts, void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null context");
  if (basis < 0) return fail(TQ_EINVAL, "basis index outside [0, 2^n)");
  if (dt == TQ_C64)
    return sv_apply_t<float>(ctx, batch, gates, n_params, d_params, d_states, opts, (hipStream_t)stream, basis);
  if (dt == TQ_C128)
    return sv_apply_t<double>(ctx, batch, gates, n_params, d_params, d_states, opts, (hipStream_t)stream, basis);
  return fail(TQ_EINVAL, "unknown dtype");
}

tq_status tq_sv_init(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, int64_t basis, void* d_states, void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null context");
  if (dt != TQ_C64 && dt != TQ_C128) return fail(TQ_EINVAL, "unknown dtype");
  std::vector<Group> groups;
  TQ_TRY(group_batch(batch, nullptr, groups));
  if (!groups.empty() && !d_states) return fail(TQ_EINVAL, "null device pointer");
  std::map<int, std::vector<int>> by_n;
  for (const Group& gr : groups) {
    if (basis < 0 || (gr.n < 63 && basis >= (int64_t(1) << gr.n)))
      return fail(TQ_EINVAL, "basis index outside [0, 2^n)");
    for (int i : gr.members) by_n[gr.n].push_back(i);
  }
  for (auto& kv : by_n) {
    std::sort(kv.second.begin(), kv.second.end());
    BatchMap smap;
    TQ_TRY(member_map(ctx, S_MISC, batch->state_off, kv.second, (hipStream_t)stream, &smap));
    if (dt == TQ_C64)
      TQ_TRY(launch_init_basis<float>(d_states, smap, kv.first, (int)kv.second.size(), basis, ctx->n_cu,
                                      (hipStream_t)stream));
    else
      TQ_TRY(launch_init_basis<double>(d_states, smap, kv.first, (int)kv.second.size(), basis, ctx->n_cu,
                                       (hipStream_t)stream));
  }
  return TQ_OK;
}

tq_status tq_sv_plan_info(tq_ctx* ctx, tq_dtype dt, int32_t n_qubits, const tq_gate* gates, int32_t n_gates,
                          const tq_sv_opts* opts, int64_t out[8]) {
  if (!out) return fail(TQ_EINVAL, "null argument");
  if (dt != TQ_C64 && dt != TQ_C128) return fail(TQ_EINVAL, "unknown dtype");
  if (n_qubits < 1 || n_qubits > 34) return fail(TQ_ENOTSUP, "n_qubits must be in 1..34");
  TQ_TRY(validate_gates(gates, n_gates, n_qubits, 0x7fffffff));
  const int mode = opts ? opts->mode : 0;
  if (mode < 0 || mode > 2) return fail(TQ_ENOTSUP, "plan mode must be 0 (fused), 1 (plain) or 2 (reverse sweep)");
  const GateView gv(gates, n_gates);
  const size_t lds_max = ctx ? ctx->lds_max : 160 * 1024;
  Schedule local;
  const Schedule* s = &local;
  int t, R, c;
  if (mode == 2) {
    TQ_TRY(adjoint_shape(lds_max, dt, n_qubits, opts, &t, &R, &c));
    build_adjoint_schedule(gv.g, gv.n, n_qubits, t, R, c, local);
  } else if (ctx) {
    Schedule* cached;
    TQ_TRY(get_schedule(ctx, dt, gv.g, gv.n, n_qubits, mode, opts, &cached));
    s = cached;
  } else {
    TQ_TRY(forward_shape(lds_max, dt, n_qubits, mode, opts, &t, &R, &c));
    build_schedule(gv.g, gv.n, n_qubits, mode, t, R, c, local);
  }
  int64_t flops = 0, mats = 0;
  for (const HostOp& o : s->ops) {
    if (o.kind == K_MAT1) flops += 14, ++mats;
    else if (o.kind == K_DIAG1 || o.kind == K_DIAG2) flops += 6;
  }
  int64_t xch = 0;
  for (const DevPhase& p : s->phases) xch += p.xchg;
  for (const DevStage& d : s->dstages) xch += d.store_xchg;
  out[0] = mode != 1 ? (int64_t)s->stages.size() : (int64_t)s->ops.size();
  out[1] = (int64_t)s->ops.size();
  out[2] = (int64_t)s->phases.size();
  out[3] = xch;
  out[4] = mode != 1 ? std::min(s->t, n_qubits) : 0;
  out[5] = mode != 1 ? std::min(s->R, std::min(s->t, n_qubits)) : 0;
  out[6] = flops;
  out[7] = mats;
  return TQ_OK;
}

tq_status tq_expval(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const void* d_states, const tq_zterm* terms,
                    int32_t n_terms, int32_t n_obs, void* d_out, void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null context");
  if (dt == TQ_C64) return expval_t<float>(ctx, batch, d_states, terms, n_terms, n_obs, d_out, (hipStream_t)stream);
  if (dt == TQ_C128) return expval_t<double>(ctx, batch, d_states, terms, n_terms, n_obs, d_out, (hipStream_t)stream);
  return fail(TQ_EINVAL, "unknown dtype");
}

}  // extern "C"

extern "C" int64_t tq_sv_backward_workspace(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates,
                                           const int32_t* n_params, const tq_zterm* terms, int32_t n_terms,
                                           int32_t n_obs, const tq_sv_opts* opts) {
  if (!ctx) {
    fail(TQ_EINVAL, "null context");
    return -1;
  }
  int64_t need = -1;
  tq_status st;
  if (dt == TQ_C64)
    st = sv_backward_t<float>(ctx, batch, gates, n_params, nullptr, nullptr, terms, n_terms, n_obs, nullptr, nullptr,
                              opts, nullptr, 0, &need, nullptr);
  else if (dt == TQ_C128)
    st = sv_backward_t<double>(ctx, batch, gates, n_params, nullptr, nullptr, terms, n_terms, n_obs, nullptr, nullptr,
                               opts, nullptr, 0, &need, nullptr);
  else
    st = fail(TQ_EINVAL, "unknown dtype");
  return st == TQ_OK ? need : -1;
}

extern "C" tq_status tq_sv_backward(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates,
                                    const int32_t* n_params, const void* d_params, const void* d_states,
                                    const tq_zterm* terms, int32_t n_terms, int32_t n_obs, const void* d_grad_out,
                                    void* d_grad, const tq_sv_opts* opts, void* d_work, int64_t work_bytes,
                                    void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null context");
  if (!d_work) return fail(TQ_EWORKSPACE, "tq_sv_backward needs a workspace (size from tq_sv_backward_workspace)");
  if (dt == TQ_C64)
    return sv_backward_t<float>(ctx, batch, gates, n_params, d_params, d_states, terms, n_terms, n_obs, d_grad_out,
                                d_grad, opts, d_work, work_bytes, nullptr, (hipStream_t)stream);
  if (dt == TQ_C128)
    return sv_backward_t<double>(ctx, batch, gates, n_params, d_params, d_states, terms, n_terms, n_obs, d_grad_out,
                                 d_grad, opts, d_work, work_bytes, nullptr, (hipStream_t)stream);
  return fail(TQ_EINVAL, "unknown dtype");
}

extern "C" tq_status tq_sv_backward_pauli(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const tq_gate* gates,
                                          const int32_t* n_params, const void* d_params, const void* d_states,
                                          const tq_pauli_term* terms, int32_t n_terms, int32_t n_obs,
                                          const void* d_grad_out, void* d_grad, const tq_sv_opts* opts, void* d_work,
                                          int64_t work_bytes, void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null context");
  if (!d_work) return fail(TQ_EWORKSPACE, "tq_sv_backward_pauli needs a workspace (size from tq_sv_backward_workspace)");
  if (n_terms < 0 || n_terms > kAdjPauliTerms || (n_terms > 0 && !terms))
    return fail(TQ_EINVAL, "the backward pass takes 0.." + std::to_string(kAdjPauliTerms) + " Pauli terms");
  if (dt == TQ_C64)
    return sv_backward_t<float>(ctx, batch, gates, n_params, d_params, d_states, nullptr, 0, n_obs, d_grad_out, d_grad,
                                opts, d_work, work_bytes, nullptr, (hipStream_t)stream, terms, n_terms);
  if (dt == TQ_C128)
    return sv_backward_t<double>(ctx, batch, gates, n_params, d_params, d_states, nullptr, 0, n_obs, d_grad_out,
                                 d_grad, opts, d_work, work_bytes, nullptr, (hipStream_t)stream, terms, n_terms);
  return fail(TQ_EINVAL, "unknown dtype");
}
