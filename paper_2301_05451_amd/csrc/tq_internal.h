// Internal declarations shared by the libtq translation units (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/tq.h"

namespace tq {

// ---------------------------------------------------------------------------------
// Error reporting
// ---------------------------------------------------------------------------------
void set_error(const std::string& msg);
tq_status fail(tq_status st, const std::string& msg);

#define TQ_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::tq::fail(TQ_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

#define TQ_TRY(expr)                 \
  do {                               \
    tq_status s_ = (expr);           \
    if (s_ != TQ_OK) return s_;      \
  } while (0)

// ---------------------------------------------------------------------------------
// Schedule: the host lowering of a gate list (built once per circuit structure).
// ---------------------------------------------------------------------------------

// Kinds of scheduled operations.
enum OpKind : uint8_t {
  K_MAT1 = 0,   // general 2x2 on one target qubit (a fused run of one-qubit gates)
  K_CX = 1,     // controlled-X: target must be register-resident, control read from index
  K_DIAG1 = 2,  // diagonal on one qubit (2 entries)
  K_DIAG2 = 3,  // diagonal on two qubits (4 entries, index 2*bit(qa)+bit(qb))
  K_CZ = 4,     // sign flip where both qubits are 1
  K_MATG = 5,   // forward stages: 2x2 matrices on several register bits of one layer
  K_ZG = 6,     // forward stages: several CZs of one layer as sign flips
};

// A matrix-table entry: how the gate-build kernel forms it from the original gates.
enum RecipeKind : int32_t { R_MAT2 = 0, R_DIAG1 = 1, R_DIAG2 = 2 };

struct HostOp {
  int kind;
  int qa;   // target (MAT1/CX) or first qubit (DIAG/CZ)
  int qb;   // control (CX) or second qubit (DIAG2/CZ), else -1
  int mat;  // matrix-table index or -1
  int src;  // original gate index for recipe-less ops (CX, CZ), else -1
  int nang = 0;  // adjoint schedules: angles of the gate (gradient slots)
};

struct Recipe {
  int kind;
  int qa, qb;
  std::vector<int> gates;  // original gate indices, application order
};

// Device-side descriptors (plain structs, copied verbatim to device memory).
struct DevOp {
  uint8_t kind;
  uint8_t rbit;  // MAT1/CX: target's register-bit index within the phase;
                 // DIAG/CZ: (register index of qa + 1) | (register index of qb + 1) << 4, 0 = none
                 // MATG: mask of the register bits, one matrix each, ascending
                 // ZG: register indices + 1 of up to two CZs whose partner is a thread or
                 //     tile bit (low and high nibble, 0 = none)
  uint8_t pa;    // x-position of qa (DIAG/CZ) or of the control (CX); ZG: first CZ's partner;
                 // MATG: sign flips after the matrices, mask over j, low byte
  uint8_t pb;    // x-position of qb (DIAG2/CZ); CX: control's register index + 1 (0 = none);
                 // ZG: second CZ's partner; MATG: flip mask, high byte
  int32_t mat;   // matrix index (MATG: of the lowest bit's matrix, the rest follow);
                 // ZG: mask over register indices j of the sign flips of the
                 // register-register CZs
};
static_assert(sizeof(DevOp) == 8, "DevOp layout");

constexpr int kMaxReg = 6;
// Reverse sweep: most one-qubit gates reversed as one op (a run on one qubit).
constexpr int kAdjMaxRun = 8;
struct DevPhase {
  int32_t op_begin, op_end;
  int32_t xchg;      // 1: the register layout differs from the previous one (LDS exchange)
  uint8_t rpos[8];   // tile-local positions of the register bits (kMaxReg used)
  uint8_t tpos[24];  // tile-local positions of the thread bits, ascending
};

constexpr int kMaxQ = 40;
struct DevStage {
  int32_t t;            // local bits
  int32_t phase_begin, phase_end;
  int32_t n_nonlocal;
  int32_t store_xchg;   // 1: last phase layout differs from the store layout
  uint8_t lpos[kMaxQ];  // global bit positions of local bits, ascending
  uint8_t npos[kMaxQ];  // global bit positions of non-local bits, ascending
};

struct StageHost {
  int t = 0;
  std::vector<int> lpos, npos;
  int phase_begin = 0, phase_end = 0;
  int n_ops = 0;
};

struct Schedule {
  int n = 0;
  int mode = 0;  // 0 fused, 1 plain
  int t = 0, R = 0, c = 0;
  std::vector<Recipe> recipes;
  std::vector<HostOp> ops;  // fused/plain op list, in a valid execution order
  // fused form
  std::vector<StageHost> stages;
  std::vector<DevPhase> phases;
  std::vector<DevOp> dops;
  std::vector<DevStage> dstages;
  // adjoint form (reverse sweep, one op per original gate; DevOp.mat = gate index)
  bool adjoint = false;
  std::vector<int32_t> dslot;         // per dop: (stage-local first slot << 2) | angle count
  std::vector<int32_t> stage_slot0;   // per stage: first global slot
  std::vector<int32_t> stage_nslot;   // per stage: slots
  int n_slots = 0;                    // total gradient slots = sum of angle counts
  std::vector<int32_t> slot_gate;     // global slot -> gate index
  std::vector<int32_t> slot_angle;    // global slot -> angle index j
  int n_params_used = 0;              // 1 + max parameter index referenced
  std::vector<int32_t> pslot_ptr;     // CSR: parameter -> global slots (with pscale)
  std::vector<int32_t> pslot_idx;
  std::vector<double> pslot_scale;
  // adjoint: runs of one-qubit gates on one qubit reversed as one op. Entries 0..n_gates are
  // offsets into the list that follows them: [adj_runs[k], adj_runs[k+1]) are the gates
  // (forward order) whose product the op at gate k applies; empty for a gate inside
  // another gate's run, {k} for a gate on its own.
  std::vector<int32_t> adj_runs;
  void* d_adj_runs = nullptr;
  void* d_dslot = nullptr;
  void* d_pslot_ptr = nullptr;
  void* d_pslot_idx = nullptr;
  void* d_pslot_scale = nullptr;
  void* d_stage_slot0 = nullptr;
  // device copies (owned)
  void* d_gates = nullptr;      // tq_gate[n_gates]
  void* d_rec = nullptr;        // int32 [n_mats][4]: kind, qa, qb, begin ; + end in next
  void* d_rec_gates = nullptr;  // int32 flat constituent gate indices
  void* d_ops = nullptr;        // DevOp
  void* d_phases = nullptr;     // DevPhase
  void* d_stages = nullptr;     // DevStage
  void* d_blob = nullptr;       // the one allocation holding all of the above
  int n_gates = 0;
  ~Schedule();
};

// Lowering passes (schedule.cpp).
void lower_ops(const tq_gate* g, int n_gates, int n, bool fuse, std::vector<Recipe>& recipes,
               std::vector<HostOp>& ops);
void build_stages(Schedule& s);
void lower_adjoint_ops(const tq_gate* g, int n_gates, std::vector<HostOp>& ops, std::vector<int32_t>& runs);
void build_adjoint_slots(Schedule& s, const tq_gate* g, int n_gates);
tq_status validate_gates(const tq_gate* g, int n_gates, int n, int n_params);
// Controlled rotations (CRX, CRY, CRZ) lowered to the gates the kernels apply (schedule.hip).
bool has_controlled(const tq_gate* g, int64_t n_gates);
void lower_controlled(const tq_gate* g, int n_gates, std::vector<tq_gate>& out);
// A gate list as the kernels see it: the caller's array, or its lowered copy.
struct GateView {
  const tq_gate* g = nullptr;
  int n = 0;
  std::vector<tq_gate> own;
  GateView(const tq_gate* src, int count) : g(src), n(count) {
    if (has_controlled(src, count)) {
      lower_controlled(src, count, own);
      g = own.data();
      n = (int)own.size();
    }
  }
};
int gate_n_angles(int op);
constexpr int kAdjMaxSlotsPerStage = 256;

// A cached device table (see cached_table).
struct TableEntry {
  void* dev = nullptr;
  size_t bytes = 0;
  uint64_t last_use = 0;
};
constexpr size_t kTableCacheBytes = size_t(256) << 20;
constexpr size_t kTableCacheEntries = 4096;

}  // namespace tq

// The context (opaque in the public header).
struct tq_ctx {
  int device = 0;
  int n_cu = 256;
  size_t lds_max = 160 * 1024;
  std::unordered_map<std::string, std::unique_ptr<tq::Schedule>> schedules;
  // grow-only device scratch buffers
  void* scratch[9] = {nullptr};
  size_t scratch_bytes[9] = {0};
  // pinned staging buffer for per-call tables (reused once the previous upload finished)
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t pinned_done = nullptr;
  bool pinned_pending = false;
  // immutable small device tables cached by content (the key is the table's bytes)
  std::unordered_map<std::string, tq::TableEntry> tables;
  size_t table_bytes = 0;
  uint64_t table_clock = 0;
  // scratch buffers replaced by larger ones (freed with the context)
  std::vector<void*> retired;
  // second stream and fork/join events of the batched TN rounds (created on first use)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // streams that run the batched TN calls' sliced networks side by side, with their join events
  hipStream_t pool[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t pool_done[4] = {nullptr, nullptr, nullptr, nullptr};
  // autotune results: key -> (t, R)
  std::unordered_map<std::string, std::pair<int, int>> tuned;
  // imported autotune results: digest of (structure, pass) -> (t, R)
  std::unordered_map<std::string, std::pair<int, int>> tuned_digest;
};

namespace tq {
// scratch slots
enum { S_MATS = 0, S_PARTIAL = 1, S_OFFS = 2, S_LAMBDA = 3, S_PSI = 4, S_GRADP = 5, S_TERMS = 6, S_MISC = 7,
       S_TNB = 8 };
// Grow-only context scratch; `zero` clears a newly allocated buffer (once, synchronously).
tq_status scratch(tq_ctx* ctx, int slot, size_t bytes, void** out, bool zero = false);
// Immutable device copy of a small host table, cached by content (no per-call upload).
tq_status cached_table(tq_ctx* ctx, const void* host, size_t bytes, void** dev);
// Stream-ordered upload of a per-call table into scratch slot `slot` (via pinned memory).
tq_status stage_upload(tq_ctx* ctx, int slot, const void* host, size_t bytes, hipStream_t stream, void** dev);
}  // namespace tq
