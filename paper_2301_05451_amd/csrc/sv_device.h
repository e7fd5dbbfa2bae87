// Device helpers for the state-vector kernels: complex arithmetic, gate matrices built
// from angles in double precision, batch offset maps.
#pragma once

#include <cstddef>
#include <type_traits>

#include "tq_internal.h"

namespace tq {

template <typename T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };

struct dcx {
  double x, y;
};

// Per-circuit offsets of a batch: off[i] if given, else base + i * stride.
struct BatchMap {
  const int64_t* off;
  int64_t base, stride;
  __host__ __device__ __forceinline__ int64_t at(int i) const { return off ? off[i] : base + stride * (int64_t)i; }
  __host__ BatchMap shifted(int c0) const {
    BatchMap m = *this;
    if (off) m.off = off + c0; else m.base += stride * (int64_t)c0;
    return m;
  }
};

template <typename C>
__host__ __device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// m0 * a + m1 * b
template <typename C>
__device__ __forceinline__ C cfma2(C m0, C a, C m1, C b) {
  C r;
  r.x = m0.x * a.x - m0.y * a.y + m1.x * b.x - m1.y * b.y;
  r.y = m0.x * a.y + m0.y * a.x + m1.x * b.y + m1.y * b.x;
  return r;
}

template <typename T>
__device__ __forceinline__ typename Cx<T>::type to_cx(dcx v) {
  typename Cx<T>::type r;
  r.x = (T)v.x;
  r.y = (T)v.y;
  return r;
}

struct dmat2 {
  dcx m[4];  // row-major: m[0]=u00 m[1]=u01 m[2]=u10 m[3]=u11
  __device__ static dmat2 identity() { return dmat2{{{1, 0}, {0, 0}, {0, 0}, {1, 0}}}; }
};

__device__ __forceinline__ dmat2 mat_mul(const dmat2& A, const dmat2& B) {
  dmat2 C;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      dcx a = cmul(A.m[2 * i + 0], B.m[0 + j]);
      dcx b = cmul(A.m[2 * i + 1], B.m[2 + j]);
      C.m[2 * i + j] = dcx{a.x + b.x, a.y + b.y};
    }
  return C;
}

__device__ __forceinline__ dcx expi(double a) {
  double s, c;
  sincos(a, &s, &c);
  return dcx{c, s};
}

template <typename T>
__device__ __forceinline__ void gate_angles(const tq_gate& g, const T* p, double* a) {
  for (int j = 0; j < 3; ++j) {
    const int pi = g.pidx[j];
    a[j] = pi >= 0 ? g.pscale[j] * (double)p[pi] : g.pscale[j];
  }
}

// 2x2 matrix of a one-qubit gate.
__device__ inline dmat2 gate_mat2(int op, const double* a) {
  const double r = 0.70710678118654752440;
  dmat2 M = dmat2::identity();
  double s, c;
  switch (op) {
    case TQ_H: M = dmat2{{{r, 0}, {r, 0}, {r, 0}, {-r, 0}}}; break;
    case TQ_X: M = dmat2{{{0, 0}, {1, 0}, {1, 0}, {0, 0}}}; break;
    case TQ_Y: M = dmat2{{{0, 0}, {0, -1}, {0, 1}, {0, 0}}}; break;
    case TQ_Z: M = dmat2{{{1, 0}, {0, 0}, {0, 0}, {-1, 0}}}; break;
    case TQ_RX:
      sincos(0.5 * a[0], &s, &c);
      M = dmat2{{{c, 0}, {0, -s}, {0, -s}, {c, 0}}};
      break;
    case TQ_RY:
      sincos(0.5 * a[0], &s, &c);
      M = dmat2{{{c, 0}, {-s, 0}, {s, 0}, {c, 0}}};
      break;
    case TQ_RZ: {
      dcx e = expi(-0.5 * a[0]);
      M = dmat2{{e, {0, 0}, {0, 0}, {e.x, -e.y}}};
      break;
    }
    case TQ_U3: {
      sincos(0.5 * a[0], &s, &c);
      dcx el = expi(a[2]), ep = expi(a[1]), epl = expi(a[1] + a[2]);
      M = dmat2{{{c, 0}, {-el.x * s, -el.y * s}, {ep.x * s, ep.y * s}, {epl.x * c, epl.y * c}}};
      break;
    }
    case TQ_ROT: {
      // RZ(omega) RY(theta) RZ(phi) with (phi, theta, omega) = (a0, a1, a2)
      double a0[1] = {a[0]}, a1[1] = {a[1]}, a2[1] = {a[2]};
      M = mat_mul(gate_mat2(TQ_RZ, a2), mat_mul(gate_mat2(TQ_RY, a1), gate_mat2(TQ_RZ, a0)));
      break;
    }
    default: break;
  }
  return M;
}

// Factor that diagonal gate g contributes to the diagonal entry with bit values (ba, bb)
// of the recipe's qubits (qa and the other one).
__device__ inline dcx diag_entry(const tq_gate& g, int qa, int ba, int bb, const double* a) {
  switch (g.op) {
    case TQ_CZ: return dcx{(ba & bb) ? -1.0 : 1.0, 0};
    case TQ_RZZ: return expi((ba ^ bb) ? 0.5 * a[0] : -0.5 * a[0]);
    case TQ_RZ: {
      int b = (g.q[0] == qa) ? ba : bb;
      return expi(b ? 0.5 * a[0] : -0.5 * a[0]);
    }
    case TQ_Z: {
      int b = (g.q[0] == qa) ? ba : bb;
      return dcx{b ? -1.0 : 1.0, 0};
    }
    default: return dcx{1, 0};
  }
}

__host__ __device__ inline int gate_n_angles_dev(int op) {
  return (op == TQ_RX || op == TQ_RY || op == TQ_RZ || op == TQ_RZZ) ? 1 : (op == TQ_U3 || op == TQ_ROT) ? 3 : 0;
}

constexpr int kAdjMatStride = 16;  // per gate: U (4 entries) then dU/da_j (4 entries each)

// ---- matrices of a gate and of its angle derivatives (double precision) ----------------
__device__ inline dmat2 d_rz(double a) {  // dRZ/da = diag(-i/2 e^{-ia/2}, i/2 e^{ia/2})
  dcx e = expi(-0.5 * a);                  // e^{-ia/2}; e^{ia/2} = conj(e)
  return dmat2{{{0.5 * e.y, -0.5 * e.x}, {0, 0}, {0, 0}, {0.5 * e.y, 0.5 * e.x}}};
}
__device__ inline dmat2 d_ry(double a) {
  double s, c;
  sincos(0.5 * a, &s, &c);
  return dmat2{{{-0.5 * s, 0}, {-0.5 * c, 0}, {0.5 * c, 0}, {-0.5 * s, 0}}};
}
__device__ inline dmat2 d_rx(double a) {
  double s, c;
  sincos(0.5 * a, &s, &c);
  return dmat2{{{-0.5 * s, 0}, {0, -0.5 * c}, {0, -0.5 * c}, {-0.5 * s, 0}}};
}

// Fills U and the derivative with respect to each angle (rows of 4, row-major 2x2, or the
// diagonal for Z/RZ (2 entries, repeated) and RZZ (4 entries, index 2*bit(q0)+bit(q1))).
__device__ inline void gate_and_derivs(int op, const double* a, dcx (&out)[kAdjMatStride]) {
  for (int i = 0; i < kAdjMatStride; ++i) out[i] = dcx{0, 0};
  auto put = [&](int slot, const dmat2& M) {
    for (int i = 0; i < 4; ++i) out[4 * slot + i] = M.m[i];
  };
  switch (op) {
    case TQ_RX: put(0, gate_mat2(TQ_RX, a)); put(1, d_rx(a[0])); break;
    case TQ_RY: put(0, gate_mat2(TQ_RY, a)); put(1, d_ry(a[0])); break;
    case TQ_RZ: {
      dcx e0 = expi(-0.5 * a[0]), e1 = expi(0.5 * a[0]);
      out[0] = e0; out[1] = e1; out[2] = e0; out[3] = e1;
      dcx d0{0.5 * e0.y, -0.5 * e0.x}, d1{-0.5 * e1.y, 0.5 * e1.x};
      out[4] = d0; out[5] = d1; out[6] = d0; out[7] = d1;
      break;
    }
    case TQ_Z: out[0] = {1, 0}; out[1] = {-1, 0}; out[2] = {1, 0}; out[3] = {-1, 0}; break;
    case TQ_RZZ: {
      dcx em = expi(-0.5 * a[0]), ep = expi(0.5 * a[0]);
      out[0] = em; out[1] = ep; out[2] = ep; out[3] = em;
      dcx dm{0.5 * em.y, -0.5 * em.x}, dp{-0.5 * ep.y, 0.5 * ep.x};
      out[4] = dm; out[5] = dp; out[6] = dp; out[7] = dm;
      break;
    }
    case TQ_U3: {
      // U3(th, ph, la) = [[c, -e^{i la} s], [e^{i ph} s, e^{i(ph+la)} c]]
      double s, c;
      sincos(0.5 * a[0], &s, &c);
      dcx el = expi(a[2]), ep = expi(a[1]), epl = expi(a[1] + a[2]);
      put(0, gate_mat2(TQ_U3, a));
      out[4] = {-0.5 * s, 0}; out[5] = {-0.5 * c * el.x, -0.5 * c * el.y};
      out[6] = {0.5 * c * ep.x, 0.5 * c * ep.y}; out[7] = {-0.5 * s * epl.x, -0.5 * s * epl.y};
      out[8] = {0, 0}; out[9] = {0, 0};
      out[10] = {-s * ep.y, s * ep.x}; out[11] = {-c * epl.y, c * epl.x};
      out[12] = {0, 0}; out[13] = {s * el.y, -s * el.x};
      out[14] = {0, 0}; out[15] = {-c * epl.y, c * epl.x};
      break;
    }
    case TQ_ROT: {
      // RZ(om) RY(th) RZ(ph) with (ph, th, om) = (a0, a1, a2)
      double a0[1] = {a[0]}, a1[1] = {a[1]}, a2[1] = {a[2]};
      dmat2 Z0 = gate_mat2(TQ_RZ, a0), Y1 = gate_mat2(TQ_RY, a1), Z2 = gate_mat2(TQ_RZ, a2);
      put(0, mat_mul(Z2, mat_mul(Y1, Z0)));
      put(1, mat_mul(Z2, mat_mul(Y1, d_rz(a[0]))));
      put(2, mat_mul(Z2, mat_mul(d_ry(a[1]), Z0)));
      put(3, mat_mul(d_rz(a[2]), mat_mul(Y1, Z0)));
      break;
    }
    default: put(0, gate_mat2(op, a)); break;  // H, X, Y (no angles); CNOT/CZ unused
  }
}


// Full 2x2 forms of a one-qubit gate and of its angle derivatives; returns the angle count.
__device__ inline int gate_full2(int op, const double* a, dmat2& U, dmat2 (&D)[3]) {
  dcx m[kAdjMatStride];
  gate_and_derivs(op, a, m);
  const int na = gate_n_angles_dev(op);
  const dcx z{0, 0};
  if (op == TQ_RZ || op == TQ_Z) {  // stored as the diagonal
    U = dmat2{{m[0], z, z, m[1]}};
    if (na > 0) D[0] = dmat2{{m[4], z, z, m[5]}};
  } else {
    U = dmat2{{m[0], m[1], m[2], m[3]}};
    for (int j = 0; j < na; ++j) D[j] = dmat2{{m[4 + 4 * j], m[5 + 4 * j], m[6 + 4 * j], m[7 + 4 * j]}};
  }
  return na;
}


// Matrix-table entry of the reverse-sweep op at gate k (runs as in the adjoint schedule: n
// offsets + 1, then the gate lists). A gate on its own keeps its own U and dU/da_j. A run
// G_L ... G_1 on one qubit gets U = G_L ... G_1 and, for angle j of gate i, the matrix
// (G_L ... G_{i+1}) dG_i/da_j (G_{i-1} ... G_1): the gradient term of that angle is then
// Re <lam| X |psi> with psi taken before the run and lam after it, the same form as for a
// single gate. Returns false for a gate inside another gate's run (no entry).
template <typename P>
__device__ inline bool adj_entry(const tq_gate* gates, int n_gates, const int32_t* runs, int k, const P* params,
                                 dcx (&out)[kAdjMatStride]) {
  const int b = runs[k], e = runs[k + 1];
  if (b == e) return false;
  if (e - b == 1) {
    double a[3];
    gate_angles(gates[k], params, a);
    gate_and_derivs(gates[k].op, a, out);
    return true;
  }
  const int32_t* lst = runs + n_gates + 1;
  const int L = e - b < kAdjMaxRun ? e - b : kAdjMaxRun;
  dmat2 G[kAdjMaxRun];
  for (int i = 0; i < L; ++i) {
    double a[3];
    gate_angles(gates[lst[b + i]], params, a);
    dmat2 D[3];
    gate_full2(gates[lst[b + i]].op, a, G[i], D);
  }
  for (int i = 0; i < kAdjMatStride; ++i) out[i] = dcx{0, 0};
  dmat2 U = dmat2::identity();
  for (int i = 0; i < L; ++i) U = mat_mul(G[i], U);
  for (int r = 0; r < 4; ++r) out[r] = U.m[r];
  int slot = 1;
  dmat2 B = dmat2::identity();  // G_{i-1} ... G_1
  for (int i = 0; i < L; ++i) {
    double a[3];
    gate_angles(gates[lst[b + i]], params, a);
    dmat2 Gi, D[3];
    const int na = gate_full2(gates[lst[b + i]].op, a, Gi, D);
    dmat2 A = dmat2::identity();  // G_L ... G_{i+1}
    for (int m = i + 1; m < L; ++m) A = mat_mul(G[m], A);
    for (int j = 0; j < na && slot < 4; ++j, ++slot) {
      const dmat2 X = mat_mul(A, mat_mul(D[j], B));
      for (int r = 0; r < 4; ++r) out[4 * slot + r] = X.m[r];
    }
    B = mat_mul(Gi, B);
  }
  return true;
}

// Schedule records, op lists and slot tables live in device (global) memory. Their
// pointers are often read from device memory themselves (the per-circuit records of a
// batch), and the compiler then only knows them as generic pointers: loads through them
// become flat loads, vector loads whose results land in vector registers even when every
// lane reads the same word. Reading through global-address-space pointers lets such
// uniform reads go through scalar loads.
#define TQ_GLOBAL __attribute__((address_space(1)))
using gword = TQ_GLOBAL const uint32_t;
template <typename P>
__device__ __forceinline__ const TQ_GLOBAL P* gptr(const P* p) {
  return (const TQ_GLOBAL P*)p;
}

// Read one 8-byte op descriptor as a single aligned 64-bit word and unpack its byte
// fields. Reading the fields one by one let the compiler split a field's address into a
// misaligned scalar base plus a misaligned immediate offset; the scalar unit does not
// add those before dropping the low address bits, so the matrix index came back as the
// op header and the matrix load left its buffer.
__device__ __forceinline__ DevOp load_op(const DevOp* ops, int o) {
  const gword* const q = reinterpret_cast<const gword*>(gptr(ops)) + 2 * (int64_t)o;
  uint2 w;
  w.x = q[0];
  w.y = q[1];
  DevOp d;
  d.kind = (uint8_t)(w.x & 0xffu);
  d.rbit = (uint8_t)((w.x >> 8) & 0xffu);
  d.pa = (uint8_t)((w.x >> 16) & 0xffu);
  d.pb = (uint8_t)(w.x >> 24);
  d.mat = (int32_t)w.y;
  return d;
}

// Schedule records (DevStage, DevPhase) are read as aligned 32-bit words with the byte
// fields unpacked in registers. A byte field read on its own is a vector load (the scalar
// unit loads whole words), a full memory round trip the wave waits for; reading words that
// every lane shares lets them come through the scalar cache, several per instruction.
constexpr int kStageWords = (int)(sizeof(DevStage) / 4);
constexpr int kPhaseWords = (int)(sizeof(DevPhase) / 4);
constexpr int kStageLposWord = (int)(offsetof(DevStage, lpos) / 4);
constexpr int kStageNposWord = (int)(offsetof(DevStage, npos) / 4);
constexpr int kPhaseRposWord = (int)(offsetof(DevPhase, rpos) / 4);
constexpr int kPhaseTposWord = (int)(offsetof(DevPhase, tpos) / 4);
static_assert(sizeof(DevStage) % 4 == 0 && sizeof(DevPhase) % 4 == 0, "word-readable records");
static_assert(offsetof(DevStage, lpos) % 4 == 0 && offsetof(DevStage, npos) % 4 == 0, "word-aligned");
static_assert(offsetof(DevPhase, rpos) % 4 == 0 && offsetof(DevPhase, tpos) % 4 == 0, "word-aligned");
static_assert(offsetof(DevStage, t) == 0 && offsetof(DevStage, phase_begin) == 4 &&
              offsetof(DevStage, phase_end) == 8 && offsetof(DevStage, n_nonlocal) == 12 &&
              offsetof(DevStage, store_xchg) == 16, "DevStage header words");
static_assert(offsetof(DevPhase, op_begin) == 0 && offsetof(DevPhase, op_end) == 4 &&
              offsetof(DevPhase, xchg) == 8, "DevPhase header words");

__device__ __forceinline__ uint32_t word_byte(const gword* w, int first_word, int k) {
  return (w[first_word + (k >> 2)] >> (8 * (k & 3))) & 0xffu;
}

// Most thread bits a stage tile has: launches use at most 512 threads.
constexpr int kMaxThreadBits = 9;

// Global offset of a tile's fixed (non-local) index bits: uniform, scalar work only. The
// tile id has no bits at or above the stage's non-local count, so every position byte may
// be visited (no branch per bit).
__device__ __forceinline__ int64_t stage_tile_base(const gword* sw, uint32_t tile) {
  int64_t base = 0;
#pragma unroll
  for (int k = 0; k < 32; ++k) base |= (int64_t)((tile >> k) & 1u) << word_byte(sw, kStageNposWord, k);
  return base;
}

// Global offset of a thread's own index bits (the low tb local bits in the load layout).
__device__ __forceinline__ int64_t stage_thread_offset(const gword* sw, int tb, uint32_t tid) {
  const uint32_t tl = tid & ((1u << tb) - 1u);
  int64_t thr = 0;
#pragma unroll
  for (int k = 0; k < kMaxThreadBits; ++k) thr |= (int64_t)((tl >> k) & 1u) << word_byte(sw, kStageLposWord, k);
  return thr;
}

// Tile-local positions of a thread's bits in a phase's layout.
__device__ __forceinline__ uint32_t phase_thread_bits(const gword* pw, int tb, uint32_t tid) {
  const uint32_t tl = tid & ((1u << tb) - 1u);
  uint32_t tp = 0;
#pragma unroll
  for (int k = 0; k < kMaxThreadBits; ++k) tp |= ((tl >> k) & 1u) << word_byte(pw, kPhaseTposWord, k);
  return tp;
}

// Largest c with pref[c] <= g (pref ascending, pref[0] = 0, pref[count] > g).
__device__ __forceinline__ int find_circ(const int64_t* __restrict__ pref, int count, int64_t g) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pref[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__host__ __device__ __forceinline__ int64_t insert_zero(int64_t k, int pos) {
  const int64_t lo = k & ((int64_t(1) << pos) - 1);
  return ((k >> pos) << (pos + 1)) | lo;
}

// One circuit of a heterogeneous batch: its schedule's device tables and its offsets into
// the batch buffers. Forward launches use the first group of fields, the reverse sweep the
// adjoint ones. All fields are 4- or 8-byte aligned at their natural offsets.
struct DevCirc {
  const DevStage* stages;
  const DevPhase* phases;
  const DevOp* ops;
  const tq_gate* gates;
  const int32_t* rec;        // forward: matrix recipes (kind, qa, qb, begin) + sentinel
  const int32_t* rec_gates;  // forward: constituent gate indices; adjoint: run table
  const int32_t* dslot;      // adjoint: per-op slot info
  const int32_t* pslot_ptr;  // adjoint: parameter -> slot CSR
  const int32_t* pslot_idx;
  const double* pslot_scale;
  const unsigned char* terms;  // adjoint: [masks u64][coeff f64][obs i32] for this n
  int64_t mats_off;   // matrix table, complex elements
  int64_t state_off;  // caller state, complex elements
  int64_t param_off;  // parameters and gradients, reals
  int64_t work_off;   // adjoint psi / lambda working copies, complex elements
  int64_t part_off;   // adjoint per-tile partial sums, doubles
  int32_t n;          // qubits
  int32_t n_mats;     // forward: matrix-table entries; adjoint: gates
  int32_t n_stages;
  int32_t n_slots;    // adjoint gradient slots
  int32_t n_params;   // gradient entries written
  int32_t n_used;     // parameters referenced by the gates
  int32_t row;        // batch index (row of grad_out)
  int32_t n_terms;
};
static_assert(sizeof(DevCirc) == 160, "DevCirc layout");

// A work item of a batched stage launch: one tile of one circuit.
struct BatchItem {
  int32_t circ;
  uint32_t tile;
};

// Batched launches over a heterogeneous batch (one kernel per stage level).
struct BatchLaunch {
  const DevCirc* d_circ = nullptr;
  const int64_t* d_pref = nullptr;   // per-circuit prefix of matrix (or gate) counts, count+1
  const int64_t* d_ppref = nullptr;  // adjoint: per-circuit prefix of gradient entries, count+1
  const BatchItem* d_items = nullptr;
  std::vector<int64_t> level_begin;  // item ranges per level, levels+1 entries
  std::vector<int32_t> level_t;      // largest tile bits at each level
  std::vector<int32_t> level_nslot;  // adjoint: largest per-stage slot count at each level
  int count = 0;
  int64_t total_mats = 0;
  int64_t total_params = 0;
  int64_t max_amps = 0;
  int T = 0, R = 0;
};
template <typename T>
tq_status launch_batch_forward(const BatchLaunch& b, const void* d_params, void* d_mats, void* d_states,
                               hipStream_t stream);
template <typename T>
tq_status launch_batch_adjoint(const BatchLaunch& b, const void* d_params, void* d_mats, const void* d_states,
                               void* d_work_psi, void* d_work_lam, double* d_partial, const T* d_grad_out,
                               int n_obs, T* d_grad, hipStream_t stream);

// Host helpers shared by the entry points (api.hip).
// Circuits of a batch grouped by structure (n, gate_off, n_gates), in first-seen order.
struct Group {
  int n;
  int64_t gate_off;
  int n_gates;
  int n_params;
  std::vector<int> members;
};
tq_status group_batch(const tq_batch* b, const int32_t* n_params, std::vector<Group>& groups);
tq_status member_map(tq_ctx* ctx, int slot, const int64_t* all, const std::vector<int>& m, hipStream_t stream,
                     BatchMap* out);
tq_status get_schedule(tq_ctx* ctx, int dt, const tq_gate* g, int n_gates, int n, int mode, const tq_sv_opts* opts,
                       Schedule** out);
tq_status get_adjoint_schedule(tq_ctx* ctx, int dt, const tq_gate* g, int n_gates, int n, const tq_sv_opts* opts,
                               Schedule** out);
tq_status term_table(tq_ctx* ctx, int n, const tq_zterm* terms, int n_terms, const unsigned char** dev);

// launchers (sv_kernels.hip)
template <typename T>
tq_status launch_gate_build(const Schedule& s, const void* d_params, BatchMap pmap, void* d_mats, int count,
                            hipStream_t stream);
template <typename T>
tq_status launch_plain(const Schedule& s, void* d_states, BatchMap smap, const void* d_mats, int count, int n_cu,
                       hipStream_t stream);
// basis >= 0: the states are not read; the first stage starts from |basis> (every stage
// of a schedule with at least one stage; the caller prepares the states otherwise).
template <typename T>
tq_status launch_stages(const Schedule& s, void* d_states, BatchMap smap, const void* d_mats, int count,
                        int64_t basis, hipStream_t stream);
template <typename T>
tq_status launch_init_basis(void* d_states, BatchMap smap, int n, int count, int64_t basis, int n_cu,
                            hipStream_t stream);
// sv_adjoint.hip
constexpr int kAdjMatEntries = kAdjMatStride;
constexpr int kAdjPauliTerms = 16;  // Pauli terms with X / Y factors per adjoint call
struct AdjPauli {              // terms over bit positions of an n-qubit index
  uint64_t f[kAdjPauliTerms];  // flip masks (X or Y)
  uint64_t m[kAdjPauliTerms];  // sign masks (Y or Z)
  double c[kAdjPauliTerms];    // coefficients
  int32_t ob[kAdjPauliTerms];  // outputs
  int32_t cls[kAdjPauliTerms]; // number of Y factors mod 4
  int32_t n;
};
// pauli == nullptr: lambda from the Z-string terms (pm, cf, ob); else from the Pauli terms.
template <typename T>
tq_status launch_adjoint(const Schedule& s, const void* d_params, BatchMap pmap, const void* d_states_in,
                         BatchMap smap_in, void* psi, void* lam, BatchMap smap_w, void* mats, double* partial,
                         const uint64_t* pm, const double* cf, const int32_t* ob, int n_terms, const T* grad_out,
                         int n_obs, T* grad, int n_params, int count, hipStream_t stream,
                         const AdjPauli* pauli = nullptr);

// expval.hip
int expval_groups(int n, int cn);
size_t expval_scratch_doubles(int n, int count, int n_obs);
template <typename T>
tq_status launch_expval(const typename Cx<T>::type* d_states, BatchMap smap, int n, int count,
                        const uint64_t* d_pmask, const double* d_coeff, const int32_t* d_obs, int n_terms, int n_obs,
                        double* d_scratch, size_t scratch_doubles, T* d_out, BatchMap rows, hipStream_t stream);

}  // namespace tq
