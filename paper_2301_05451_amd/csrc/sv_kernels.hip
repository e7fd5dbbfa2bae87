// State-vector kernels for gfx950 (wave64): gate-matrix build, plain one-gate sweeps,
// fused LDS-tile stages, and Z-string expectation values.
//
// Layout: one circuit's state is 2^n interleaved complex amplitudes (float2 or double2);
// qubit q is bit n-1-q of the index. A batch of states sits in one allocation at per-
// circuit offsets (BatchMap).
#include "sv_device.h"

namespace tq {

// ---------------------------------------------------------------------------------
// Gate-matrix build: one thread per (circuit, matrix-table entry). Products are formed in
// double precision from the circuit's parameters and rounded once to the state dtype.
// ---------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void build_mat(const tq_gate* __restrict__ gates, const int32_t* __restrict__ rec,
                                          const int32_t* __restrict__ rec_gates, int m, const T* __restrict__ p,
                                          typename Cx<T>::type* __restrict__ out) {
  const int kind = rec[4 * m + 0], qa = rec[4 * m + 1];
  const int b0 = rec[4 * m + 3], b1 = rec[4 * (m + 1) + 3];
  if (kind == R_MAT2) {
    dmat2 M = dmat2::identity();
    for (int i = b0; i < b1; ++i) {
      const tq_gate& g = gates[rec_gates[i]];
      double a[3];
      gate_angles(g, p, a);
      M = mat_mul(gate_mat2(g.op, a), M);
    }
    for (int k = 0; k < 4; ++k) out[k] = to_cx<T>(M.m[k]);
  } else {
    // diagonal: entries indexed by 2*bit(qa) + bit(qb) (R_DIAG2) or bit(qa) (R_DIAG1)
    dcx d[4] = {{1, 0}, {1, 0}, {1, 0}, {1, 0}};
    for (int i = b0; i < b1; ++i) {
      const tq_gate& g = gates[rec_gates[i]];
      double a[3];
      gate_angles(g, p, a);
      for (int idx = 0; idx < 4; ++idx) {
        int ba = (kind == R_DIAG2) ? (idx >> 1) : (idx & 1);
        int bb = idx & 1;
        d[idx] = cmul(d[idx], diag_entry(g, qa, ba, bb, a));
      }
    }
    for (int k = 0; k < 4; ++k) out[k] = to_cx<T>(d[k]);
  }
}

template <typename T>
__global__ void gate_build_kernel(const tq_gate* __restrict__ gates, const int32_t* __restrict__ rec,
                                  const int32_t* __restrict__ rec_gates, int n_mats,
                                  const T* __restrict__ params, BatchMap pmap,
                                  typename Cx<T>::type* __restrict__ mats, int count) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)n_mats * count) return;
  const int m = (int)(gid % n_mats);
  const int circ = (int)(gid / n_mats);
  build_mat<T>(gates, rec, rec_gates, m, params + pmap.at(circ), mats + ((int64_t)circ * n_mats + m) * 4);
}

// Heterogeneous batch: one thread per (circuit, matrix entry) over the concatenated tables.
template <typename T>
__global__ void batch_gate_build_kernel(const DevCirc* __restrict__ circs, const int64_t* __restrict__ pref,
                                        int count, const T* __restrict__ params,
                                        typename Cx<T>::type* __restrict__ mats) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= pref[count]) return;
  const int c = find_circ(pref, count, gid);
  const DevCirc& d = circs[c];
  const int m = (int)(gid - pref[c]);
  build_mat<T>(d.gates, d.rec, d.rec_gates, m, params + d.param_off, mats + d.mats_off + 4 * (int64_t)m);
}

// ---------------------------------------------------------------------------------
// Plain sweeps: one HBM pass per scheduled op (grid-stride; y = circuit).
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) plain_mat1_kernel(typename Cx<T>::type* __restrict__ st, BatchMap smap,
                                                         int pos, int64_t npairs,
                                                         const typename Cx<T>::type* __restrict__ mats,
                                                         int64_t mats_stride, int mat) {
  using C = typename Cx<T>::type;
  C* s = st + smap.at(blockIdx.y);
  const C* M = mats + (int64_t)blockIdx.y * mats_stride + 4 * (int64_t)mat;
  const C m0 = M[0], m1 = M[1], m2 = M[2], m3 = M[3];
  const int64_t lo_mask = (int64_t(1) << pos) - 1;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npairs; k += (int64_t)gridDim.x * blockDim.x) {
    int64_t i0 = ((k & ~lo_mask) << 1) | (k & lo_mask);
    int64_t i1 = i0 | (int64_t(1) << pos);
    C a = s[i0], b = s[i1];
    s[i0] = cfma2(m0, a, m1, b);
    s[i1] = cfma2(m2, a, m3, b);
  }
}

// Controlled-X: swap the target pair where the control bit is 1 (touches half the state).
template <typename T>
__global__ void __launch_bounds__(256) plain_cx_kernel(typename Cx<T>::type* __restrict__ st, BatchMap smap,
                                                       int pc, int pt, int64_t nquads) {
  using C = typename Cx<T>::type;
  C* s = st + smap.at(blockIdx.y);
  const int plo = pc < pt ? pc : pt, phi = pc < pt ? pt : pc;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nquads; k += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = insert_zero(insert_zero(k, plo), phi) | (int64_t(1) << pc);
    int64_t j = i | (int64_t(1) << pt);
    C a = s[i], b = s[j];
    s[i] = b;
    s[j] = a;
  }
}

// CZ: negate the quarter of amplitudes with both bits 1.
template <typename T>
__global__ void __launch_bounds__(256) plain_cz_kernel(typename Cx<T>::type* __restrict__ st, BatchMap smap,
                                                       int pa, int pb, int64_t nquads) {
  using C = typename Cx<T>::type;
  C* s = st + smap.at(blockIdx.y);
  const int plo = pa < pb ? pa : pb, phi = pa < pb ? pb : pa;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nquads; k += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = insert_zero(insert_zero(k, plo), phi) | (int64_t(1) << pa) | (int64_t(1) << pb);
    C a = s[i];
    a.x = -a.x;
    a.y = -a.y;
    s[i] = a;
  }
}

// Diagonal on one or two qubits: every amplitude times d[2*bit(pa)+bit(pb)] (pb < 0: d[bit(pa)]).
template <typename T>
__global__ void __launch_bounds__(256) plain_diag_kernel(typename Cx<T>::type* __restrict__ st, BatchMap smap,
                                                         int pa, int pb, int64_t namps,
                                                         const typename Cx<T>::type* __restrict__ mats,
                                                         int64_t mats_stride, int mat) {
  using C = typename Cx<T>::type;
  C* s = st + smap.at(blockIdx.y);
  const C* D = mats + (int64_t)blockIdx.y * mats_stride + 4 * (int64_t)mat;
  const C d0 = D[0], d1 = D[1], d2 = D[2], d3 = D[3];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < namps; i += (int64_t)gridDim.x * blockDim.x) {
    const int ba = (int)((i >> pa) & 1);
    const int bb = pb < 0 ? ba : (int)((i >> pb) & 1);
    const bool two = pb >= 0;
    C d;
    d.x = ba ? (two ? (bb ? d3.x : d2.x) : d1.x) : (two ? (bb ? d1.x : d0.x) : d0.x);
    d.y = ba ? (two ? (bb ? d3.y : d2.y) : d1.y) : (two ? (bb ? d1.y : d0.y) : d0.y);
    s[i] = cmul(d, s[i]);
  }
}

// ---------------------------------------------------------------------------------
// Fused LDS-tile stage. A work-group owns one tile: 2^t amplitudes whose index varies
// over the stage's local bit positions (lpos) with the other bits fixed by the tile id.
// Each thread holds 2^R amplitudes in registers. Loads and stores use the layout where
// the register bits are the top R local bits, so consecutive threads touch consecutive
// addresses (the lowest local positions are the lowest index bits). Each phase applies
// its ops on the register-resident target bits; switching the register bit set is one
// exchange through LDS (XOR-swizzled to spread banks).
// ---------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ uint32_t lds_swz(uint32_t li) {
  // fold higher G-bit groups into the low G bits (a bijection on [0, 2^t))
  constexpr int G = sizeof(T) == 4 ? 5 : 4;
  constexpr uint32_t mask = (1u << G) - 1;
  return li ^ (((li >> G) ^ (li >> (2 * G)) ^ (li >> (3 * G))) & mask);
}

template <typename T, int R, int B>
__device__ __forceinline__ void reg_mat(typename Cx<T>::type (&v)[1 << R], typename Cx<T>::type m0,
                                        typename Cx<T>::type m1, typename Cx<T>::type m2,
                                        typename Cx<T>::type m3) {
#pragma unroll
  for (int j = 0; j < (1 << R); ++j) {
    if (j & (1 << B)) continue;
    const int j1 = j | (1 << B);
    auto a = v[j], b = v[j1];
    v[j] = cfma2(m0, a, m1, b);
    v[j1] = cfma2(m2, a, m3, b);
  }
}

// Bit `pos` of the tile-local index of this thread's amplitudes when it is not a register
// bit: a thread bit (tp holds the thread bits at their local positions) or a tile bit.
__device__ __forceinline__ uint32_t idx_bit(int pos, uint32_t tp, int t, uint32_t tile) {
  return pos < t ? ((tp >> pos) & 1u) : ((tile >> (pos - t)) & 1u);
}

__device__ __forceinline__ float flip_sign(float x, uint32_t s) { return __uint_as_float(__float_as_uint(x) ^ s); }
__device__ __forceinline__ double flip_sign(double x, uint32_t s) {
  return __longlong_as_double(__double_as_longlong(x) ^ ((long long)s << 32));
}

// Masks over the register index j (bit j set when bit k of j is 1), for register bit k.
__device__ __forceinline__ uint32_t reg_mask(int k) {
  // a select chain (a table indexed at run time would live in scratch memory)
  return k == 0 ? 0xAAAAAAAAu
       : k == 1 ? 0xCCCCCCCCu
       : k == 2 ? 0xF0F0F0F0u
       : k == 3 ? 0xFF00FF00u
       : k == 4 ? 0xFFFF0000u
                : 0xFFFFFFFFu;
}

// CX with the target on register bit B: the pairs with (mc >> j) & 1 are swapped where the
// per-thread flag cb is set. A register control gives a uniform mc and cb = 1; a thread or
// tile control gives mc = all and a per-thread cb.
template <typename T, int R, int B>
__device__ __forceinline__ void reg_cx(typename Cx<T>::type (&v)[1 << R], uint32_t mc, uint32_t cb) {
#pragma unroll
  for (int j = 0; j < (1 << R); ++j) {
    if (j & (1 << B)) continue;
    const int j1 = j | (1 << B);
    if ((mc >> j) & 1u) {
      auto a = v[j], b = v[j1];
      v[j].x = cb ? b.x : a.x;
      v[j].y = cb ? b.y : a.y;
      v[j1].x = cb ? a.x : b.x;
      v[j1].y = cb ? a.y : b.y;
    }
  }
}

// CZ: amplitudes with (m >> j) & 1 (register operands both 1) get the per-thread sign s (the
// product of the non-register operand bits).
template <typename T, int R>
__device__ __forceinline__ void reg_cz(typename Cx<T>::type (&v)[1 << R], uint32_t m, uint32_t s) {
#pragma unroll
  for (int j = 0; j < (1 << R); ++j) {
    if ((m >> j) & 1u) {
      v[j].x = flip_sign(v[j].x, s);
      v[j].y = flip_sign(v[j].y, s);
    }
  }
}

// A layer of one-qubit matrices on the register bits in MASK, ascending bit order; the
// matrices are consecutive in the table (m, then m + 4, ...). Straight-line code: one loop
// iteration of the op list covers the whole layer.
template <typename T, int R, int MASK, int B = 0, int RANK = 0>
__device__ __forceinline__ void reg_mat_group(typename Cx<T>::type (&v)[1 << R],
                                              const typename Cx<T>::type* __restrict__ m) {
  if constexpr (B < R) {
    if constexpr (((MASK >> B) & 1) != 0) {
      reg_mat<T, R, B>(v, m[4 * RANK], m[4 * RANK + 1], m[4 * RANK + 2], m[4 * RANK + 3]);
      // keep the matrices' passes apart (interleaving them only raises register pressure)
      __builtin_amdgcn_sched_barrier(0);
      reg_mat_group<T, R, MASK, B + 1, RANK + 1>(v, m);
    } else {
      reg_mat_group<T, R, MASK, B + 1, RANK>(v, m);
    }
  }
}

// Per-thread CZ signs without register-register flips: the CZs with register operands K1
// and K2 (K2 < 0: none) whose partners are thread or tile bits, with sign words s1, s2 of
// those bits. Which amplitudes a word applies to is fixed by K1 and K2, so only the flipped
// ones cost instructions (two XORs each).
template <typename T, int R, int K1, int K2>
__device__ __forceinline__ void zg_thread_flips(typename Cx<T>::type (&v)[1 << R], uint32_t s1, uint32_t s2) {
  const uint32_t s12 = s1 ^ s2;
#pragma unroll
  for (int j = 0; j < (1 << R); ++j) {
    const bool b1 = ((j >> K1) & 1) != 0, b2 = K2 >= 0 && ((j >> (K2 < 0 ? 0 : K2)) & 1) != 0;
    if (!b1 && !b2) continue;
    const uint32_t sg = b1 && b2 ? s12 : (b1 ? s1 : s2);
    v[j].x = flip_sign(v[j].x, sg);
    v[j].y = flip_sign(v[j].y, sg);
  }
}

template <typename T, int R>
__device__ __forceinline__ void apply_op(typename Cx<T>::type (&v)[1 << R], const DevOp op, uint32_t tp,
                                         const typename Cx<T>::type* __restrict__ M, int t, uint32_t tile) {
  using C = typename Cx<T>::type;
  {
    if constexpr (R <= 4) {
      if (op.kind == K_MATG) {
        const C* m = M + 4 * (int64_t)op.mat;
#define TQ_MATG_CASE(K) \
  case K:               \
    reg_mat_group<T, R, K>(v, m); \
    break;
        switch (op.rbit) {
          TQ_MATG_CASE(1) TQ_MATG_CASE(2) TQ_MATG_CASE(3) TQ_MATG_CASE(4) TQ_MATG_CASE(5)
          TQ_MATG_CASE(6) TQ_MATG_CASE(7) TQ_MATG_CASE(8) TQ_MATG_CASE(9) TQ_MATG_CASE(10)
          TQ_MATG_CASE(11) TQ_MATG_CASE(12) TQ_MATG_CASE(13) TQ_MATG_CASE(14)
          default: reg_mat_group<T, R, 15>(v, m); break;
        }
#undef TQ_MATG_CASE
        // the layer's register-register CZs as uniform sign flips
        const uint32_t fl = (uint32_t)op.pa | ((uint32_t)op.pb << 8);
        if (fl) {
#pragma unroll
          for (int j = 0; j < (1 << R); ++j)
            if ((fl >> j) & 1u) {
              v[j].x = flip_sign(v[j].x, 0x80000000u);
              v[j].y = flip_sign(v[j].y, 0x80000000u);
            }
        }
        return;
      }
      if (op.kind == K_ZG) {
        // sign flips: uniform ones from the register-register CZs, per-thread ones from up
        // to two CZs whose partner is a thread or tile bit
        const uint32_t uni = (uint32_t)op.mat;
        const int k1 = (op.rbit & 15) - 1, k2 = (op.rbit >> 4) - 1;
        if (k1 < 0) {
          if (uni == 0) return;  // an empty op (phases are padded to an even op count)
#pragma unroll
          for (int j = 0; j < (1 << R); ++j)
            if ((uni >> j) & 1u) {
              v[j].x = flip_sign(v[j].x, 0x80000000u);
              v[j].y = flip_sign(v[j].y, 0x80000000u);
            }
        } else if (uni == 0) {
          const uint32_t s1 = idx_bit(op.pa, tp, t, tile) << 31;
          const uint32_t s2 = k2 >= 0 ? idx_bit(op.pb, tp, t, tile) << 31 : 0u;
#define TQ_ZG_K(A, B) zg_thread_flips<T, R, (R > A ? A : R - 1), (R > B ? B : R - 1)>(v, s1, s2)
#define TQ_ZG_CASE(A)                                       \
  case A:                                                   \
    switch (k2) {                                           \
      case -1: zg_thread_flips<T, R, (R > A ? A : R - 1), -1>(v, s1, s2); break; \
      case 0: TQ_ZG_K(A, 0); break;                         \
      case 1: TQ_ZG_K(A, 1); break;                         \
      case 2: TQ_ZG_K(A, 2); break;                         \
      default: TQ_ZG_K(A, 3); break;                        \
    }                                                       \
    break;
          switch (k1) { TQ_ZG_CASE(0) TQ_ZG_CASE(1) TQ_ZG_CASE(2) default: switch (k2) {
              case -1: zg_thread_flips<T, R, (R > 3 ? 3 : R - 1), -1>(v, s1, s2); break;
              case 0: TQ_ZG_K(3, 0); break;
              case 1: TQ_ZG_K(3, 1); break;
              case 2: TQ_ZG_K(3, 2); break;
              default: TQ_ZG_K(3, 3); break;
            } }
#undef TQ_ZG_CASE
#undef TQ_ZG_K
        } else {
          // this thread's flip mask over j, then bit j moved to the sign position
          uint32_t f = uni;
          if (idx_bit(op.pa, tp, t, tile)) f ^= reg_mask(k1);
          if (k2 >= 0 && idx_bit(op.pb, tp, t, tile)) f ^= reg_mask(k2);
#pragma unroll
          for (int j = 0; j < (1 << R); ++j) {
            const uint32_t sg = (f << (31 - j)) & 0x80000000u;
            v[j].x = flip_sign(v[j].x, sg);
            v[j].y = flip_sign(v[j].y, sg);
          }
        }
        return;
      }
    }
    C m0{}, m1{}, m2{}, m3{};
    if (op.kind == K_MAT1 || op.kind == K_DIAG1 || op.kind == K_DIAG2) {
      const C* m = M + 4 * (int64_t)op.mat;
      m0 = m[0]; m1 = m[1]; m2 = m[2]; m3 = m[3];
    }
    if (op.kind == K_MAT1) {
      // every path applies the gate (register bits >= R never occur; they fall to the top
      // bit), so the tile is updated in place on all branches
#define TQ_MAT_CASE(B) \
  case B:              \
    reg_mat<T, R, (R > B ? B : R - 1)>(v, m0, m1, m2, m3); \
    break;
      switch (op.rbit) { TQ_MAT_CASE(0) TQ_MAT_CASE(1) TQ_MAT_CASE(2) TQ_MAT_CASE(3)
        default: reg_mat<T, R, (R > 4 ? 4 : R - 1)>(v, m0, m1, m2, m3); break; }
#undef TQ_MAT_CASE
    } else if (op.kind == K_CX) {
      const int kc = (int)op.pb - 1;
      const uint32_t cb = kc < 0 ? idx_bit(op.pa, tp, t, tile) : 1u;
      const uint32_t mc = reg_mask(kc);
#define TQ_CX_CASE(B) \
  case B:             \
    reg_cx<T, R, (R > B ? B : R - 1)>(v, mc, cb); \
    break;
      switch (op.rbit) { TQ_CX_CASE(0) TQ_CX_CASE(1) TQ_CX_CASE(2) TQ_CX_CASE(3)
        default: reg_cx<T, R, (R > 4 ? 4 : R - 1)>(v, mc, cb); break; }
#undef TQ_CX_CASE
    } else if (op.kind == K_CZ) {
      const int ka = (op.rbit & 15) - 1, kb = (op.rbit >> 4) - 1;
      uint32_t f = 1u;
      if (ka < 0) f &= idx_bit(op.pa, tp, t, tile);
      if (kb < 0) f &= idx_bit(op.pb, tp, t, tile);
      reg_cz<T, R>(v, reg_mask(ka) & reg_mask(kb), f << 31);
    } else {
      // diagonal on one (entries d[bit a]) or two qubits (entries d[2 bit a + bit b]); an
      // operand is a register bit (index ka / kb) or a thread or tile bit
      const C d0 = m0, d1 = m1, d2 = m2, d3 = m3;
      const bool two = op.kind == K_DIAG2;
      const int ka = (op.rbit & 15) - 1, kb = (op.rbit >> 4) - 1;
      const uint32_t xa = ka < 0 ? idx_bit(op.pa, tp, t, tile) : 0u;
      const uint32_t xb = (two && kb < 0) ? idx_bit(op.pb, tp, t, tile) : 0u;
#pragma unroll
      for (int j = 0; j < (1 << R); ++j) {
        const uint32_t ba = ka >= 0 ? (((uint32_t)j >> ka) & 1u) : xa;
        const uint32_t bb = !two ? ba : (kb >= 0 ? (((uint32_t)j >> kb) & 1u) : xb);
        C f;
        f.x = ba ? (two ? (bb ? d3.x : d2.x) : d1.x) : (two ? (bb ? d1.x : d0.x) : d0.x);
        f.y = ba ? (two ? (bb ? d3.y : d2.y) : d1.y) : (two ? (bb ? d1.y : d0.y) : d0.y);
        v[j] = cmul(f, v[j]);
      }
    }
  }
}

// A phase's ops in order. Forward schedules with grouped layers (R <= 4) pad every phase
// to an even op count, and the loop takes two ops per trip: the first op's results can then
// live in other registers than the loop-carried ones and the second op's results land back
// in them, instead of every trip ending with a copy of all amplitudes.
template <typename T, int R>
__device__ __forceinline__ void apply_phase_ops(typename Cx<T>::type (&v)[1 << R], uint32_t tp,
                                                const DevOp* __restrict__ ops, int ob, int oe,
                                                const typename Cx<T>::type* __restrict__ M, int t,
                                                uint32_t tile) {
  if constexpr (R <= 4) {
    for (int o = ob; o < oe; o += 2) {
      apply_op<T, R>(v, load_op(ops, o), tp, M, t, tile);
      apply_op<T, R>(v, load_op(ops, o + 1), tp, M, t, tile);
    }
  } else {
    for (int o = ob; o < oe; ++o) apply_op<T, R>(v, load_op(ops, o), tp, M, t, tile);
  }
}

// One stage over one tile. Threads with act == false (past the 2^(t-R) a tile of a smaller
// circuit needs, in a batched work-group sized for the largest) hold no amplitudes and only
// take part in the barriers. basis >= 0: the tile is not read but starts as that part of
// the basis state |basis> (1 at index basis, 0 elsewhere).
//
// LDS addresses: amplitude j of a thread sits at local index tp | rp_j (thread bits and
// register bits occupy disjoint positions). The swizzle is linear over XOR, so its byte
// address is swz(tp) ^ swz(rp_j): one per-thread term and one uniform term per register
// index, kept in scalar registers.
template <typename T, int R, bool kLoadPrio = true>
__device__ __forceinline__ void stage_tile(const DevStage* __restrict__ stg, const DevPhase* __restrict__ phases,
                                           const DevOp* __restrict__ ops,
                                           const typename Cx<T>::type* __restrict__ M,
                                           typename Cx<T>::type* __restrict__ st, uint32_t tile, uint32_t tid,
                                           bool act, typename Cx<T>::type* lds, int64_t basis) {
  using C = typename Cx<T>::type;
  constexpr uint32_t E = sizeof(C);
  const gword* const sw = reinterpret_cast<const gword*>(gptr(stg));
  const int t = (int)sw[0];
  const int tb = t - R;
  unsigned char* const lb = reinterpret_cast<unsigned char*>(lds);

  // global offsets of this thread's amplitudes in the load/store layout
  const int64_t off = stage_tile_base(sw, tile) | stage_thread_offset(sw, tb, tid);
  C* const sb = st + off;
  C v[1 << R];
  // One circuit's stage: the tile's loads are issued at raised wave priority. A work-group
  // that starts while the CU's other groups compute would otherwise wait for issue slots
  // behind them (issue goes to the oldest wave first) and stall on its loads later, with
  // nothing to overlap (2.5 % on the 24-qubit step; the exchanges below at priority 1 gave
  // another 2.6 %). The batched kernel's short groups of many circuits ran about 10 % slower
  // with raised load priority, so it keeps the default priority throughout.
  if constexpr (kLoadPrio) __builtin_amdgcn_s_setprio(2);
#pragma unroll
  for (int j = 0; j < (1 << R); ++j) {
    int64_t hi = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) hi |= (int64_t)((j >> k) & 1) << word_byte(sw, kStageLposWord, tb + k);
    if (!act) v[j] = C{(T)0, (T)0};
    else if (basis < 0) v[j] = sb[hi];
    else v[j] = C{(off | hi) == basis ? (T)1 : (T)0, (T)0};
  }

  if constexpr (kLoadPrio) __builtin_amdgcn_s_setprio(0);
  // load layout: thread bits are the low tb local bits, registers the top R
  uint32_t tp = tid & ((1u << tb) - 1u);
  uint32_t ta = lds_swz<T>(tp) * E;
  uint32_t ra[1 << R];
#pragma unroll
  for (int j = 0; j < (1 << R); ++j) ra[j] = lds_swz<T>((uint32_t)j << tb) * E;

  bool first_x = true;
  const int p_end = (int)sw[2];
  for (int p = (int)sw[1]; p < p_end; ++p) {
    const gword* const pw = reinterpret_cast<const gword*>(gptr(phases)) + (int64_t)p * kPhaseWords;
    if (pw[2]) {
      // an exchange at priority 1: the group's waves reach its barriers sooner, instead of
      // queueing for issue behind other groups' arithmetic while their partners wait
      if constexpr (kLoadPrio) __builtin_amdgcn_s_setprio(1);
      if (!first_x) __syncthreads();
      first_x = false;
      if (act)
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) *reinterpret_cast<C*>(lb + (ta ^ ra[j])) = v[j];
      tp = phase_thread_bits(pw, tb, tid);
      ta = lds_swz<T>(tp) * E;
#pragma unroll
      for (int j = 0; j < (1 << R); ++j) {
        uint32_t rp = 0;
#pragma unroll
        for (int k = 0; k < R; ++k) rp |= (uint32_t)((j >> k) & 1) << word_byte(pw, kPhaseRposWord, k);
        ra[j] = lds_swz<T>(rp) * E;
      }
      __syncthreads();
      if (act)
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) v[j] = *reinterpret_cast<const C*>(lb + (ta ^ ra[j]));
      if constexpr (kLoadPrio) __builtin_amdgcn_s_setprio(0);
    }
    apply_phase_ops<T, R>(v, tp, ops, (int)pw[0], (int)pw[1], M, t, tile);
  }
  if (sw[4]) {
    if (!first_x) __syncthreads();
    if (act)
#pragma unroll
      for (int j = 0; j < (1 << R); ++j) *reinterpret_cast<C*>(lb + (ta ^ ra[j])) = v[j];
    __syncthreads();
    const uint32_t ts = lds_swz<T>(tid & ((1u << tb) - 1u)) * E;
    if (act)
#pragma unroll
      for (int j = 0; j < (1 << R); ++j)
        v[j] = *reinterpret_cast<const C*>(lb + (ts ^ (lds_swz<T>((uint32_t)j << tb) * E)));
  }
  if (act) {
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
      int64_t hi = 0;
#pragma unroll
      for (int k = 0; k < R; ++k) hi |= (int64_t)((j >> k) & 1) << word_byte(sw, kStageLposWord, tb + k);
      sb[hi] = v[j];
    }
  }
}

// Waves per SIMD the stage kernel is compiled for. A complex64 tile of 2^12 amplitudes takes
// 32 KiB of LDS, so five work-groups fit a CU; with R = 4 that needs at most 96 registers,
// which the code meets without spilling. Other shapes leave the choice to the compiler.
template <typename T, int R>
constexpr int stage_waves() {
  return (sizeof(T) == 4 && R == 4) ? 5 : 1;
}

template <typename T, int R>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(stage_waves<T, R>()))) sv_stage_kernel(const DevStage* __restrict__ stg,
                                                        const DevPhase* __restrict__ phases,
                                                        const DevOp* __restrict__ ops,
                                                        const typename Cx<T>::type* __restrict__ mats,
                                                        int64_t mats_stride, typename Cx<T>::type* __restrict__ state,
                                                        BatchMap smap, int64_t basis) {
  using C = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  stage_tile<T, R>(stg, phases, ops, mats + (int64_t)blockIdx.y * mats_stride, state + smap.at(blockIdx.y),
                   blockIdx.x, threadIdx.x, true, reinterpret_cast<C*>(smem_raw), basis);
}

// The same kernel for the default tile of 2^12 amplitudes, its LDS declared with a fixed
// size. A dynamically sized LDS array starts at a link-time symbol, which the compiler adds
// to every LDS address (one extra instruction per access); a fixed array's base folds away.
constexpr int kStaticTileBits = 12;

template <typename T, int R>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(stage_waves<T, R>()))) sv_stage_kernel_t12(const DevStage* __restrict__ stg,
                                                            const DevPhase* __restrict__ phases,
                                                            const DevOp* __restrict__ ops,
                                                            const typename Cx<T>::type* __restrict__ mats,
                                                            int64_t mats_stride,
                                                            typename Cx<T>::type* __restrict__ state,
                                                            BatchMap smap, int64_t basis) {
  using C = typename Cx<T>::type;
  __shared__ __align__(16) C tile_lds[1 << kStaticTileBits];
  stage_tile<T, R>(stg, phases, ops, mats + (int64_t)blockIdx.y * mats_stride, state + smap.at(blockIdx.y),
                   blockIdx.x, threadIdx.x, true, tile_lds, basis);
}

// Heterogeneous batch, one stage level: work-group i runs items[i] (a tile of one circuit's
// stage `level`). The work-group is sized for the level's largest tile.
template <typename T, int R>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(stage_waves<T, R>()))) sv_batch_stage_kernel(const DevCirc* __restrict__ circs,
                                                              const BatchItem* __restrict__ items, int level,
                                                              const typename Cx<T>::type* __restrict__ mats,
                                                              typename Cx<T>::type* __restrict__ states) {
  using C = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint2 w = reinterpret_cast<const uint2*>(items)[blockIdx.x];
  const DevCirc& d = circs[(int)w.x];
  const DevStage* stg = d.stages + level;
  const bool act = threadIdx.x < (1u << ((int)reinterpret_cast<const gword*>(gptr(stg))[0] - R));
  stage_tile<T, R, false>(stg, d.phases, d.ops, mats + d.mats_off, states + d.state_off, w.y, threadIdx.x, act,
                          reinterpret_cast<C*>(smem_raw), -1);
}

// Basis-state initialisation |b> (Sec. 3.1 default |0..0> for b = 0): vector stores only,
// two complex64 amplitudes per 16-byte store where the state is 16-byte aligned (2^n is even).
template <typename T>
__global__ void __launch_bounds__(256) init_basis_kernel(typename Cx<T>::type* __restrict__ st, BatchMap smap,
                                                         int64_t namps, int64_t basis) {
  using C = typename Cx<T>::type;
  C* s = st + smap.at(blockIdx.y);
  if constexpr (sizeof(C) == 8) {
    if ((reinterpret_cast<uintptr_t>(s) & 15) == 0 && (namps & 1) == 0) {
      float4* s4 = reinterpret_cast<float4*>(s);
      for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < namps / 2;
           i += (int64_t)gridDim.x * blockDim.x) {
        float4 v;
        v.x = (2 * i == basis) ? 1.0f : 0.0f;
        v.y = 0.0f;
        v.z = (2 * i + 1 == basis) ? 1.0f : 0.0f;
        v.w = 0.0f;
        s4[i] = v;
      }
      return;
    }
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < namps; i += (int64_t)gridDim.x * blockDim.x) {
    C v;
    v.x = (i == basis) ? (T)1 : (T)0;
    v.y = (T)0;
    s[i] = v;
  }
}

// ---------------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------------
template <typename T>
tq_status launch_init_basis(void* d_states, BatchMap smap, int n, int count, int64_t basis, int n_cu,
                            hipStream_t stream) {
  using C = typename Cx<T>::type;
  const int64_t namps = int64_t(1) << n;
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int cn = std::min(65535, count - c0);
    int64_t b = (namps + 255) / 256;
    int64_t cap = std::max<int64_t>(1, (int64_t)n_cu * 16 / cn);
    if (b > cap) b = cap;
    hipLaunchKernelGGL(init_basis_kernel<T>, dim3((unsigned)b, cn), dim3(256), 0, stream, (C*)d_states,
                       smap.shifted(c0), namps, basis);
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}
template tq_status launch_init_basis<float>(void*, BatchMap, int, int, int64_t, int, hipStream_t);
template tq_status launch_init_basis<double>(void*, BatchMap, int, int, int64_t, int, hipStream_t);

template <typename T>
tq_status launch_gate_build(const Schedule& s, const void* d_params, BatchMap pmap, void* d_mats, int count,
                            hipStream_t stream) {
  const int n_mats = (int)s.recipes.size();
  if (n_mats == 0 || count == 0) return TQ_OK;
  const int64_t total = (int64_t)n_mats * count;
  const int threads = 128;
  const int64_t blocks = (total + threads - 1) / threads;
  hipLaunchKernelGGL(gate_build_kernel<T>, dim3((unsigned)blocks), dim3(threads), 0, stream,
                     (const tq_gate*)s.d_gates, (const int32_t*)s.d_rec, (const int32_t*)s.d_rec_gates, n_mats,
                     (const T*)d_params, pmap, (typename Cx<T>::type*)d_mats, count);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

static inline unsigned sweep_blocks(int64_t work, int n_cu) {
  int64_t b = (work + 255) / 256;
  int64_t cap = (int64_t)n_cu * 16;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

template <typename T>
tq_status launch_plain(const Schedule& s, void* d_states, BatchMap smap, const void* d_mats, int count,
                       int n_cu, hipStream_t stream) {
  using C = typename Cx<T>::type;
  const int n = s.n;
  const int64_t namps = int64_t(1) << n;
  const int64_t mstride = 4 * (int64_t)s.recipes.size();
  C* st = (C*)d_states;
  const C* M = (const C*)d_mats;
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int cn = std::min(65535, count - c0);
    BatchMap sm = smap.shifted(c0);
    const C* Mc = M + (int64_t)c0 * mstride;
    for (const HostOp& o : s.ops) {
      const int pa = n - 1 - o.qa;
      const int pb = o.qb >= 0 ? n - 1 - o.qb : -1;
      if (o.kind == K_MAT1) {
        hipLaunchKernelGGL(plain_mat1_kernel<T>, dim3(sweep_blocks(namps / 2, n_cu), cn), dim3(256), 0, stream,
                           st, sm, pa, namps / 2, Mc, mstride, o.mat);
      } else if (o.kind == K_CX) {
        // qa = target, qb = control
        hipLaunchKernelGGL(plain_cx_kernel<T>, dim3(sweep_blocks(namps / 4, n_cu), cn), dim3(256), 0, stream,
                           st, sm, pb, pa, namps / 4);
      } else if (o.kind == K_CZ) {
        hipLaunchKernelGGL(plain_cz_kernel<T>, dim3(sweep_blocks(namps / 4, n_cu), cn), dim3(256), 0, stream,
                           st, sm, pa, pb, namps / 4);
      } else {
        hipLaunchKernelGGL(plain_diag_kernel<T>, dim3(sweep_blocks(namps, n_cu), cn), dim3(256), 0, stream, st, sm,
                           pa, o.kind == K_DIAG2 ? pb : -1, namps, Mc, mstride, o.mat);
      }
      TQ_HIP(hipGetLastError());
    }
  }
  return TQ_OK;
}

template <typename T, int R>
static tq_status launch_stages_R(const Schedule& s, void* d_states, BatchMap smap, const void* d_mats, int count,
                                 int64_t basis, hipStream_t stream) {
  using C = typename Cx<T>::type;
  const int64_t mstride = 4 * (int64_t)s.recipes.size();
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int cn = std::min(65535, count - c0);
    BatchMap sm = smap.shifted(c0);
    const C* Mc = (const C*)d_mats + (int64_t)c0 * mstride;
    for (size_t k = 0; k < s.stages.size(); ++k) {
      const int t = s.stages[k].t;
      const unsigned tiles = 1u << (s.n - t);
      const unsigned threads = 1u << (t - R);
      const size_t lds = sizeof(C) << t;
      const int64_t b = k == 0 ? basis : -1;  // only the first stage starts from |basis>
      if (t == kStaticTileBits)
        hipLaunchKernelGGL((sv_stage_kernel_t12<T, R>), dim3(tiles, cn), dim3(threads), 0, stream,
                           (const DevStage*)s.d_stages + k, (const DevPhase*)s.d_phases, (const DevOp*)s.d_ops, Mc,
                           mstride, (C*)d_states, sm, b);
      else
        hipLaunchKernelGGL((sv_stage_kernel<T, R>), dim3(tiles, cn), dim3(threads), lds, stream,
                           (const DevStage*)s.d_stages + k, (const DevPhase*)s.d_phases, (const DevOp*)s.d_ops, Mc,
                           mstride, (C*)d_states, sm, b);
      TQ_HIP(hipGetLastError());
    }
  }
  return TQ_OK;
}

template <typename T>
tq_status launch_stages(const Schedule& s, void* d_states, BatchMap smap, const void* d_mats, int count,
                        int64_t basis, hipStream_t stream) {
  const int R = std::min(s.R, std::min(s.t, s.n));
  switch (R) {
    case 1: return launch_stages_R<T, 1>(s, d_states, smap, d_mats, count, basis, stream);
    case 2: return launch_stages_R<T, 2>(s, d_states, smap, d_mats, count, basis, stream);
    case 3: return launch_stages_R<T, 3>(s, d_states, smap, d_mats, count, basis, stream);
    case 4: return launch_stages_R<T, 4>(s, d_states, smap, d_mats, count, basis, stream);
    case 5: return launch_stages_R<T, 5>(s, d_states, smap, d_mats, count, basis, stream);
    default: return fail(TQ_ENOTSUP, "register bits must be 1..5");
  }
}

template tq_status launch_gate_build<float>(const Schedule&, const void*, BatchMap, void*, int, hipStream_t);
template tq_status launch_gate_build<double>(const Schedule&, const void*, BatchMap, void*, int, hipStream_t);
template tq_status launch_plain<float>(const Schedule&, void*, BatchMap, const void*, int, int, hipStream_t);
template tq_status launch_plain<double>(const Schedule&, void*, BatchMap, const void*, int, int, hipStream_t);
template tq_status launch_stages<float>(const Schedule&, void*, BatchMap, const void*, int, int64_t, hipStream_t);
template tq_status launch_stages<double>(const Schedule&, void*, BatchMap, const void*, int, int64_t, hipStream_t);

// ---- heterogeneous batch ---------------------------------------------------------------
template <typename T, int R>
static tq_status launch_batch_stages_R(const BatchLaunch& b, const void* d_mats, void* d_states,
                                       hipStream_t stream) {
  using C = typename Cx<T>::type;
  for (size_t L = 0; L + 1 < b.level_begin.size(); ++L) {
    const int64_t items = b.level_begin[L + 1] - b.level_begin[L];
    if (items == 0) continue;
    const int t = b.level_t[L];
    hipLaunchKernelGGL((sv_batch_stage_kernel<T, R>), dim3((unsigned)items), dim3(1u << (t - R)), sizeof(C) << t,
                       stream, b.d_circ, b.d_items + b.level_begin[L], (int)L, (const C*)d_mats, (C*)d_states);
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}

template <typename T>
tq_status launch_batch_forward(const BatchLaunch& b, const void* d_params, void* d_mats, void* d_states,
                               hipStream_t stream) {
  using C = typename Cx<T>::type;
  if (b.total_mats > 0) {
    hipLaunchKernelGGL(batch_gate_build_kernel<T>, dim3((unsigned)((b.total_mats + 127) / 128)), dim3(128), 0,
                       stream, b.d_circ, b.d_pref, b.count, (const T*)d_params, (C*)d_mats);
    TQ_HIP(hipGetLastError());
  }
  switch (b.R) {
    case 1: return launch_batch_stages_R<T, 1>(b, d_mats, d_states, stream);
    case 2: return launch_batch_stages_R<T, 2>(b, d_mats, d_states, stream);
    case 3: return launch_batch_stages_R<T, 3>(b, d_mats, d_states, stream);
    case 4: return launch_batch_stages_R<T, 4>(b, d_mats, d_states, stream);
    case 5: return launch_batch_stages_R<T, 5>(b, d_mats, d_states, stream);
    default: return fail(TQ_ENOTSUP, "register bits must be 1..5");
  }
}
template tq_status launch_batch_forward<float>(const BatchLaunch&, const void*, void*, void*, hipStream_t);
template tq_status launch_batch_forward<double>(const BatchLaunch&, const void*, void*, void*, hipStream_t);

}  // namespace tq
