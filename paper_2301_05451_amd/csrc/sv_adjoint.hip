// Adjoint (reverse-sweep) gradients of Z-string expectation values.
//
// For f = <psi_N| O |psi_N> with psi_k = U_k psi_{k-1}, the derivative with respect to an
// angle a of gate k is 2 Re <lambda_k| dU_k/da |psi_{k-1}>, where lambda_k =
// U_{k+1}^dag .. U_N^dag O psi_N. One reverse pass produces every such term: starting from
// lambda = O psi_N, for k = N..1: psi <- U_k^dag psi, record 2 Re <lambda| dU_k psi>,
// lambda <- U_k^dag lambda. These are the exact derivatives, equal to the parameter-shift
// values of the paper's Sec. 4.2; the paper itself obtains them by library backpropagation
// (Sec. 4.1), which stores every intermediate state instead of two.
//
// The reverse gate list is scheduled into LDS-tile stages exactly like the forward pass
// (one op per original gate). Each stage keeps tiles of psi and lambda in registers/LDS,
// and every angle gets a "slot": per-thread partial inner products are wave-reduced into
// LDS and written once per tile; a final pass sums tiles and parameter occurrences in a
// fixed order (deterministic).
#include "sv_device.h"

namespace tq {

template <typename T>
__global__ void adj_gate_build_kernel(const tq_gate* __restrict__ gates, int n_gates, const int32_t* __restrict__ runs,
                                      const T* __restrict__ params, BatchMap pmap,
                                      typename Cx<T>::type* __restrict__ mats, int count) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)n_gates * count) return;
  const int k = (int)(gid % n_gates);
  const int circ = (int)(gid / n_gates);
  dcx m[kAdjMatStride];
  if (!adj_entry(gates, n_gates, runs, k, params + pmap.at(circ), m)) return;
  typename Cx<T>::type* out = mats + ((int64_t)circ * n_gates + k) * kAdjMatStride;
  for (int i = 0; i < kAdjMatStride; ++i) out[i] = to_cx<T>(m[i]);
}

// lambda = sum_o w_o O_o psi with w = grad_out; psi copied to the working buffer.
template <typename T>
__global__ void __launch_bounds__(256)
    adj_init_kernel(const typename Cx<T>::type* __restrict__ psi_in, BatchMap smap_in,
                    typename Cx<T>::type* __restrict__ psi, typename Cx<T>::type* __restrict__ lam, BatchMap smap_w,
                    int64_t namps, const uint64_t* __restrict__ pmask, const double* __restrict__ coeff,
                    const int32_t* __restrict__ obs, int n_terms, const T* __restrict__ grad_out, int n_obs) {
  using C = typename Cx<T>::type;
  const int circ = blockIdx.y;
  const C* src = psi_in + smap_in.at(circ);
  C* p = psi + smap_w.at(circ);
  C* l = lam + smap_w.at(circ);
  const T* w = grad_out + (int64_t)circ * n_obs;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < namps; i += (int64_t)gridDim.x * blockDim.x) {
    double sgn = 0.0;
    for (int k = 0; k < n_terms; ++k) {
      const double wc = (double)w[obs[k]] * coeff[k];
      sgn += (__popcll((uint64_t)i & pmask[k]) & 1) ? -wc : wc;
    }
    const C a = src[i];
    p[i] = a;
    C b;
    b.x = (T)(sgn * (double)a.x);
    b.y = (T)(sgn * (double)a.y);
    l[i] = b;
  }
}

// lambda = sum_k w_{obs_k} coeff_k P_k psi for Pauli strings with X / Y factors, with
// (P psi)_x = i^nY (-1)^{|(x ^ f) & m|} psi_{x ^ f} (f = flip mask, m = sign mask over bit
// positions, nY = number of Y factors, all per term); psi copied to the working buffer.

template <typename T>
__global__ void __launch_bounds__(256)
    adj_init_pauli_kernel(const typename Cx<T>::type* __restrict__ psi_in, BatchMap smap_in,
                          typename Cx<T>::type* __restrict__ psi, typename Cx<T>::type* __restrict__ lam,
                          BatchMap smap_w, int64_t namps, AdjPauli P, const T* __restrict__ grad_out, int n_obs) {
  using C = typename Cx<T>::type;
  const int circ = blockIdx.y;
  const C* src = psi_in + smap_in.at(circ);
  C* p = psi + smap_w.at(circ);
  C* l = lam + smap_w.at(circ);
  const T* w = grad_out + (int64_t)circ * n_obs;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < namps; i += (int64_t)gridDim.x * blockDim.x) {
    double lr = 0.0, li = 0.0;
    for (int k = 0; k < P.n; ++k) {
      const uint64_t y = (uint64_t)i ^ P.f[k];
      const C a = src[y];
      double s = (double)w[P.ob[k]] * P.c[k];
      if (__popcll(y & P.m[k]) & 1) s = -s;
      // multiply a by s * i^cls
      const double ar = (double)a.x, ai = (double)a.y;
      switch (P.cls[k]) {
        case 0: lr += s * ar; li += s * ai; break;
        case 1: lr -= s * ai; li += s * ar; break;
        case 2: lr -= s * ar; li -= s * ai; break;
        default: lr += s * ai; li -= s * ar; break;
      }
    }
    p[i] = src[i];
    C b;
    b.x = (T)lr;
    b.y = (T)li;
    l[i] = b;
  }
}

template <typename T>
__device__ __forceinline__ uint32_t adj_swz(uint32_t li) {
  constexpr int G = sizeof(T) == 4 ? 5 : 4;
  constexpr uint32_t mask = (1u << G) - 1;
  return li ^ (((li >> G) ^ (li >> (2 * G)) ^ (li >> (3 * G))) & mask);
}

template <typename C>
__device__ __forceinline__ C cconj_mul(C a, C b) {  // conj(a) * b
  C r;
  r.x = a.x * b.x + a.y * b.y;
  r.y = a.x * b.y - a.y * b.x;
  return r;
}

// Re(conj(x) * y)
template <typename C>
__device__ __forceinline__ auto re_dot(C x, C y) -> decltype(x.x) {
  return x.x * y.x + x.y * y.y;
}

// Sum over the active lanes of a wave; `active` lanes (a power of two, or 64) are 0..active-1.
// Lanes past `active` (a work-group smaller than one wave) hold stale registers and are
// masked out of every butterfly step.
template <typename T>
__device__ __forceinline__ T wave_sum(T v, int lane, int active) {
  for (int off = 32; off > 0; off >>= 1) {
    const T o = __shfl_xor(v, off, 64);
    v += ((lane ^ off) < active) ? o : (T)0;
  }
  return v;
}

// v + (v moved across lanes by the data-parallel-primitive control CTRL); rows outside
// ROWS receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}

// Sum over all 64 lanes of a full wave without the LDS crossbar: pair sums within quads,
// mirrors within half-rows and rows, then row broadcasts; lane 63 holds the total, which
// is returned to every lane.
__device__ __forceinline__ float wave_sum_full(float v) {
  v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);  // row_mirror
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// conj(x) * y accumulated into acc
template <typename C>
__device__ __forceinline__ void cconj_fma(C& acc, C x, C y) {
  acc.x += x.x * y.x + x.y * y.y;
  acc.y += x.x * y.y - x.y * y.x;
}

// One register-resident target bit B: psi <- U^dag psi, lam <- U^dag lam, and the gradient
// terms Re <lam| dU_q psi> for the gate's angles q. Per thread, M[r][c] = sum over its pairs
// of conj(lam_r) psi_c (psi after U^dag, lam before it) is accumulated once; each angle's term
// is then Re sum_rc dU_q[r][c] M[r][c] (the derivative matrices never touch the amplitudes).
template <typename T, int R, int B>
__device__ __forceinline__ void adj_mat(typename Cx<T>::type (&vp)[1 << R], typename Cx<T>::type (&vl)[1 << R],
                                        const typename Cx<T>::type* __restrict__ m, int na, T (&acc)[3]) {
  using C = typename Cx<T>::type;
  const C u00 = m[0], u01 = m[1], u10 = m[2], u11 = m[3];
  // U^dag = [[conj u00, conj u10], [conj u01, conj u11]]
  C h00{u00.x, -u00.y}, h01{u10.x, -u10.y}, h10{u01.x, -u01.y}, h11{u11.x, -u11.y};
  C M00{(T)0, (T)0}, M01{(T)0, (T)0}, M10{(T)0, (T)0}, M11{(T)0, (T)0};
#pragma unroll
  for (int j = 0; j < (1 << R); ++j) {
    if (j & (1 << B)) continue;
    const int j1 = j | (1 << B);
    const C a = cfma2(h00, vp[j], h01, vp[j1]);
    const C b = cfma2(h10, vp[j], h11, vp[j1]);
    vp[j] = a;
    vp[j1] = b;
    const C la = vl[j], lb = vl[j1];
    if (na > 0) {
      cconj_fma(M00, la, a);
      cconj_fma(M01, la, b);
      cconj_fma(M10, lb, a);
      cconj_fma(M11, lb, b);
    }
    vl[j] = cfma2(h00, la, h01, lb);
    vl[j1] = cfma2(h10, la, h11, lb);
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (q < na) {
      const C* d = m + 4 + 4 * q;
      acc[q] += re_dot(C{d[0].x, -d[0].y}, M00) + re_dot(C{d[1].x, -d[1].y}, M01) +
                re_dot(C{d[2].x, -d[2].y}, M10) + re_dot(C{d[3].x, -d[3].y}, M11);
    }
  }
}

// CX with the target on register bit B on both tiles: pairs with (mc >> j) & 1 swap where cb.
template <typename T, int R, int B>
__device__ __forceinline__ void adj_cx(typename Cx<T>::type (&vp)[1 << R], typename Cx<T>::type (&vl)[1 << R],
                                       uint32_t mc, uint32_t cb) {
#pragma unroll
  for (int j = 0; j < (1 << R); ++j) {
    if (j & (1 << B)) continue;
    const int j1 = j | (1 << B);
    if ((mc >> j) & 1u) {
      auto a = vp[j], b = vp[j1];
      vp[j].x = cb ? b.x : a.x;
      vp[j].y = cb ? b.y : a.y;
      vp[j1].x = cb ? a.x : b.x;
      vp[j1].y = cb ? a.y : b.y;
      a = vl[j];
      b = vl[j1];
      vl[j].x = cb ? b.x : a.x;
      vl[j].y = cb ? b.y : a.y;
      vl[j1].x = cb ? a.x : b.x;
      vl[j1].y = cb ? a.y : b.y;
    }
  }
}

__device__ __forceinline__ uint32_t adj_reg_mask(int k) {
  return k == 0 ? 0xAAAAAAAAu
       : k == 1 ? 0xCCCCCCCCu
       : k == 2 ? 0xF0F0F0F0u
       : k == 3 ? 0xFF00FF00u
       : k == 4 ? 0xFFFF0000u
                : 0xFFFFFFFFu;
}
__device__ __forceinline__ uint32_t adj_idx_bit(int pos, uint32_t tp, int t, uint32_t tile) {
  return pos < t ? ((tp >> pos) & 1u) : ((tile >> (pos - t)) & 1u);
}
__device__ __forceinline__ float adj_flip(float x, uint32_t s) { return __uint_as_float(__float_as_uint(x) ^ s); }
__device__ __forceinline__ double adj_flip(double x, uint32_t s) {
  return __longlong_as_double(__double_as_longlong(x) ^ ((long long)s << 32));
}

// One reverse stage over one tile of psi and lambda. `nact` threads (a power of two) hold
// amplitudes; the rest of a larger batched work-group only joins the barriers. Partial
// inner products of the stage's slots go to part[(slot0 + s) * ntiles + tile].
template <typename T, int R>
__device__ __forceinline__ void adj_tile(const DevStage* __restrict__ stg, const DevPhase* __restrict__ phases,
                                         const DevOp* __restrict__ ops, const int32_t* __restrict__ dslot,
                                         const typename Cx<T>::type* __restrict__ M,
                                         typename Cx<T>::type* __restrict__ sp, typename Cx<T>::type* __restrict__ sl,
                                         uint32_t tile, uint32_t tid, int nact, int slot0, int nslot, int64_t ntiles,
                                         double* __restrict__ part, unsigned char* smem_raw) {
  using C = typename Cx<T>::type;
  constexpr uint32_t E = sizeof(C);
  const gword* const sw = reinterpret_cast<const gword*>(gptr(stg));
  const int t = (int)sw[0];
  const int tb = t - R;
  // LDS: psi tile, lambda tile, then the per-wave partial sums. Amplitude j of a thread sits
  // at local index tp | rp_j; the swizzle is linear over XOR, so its byte offset is
  // swz(tp) ^ swz(rp_j) (a per-thread term and a uniform one per register index).
  unsigned char* const lbp = smem_raw;
  unsigned char* const lbl = smem_raw + ((size_t)E << t);
  T* red = reinterpret_cast<T*>(smem_raw + 2 * ((size_t)E << t));  // [nslot][waves]
  const int nwaves = (nact + 63) >> 6;
  const int lane = tid & 63, wv = tid >> 6;
  const int active = nact < 64 ? nact : 64;
  const bool act = (int)tid < nact;

  const int64_t off = stage_tile_base(sw, tile) | stage_thread_offset(sw, tb, tid);
  C vp[1 << R], vl[1 << R];
#pragma unroll
  for (int j = 0; j < (1 << R); ++j) {
    int64_t hi = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) hi |= (int64_t)((j >> k) & 1) << word_byte(sw, kStageLposWord, tb + k);
    if (act) {
      vp[j] = sp[off + hi];
      vl[j] = sl[off + hi];
    } else {
      vp[j] = C{(T)0, (T)0};
      vl[j] = C{(T)0, (T)0};
    }
  }
  uint32_t tp = tid & ((1u << tb) - 1u);  // this thread's own bits at their local positions
  uint32_t ta = adj_swz<T>(tp) * E;
  uint32_t ra[1 << R];
#pragma unroll
  for (int j = 0; j < (1 << R); ++j) ra[j] = adj_swz<T>((uint32_t)j << tb) * E;

  const int p_end = (int)sw[2];
  for (int p = (int)sw[1]; p < p_end; ++p) {
    const gword* const pw = reinterpret_cast<const gword*>(gptr(phases)) + (int64_t)p * kPhaseWords;
    if (pw[2]) {
      __syncthreads();
      if (act)
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) {
          *reinterpret_cast<C*>(lbp + (ta ^ ra[j])) = vp[j];
          *reinterpret_cast<C*>(lbl + (ta ^ ra[j])) = vl[j];
        }
      tp = phase_thread_bits(pw, tb, tid);
      ta = adj_swz<T>(tp) * E;
#pragma unroll
      for (int j = 0; j < (1 << R); ++j) {
        uint32_t rp = 0;
#pragma unroll
        for (int k = 0; k < R; ++k) rp |= (uint32_t)((j >> k) & 1) << word_byte(pw, kPhaseRposWord, k);
        ra[j] = adj_swz<T>(rp) * E;
      }
      __syncthreads();
      if (act)
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) {
          vp[j] = *reinterpret_cast<const C*>(lbp + (ta ^ ra[j]));
          vl[j] = *reinterpret_cast<const C*>(lbl + (ta ^ ra[j]));
        }
    }
    const int o_end = (int)pw[1];
    // one op of the phase; two per loop trip, so that the loop-carried amplitudes need no
    // register copies at the end of every trip
    auto do_op = [&](int o) {
      const DevOp op = load_op(ops, o);
      const int sl_info = gptr(dslot)[o];
      const int na = sl_info & 3, s0 = sl_info >> 2;
      const C* m = M + (int64_t)op.mat * kAdjMatStride;
      T acc[3] = {(T)0, (T)0, (T)0};
      if (op.kind == K_MAT1) {
#define TQ_ADJ_CASE(B) \
  case B:              \
    adj_mat<T, R, (R > B ? B : R - 1)>(vp, vl, m, na, acc); \
    break;
        switch (op.rbit) { TQ_ADJ_CASE(0) TQ_ADJ_CASE(1) TQ_ADJ_CASE(2) TQ_ADJ_CASE(3)
          default: adj_mat<T, R, (R > 4 ? 4 : R - 1)>(vp, vl, m, na, acc); break; }
#undef TQ_ADJ_CASE
      } else if (op.kind == K_CX) {
        const int kc = (int)op.pb - 1;  // control's register index, or -1
        const uint32_t cb = kc < 0 ? adj_idx_bit(op.pa, tp, t, tile) : 1u;
        const uint32_t mc = adj_reg_mask(kc);
#define TQ_ADJX_CASE(B) \
  case B:               \
    adj_cx<T, R, (R > B ? B : R - 1)>(vp, vl, mc, cb); \
    break;
        switch (op.rbit) { TQ_ADJX_CASE(0) TQ_ADJX_CASE(1) TQ_ADJX_CASE(2) TQ_ADJX_CASE(3)
          default: adj_cx<T, R, (R > 4 ? 4 : R - 1)>(vp, vl, mc, cb); break; }
#undef TQ_ADJX_CASE
      } else if (op.kind == K_CZ) {
        const int ka = (op.rbit & 15) - 1, kb = (op.rbit >> 4) - 1;
        uint32_t f = 1u;
        if (ka < 0) f &= adj_idx_bit(op.pa, tp, t, tile);
        if (kb < 0) f &= adj_idx_bit(op.pb, tp, t, tile);
        const uint32_t msk = adj_reg_mask(ka) & adj_reg_mask(kb), sg = f << 31;
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) {
          if ((msk >> j) & 1u) {
            vp[j].x = adj_flip(vp[j].x, sg); vp[j].y = adj_flip(vp[j].y, sg);
            vl[j].x = adj_flip(vl[j].x, sg); vl[j].y = adj_flip(vl[j].y, sg);
          }
        }
      } else {
        const bool two = op.kind == K_DIAG2;
        const C d0 = m[0], d1 = m[1], d2 = m[2], d3 = m[3];
        const C e0 = m[4], e1 = m[5], e2 = m[6], e3 = m[7];
        // an operand is a register bit (index ka / kb) or a thread or tile bit
        const int ka = (op.rbit & 15) - 1, kb = (op.rbit >> 4) - 1;
        const uint32_t xa = ka < 0 ? adj_idx_bit(op.pa, tp, t, tile) : 0u;
        const uint32_t xb = (two && kb < 0) ? adj_idx_bit(op.pb, tp, t, tile) : 0u;
#pragma unroll
        for (int j = 0; j < (1 << R); ++j) {
          const uint32_t ba = ka >= 0 ? (((uint32_t)j >> ka) & 1u) : xa;
          const uint32_t bb = !two ? ba : (kb >= 0 ? (((uint32_t)j >> kb) & 1u) : xb);
          C f, g;
          f.x = ba ? (two ? (bb ? d3.x : d2.x) : d1.x) : (two ? (bb ? d1.x : d0.x) : d0.x);
          f.y = ba ? (two ? (bb ? d3.y : d2.y) : d1.y) : (two ? (bb ? d1.y : d0.y) : d0.y);
          g.x = ba ? (two ? (bb ? e3.x : e2.x) : e1.x) : (two ? (bb ? e1.x : e0.x) : e0.x);
          g.y = ba ? (two ? (bb ? e3.y : e2.y) : e1.y) : (two ? (bb ? e1.y : e0.y) : e0.y);
          const C a = cconj_mul(f, vp[j]);  // psi <- conj(d) psi
          vp[j] = a;
          if (na > 0) acc[0] += re_dot(vl[j], cmul(g, a));
          vl[j] = cconj_mul(f, vl[j]);
        }
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (q < na) {
          T s;
          if constexpr (sizeof(T) == 4) s = active == 64 ? wave_sum_full(acc[q]) : wave_sum<T>(acc[q], lane, active);
          else s = wave_sum<T>(acc[q], lane, active);
          if (lane == 0 && wv < nwaves) red[(s0 + q) * nwaves + wv] = s;
        }
      }
    };
    for (int o = (int)pw[0]; o < o_end; o += 2) {
      do_op(o);
      if (o + 1 < o_end) do_op(o + 1);
    }
  }
  // store both tiles in the load layout
  if (sw[4]) {
    __syncthreads();
    if (act)
#pragma unroll
      for (int j = 0; j < (1 << R); ++j) {
        *reinterpret_cast<C*>(lbp + (ta ^ ra[j])) = vp[j];
        *reinterpret_cast<C*>(lbl + (ta ^ ra[j])) = vl[j];
      }
    __syncthreads();
    const uint32_t ts = adj_swz<T>(tid & ((1u << tb) - 1u)) * E;
    if (act)
#pragma unroll
      for (int j = 0; j < (1 << R); ++j) {
        const uint32_t a0 = ts ^ (adj_swz<T>((uint32_t)j << tb) * E);
        vp[j] = *reinterpret_cast<const C*>(lbp + a0);
        vl[j] = *reinterpret_cast<const C*>(lbl + a0);
      }
  }
  if (act)
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) {
      int64_t hi = 0;
#pragma unroll
      for (int k = 0; k < R; ++k) hi |= (int64_t)((j >> k) & 1) << word_byte(sw, kStageLposWord, tb + k);
      sp[off + hi] = vp[j];
      sl[off + hi] = vl[j];
    }
  __syncthreads();
  if (act)
    for (int s = tid; s < nslot; s += nact) {
      double x = 0.0;
      for (int w = 0; w < nwaves; ++w) x += (double)red[s * nwaves + w];
      part[(int64_t)(slot0 + s) * ntiles + tile] = x;
    }
}

template <typename T, int R>
__global__ void __launch_bounds__(512)
    adj_stage_kernel(const DevStage* __restrict__ stg, const DevPhase* __restrict__ phases,
                     const DevOp* __restrict__ ops, const int32_t* __restrict__ dslot,
                     const typename Cx<T>::type* __restrict__ mats, int64_t mats_stride,
                     typename Cx<T>::type* __restrict__ psi, typename Cx<T>::type* __restrict__ lam, BatchMap smap,
                     int slot0, int nslot, int n_slots, double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t ntiles = gridDim.x;
  adj_tile<T, R>(stg, phases, ops, dslot, mats + (int64_t)blockIdx.y * mats_stride, psi + smap.at(blockIdx.y),
                 lam + smap.at(blockIdx.y), blockIdx.x, threadIdx.x, (int)blockDim.x, slot0, nslot, ntiles,
                 partial + (int64_t)blockIdx.y * n_slots * ntiles, smem_raw);
}

// Heterogeneous batch, one reverse-stage level: work-group i runs items[i]. The circuit's
// per-stage (first slot, slot count) pairs sit in its `rec` table.
template <typename T, int R>
__global__ void __launch_bounds__(512)
    adj_batch_stage_kernel(const DevCirc* __restrict__ circs, const BatchItem* __restrict__ items, int level,
                           const typename Cx<T>::type* __restrict__ mats, typename Cx<T>::type* __restrict__ psi,
                           typename Cx<T>::type* __restrict__ lam, double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint2 w = reinterpret_cast<const uint2*>(items)[blockIdx.x];
  const DevCirc& d = circs[(int)w.x];
  const DevStage* stg = d.stages + level;
  const gword* const rw = reinterpret_cast<const gword*>(gptr(d.rec)) + 2 * level;
  const int slot0 = (int)rw[0], nslot = (int)rw[1];
  const int t = (int)reinterpret_cast<const gword*>(gptr(stg))[0];
  adj_tile<T, R>(stg, d.phases, d.ops, d.dslot, mats + d.mats_off, psi + d.work_off, lam + d.work_off, w.y,
                 threadIdx.x, 1 << (t - R), slot0, nslot, int64_t(1) << (d.n - t), partial + d.part_off, smem_raw);
}

// grad[p] = sum over occurrences s of p: pscale_s * 2 * sum_tiles partial[s][tile] (fixed order)
template <typename T>
__global__ void adj_final_kernel(const double* __restrict__ partial, int n_slots, int64_t ntiles,
                                 const int32_t* __restrict__ pptr, const int32_t* __restrict__ pidx,
                                 const double* __restrict__ pscale, int n_used, int n_params, T* __restrict__ grad,
                                 BatchMap pmap, int count) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)n_params * count) return;
  const int p = (int)(gid % n_params);
  const int circ = (int)(gid / n_params);
  double g = 0.0;
  if (p < n_used) {
    const double* part = partial + (int64_t)circ * n_slots * ntiles;
    for (int e = pptr[p]; e < pptr[p + 1]; ++e) {
      double x = 0.0;
      const double* row = part + (int64_t)pidx[e] * ntiles;
      for (int64_t tl = 0; tl < ntiles; ++tl) x += row[tl];
      g += 2.0 * pscale[e] * x;
    }
  }
  grad[pmap.at(circ) + p] = (T)g;
}

// ---- host launchers --------------------------------------------------------------------
template <typename T, int R>
static tq_status launch_adj_stages_R(const Schedule& s, void* psi, void* lam, BatchMap smap, const void* mats,
                                     int count, double* partial, hipStream_t stream) {
  using C = typename Cx<T>::type;
  const int64_t mstride = (int64_t)s.n_gates * kAdjMatStride;
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int cn = std::min(65535, count - c0);
    for (size_t k = 0; k < s.stages.size(); ++k) {
      const int t = s.stages[k].t;
      const unsigned tiles = 1u << (s.n - t);
      const unsigned threads = 1u << (t - R);
      const unsigned waves = (threads + 63) / 64;
      const size_t lds = 2 * (sizeof(C) << t) + (size_t)std::max(1, s.stage_nslot[k]) * waves * sizeof(T);
      double* part = partial + (int64_t)c0 * s.n_slots * tiles;
      hipLaunchKernelGGL((adj_stage_kernel<T, R>), dim3(tiles, cn), dim3(threads), lds, stream,
                         (const DevStage*)s.d_stages + k, (const DevPhase*)s.d_phases, (const DevOp*)s.d_ops,
                         (const int32_t*)s.d_dslot, (const C*)mats + (int64_t)c0 * mstride, mstride, (C*)psi,
                         (C*)lam, smap.shifted(c0), s.stage_slot0[k], s.stage_nslot[k], s.n_slots, part);
      TQ_HIP(hipGetLastError());
    }
  }
  return TQ_OK;
}

template <typename T>
tq_status launch_adjoint(const Schedule& s, const void* d_params, BatchMap pmap, const void* d_states_in,
                         BatchMap smap_in, void* psi, void* lam, BatchMap smap_w, void* mats, double* partial,
                         const uint64_t* pm, const double* cf, const int32_t* ob, int n_terms, const T* grad_out,
                         int n_obs, T* grad, int n_params, int count, hipStream_t stream, const AdjPauli* pauli) {
  using C = typename Cx<T>::type;
  const int n = s.n;
  const int64_t namps = int64_t(1) << n;
  // matrices and derivatives of every gate
  if (s.n_gates > 0) {
    const int64_t total = (int64_t)s.n_gates * count;
    hipLaunchKernelGGL(adj_gate_build_kernel<T>, dim3((unsigned)((total + 127) / 128)), dim3(128), 0, stream,
                       (const tq_gate*)s.d_gates, s.n_gates, (const int32_t*)s.d_adj_runs, (const T*)d_params, pmap,
                       (C*)mats, count);
    TQ_HIP(hipGetLastError());
  }
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int cn = std::min(65535, count - c0);
    int64_t b = (namps + 255) / 256;
    b = std::min<int64_t>(b, std::max<int64_t>(1, 4096 / cn));
    if (pauli)
      hipLaunchKernelGGL(adj_init_pauli_kernel<T>, dim3((unsigned)b, cn), dim3(256), 0, stream, (const C*)d_states_in,
                         smap_in.shifted(c0), (C*)psi, (C*)lam, smap_w.shifted(c0), namps, *pauli,
                         grad_out + (int64_t)c0 * n_obs, n_obs);
    else
      hipLaunchKernelGGL(adj_init_kernel<T>, dim3((unsigned)b, cn), dim3(256), 0, stream, (const C*)d_states_in,
                         smap_in.shifted(c0), (C*)psi, (C*)lam, smap_w.shifted(c0), namps, pm, cf, ob, n_terms,
                         grad_out + (int64_t)c0 * n_obs, n_obs);
    TQ_HIP(hipGetLastError());
  }
  const int R = std::min(s.R, std::min(s.t, s.n));
  tq_status st;
  switch (R) {
    case 1: st = launch_adj_stages_R<T, 1>(s, psi, lam, smap_w, mats, count, partial, stream); break;
    case 2: st = launch_adj_stages_R<T, 2>(s, psi, lam, smap_w, mats, count, partial, stream); break;
    case 3: st = launch_adj_stages_R<T, 3>(s, psi, lam, smap_w, mats, count, partial, stream); break;
    case 4: st = launch_adj_stages_R<T, 4>(s, psi, lam, smap_w, mats, count, partial, stream); break;
    default: return fail(TQ_ENOTSUP, "adjoint register bits must be 1..4");
  }
  TQ_TRY(st);
  const int64_t ntiles = s.stages.empty() ? 1 : (int64_t(1) << (s.n - s.stages[0].t));
  const int64_t tot = (int64_t)n_params * count;
  if (tot > 0) {
    hipLaunchKernelGGL(adj_final_kernel<T>, dim3((unsigned)((tot + 127) / 128)), dim3(128), 0, stream,
                       (const double*)partial, s.n_slots, ntiles, (const int32_t*)s.d_pslot_ptr,
                       (const int32_t*)s.d_pslot_idx, (const double*)s.d_pslot_scale, s.n_params_used, n_params,
                       grad, pmap, count);
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}

// ---- heterogeneous batch ---------------------------------------------------------------
template <typename T>
__global__ void adj_batch_gate_build_kernel(const DevCirc* __restrict__ circs, const int64_t* __restrict__ pref,
                                            int count, const T* __restrict__ params,
                                            typename Cx<T>::type* __restrict__ mats) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= pref[count]) return;
  const int c = find_circ(pref, count, gid);
  const DevCirc& d = circs[c];
  const int k = (int)(gid - pref[c]);
  dcx m[kAdjMatStride];
  if (!adj_entry(d.gates, d.n_mats, d.rec_gates, k, params + d.param_off, m)) return;
  typename Cx<T>::type* out = mats + d.mats_off + (int64_t)k * kAdjMatStride;
  for (int i = 0; i < kAdjMatStride; ++i) out[i] = to_cx<T>(m[i]);
}

// y = circuit; lambda = sum_o w_o O_o psi with the circuit's own term table.
template <typename T>
__global__ void __launch_bounds__(256)
    adj_batch_init_kernel(const DevCirc* __restrict__ circs, const typename Cx<T>::type* __restrict__ states,
                          typename Cx<T>::type* __restrict__ psi, typename Cx<T>::type* __restrict__ lam,
                          const T* __restrict__ grad_out, int n_obs) {
  using C = typename Cx<T>::type;
  const DevCirc& d = circs[blockIdx.y];
  const int64_t namps = int64_t(1) << d.n;
  const int nt = d.n_terms;
  const uint64_t* pmask = reinterpret_cast<const uint64_t*>(d.terms);
  const double* coeff = reinterpret_cast<const double*>(d.terms + 8 * (size_t)nt);
  const int32_t* obs = reinterpret_cast<const int32_t*>(d.terms + 16 * (size_t)nt);
  const T* w = grad_out + (int64_t)d.row * n_obs;
  const C* src = states + d.state_off;
  C* p = psi + d.work_off;
  C* l = lam + d.work_off;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < namps; i += (int64_t)gridDim.x * blockDim.x) {
    double sgn = 0.0;
    for (int k = 0; k < nt; ++k) {
      const double wc = (double)w[obs[k]] * coeff[k];
      sgn += (__popcll((uint64_t)i & pmask[k]) & 1) ? -wc : wc;
    }
    const C a = src[i];
    p[i] = a;
    C b;
    b.x = (T)(sgn * (double)a.x);
    b.y = (T)(sgn * (double)a.y);
    l[i] = b;
  }
}

template <typename T>
__global__ void adj_batch_final_kernel(const DevCirc* __restrict__ circs, const int64_t* __restrict__ ppref,
                                       int count, const double* __restrict__ partial, T* __restrict__ grad) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= ppref[count]) return;
  const int c = find_circ(ppref, count, gid);
  const DevCirc& d = circs[c];
  const int p = (int)(gid - ppref[c]);
  const int64_t ntiles = d.n_stages > 0 ? (int64_t(1) << (d.n - d.stages[0].t)) : 1;
  double g = 0.0;
  if (p < d.n_used) {
    const double* part = partial + d.part_off;
    for (int e = d.pslot_ptr[p]; e < d.pslot_ptr[p + 1]; ++e) {
      double x = 0.0;
      const double* row = part + (int64_t)d.pslot_idx[e] * ntiles;
      for (int64_t tl = 0; tl < ntiles; ++tl) x += row[tl];
      g += 2.0 * d.pslot_scale[e] * x;
    }
  }
  grad[d.param_off + p] = (T)g;
}

template <typename T, int R>
static tq_status launch_adj_batch_stages_R(const BatchLaunch& b, const void* mats, void* psi, void* lam,
                                           double* partial, hipStream_t stream) {
  using C = typename Cx<T>::type;
  for (size_t L = 0; L + 1 < b.level_begin.size(); ++L) {
    const int64_t items = b.level_begin[L + 1] - b.level_begin[L];
    if (items == 0) continue;
    const int t = b.level_t[L];
    const unsigned threads = 1u << (t - R);
    const unsigned waves = (threads + 63) / 64;
    const size_t lds = 2 * (sizeof(C) << t) + (size_t)std::max(1, b.level_nslot[L]) * waves * sizeof(T);
    hipLaunchKernelGGL((adj_batch_stage_kernel<T, R>), dim3((unsigned)items), dim3(threads), lds, stream, b.d_circ,
                       b.d_items + b.level_begin[L], (int)L, (const C*)mats, (C*)psi, (C*)lam, partial);
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}

template <typename T>
tq_status launch_batch_adjoint(const BatchLaunch& b, const void* d_params, void* d_mats, const void* d_states,
                               void* d_work_psi, void* d_work_lam, double* d_partial, const T* d_grad_out,
                               int n_obs, T* d_grad, hipStream_t stream) {
  using C = typename Cx<T>::type;
  if (b.count == 0) return TQ_OK;
  if (b.total_mats > 0) {
    hipLaunchKernelGGL(adj_batch_gate_build_kernel<T>, dim3((unsigned)((b.total_mats + 127) / 128)), dim3(128), 0,
                       stream, b.d_circ, b.d_pref, b.count, (const T*)d_params, (C*)d_mats);
    TQ_HIP(hipGetLastError());
  }
  for (int c0 = 0; c0 < b.count; c0 += 65535) {
    const int cn = std::min(65535, b.count - c0);
    int64_t bx = (b.max_amps + 255) / 256;
    bx = std::min<int64_t>(bx, std::max<int64_t>(1, 8192 / cn));
    hipLaunchKernelGGL(adj_batch_init_kernel<T>, dim3((unsigned)bx, cn), dim3(256), 0, stream, b.d_circ + c0,
                       (const C*)d_states, (C*)d_work_psi, (C*)d_work_lam, d_grad_out, n_obs);
    TQ_HIP(hipGetLastError());
  }
  tq_status st;
  switch (b.R) {
    case 1: st = launch_adj_batch_stages_R<T, 1>(b, d_mats, d_work_psi, d_work_lam, d_partial, stream); break;
    case 2: st = launch_adj_batch_stages_R<T, 2>(b, d_mats, d_work_psi, d_work_lam, d_partial, stream); break;
    case 3: st = launch_adj_batch_stages_R<T, 3>(b, d_mats, d_work_psi, d_work_lam, d_partial, stream); break;
    case 4: st = launch_adj_batch_stages_R<T, 4>(b, d_mats, d_work_psi, d_work_lam, d_partial, stream); break;
    default: return fail(TQ_ENOTSUP, "adjoint register bits must be 1..4");
  }
  TQ_TRY(st);
  if (b.total_params > 0) {
    hipLaunchKernelGGL(adj_batch_final_kernel<T>, dim3((unsigned)((b.total_params + 127) / 128)), dim3(128), 0,
                       stream, b.d_circ, b.d_ppref, b.count, (const double*)d_partial, d_grad);
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}
template tq_status launch_batch_adjoint<float>(const BatchLaunch&, const void*, void*, const void*, void*, void*,
                                               double*, const float*, int, float*, hipStream_t);
template tq_status launch_batch_adjoint<double>(const BatchLaunch&, const void*, void*, const void*, void*, void*,
                                                double*, const double*, int, double*, hipStream_t);

template tq_status launch_adjoint<float>(const Schedule&, const void*, BatchMap, const void*, BatchMap, void*, void*,
                                         BatchMap, void*, double*, const uint64_t*, const double*, const int32_t*, int,
                                         const float*, int, float*, int, int, hipStream_t, const AdjPauli*);
template tq_status launch_adjoint<double>(const Schedule&, const void*, BatchMap, const void*, BatchMap, void*, void*,
                                          BatchMap, void*, double*, const uint64_t*, const double*, const int32_t*,
                                          int, const double*, int, double*, int, int, hipStream_t, const AdjPauli*);

}  // namespace tq
