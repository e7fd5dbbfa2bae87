// Expectation values of sums of Pauli-Z strings (the VQC cost of Sec. 4):
// <O_o> = sum over terms k with obs_k = o of coeff_k * sum_x |psi_x|^2 (-1)^popcount(x & m_k).
//
// The state is read in chunks of 2^12 contiguous amplitudes, so the index bits at and above
// 12 are fixed per chunk: their parity is one uniform sign per term. Within a chunk, a
// thread holds 16 amplitudes; the sums of all terms over them are read off one
// Walsh-Hadamard transform of the thread's |psi|^2 values, in the state's precision, as is the
// thread's running sum over its chunks. Everything above a thread (the threads of a group, the
// groups of a circuit) is summed in double in a fixed order, so repeated runs are bitwise equal.
#include <mutex>
#include <type_traits>

#include "sv_device.h"

namespace tq {

constexpr int kExpThreads = 256;

// +1 or -1 built from the parity bit with integer operations (a wave-uniform parity stays in
// scalar registers, so the multiply-add takes it as a scalar operand)
template <typename T>
__device__ __forceinline__ T unit_sign(uint32_t parity);
template <>
__device__ __forceinline__ float unit_sign<float>(uint32_t parity) {
  return __uint_as_float(0x3f800000u | (parity << 31));
}
template <>
__device__ __forceinline__ double unit_sign<double>(uint32_t parity) {
  return __longlong_as_double((long long)(0x3ff0000000000000ull | ((unsigned long long)parity << 63)));
}

// v + (v moved across lanes by the data-parallel-primitive control CTRL), in double: both
// 32-bit halves move with the same control; rows outside ROWS receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_add_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffull), CTRL, ROWS, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return v + __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over each aligned group of P lanes (P = 16: a row of 16 lanes; P = 32: two rows) in a
// fixed order: pairs in quads, quads, half-row and row mirrors, and for P = 32 a row broadcast
// into the odd rows. The group's total is then in its last lane.
template <int P>
__device__ __forceinline__ double lanes_sum_f64(double v) {
  static_assert(P == 16 || P == 32, "groups of 16 or 32 lanes");
  v = dpp_add_f64<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add_f64<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add_f64<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add_f64<0x140, 0xf>(v);  // row_mirror: every lane of a row holds the row's total
  if constexpr (P == 32) v = dpp_add_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  return v;
}

// Chunk size of the partial-sum kernel: 2^kExpChunkBits amplitudes, 16 per thread.
constexpr int kExpChunkBits = 12;
constexpr int kExpVals = 16;

// Work-groups per circuit of the partial-sum kernel: about kExpGroups over the launch, at
// most one per 2^12-amplitude chunk.
constexpr int kExpGroups = 512;

int expval_groups(int n, int cn) {
  const int cb = n < kExpChunkBits ? n : kExpChunkBits;
  const int64_t chunks = int64_t(1) << (n - cb);
  const int64_t want = std::max<int64_t>(1, kExpGroups / std::max(cn, 1));
  return (int)std::min<int64_t>(chunks, want);
}

// Vector width of the partial-sum kernel's loads: A amplitudes per 16-byte load (2 for
// complex64, 1 for complex128). A circuit whose state is not 16-byte aligned, or holds fewer
// than 2^12 amplitudes, is read one amplitude per load instead (the same sums, in another
// order).
template <typename T>
struct ExpVec {
  static constexpr int A = 16 / (int)sizeof(typename Cx<T>::type);
};

// One work-group's share of one circuit: a contiguous range of its 2^cb-amplitude chunks,
// the next chunk's loads in flight while the current one is transformed. In a chunk a thread
// reads A amplitudes per load at index (it << (lgA + 8)) | (tid << lgA) | e, it < nit, e < A:
// their |psi|^2 values p[(it << lgA) | e] go through one Walsh-Hadamard transform
// W[u] = sum_v (-1)^{|v & u|} p[v], and a term with mask m reads W at u = the mask's bits over
// (it, e). The sign of the mask's chunk bits is the same for the whole wave: lane k of every
// wave holds term k's chunk mask, and one ballot per chunk gives all terms' signs as a scalar
// bit mask, applied in a multiply-add with a scalar +-1. The sign of the mask's thread bits
// is fixed per thread and applied once, after the last chunk. The transform and a thread's
// sum over its chunks are in the state's precision; the partial sums below are in double.
template <typename T, int KT, int A, bool FULL>
__device__ __forceinline__ void expval_partial_body(const typename Cx<T>::type* __restrict__ s, int n,
                                                    const uint64_t* __restrict__ pmask, int nk, T (&acc)[KT],
                                                    T (*wsh)[kExpThreads]) {
  using C = typename Cx<T>::type;
  using V = typename std::conditional<A == 2, typename std::conditional<sizeof(T) == 4, float4, double4>::type,
                                      C>::type;
  constexpr int lgA = A == 2 ? 1 : 0;
  constexpr int kLoads = kExpVals / A;  // loads per thread and chunk
  // FULL: n >= kExpChunkBits, so every thread holds 16 live values of every chunk
  const int cb = FULL ? kExpChunkBits : (n < kExpChunkBits ? n : kExpChunkBits);
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const int tb = FULL ? 8 : (cb - lgA < 8 ? cb - lgA : 8);  // thread bits of a chunk index
  const int nit = FULL ? kLoads : 1 << (cb - lgA - tb);
  const uint32_t tcl = tid & ((1u << tb) - 1);
  const bool live = FULL || tid < (1u << tb);
  const int64_t nchunk = int64_t(1) << (n - cb);
  const V* sv = (const V*)s;  // index in units of A amplitudes
  V buf0[kLoads], buf1[kLoads];
  auto load = [&](V(&nxt)[kLoads], int64_t j) {
#pragma unroll
    for (int it = 0; it < kLoads; ++it) {
      const uint32_t itc = FULL ? (uint32_t)it : (uint32_t)(it < nit ? it : nit - 1);
      nxt[it] = sv[(((uint64_t)j << cb) >> lgA) + ((itc << 8) | tcl)];
    }
  };
  // this group's chunks: a contiguous range (a fixed sequence, so the sums repeat bitwise);
  // every load is issued unconditionally (past the range: the group's last chunk again), so
  // the number of loads in flight is the same on every path and each wait covers one buffer
  const int64_t per = (nchunk + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * per;
  const int64_t j1 = j0 + per < nchunk ? j0 + per : nchunk;
  if (j0 >= j1) return;
  const int64_t last = j1 - 1;
  load(buf0, j0);  // in flight during the term set-up below
  // lane k < nk: term k's chunk mask, its mask over the thread bits, and the element offset
  // of its W[u] column in wsh; lanes past nk hold zeros, so the padding terms k >= nk of the
  // template read W[0] with sign +1 (their sums are never reduced) and no loop below branches
  uint32_t lane_cm = 0, lane_tm = 0, lane_uo = 0;
  if (lane < (uint32_t)nk) {
    const uint64_t m = pmask[lane];
    const uint32_t u = ((((uint32_t)m >> (lgA + 8)) & (uint32_t)(nit - 1)) << lgA) | ((uint32_t)m & (uint32_t)(A - 1));
    lane_cm = (uint32_t)(m >> cb);  // n - cb <= 28 chunk bits
    lane_tm = ((uint32_t)m >> lgA) & 0xffu;
    lane_uo = u * kExpThreads;
  }
  uint32_t tpar = 0;  // bit k: parity of term k's mask over this thread's index bits
#pragma unroll
  for (int k = 0; k < KT; ++k)
    tpar |= ((uint32_t)__popc(tid & (uint32_t)__builtin_amdgcn_readlane((int)lane_tm, k)) & 1u) << k;
  T* const wcol = &wsh[0][tid];
  // Chunk j from buffer `cur` (when `use`); the other buffer's loads, issued just before, stay
  // in flight meanwhile. The two buffers alternate, so nothing is copied between them.
  auto chunk = [&](V(&cur)[kLoads], int64_t j, bool use) {
    T pv[kExpVals];
#pragma unroll
    for (int it = 0; it < kLoads; ++it) {
      const bool on = FULL || (it < nit && live);
      if constexpr (A == 2) {
        const T p0 = cur[it].x * cur[it].x + cur[it].y * cur[it].y;
        const T p1 = cur[it].z * cur[it].z + cur[it].w * cur[it].w;
        pv[2 * it] = on ? p0 : (T)0;
        pv[2 * it + 1] = on ? p1 : (T)0;
      } else {
        const T p = cur[it].x * cur[it].x + cur[it].y * cur[it].y;
        pv[it] = on ? p : (T)0;
      }
    }
    if (!use) return;
#pragma unroll
    for (int h = 1; h < kExpVals; h <<= 1) {
#pragma unroll
      for (int i = 0; i < kExpVals; ++i)
        if ((i & h) == 0) {
          const T a = pv[i], b = pv[i | h];
          pv[i] = a + b;
          pv[i | h] = a - b;
        }
    }
    // all 16 coefficients are stored (those past nit * A belong to the zero padding of a
    // small chunk and are read by no term), so the stores do not branch
#pragma unroll
    for (int v = 0; v < kExpVals; ++v) wcol[v * kExpThreads] = pv[v];
    // bit k: parity of term k's chunk bits in chunk j (the same in every wave of the group)
    const uint64_t cpar = __builtin_amdgcn_ballot_w64((__popc((uint32_t)j & lane_cm) & 1) != 0);
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const uint32_t uo = (uint32_t)__builtin_amdgcn_readlane((int)lane_uo, k);
      acc[k] = fma(unit_sign<T>((uint32_t)(cpar >> k) & 1u), wcol[uo], acc[k]);
    }
  };
  for (int64_t j = j0; j < j1; j += 2) {
    load(buf1, j + 1 < j1 ? j + 1 : last);
    chunk(buf0, j, true);
    load(buf0, j + 2 < j1 ? j + 2 : last);
    chunk(buf1, j + 1, j + 1 < j1);
  }
#pragma unroll
  for (int k = 0; k < KT; ++k)
    if ((tpar >> k) & 1u) acc[k] = -acc[k];
}

// Partial sums of every term over one work-group's chunks of circuit blockIdx.y.
template <typename T, int KT>
__global__ void __launch_bounds__(kExpThreads)
    expval_partial_kernel(const typename Cx<T>::type* __restrict__ st, BatchMap smap, int n,
                          const uint64_t* __restrict__ pmask, int nk, double* __restrict__ partial) {
  const typename Cx<T>::type* s = st + smap.at(blockIdx.y);
  __shared__ T wsh[kExpVals][kExpThreads];  // per-thread column: indexable storage for W[u]
  T acc[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) acc[k] = (T)0;
  constexpr int A = ExpVec<T>::A;
  if (n < kExpChunkBits)  // a small state: one chunk, read one amplitude per load
    expval_partial_body<T, KT, 1, false>(s, n, pmask, nk, acc, wsh);
  else if (A > 1 && (reinterpret_cast<uintptr_t>(s) & 15) == 0)
    expval_partial_body<T, KT, A, true>(s, n, pmask, nk, acc, wsh);
  else
    expval_partial_body<T, KT, 1, true>(s, n, pmask, nk, acc, wsh);
  // The group's sums of its terms, in rounds of RT terms: every thread stores its sums of the
  // round's terms, as double, over the transform's LDS array; P = 256 / RT threads per term
  // each add RT of them (threads s, s + P, s + 2P, ...) in order, P-lane sums finish the term
  // and the group's last lane writes it. A fixed order, so repeated runs are bitwise equal.
  constexpr int RT = (int)(sizeof(wsh) / (kExpThreads * sizeof(double)));  // 8 (float), 16 (double)
  constexpr int P = kExpThreads / RT;
  double* const red = reinterpret_cast<double*>(&wsh[0][0]);
  const int tid = threadIdx.x, rk = tid / P, rs = tid % P;  // this thread's term of a round, first thread
#pragma unroll
  for (int r = 0; r < KT; r += RT) {
    __syncthreads();  // the array is free: every thread is past its chunks / the last round's reads
#pragma unroll
    for (int k = 0; k < RT; ++k) red[k * kExpThreads + tid] = r + k < KT ? (double)acc[r + k < KT ? r + k : 0] : 0.0;
    __syncthreads();
    double x = 0.0;
#pragma unroll
    for (int i = 0; i < RT; ++i) x += red[rk * kExpThreads + rs + P * i];
    x = lanes_sum_f64<P>(x);
    const int k = r + rk;
    if (rs == P - 1 && k < nk)  // terms past nk (the template's padding) are not written
      partial[((int64_t)blockIdx.y * KT + k) * gridDim.x + blockIdx.x] = x;
  }
}

// One work-group of 16 waves per circuit: wave w sums the partials of terms w, w + 16, ...;
// a lane adds groups lane + 64 c (c < 8) of each of its terms per block of 512 groups, all
// loads of a block issued before any add, in eight chains per term, then chains and lanes
// are combined in a fixed order; each observable's thread accumulates coeff * S_k over its
// terms in term order. Circuit i of the launch writes output row rows.at(i).
constexpr int kExpFinalThreads = 1024;

template <typename T, int KT>
__global__ void __launch_bounds__(kExpFinalThreads)
    expval_final_kernel(const double* __restrict__ partial, int nb, int nk, const double* __restrict__ coeff,
                        const int32_t* __restrict__ obs, int n_obs, double* __restrict__ outacc, int first,
                        int last, T* __restrict__ out, BatchMap rows) {
  constexpr int kW = kExpFinalThreads / 64;
  constexpr int TPW = (KT + kW - 1) / kW;  // terms per wave
  __shared__ double sk[KT], sc[KT];
  __shared__ int32_t so[KT];
  const int circ = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x < nk) {  // the terms' coefficients and observables, read once per group
    sc[threadIdx.x] = coeff[threadIdx.x];
    so[threadIdx.x] = obs[threadIdx.x];
  }
  double x[TPW][8];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int c = 0; c < 8; ++c) x[t][c] = 0.0;
  for (int b0 = 0; b0 < nb; b0 += 512) {
    double v[TPW][8];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int k = wv + kW * t;
      const double* pk = partial + ((int64_t)circ * KT + (k < nk ? k : 0)) * nb;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int b = b0 + lane + 64 * c;
        v[t][c] = (k < nk && b < nb) ? pk[b] : 0.0;
      }
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int c = 0; c < 8; ++c) x[t][c] += v[t][c];
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int k = wv + kW * t;
    double y = ((x[t][0] + x[t][1]) + (x[t][2] + x[t][3])) + ((x[t][4] + x[t][5]) + (x[t][6] + x[t][7]));
    for (int off = 32; off > 0; off >>= 1) y += __shfl_xor(y, off, 64);
    if (k < nk && lane == 0) sk[k] = y;
  }
  __syncthreads();
  // thread o owns observable o: its terms' coeff * S_k added in term order (onto what the
  // earlier term chunks left in outacc), written out after the last chunk
  for (int o = threadIdx.x; o < n_obs; o += kExpFinalThreads) {
    double* acc = outacc + (int64_t)circ * n_obs + o;
    double a = first ? 0.0 : *acc;
    for (int k = 0; k < nk; ++k)
      if (so[k] == o) a += sc[k] * sk[k];
    if (last)
      out[rows.at(circ) * n_obs + o] = (T)a;
    else
      *acc = a;
  }
}

template <typename T, int KT>
static void launch_chunk(const typename Cx<T>::type* d_states, BatchMap smap, int n, int nb, int cn,
                         const uint64_t* pm, const double* cf, const int32_t* ob, int nk, int n_obs, double* partial,
                         double* outacc, int first, int last, T* out, BatchMap rows, hipStream_t stream) {
  hipLaunchKernelGGL((expval_partial_kernel<T, KT>), dim3((unsigned)nb, (unsigned)cn), dim3(kExpThreads), 0, stream,
                     d_states, smap, n, pm, nk, partial);
  hipLaunchKernelGGL((expval_final_kernel<T, KT>), dim3((unsigned)cn), dim3(kExpFinalThreads), 0, stream, partial, nb, nk,
                     cf, ob, n_obs, outacc, first, last, out, rows);
}

size_t expval_scratch_doubles(int n, int count, int n_obs) {
  const int cn = std::min(count, 65535);
  const int nb = expval_groups(n, cn);
  return (size_t)cn * n_obs + (size_t)cn * nb * 32 + 64;
}

template <typename T>
tq_status launch_expval(const typename Cx<T>::type* d_states, BatchMap smap, int n, int count,
                        const uint64_t* d_pmask, const double* d_coeff, const int32_t* d_obs, int n_terms, int n_obs,
                        double* d_scratch, size_t scratch_doubles, T* d_out, BatchMap rows, hipStream_t stream) {
  if (expval_scratch_doubles(n, count, n_obs) > scratch_doubles) return fail(TQ_ENOMEM, "expval scratch too small");
  for (int c0 = 0; c0 < count; c0 += 65535) {
    const int cn = std::min(65535, count - c0);
    const int nb = expval_groups(n, cn);
    double* outacc = d_scratch;
    double* partial = d_scratch + (size_t)cn * n_obs;
    const BatchMap sm = smap.shifted(c0), rm = rows.shifted(c0);
    if (n_terms == 0)
      launch_chunk<T, 1>(d_states, sm, n, nb, cn, d_pmask, d_coeff, d_obs, 0, n_obs, partial, outacc, 1, 1, d_out, rm,
                         stream);
    for (int k0 = 0; k0 < n_terms; k0 += 32) {
      const int nk = std::min(32, n_terms - k0);
      const int first = k0 == 0, last = k0 + 32 >= n_terms;
      // the smallest term count of the templates that holds nk (every template term costs
      // the same per chunk, used or not)
      auto go = [&](auto kt) {
        launch_chunk<T, decltype(kt)::value>(d_states, sm, n, nb, cn, d_pmask + k0, d_coeff + k0, d_obs + k0, nk,
                                             n_obs, partial, outacc, first, last, d_out, rm, stream);
      };
      if (nk <= 4)
        go(std::integral_constant<int, 4>());
      else if (nk <= 8)
        go(std::integral_constant<int, 8>());
      else if (nk <= 16)
        go(std::integral_constant<int, 16>());
      else if (nk <= 24)
        go(std::integral_constant<int, 24>());
      else
        go(std::integral_constant<int, 32>());
    }
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}

template tq_status launch_expval<float>(const float2*, BatchMap, int, int, const uint64_t*, const double*,
                                        const int32_t*, int, int, double*, size_t, float*, BatchMap, hipStream_t);
template tq_status launch_expval<double>(const double2*, BatchMap, int, int, const uint64_t*, const double*,
                                         const int32_t*, int, int, double*, size_t, double*, BatchMap, hipStream_t);

}  // namespace tq

// ---------------------------------------------------------------------------------------
// Allocation-free expectation values, for callers that cannot allocate (code under HIP graph
// capture, tight serving loops). The term table, the accumulators and the partial sums
// live in one static device array per GPU, whose device address is looked up once per device
// (hipGetSymbolAddress with that device current); host code only ever passes that address.
// Every call on a GPU shares the array and it keeps the last call's contents, so calls that
// overlap on one GPU (several streams or host threads at once) race.
// ---------------------------------------------------------------------------------------
namespace tq {
namespace {

constexpr size_t kStaticScratchBytes = size_t(8) << 20;
constexpr int kStaticMaxTerms = 64;
constexpr size_t kStaticTableBytes = 2048;  // 64 masks + 64 coefficients + 64 observables
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char expval_static_scratch[kStaticScratchBytes];

struct StaticTerms {
  uint64_t pm[kStaticMaxTerms];
  double cf[kStaticMaxTerms];
  int32_t ob[kStaticMaxTerms];
};

// Writes the term table at the start of the array.
__global__ void expval_static_setup_kernel(StaticTerms terms, int n_terms, unsigned char* base) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t* pm = (uint64_t*)base;
  double* cf = (double*)(base + 8 * kStaticMaxTerms);
  int32_t* ob = (int32_t*)(base + 16 * kStaticMaxTerms);
  if (i < n_terms) {
    pm[i] = terms.pm[i];
    cf[i] = terms.cf[i];
    ob[i] = terms.ob[i];
  }
}

std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {nullptr};

tq_status static_scratch_address(void** out) {
  int dev = -1;
  TQ_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TQ_ENOTSUP, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(expval_static_scratch));
    if (e != hipSuccess || !p)
      return fail(TQ_EHIP, std::string("hipGetSymbolAddress of the static scratch: ") + hipGetErrorString(e));
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  return TQ_OK;
}

template <typename T>
tq_status expval_noalloc_t(int n, int count, int64_t stride, const void* d_states, const StaticTerms& st,
                           int n_terms, int n_obs, void* d_out, hipStream_t stream) {
  void* base;
  TQ_TRY(static_scratch_address(&base));
  const size_t avail = (kStaticScratchBytes - kStaticTableBytes) / sizeof(double);
  const size_t need = expval_scratch_doubles(n, count, n_obs);
  if (need > avail)
    return fail(TQ_EWORKSPACE, "tq_expval_noalloc: " + std::to_string(count) + " circuits of " + std::to_string(n) +
                                   " qubits with " + std::to_string(n_obs) + " outputs need " +
                                   std::to_string(need * sizeof(double)) + " bytes of scratch, above the " +
                                   std::to_string(avail * sizeof(double)) + "-byte static limit");
  unsigned char* b = (unsigned char*)base;
  hipLaunchKernelGGL(expval_static_setup_kernel, dim3(1), dim3(kStaticMaxTerms), 0, stream, st, n_terms, b);
  TQ_HIP(hipGetLastError());
  BatchMap smap{nullptr, 0, stride};
  BatchMap rows{nullptr, 0, 1};
  return launch_expval<T>((const typename Cx<T>::type*)d_states, smap, n, count, (const uint64_t*)b,
                          (const double*)(b + 8 * kStaticMaxTerms), (const int32_t*)(b + 16 * kStaticMaxTerms), n_terms,
                          n_obs, (double*)(b + kStaticTableBytes), avail, (T*)d_out, rows, stream);
}

}  // namespace
}  // namespace tq

extern "C" tq_status tq_expval_noalloc(tq_dtype dt, int32_t n_qubits, int32_t count, int64_t state_stride,
                                       const void* d_states, const tq_zterm* terms, int32_t n_terms, int32_t n_obs,
                                       void* d_out, void* stream) {
  using namespace tq;
  if (dt != TQ_C64 && dt != TQ_C128) return fail(TQ_EINVAL, "unknown dtype");
  if (n_qubits < 1 || n_qubits > 34) return fail(TQ_ENOTSUP, "n_qubits must be in 1..34");
  if (count < 0) return fail(TQ_EINVAL, "negative count");
  if (count == 0) return TQ_OK;
  if (state_stride < (int64_t(1) << n_qubits)) return fail(TQ_EINVAL, "state_stride is smaller than 2^n_qubits");
  if (n_obs < 1) return fail(TQ_EINVAL, "n_obs must be >= 1");
  if (n_terms < 0 || n_terms > kStaticMaxTerms || (n_terms > 0 && !terms))
    return fail(TQ_EINVAL, "tq_expval_noalloc takes 0.." + std::to_string(kStaticMaxTerms) + " terms");
  if (!d_states || !d_out) return fail(TQ_EINVAL, "null device pointer");
  StaticTerms st{};
  for (int k = 0; k < n_terms; ++k) {
    if (terms[k].obs < 0 || terms[k].obs >= n_obs) return fail(TQ_EINVAL, "term obs index out of range");
    if (n_qubits < 64 && (terms[k].mask >> n_qubits) != 0) return fail(TQ_EINVAL, "term names a qubit >= n");
    uint64_t m = 0;
    for (int q = 0; q < n_qubits; ++q)
      if ((terms[k].mask >> q) & 1ull) m |= 1ull << (n_qubits - 1 - q);
    st.pm[k] = m;
    st.cf[k] = terms[k].coeff;
    st.ob[k] = terms[k].obs;
  }
  if (dt == TQ_C64)
    return expval_noalloc_t<float>(n_qubits, count, state_stride, d_states, st, n_terms, n_obs, d_out,
                                   (hipStream_t)stream);
  return expval_noalloc_t<double>(n_qubits, count, state_stride, d_states, st, n_terms, n_obs, d_out,
                                  (hipStream_t)stream);
}
