// Tensor-network mode: execution of a contraction tree as pairwise complex contractions
// (the paper's Sec. 3.2, step (e)), optionally sliced (Sec. 3.2.3), and its reverse pass.
//
// Every index has dimension 2, so a tensor of rank r is 2^r complex numbers and an index
// is one bit of the element offset (first index = most significant bit). A pairwise step
// contracts X and Y into Z; each index of the step falls in one class:
//   batch      in X, Y and Z          (a hyperedge kept for later tensors)
//   kept       in X (or Y) and Z      (the M, N of a GEMM)
//   contracted in X and Y, not in Z   (the K of a GEMM)
//   summed     in X only (or Y only), not in Z
//   broadcast  in Z only              (reverse pass of a summed index)
// The generic "direct" kernel handles all classes with bit deposits. Steps whose indices are
// only batch / kept / contracted and whose M, N, K are all large go to a bit-permute of X
// and Y into [batch][M][K] and [batch][K][N] followed by a complex GEMM on FP32 MFMA
// (a real GEMM on interleaved complex data with Y expanded to 2x2 real blocks, i.e. the
// four-real-product form with FP32 accumulation).
//
// Slices run in groups of G: a tensor that does not depend on a sliced index is computed
// once and shared by the G slices (stride 0); the others get G copies.
#include <algorithm>
#include <map>
#include <set>

#include "sv_device.h"

namespace tq {

constexpr int kTnMaxBits = 40;
constexpr uint8_t kNone = 0xff;

// Device-side compact step: bit-position tables.
struct DevTnStep {
  int32_t zr;               // output rank
  int32_t ks;               // summed bits
  uint8_t xo[kTnMaxBits];   // for output bit i (from LSB): position in X or kNone
  uint8_t yo[kTnMaxBits];
  uint8_t xs[kTnMaxBits];   // for summed bit j: position in X or kNone
  uint8_t ys[kTnMaxBits];
};

struct TnTensorInfo {
  int rank = 0;
  std::vector<int> inds;    // most significant first
  bool sdep = false;        // depends on a sliced index
  int64_t off = -1;         // workspace offset (complex elements) of copy 0
  int leaf = -1;            // leaf id (>= 0 for leaves)
  std::vector<int> sliced_pos;  // leaves: positions (from LSB, in the full leaf) of sliced indices
  std::vector<int> sliced_bits; // leaves: for each entry of sliced_pos, its bit in the slice number
  int gather = -1;              // leaves: row of the plan's gather table
};

struct TnExec {              // one pairwise contraction as executed
  int x, y, z;               // tensor ids (z may be an environment slot in the reverse pass)
  int method = 0;            // 0 direct, 1 gemm
  DevTnStep dev{};
  int64_t flops = 0;         // real flops per slice
  // gemm
  int64_t B = 1, M = 1, N = 1, K = 1;
  bool permx = false, permy = false;
  std::vector<uint8_t> px, py;   // for each bit of the permuted operand (from LSB): source bit
};

}  // namespace tq

struct tq_tn_plan {
  int dtype = 0;
  int n_leaves = 0;
  std::vector<tq::TnTensorInfo> t;     // leaves then intermediates
  std::vector<std::pair<int, int>> pairs;
  std::vector<int> sliced;
  std::vector<int> out_inds;
  int root = -1;
  std::vector<int64_t> leaf_off;       // packed leaf buffer offsets
  int64_t leaf_elems = 0;
  int64_t n_slices = 1, G = 1;
  std::vector<tq::TnExec> fwd;         // forward steps
  std::vector<tq::TnExec> bwd;         // reverse steps (2 per forward step)
  int64_t ws_fwd = 0, ws_bwd = 0;      // complex elements
  int64_t perm_elems = 0;              // permute scratch (per slice)
  int64_t perm_off = 0;                // workspace offset of the permute scratch
  int64_t env_off0 = 0;                // reverse pass: environment offsets per tensor
  std::vector<int64_t> env_off;
  int64_t split_off = 0, split_elems = 0;  // partial sums of steps split over the summed range
  int64_t flops = 0, gemm_flops = 0, max_elems = 0;
  int n_direct = 0, n_gemm = 0;
  // device copies
  void* d_fwd = nullptr;               // DevTnStep[fwd.size()]
  void* d_bwd = nullptr;
  void* d_perm = nullptr;              // uint8 tables for permutes: [2 * steps][kTnMaxBits]
  void* d_bperm = nullptr;
  std::vector<int> sliced_leaves;      // leaf tensor ids that depend on a sliced index
  void* d_gather = nullptr;            // per sliced leaf: [keep pos][slice pos][slice bit] x kTnMaxBits
  // execution segments: runs of small steps (one fused launch each) and single large steps
  struct Seg {
    int fused = 0;       // 1: run of small direct steps in tn_fused_kernel
    int first = 0;       // first step (index into fwd / bwd)
    int count = 0;
    int64_t list = 0;    // fused: first entry in the DevFused table
    int shared = 0;      // forward: outputs do not depend on a sliced index (one copy)
  };
  std::vector<Seg> fseg, bseg;
  void* d_ffused = nullptr;            // DevFused entries of the forward runs
  void* d_bfused = nullptr;            // ... of the reverse runs
  void* d_leaf_env = nullptr;          // (leaf offset, environment offset, elements) of unsliced leaves
  int n_leaf_env = 0;
  bool store = false;                  // the reverse pass reuses the forward's intermediates
  bool host_only = false;              // built without a context: no device tables, cannot run
  ~tq_tn_plan();
};

namespace tq {

// ---------------------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int64_t deposit_bits(uint64_t v, const uint8_t* pos, int n) {
  int64_t r = 0;
  for (int i = 0; i < n; ++i)
    if (pos[i] != kNone) r |= (int64_t)((v >> i) & 1ull) << pos[i];
  return r;
}

// A pairwise step by bit deposits: Z[e] = sum_s X[xoff(e) + xsum(s)] * Y[yoff(e) + ysum(s)].
// 2^tb consecutive lanes share one output e: lane l sums the assignments s = l, l + 2^tb, ..
// of the summed bits, then the group adds its partial sums by a butterfly (and, for groups
// wider than a wave, through LDS): a fixed order, so results repeat bitwise. The offsets of
// the low kt summed bits come from LDS tables built by the whole work-group.
constexpr int kTnTabBits = 9;

// Per-step LDS state of a work-group: the step record itself (its position bytes would
// otherwise be re-read from device memory one byte per bit, each a memory round trip) and
// offset tables of the low 16 output bits in X and Y, 8 bits per table.
struct TnStepLds {
  DevTnStep st;
  int64_t ox[2][256], oy[2][256];
};
static_assert(sizeof(DevTnStep) % 4 == 0, "word copy of the step record");

// Work-group-wide: stage the step, then build the summed-bit tables (tx, ty) and the
// output-bit tables. The caller synchronises before using them.
template <typename T>
__device__ __forceinline__ void tn_build_tables(const DevTnStep* __restrict__ gst, TnStepLds* L, int64_t* tx,
                                                int64_t* ty) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(gst);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&L->st);
  for (int i = threadIdx.x; i < (int)(sizeof(DevTnStep) / 4); i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  const DevTnStep* st = &L->st;
  const int kt = st->ks < kTnTabBits ? st->ks : kTnTabBits;
  for (int i = threadIdx.x; i < (1 << kt); i += blockDim.x) {
    tx[i] = deposit_bits((uint64_t)i, st->xs, kt);
    ty[i] = deposit_bits((uint64_t)i, st->ys, kt);
  }
  // only the entries an output index can select are built (2^z0 and 2^z1 of them; entry 0
  // of the second table is 0 for outputs below 2^8)
  const int z0 = st->zr < 8 ? st->zr : 8;
  const int z1 = st->zr < 8 ? 0 : (st->zr < 16 ? st->zr - 8 : 8);
  for (int i = threadIdx.x; i < (1 << z0); i += blockDim.x) {
    L->ox[0][i] = deposit_bits((uint64_t)i, st->xo, z0);
    L->oy[0][i] = deposit_bits((uint64_t)i, st->yo, z0);
  }
  for (int i = threadIdx.x; i < (1 << z1); i += blockDim.x) {
    L->ox[1][i] = deposit_bits((uint64_t)i, st->xo + 8, z1);
    L->oy[1][i] = deposit_bits((uint64_t)i, st->yo + 8, z1);
  }
}

// Outputs of groups g = g0, g0 + gstride, ... (one group = 2^tb lanes). Every thread of the
// work-group calls this with the same g0 / gstride trip count (barriers inside when tb > 6).
// Summed assignments are walked as outer chunks so0 .. so1 of the table (all of them by
// default); output e goes to z[e * zstride] (zstride > 1: partial sums of one chunk range).
template <typename T>
__device__ __forceinline__ void tn_step_outputs(const TnStepLds* L, const int64_t* tx,
                                                const int64_t* ty, const typename Cx<T>::type* __restrict__ x,
                                                const typename Cx<T>::type* __restrict__ y,
                                                typename Cx<T>::type* __restrict__ z, int tb, int64_t gfirst,
                                                int64_t gstride, T* red, int64_t so0 = 0, int64_t so1 = -1,
                                                int64_t zstride = 1) {
  using C = typename Cx<T>::type;
  const DevTnStep* st = &L->st;
  const int zr = st->zr, ks = st->ks;
  const int kt = ks < kTnTabBits ? ks : kTnTabBits;
  const int nt = 1 << kt;
  const int G = 1 << tb;
  const int lane = threadIdx.x & (G - 1);
  const int gpb = (int)blockDim.x >> tb;  // groups per block
  const int64_t nz = int64_t(1) << zr;
  const int64_t nouter = so1 < 0 ? (int64_t(1) << (ks - kt)) : so1;
  const int64_t ngroups = (nz + gpb - 1) / gpb;  // rounds of the block's group slots
  for (int64_t r = gfirst; r < ngroups; r += gstride) {
    const int64_t e0 = r * gpb;  // first output of the round (gpb divides 2^16)
    const int64_t e = e0 + (threadIdx.x >> tb);
    const bool valid = e < nz;
    // output bits 16 and up are the same for the whole round: deposited once, in scalar
    // registers, rather than per lane
    int64_t xhi = 0, yhi = 0;
    if (zr > 16) {
      xhi = deposit_bits((uint64_t)e0 >> 16, st->xo + 16, zr - 16);
      yhi = deposit_bits((uint64_t)e0 >> 16, st->yo + 16, zr - 16);
    }
    T ar = 0, ai = 0;
    if (valid) {
      const int64_t xb = xhi + L->ox[0][e & 255] + L->ox[1][(e >> 8) & 255];
      const int64_t yb = yhi + L->oy[0][e & 255] + L->oy[1][(e >> 8) & 255];
      for (int64_t so = so0; so < nouter; ++so) {
        const int64_t xo2 = xb + deposit_bits((uint64_t)so, st->xs + kt, ks - kt);
        const int64_t yo2 = yb + deposit_bits((uint64_t)so, st->ys + kt, ks - kt);
        for (int sl = lane; sl < nt; sl += G) {
          const C a = x[xo2 + tx[sl]], b = y[yo2 + ty[sl]];
          ar += a.x * b.x - a.y * b.y;
          ai += a.x * b.y + a.y * b.x;
        }
      }
    }
    const int wl = tb < 6 ? tb : 6;  // butterfly inside the wave
    for (int off = 1; off < (1 << wl); off <<= 1) {
      ar += __shfl_xor(ar, off, 64);
      ai += __shfl_xor(ai, off, 64);
    }
    if (tb > 6) {  // groups of 128 or 256 lanes: add the waves' sums in wave order
      const int wv = threadIdx.x >> 6;
      if ((threadIdx.x & 63) == 0) {
        red[2 * wv] = ar;
        red[2 * wv + 1] = ai;
      }
      __syncthreads();
      if (lane == 0) {
        ar = 0;
        ai = 0;
        for (int w = 0; w < (G >> 6); ++w) {
          ar += red[2 * (wv + w)];
          ai += red[2 * (wv + w) + 1];
        }
      }
      __syncthreads();
    }
    if (valid && lane == 0) {
      C o;
      o.x = ar;
      o.y = ai;
      z[e * zstride] = o;
    }
  }
}

// Wide steps with one lane per output and few summed bits (ks <= kTnWideMaxKs): each lane
// takes kTnWideOpl outputs per round (e = e0 + tid + 256 j, so every load instruction stays
// coalesced across the lanes), and issues all their loads before any multiply, which keeps
// several times more bytes in flight per lane than one output at a time. Same sums in the
// same order as tn_step_outputs with 2^0 lanes per output.
constexpr int kTnWideOpl = 4;
constexpr int kTnWideMaxKs = 3;

template <typename T>
__device__ __forceinline__ void tn_step_outputs_wide(const TnStepLds* L, const int64_t* tx, const int64_t* ty,
                                                     const typename Cx<T>::type* __restrict__ x,
                                                     const typename Cx<T>::type* __restrict__ y,
                                                     typename Cx<T>::type* __restrict__ z, int64_t gfirst,
                                                     int64_t gstride) {
  using C = typename Cx<T>::type;
  const DevTnStep* st = &L->st;
  const int zr = st->zr, nt = 1 << st->ks;
  const int64_t nz = int64_t(1) << zr;
  const int64_t per = (int64_t)blockDim.x * kTnWideOpl;  // outputs per round (divides 2^16)
  for (int64_t r = gfirst; r * per < nz; r += gstride) {
    const int64_t e0 = r * per;
    int64_t xhi = 0, yhi = 0;  // output bits 16 and up: the same for the whole round
    if (zr > 16) {
      xhi = deposit_bits((uint64_t)e0 >> 16, st->xo + 16, zr - 16);
      yhi = deposit_bits((uint64_t)e0 >> 16, st->yo + 16, zr - 16);
    }
    int64_t xb[kTnWideOpl], yb[kTnWideOpl];
    bool ok[kTnWideOpl];
#pragma unroll
    for (int j = 0; j < kTnWideOpl; ++j) {
      const int64_t e = e0 + threadIdx.x + (int64_t)blockDim.x * j;
      ok[j] = e < nz;
      xb[j] = xhi + L->ox[0][e & 255] + L->ox[1][(e >> 8) & 255];
      yb[j] = yhi + L->oy[0][e & 255] + L->oy[1][(e >> 8) & 255];
    }
    T ar[kTnWideOpl], ai[kTnWideOpl];
#pragma unroll
    for (int j = 0; j < kTnWideOpl; ++j) ar[j] = ai[j] = 0;
    for (int sl = 0; sl < nt; ++sl) {
      C a[kTnWideOpl], b[kTnWideOpl];
#pragma unroll
      for (int j = 0; j < kTnWideOpl; ++j)
        if (ok[j]) {
          a[j] = x[xb[j] + tx[sl]];
          b[j] = y[yb[j] + ty[sl]];
        }
#pragma unroll
      for (int j = 0; j < kTnWideOpl; ++j)
        if (ok[j]) {
          ar[j] += a[j].x * b[j].x - a[j].y * b[j].y;
          ai[j] += a[j].x * b[j].y + a[j].y * b[j].x;
        }
    }
#pragma unroll
    for (int j = 0; j < kTnWideOpl; ++j)
      if (ok[j]) {
        C o;
        o.x = ar[j];
        o.y = ai[j];
        z[e0 + threadIdx.x + (int64_t)blockDim.x * j] = o;
      }
  }
}

// The kernel takes the wide form for these steps (the host sizes the grid alike).
__host__ __device__ __forceinline__ bool tn_wide_form(int tb, int ks) { return tb == 0 && ks <= kTnWideMaxKs; }

// One step over the whole device; blockIdx.y = slice copy (stride 0 for shared tensors).
// With kb > 0 the summed range is also split over 2^kb chunks of work-groups: block x runs
// output rounds (x mod rb) for chunk (x / rb) and writes partial sums P[e][chunk]; the
// chunks are added afterwards in order by tn_chunk_sum_kernel.
template <typename T>
__global__ void __launch_bounds__(256)
    tn_direct_kernel(const DevTnStep* __restrict__ st, const typename Cx<T>::type* __restrict__ X, int64_t xs,
                     const typename Cx<T>::type* __restrict__ Y, int64_t ys, typename Cx<T>::type* __restrict__ Z,
                     int64_t zs, int tb, int kb, int rb, typename Cx<T>::type* __restrict__ P, int64_t ps) {
  __shared__ int64_t tx[1 << kTnTabBits], ty[1 << kTnTabBits];
  __shared__ T red[16];
  __shared__ TnStepLds L;
  tn_build_tables<T>(st, &L, tx, ty);
  __syncthreads();
  const typename Cx<T>::type* x = X + xs * blockIdx.y;
  const typename Cx<T>::type* y = Y + ys * blockIdx.y;
  if (kb == 0) {
    if (tn_wide_form(tb, L.st.ks))
      tn_step_outputs_wide<T>(&L, tx, ty, x, y, Z + zs * blockIdx.y, blockIdx.x, gridDim.x);
    else
      tn_step_outputs<T>(&L, tx, ty, x, y, Z + zs * blockIdx.y, tb, blockIdx.x, gridDim.x, red);
    return;
  }
  const int kt = L.st.ks < kTnTabBits ? L.st.ks : kTnTabBits;
  const int64_t per = (int64_t(1) << (L.st.ks - kt)) >> kb;  // outer chunks per split
  const int64_t c = blockIdx.x / rb;
  tn_step_outputs<T>(&L, tx, ty, x, y, P + ps * blockIdx.y + c, tb, blockIdx.x % rb, rb, red, c * per,
                     (c + 1) * per, int64_t(1) << kb);
}

// z[e] = sum over chunks c in order of P[e][c]; blockIdx.y = slice copy.
template <typename T>
__global__ void __launch_bounds__(256)
    tn_chunk_sum_kernel(const typename Cx<T>::type* __restrict__ P, int64_t ps, typename Cx<T>::type* __restrict__ Z,
                        int64_t zs, int64_t nz, int nchunks) {
  using C = typename Cx<T>::type;
  const C* p = P + ps * blockIdx.y;
  C* z = Z + zs * blockIdx.y;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nz; e += (int64_t)gridDim.x * blockDim.x) {
    C v{(T)0, (T)0};
    for (int c = 0; c < nchunks; ++c) {
      const C q = p[e * nchunks + c];
      v.x += q.x;
      v.y += q.y;
    }
    z[e] = v;
  }
}

// Large direct steps of many networks in one launch (a round of a batch): item i owns
// blocks first[i] .. first[i + 1] - 1 and runs them as tn_direct_kernel would: kb = 0 writes
// the outputs; kb > 0 splits the summed range over 2^kb chunks of rb blocks each and writes
// partial sums P[e][chunk], added afterwards by tn_chunk_sum_multi_kernel.
struct DevDirectItem {
  const DevTnStep* st;
  const void* x;
  const void* y;
  void* z;
  void* P;  // partial sums (kb > 0)
  int32_t tb, rb, kb, pad;
};
static_assert(sizeof(DevDirectItem) == 56, "DevDirectItem layout");
constexpr int kTnMultiMaxItems = 1024;

// The item of block b: the largest i with fb[i] <= b (fb in LDS, n items).
__device__ __forceinline__ int tn_item_of(const int32_t* fb, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fb[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__global__ void __launch_bounds__(256)
    tn_direct_multi_kernel(const int32_t* __restrict__ first, const DevDirectItem* __restrict__ items, int n) {
  using C = typename Cx<T>::type;
  __shared__ int32_t fb[kTnMultiMaxItems + 1];
  __shared__ int64_t tx[1 << kTnTabBits], ty[1 << kTnTabBits];
  __shared__ T red[16];
  __shared__ TnStepLds L;
  for (int i = threadIdx.x; i <= n; i += blockDim.x) fb[i] = first[i];
  __syncthreads();
  const int b = (int)blockIdx.x;
  const int it = tn_item_of(fb, n, b);
  const DevDirectItem d = items[it];
  const int lb = b - fb[it];
  tn_build_tables<T>(d.st, &L, tx, ty);
  __syncthreads();
  if (d.kb == 0) {
    if (tn_wide_form(d.tb, L.st.ks))
      tn_step_outputs_wide<T>(&L, tx, ty, (const C*)d.x, (const C*)d.y, (C*)d.z, lb, d.rb);
    else
      tn_step_outputs<T>(&L, tx, ty, (const C*)d.x, (const C*)d.y, (C*)d.z, d.tb, lb, d.rb, red);
    return;
  }
  const int kt = L.st.ks < kTnTabBits ? L.st.ks : kTnTabBits;
  const int64_t per = (int64_t(1) << (L.st.ks - kt)) >> d.kb;  // outer chunks per split
  const int64_t c = lb / d.rb;
  tn_step_outputs<T>(&L, tx, ty, (const C*)d.x, (const C*)d.y, (C*)d.P + c, d.tb, lb % d.rb, d.rb, red, c * per,
                     (c + 1) * per, int64_t(1) << d.kb);
}

// z[e] = sum over chunks in order of P[e][chunk] for the kb > 0 items of a round: item i owns
// blocks first[i] .. first[i + 1] - 1 (the same sums, in the same order, as
// tn_chunk_sum_kernel).
struct DevChunkItem {
  const void* P;
  void* z;
  int64_t nz;
  int32_t nchunks, pad;
};
static_assert(sizeof(DevChunkItem) == 32, "DevChunkItem layout");

template <typename T>
__global__ void __launch_bounds__(256)
    tn_chunk_sum_multi_kernel(const int32_t* __restrict__ first, const DevChunkItem* __restrict__ items, int n) {
  using C = typename Cx<T>::type;
  __shared__ int32_t fb[kTnMultiMaxItems + 1];
  for (int i = threadIdx.x; i <= n; i += blockDim.x) fb[i] = first[i];
  __syncthreads();
  const int b = (int)blockIdx.x;
  const int it = tn_item_of(fb, n, b);
  const DevChunkItem d = items[it];
  const int nblk = fb[it + 1] - fb[it];
  const C* p = (const C*)d.P;
  C* z = (C*)d.z;
  for (int64_t e = (int64_t)(b - fb[it]) * blockDim.x + threadIdx.x; e < d.nz; e += (int64_t)nblk * blockDim.x) {
    C v{(T)0, (T)0};
    for (int c = 0; c < d.nchunks; ++c) {
      const C q = p[e * d.nchunks + c];
      v.x += q.x;
      v.y += q.y;
    }
    z[e] = v;
  }
}

// A run of small steps in one launch: one work-group per slice copy. The host orders a run's
// steps by dependency level (a step's level is one more than the levels of the steps that
// produce its operands); the steps of one level are independent and run on different waves
// at once, with one barrier between levels (each level reads tensors the earlier ones wrote).
struct DevFused {
  int32_t step;   // index in the plan's step table
  int32_t flags;  // bit 0: X from the leaf buffer, bit 1: Y from the leaf buffer; bits 8..31 on
                  // the first entry of a level: the number of entries in that level
  int32_t r0;     // first output round of this step in its level's list of rounds
  int32_t rn;     // output rounds of this step (tn_wave_rounds)
  int32_t lw;     // on the first entry of a level: the level's total rounds
  int32_t pad;
  int64_t xo, xs, yo, ys, zo, zs;  // complex-element offsets and per-copy strides
};
static_assert(sizeof(DevFused) == 72, "DevFused layout");

// Output rounds of a small step on one wave: 64 / 2^tb outputs per round, tb = the lanes per
// output (6 - zr, within 0..ks).
__host__ __device__ __forceinline__ int tn_wave_rounds(int zr, int ks) {
  int tb = 6 - zr;
  tb = tb < 0 ? 0 : (tb > ks ? ks : tb);
  const int opr = 64 >> tb;
  return ((1 << zr) + opr - 1) / opr;
}

// Steps run inside a fused run when their output has at most 2^12 elements and their work
// (outputs x summed assignments) at most 2^16 complex products.
constexpr int kTnFusedMaxOut = 12;
constexpr int kTnFusedMaxWork = 16;
constexpr int kTnFusedThreads = 1024;  // 16 waves: up to 16 steps of a level at once

// A small step's record as a fused run keeps it in LDS: output rank, summed bits, and the
// first 16 entries of each position array (a small step has at most 16 bits in all).
struct TnSmallStep {
  int32_t zr, ks;
  uint8_t pos[4][16];  // output bits in X, in Y; summed bits in X, in Y (kNone if absent)
};
static_assert(sizeof(TnSmallStep) == 72, "TnSmallStep layout");
constexpr int kTnRunCap = 512;  // entries of one fused run (the host splits longer runs)

// One wave's share of one small step (output rank zr, ks summed bits, zr + ks <= 16, so
// every operand index fits 32 bits): output rounds r0 <= r < r1 of 64 / 2^tb outputs, 2^tb
// lanes per output. A lane's summed assignments are its low tb bits (from the
// lane), the next cb <= 3 bits (unrolled, offsets from uniform registers) and the remaining
// bits walked in Gray-code order (one uniform bit toggle per block of 2^cb products). The
// lanes of an output add their sums by a butterfly: a fixed order, so results repeat bitwise.
template <typename T>
__device__ __forceinline__ void tn_wave_step(const TnSmallStep* stp, const typename Cx<T>::type* __restrict__ x,
                                             const typename Cx<T>::type* __restrict__ y,
                                             typename Cx<T>::type* __restrict__ z, int r0, int r1) {
  using C = typename Cx<T>::type;
  const int zr = stp->zr, ks = stp->ks;
  constexpr int XO = 0, YO = 1, XS = 2, YS = 3;
  auto tn_pos_byte = [stp](int arr, int i) -> int { return stp->pos[arr][i]; };
  const int lane = threadIdx.x & 63;
  int tb = 6 - zr;
  tb = tb < 0 ? 0 : (tb > ks ? ks : tb);
  const int opr = 64 >> tb;  // outputs per round
  const int lsub = lane & ((1 << tb) - 1), lhi = lane >> tb;
  // summed bits 0..tb-1: from the lane
  uint32_t xl = 0, yl = 0;
  for (int j = 0; j < tb; ++j) {
    const int px = tn_pos_byte(XS, j), py = tn_pos_byte(YS, j);
    const uint32_t bit = (uint32_t)(lsub >> j) & 1u;
    if (px != kNone) xl |= bit << px;
    if (py != kNone) yl |= bit << py;
  }
  // output bits below lo: from the lane (opr = 2^(6 - tb) outputs per round)
  const int lo = zr < 6 - tb ? zr : 6 - tb;
  for (int i = 0; i < lo; ++i) {
    const int px = tn_pos_byte(XO, i), py = tn_pos_byte(YO, i);
    const uint32_t bit = (uint32_t)(lhi >> i) & 1u;
    if (px != kNone) xl |= bit << px;
    if (py != kNone) yl |= bit << py;
  }
  // summed bits tb..tb+cb-1: 2^cb uniform offsets
  const int nhb = ks - tb;
  const int cb = nhb < 3 ? nhb : 3;
  const int nin = 1 << cb;
  uint32_t ix[8], iy[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    ix[v] = 0;
    iy[v] = 0;
    for (int j = 0; j < cb; ++j) {
      const int px = tn_pos_byte(XS, tb + j), py = tn_pos_byte(YS, tb + j);
      if (((v >> j) & 1) && px != kNone) ix[v] |= 1u << px;
      if (((v >> j) & 1) && py != kNone) iy[v] |= 1u << py;
    }
  }
  const int nu = 1 << (nhb - cb);
  const int nz = 1 << zr;
  for (int r = r0; r < r1 && r * opr < nz; ++r) {
    // output bits lo.. of the round: uniform
    const int e0 = r * opr;
    uint32_t xr = 0, yr = 0;
    for (int i = lo; i < zr; ++i) {
      const int px = tn_pos_byte(XO, i), py = tn_pos_byte(YO, i);
      const uint32_t bit = (uint32_t)(e0 >> i) & 1u;
      if (px != kNone) xr |= bit << px;
      if (py != kNone) yr |= bit << py;
    }
    const int e = e0 + lhi;
    const bool valid = e < nz;
    uint32_t xb = xr | xl, yb = yr | yl;
    T ar = 0, ai = 0;
    for (int u = 0; u < nu; ++u) {
      if (valid) {
        C a[8], b[8];
#pragma unroll
        for (int v = 0; v < 8; ++v)
          if (v < nin) {
            a[v] = x[xb | ix[v]];
            b[v] = y[yb | iy[v]];
          }
#pragma unroll
        for (int v = 0; v < 8; ++v)
          if (v < nin) {
            ar += a[v].x * b[v].x - a[v].y * b[v].y;
            ai += a[v].x * b[v].y + a[v].y * b[v].x;
          }
      }
      if (u + 1 < nu) {  // Gray code: the next block differs in one summed bit
        const int j = tb + cb + __builtin_ctz((unsigned)(u + 1));
        const int px = tn_pos_byte(XS, j), py = tn_pos_byte(YS, j);
        if (px != kNone) xb ^= 1u << px;
        if (py != kNone) yb ^= 1u << py;
      }
    }
    for (int off = 1; off < (1 << tb); off <<= 1) {
      ar += __shfl_xor(ar, off, 64);
      ai += __shfl_xor(ai, off, 64);
    }
    if (valid && lsub == 0) {
      C o;
      o.x = ar;
      o.y = ai;
      z[e] = o;
    }
  }
}

// A fused run (n <= kTnRunCap entries): its entry list and compact step records are first
// copied to LDS, then the levels run as below, reading all of their metadata from LDS.
template <typename T>
__device__ __forceinline__ void tn_run_list(const DevTnStep* __restrict__ steps, const DevFused* __restrict__ list,
                                            int n, const typename Cx<T>::type* __restrict__ leaves,
                                            typename Cx<T>::type* __restrict__ ws, int64_t c, DevFused* lf,
                                            TnSmallStep* ls) {
  using C = typename Cx<T>::type;
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(list);
    uint32_t* dst = reinterpret_cast<uint32_t*>(lf);
    constexpr int kw = (int)(sizeof(DevFused) / 4);
    for (int i = threadIdx.x; i < n * kw; i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  {
    // words 0-1: zr, ks; then 4 words from each position array (byte offsets 8, 8 + 40, ...)
    constexpr int kw = (int)(sizeof(TnSmallStep) / 4);  // 18
    for (int i = threadIdx.x; i < n * kw; i += blockDim.x) {
      const int e = i / kw, w = i % kw;
      const uint32_t* st = reinterpret_cast<const uint32_t*>(steps + lf[e].step);
      const int sw = w < 2 ? w : 2 + ((w - 2) >> 2) * (kTnMaxBits / 4) + ((w - 2) & 3);
      reinterpret_cast<uint32_t*>(ls + e)[w] = st[sw];
    }
  }
  __syncthreads();
  const int W = (int)(blockDim.x >> 6), wave = (int)(threadIdx.x >> 6);
  for (int k = 0; k < n;) {
    const int m = max(1, lf[k].flags >> 8);  // entries of this level
    // the level's output rounds, in entry order, split into W contiguous shares: a wave runs
    // its share's rounds entry by entry (a large step spreads over several waves)
    const int total = lf[k].lw;
    const int share = (total + W - 1) / W;
    int w0 = wave * share;
    const int w1 = min(total, w0 + share);
    if (w0 < w1) {
      int lo = 0, hi = m - 1;  // the entry holding round w0
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (lf[k + mid].r0 <= w0) lo = mid; else hi = mid - 1;
      }
      for (int i = lo; w0 < w1 && i < m; ++i) {
        const DevFused& f = lf[k + i];
        const int end = min(w1, f.r0 + f.rn);
        if (end > w0) {
          const C* x = ((f.flags & 1) ? leaves : ws) + f.xo + f.xs * c;
          const C* y = ((f.flags & 2) ? leaves : ws) + f.yo + f.ys * c;
          C* z = ws + f.zo + f.zs * c;
          tn_wave_step<T>(ls + k + i, x, y, z, w0 - f.r0, end - f.r0);
          w0 = end;
        }
      }
    }
    __syncthreads();
    k += m;
  }
}

template <typename T>
__global__ void __launch_bounds__(kTnFusedThreads)
    tn_fused_kernel(const DevTnStep* __restrict__ steps, const DevFused* __restrict__ list, int n,
                    const typename Cx<T>::type* __restrict__ leaves, typename Cx<T>::type* __restrict__ ws) {
  __shared__ DevFused lf[kTnRunCap];
  __shared__ TnSmallStep ls[kTnRunCap];
  tn_run_list<T>(steps, list, n, leaves, ws, blockIdx.x, lf, ls);
}

// Many networks at once: items of one launch, one work-group each.
struct DevFusedItem {  // a run of small steps of one network
  const DevTnStep* steps;
  const DevFused* list;
  const void* leaves;
  void* ws;
  int32_t n;
  int32_t pad;
};
static_assert(sizeof(DevFusedItem) == 40, "DevFusedItem layout");
struct DevCopyItem {  // dst[0, n) = src[0, n)
  const void* src;
  void* dst;
  int64_t n;
};
static_assert(sizeof(DevCopyItem) == 24, "DevCopyItem layout");
struct DevEnvItem {  // leaf environments of one unsliced network into its gradient buffer
  const int64_t* tab;  // rows (leaf offset, environment offset, elements)
  const void* ws;
  void* grad;
  int32_t rows;
  int32_t pad;
};
static_assert(sizeof(DevEnvItem) == 32, "DevEnvItem layout");

template <typename T>
__global__ void __launch_bounds__(kTnFusedThreads) tn_fused_multi_kernel(const DevFusedItem* __restrict__ items) {
  __shared__ DevFused lf[kTnRunCap];
  __shared__ TnSmallStep ls[kTnRunCap];
  const DevFusedItem& d = items[blockIdx.x];
  tn_run_list<T>(d.steps, d.list, d.n, (const typename Cx<T>::type*)d.leaves, (typename Cx<T>::type*)d.ws, 0, lf,
                 ls);
}

template <typename T>
__global__ void __launch_bounds__(256) tn_copy_multi_kernel(const DevCopyItem* __restrict__ items) {
  using C = typename Cx<T>::type;
  const DevCopyItem& d = items[blockIdx.x];
  const C* src = (const C*)d.src;
  C* dst = (C*)d.dst;
  for (int64_t j = threadIdx.x; j < d.n; j += blockDim.x) dst[j] = src[j];
}

// Unsliced networks: every leaf has one environment, so the gradient is a copy.
template <typename T>
__global__ void __launch_bounds__(256) tn_env_multi_kernel(const DevEnvItem* __restrict__ items) {
  using C = typename Cx<T>::type;
  const DevEnvItem& d = items[blockIdx.x];
  const C* ws = (const C*)d.ws;
  C* grad = (C*)d.grad;
  for (int r = 0; r < d.rows; ++r) {
    const int64_t lo = d.tab[3 * r], eo = d.tab[3 * r + 1], n = d.tab[3 * r + 2];
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) grad[lo + j] = ws[eo + j];
  }
}

// Leaf environments -> gradient buffer: row i of the table is (leaf offset, environment
// offset, elements); out[leaf + j] += sum over the G copies of env[j] (copies in order).
template <typename T>
__global__ void __launch_bounds__(256)
    tn_leaf_env_kernel(const int64_t* __restrict__ tab, const typename Cx<T>::type* __restrict__ ws, int G,
                       typename Cx<T>::type* __restrict__ grad) {
  using C = typename Cx<T>::type;
  const int64_t lo = tab[3 * blockIdx.x], eo = tab[3 * blockIdx.x + 1], n = tab[3 * blockIdx.x + 2];
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    C v = grad[lo + j];
    for (int g = 0; g < G; ++g) {
      const C e = ws[eo + n * g + j];
      v.x += e.x;
      v.y += e.y;
    }
    grad[lo + j] = v;
  }
}

// The upstream value as the result's environment, one copy per slice of the group.
template <typename T>
__global__ void __launch_bounds__(256)
    tn_broadcast_kernel(const typename Cx<T>::type* __restrict__ in, typename Cx<T>::type* __restrict__ out,
                        int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    out[n * blockIdx.y + j] = in[j];
}

// Bit permutation: out[j] = in[i(j)], out bit q taken from in bit perm[q].
template <typename T>
__global__ void __launch_bounds__(256)
    tn_permute_kernel(const typename Cx<T>::type* __restrict__ in, int64_t is, typename Cx<T>::type* __restrict__ out,
                      int64_t os, const uint8_t* __restrict__ perm, int r) {
  const typename Cx<T>::type* src = in + is * blockIdx.y;
  typename Cx<T>::type* dst = out + os * blockIdx.y;
  const int64_t n = int64_t(1) << r;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    dst[j] = src[deposit_bits((uint64_t)j, perm, r)];
}

// Batched complex GEMM on FP32 MFMA: C[b] (M x N) = A[b] (M x K) * B[b] (K x N), complex64,
// row-major, interleaved. Real view: C^ (M x 2N) = A^ (M x 2K) * B^ (2K x 2N) with every
// complex b of B becoming the real block [[br, bi], [-bi, br]]. Work-group tile 64 x 64 real
// (64 complex rows x 32 complex columns), 4 waves in 2 x 2, each wave 2 x 2 MFMA 16x16x4
// blocks. Requires M % 64 == 0, N % 32 == 0, K % 8 == 0.
constexpr int kGemmBM = 64, kGemmBN = 64, kGemmBK = 16;

__global__ void __launch_bounds__(256)
    tn_cgemm_mfma_kernel(const float2* __restrict__ A, int64_t as, const float2* __restrict__ B, int64_t bs,
                         float2* __restrict__ Cm, int64_t cs, int M, int N, int K) {
  __shared__ float sA[kGemmBK][kGemmBM + 4];   // [k][m]
  __shared__ float sB[kGemmBK][kGemmBN + 4];   // [k][n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int m0 = blockIdx.y * kGemmBM;
  const int n0c = blockIdx.x * (kGemmBN / 2);  // complex column
  const float2* a = A + as * blockIdx.z;
  const float2* b = B + bs * blockIdx.z;
  float2* c = Cm + cs * blockIdx.z;
  typedef float float4v __attribute__((ext_vector_type(4)));
  float4v acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = float4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += kGemmBK / 2) {  // complex k
    // A tile: 64 rows x 8 complex = 64 x 16 real; thread loads 2 complex of one row
    {
      const int r = tid >> 2, kk = (tid & 3) * 2;
      const float2 v0 = a[(int64_t)(m0 + r) * K + k0 + kk];
      const float2 v1 = a[(int64_t)(m0 + r) * K + k0 + kk + 1];
      sA[2 * kk + 0][r] = v0.x;
      sA[2 * kk + 1][r] = v0.y;
      sA[2 * kk + 2][r] = v1.x;
      sA[2 * kk + 3][r] = v1.y;
    }
    // B tile: 8 complex rows x 32 complex cols -> 16 x 64 real
    {
      const int kr = tid >> 5, cc = tid & 31;
      const float2 v = b[(int64_t)(k0 + kr) * N + n0c + cc];
      sB[2 * kr + 0][2 * cc + 0] = v.x;
      sB[2 * kr + 0][2 * cc + 1] = v.y;
      sB[2 * kr + 1][2 * cc + 0] = -v.y;
      sB[2 * kr + 1][2 * cc + 1] = v.x;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGemmBK; kk += 4) {
      const int kl = kk + (lane >> 4);
      float av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = sA[kl][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = sB[kl][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of 16x16x4: lane l, register r -> row 4*(l/16) + r, column l % 16
  float* cf = reinterpret_cast<float*>(c);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int col = 2 * n0c + wn + 16 * j + (lane & 15);
        cf[(int64_t)row * (2 * N) + col] = acc[i][j][r];
      }
}

// The same product with a 128 x 128 real tile per work-group (128 complex rows, 64 complex
// columns), each wave 64 x 64 as 4 x 4 MFMA blocks: four times the matrix-core work per
// barrier and half the L2 reads of the 64 x 64 tile. Requires M % 128 == 0, N % 64 == 0,
// K % 8 == 0 (the host takes the 64 x 64 kernel otherwise).
constexpr int kGemm2BM = 128, kGemm2BN = 128, kGemm2BK = 32;

__global__ void __launch_bounds__(256)
    tn_cgemm_mfma128_kernel(const float2* __restrict__ A, int64_t as, const float2* __restrict__ B, int64_t bs,
                            float2* __restrict__ Cm, int64_t cs, int M, int N, int K) {
  __shared__ float sA[kGemm2BK][kGemm2BM + 4];   // [k][m]
  __shared__ float sB[kGemm2BK][kGemm2BN + 4];   // [k][n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int m0 = blockIdx.y * kGemm2BM;
  const int n0c = blockIdx.x * (kGemm2BN / 2);  // complex column
  const float2* a = A + as * blockIdx.z;
  const float2* b = B + bs * blockIdx.z;
  float2* c = Cm + cs * blockIdx.z;
  typedef float float4v __attribute__((ext_vector_type(4)));
  float4v acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = float4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += kGemm2BK / 2) {  // complex k
    // A tile: 128 rows x 16 complex = 128 x 32 real; a thread loads 8 complex of one row
    {
      const int r = tid >> 1, kk = (tid & 1) * 8;
      const float2* src = a + (int64_t)(m0 + r) * K + k0 + kk;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float2 v = src[q];
        sA[2 * (kk + q) + 0][r] = v.x;
        sA[2 * (kk + q) + 1][r] = v.y;
      }
    }
    // B tile: 16 complex rows x 64 complex cols -> 32 x 128 real; a thread loads 4 complex
    {
      const int kr = tid >> 4, cc = (tid & 15) * 4;
      const float2* src = b + (int64_t)(k0 + kr) * N + n0c + cc;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float2 v = src[q];
        const int col = 2 * (cc + q);
        sB[2 * kr + 0][col + 0] = v.x;
        sB[2 * kr + 0][col + 1] = v.y;
        sB[2 * kr + 1][col + 0] = -v.y;
        sB[2 * kr + 1][col + 1] = v.x;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGemm2BK; kk += 4) {
      const int kl = kk + (lane >> 4);
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sA[kl][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sB[kl][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of 16x16x4: lane l, register r -> row 4*(l/16) + r, column l % 16
  float* cf = reinterpret_cast<float*>(c);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int col = 2 * n0c + wn + 16 * j + (lane & 15);
        cf[(int64_t)row * (2 * N) + col] = acc[i][j][r];
      }
}

// The same batched complex GEMM for complex128 on FP64 MFMA (16x16x4, double operands and
// accumulation); identical tiling and real view, so the same size requirements.
__global__ void __launch_bounds__(256)
    tn_zgemm_mfma_kernel(const double2* __restrict__ A, int64_t as, const double2* __restrict__ B, int64_t bs,
                         double2* __restrict__ Cm, int64_t cs, int M, int N, int K) {
  __shared__ double sA[kGemmBK][kGemmBM + 2];   // [k][m]
  __shared__ double sB[kGemmBK][kGemmBN + 2];   // [k][n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int m0 = blockIdx.y * kGemmBM;
  const int n0c = blockIdx.x * (kGemmBN / 2);  // complex column
  const double2* a = A + as * blockIdx.z;
  const double2* b = B + bs * blockIdx.z;
  double2* c = Cm + cs * blockIdx.z;
  typedef double double4v __attribute__((ext_vector_type(4)));
  double4v acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = double4v{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += kGemmBK / 2) {  // complex k
    {
      const int r = tid >> 2, kk = (tid & 3) * 2;
      const double2 v0 = a[(int64_t)(m0 + r) * K + k0 + kk];
      const double2 v1 = a[(int64_t)(m0 + r) * K + k0 + kk + 1];
      sA[2 * kk + 0][r] = v0.x;
      sA[2 * kk + 1][r] = v0.y;
      sA[2 * kk + 2][r] = v1.x;
      sA[2 * kk + 3][r] = v1.y;
    }
    {
      const int kr = tid >> 5, cc = tid & 31;
      const double2 v = b[(int64_t)(k0 + kr) * N + n0c + cc];
      sB[2 * kr + 0][2 * cc + 0] = v.x;
      sB[2 * kr + 0][2 * cc + 1] = v.y;
      sB[2 * kr + 1][2 * cc + 0] = -v.y;
      sB[2 * kr + 1][2 * cc + 1] = v.x;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGemmBK; kk += 4) {
      const int kl = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = sA[kl][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = sB[kl][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of the FP64 16x16x4 (checked on the device; it differs from the FP32 one):
  // lane l, register r -> row l/16 + 4 r, column l % 16
  double* cf = reinterpret_cast<double*>(c);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * i + (lane >> 4) + 4 * r;
        const int col = 2 * n0c + wn + 16 * j + (lane & 15);
        cf[(int64_t)row * (2 * N) + col] = acc[i][j][r];
      }
}

// The FP64 product with the large tile: 128 x 128 real per work-group, each wave 64 x 64 as
// 4 x 4 MFMA 16x16x4 FP64 blocks, 16 real k per barrier. Requires M % 128 == 0, N % 64 == 0,
// K % 8 == 0 (the host takes the 64 x 64 kernel otherwise).
__global__ void __launch_bounds__(256)
    tn_zgemm_mfma128_kernel(const double2* __restrict__ A, int64_t as, const double2* __restrict__ B, int64_t bs,
                            double2* __restrict__ Cm, int64_t cs, int M, int N, int K) {
  __shared__ double sA[kGemmBK][kGemm2BM + 2];   // [k][m]
  __shared__ double sB[kGemmBK][kGemm2BN + 2];   // [k][n]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int m0 = blockIdx.y * kGemm2BM;
  const int n0c = blockIdx.x * (kGemm2BN / 2);  // complex column
  const double2* a = A + as * blockIdx.z;
  const double2* b = B + bs * blockIdx.z;
  double2* c = Cm + cs * blockIdx.z;
  typedef double double4v __attribute__((ext_vector_type(4)));
  double4v acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = double4v{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += kGemmBK / 2) {  // complex k
    // A tile: 128 rows x 8 complex = 128 x 16 real; a thread loads 4 complex of one row
    {
      const int r = tid >> 1, kk = (tid & 1) * 4;
      const double2* src = a + (int64_t)(m0 + r) * K + k0 + kk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 v = src[q];
        sA[2 * (kk + q) + 0][r] = v.x;
        sA[2 * (kk + q) + 1][r] = v.y;
      }
    }
    // B tile: 8 complex rows x 64 complex cols -> 16 x 128 real; a thread loads 2 complex
    {
      const int kr = tid >> 5, cc = (tid & 31) * 2;
      const double2* src = b + (int64_t)(k0 + kr) * N + n0c + cc;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double2 v = src[q];
        const int col = 2 * (cc + q);
        sB[2 * kr + 0][col + 0] = v.x;
        sB[2 * kr + 0][col + 1] = v.y;
        sB[2 * kr + 1][col + 0] = -v.y;
        sB[2 * kr + 1][col + 1] = v.x;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGemmBK; kk += 4) {
      const int kl = kk + (lane >> 4);
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sA[kl][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sB[kl][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of the FP64 16x16x4: lane l, register r -> row l/16 + 4 r, column l % 16
  double* cf = reinterpret_cast<double*>(c);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * i + (lane >> 4) + 4 * r;
        const int col = 2 * n0c + wn + 16 * j + (lane & 15);
        cf[(int64_t)row * (2 * N) + col] = acc[i][j][r];
      }
}

// Sliced leaf restriction: out[g][j] = leaf[j with the sliced bits of slice s0+g inserted].
template <typename T>
__global__ void tn_slice_gather_kernel(const typename Cx<T>::type* __restrict__ leaf, typename Cx<T>::type* __restrict__ out,
                                       int r_out, const uint8_t* __restrict__ keep_pos, const uint8_t* __restrict__ sl_pos,
                                       const uint8_t* __restrict__ sl_bit, int nsl, int64_t s0) {
  const int g = blockIdx.y;
  const int64_t s = s0 + g;
  int64_t base = 0;
  for (int q = 0; q < nsl; ++q) base |= ((s >> sl_bit[q]) & 1) << sl_pos[q];
  const int64_t n = int64_t(1) << r_out;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    out[(int64_t)g * n + j] = leaf[base | deposit_bits((uint64_t)j, keep_pos, r_out)];
}

// Reverse of the gather: grad_leaf[slice bits of s0+g inserted][j] += env[g][j], g in order.
template <typename T>
__global__ void tn_slice_scatter_kernel(const typename Cx<T>::type* __restrict__ env, int64_t es, int G,
                                        typename Cx<T>::type* __restrict__ grad, int r_env,
                                        const uint8_t* __restrict__ keep_pos, const uint8_t* __restrict__ sl_pos,
                                        const uint8_t* __restrict__ sl_bit, int nsl, int64_t s0) {
  using C = typename Cx<T>::type;
  const int64_t n = int64_t(1) << r_env;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t lj = deposit_bits((uint64_t)j, keep_pos, r_env);
    for (int g = 0; g < G; ++g) {
      const int64_t s = s0 + g;
      int64_t base = 0;
      for (int q = 0; q < nsl; ++q) base |= ((s >> sl_bit[q]) & 1) << sl_pos[q];
      const C e = env[es * g + j];
      C v = grad[base | lj];
      v.x += e.x;
      v.y += e.y;
      grad[base | lj] = v;
    }
  }
}

// out[j] (+)= sum_g in[g][j] in slice order.
template <typename T>
__global__ void tn_sum_copies_kernel(const typename Cx<T>::type* __restrict__ in, int64_t is, int G,
                                     typename Cx<T>::type* __restrict__ out, int64_t n, int accumulate) {
  using C = typename Cx<T>::type;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    C v = accumulate ? out[j] : C{0, 0};
    for (int g = 0; g < G; ++g) {
      const C e = in[is * g + j];
      v.x += e.x;
      v.y += e.y;
    }
    out[j] = v;
  }
}

template <typename T>
__global__ void tn_fill_kernel(typename Cx<T>::type* __restrict__ p, int64_t n, typename Cx<T>::type v) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    p[j] = v;
}

// ---- leaves from circuit parameters ------------------------------------------------------
struct DevLeaf {
  int32_t kind, gate, conj, const_off;
  int64_t off;
  int32_t flip, _pad;  // element e holds the kind's entry e ^ flip
};

// Leaf li of one network (one thread per leaf).
template <typename T>
__device__ __forceinline__ void tn_leaf_build_one(const DevLeaf* __restrict__ lv, int li,
                                                  const tq_gate* __restrict__ gates, const double* __restrict__ cv,
                                                  const T* __restrict__ params,
                                                  typename Cx<T>::type* __restrict__ out) {
  const DevLeaf L = lv[li];
  typename Cx<T>::type* o = out + L.off;
  const int f = L.flip;  // entry i of the kind's tensor goes to element i ^ f
  const double sg = L.conj ? -1.0 : 1.0;
  if (L.kind == 0) {
    // constants are copied as given (the caller supplies conjugated values if needed)
    const int r = L.gate;  // number of entries for constants is carried in gate
    for (int i = 0; i < r; ++i)
      o[i ^ f] = to_cx<T>(dcx{cv[2 * (L.const_off + i)], cv[2 * (L.const_off + i) + 1]});
    return;
  }
  const tq_gate& g = gates[L.gate];
  double a[3];
  gate_angles(g, params, a);
  if (L.kind == 1) {
    const dmat2 M = gate_mat2(g.op, a);
    for (int i = 0; i < 4; ++i) o[i ^ f] = to_cx<T>(dcx{M.m[i].x, sg * M.m[i].y});
  } else if (L.kind == 2) {
    for (int b = 0; b < 2; ++b) {
      dcx d = diag_entry(g, g.q[0], b, b, a);
      o[b ^ f] = to_cx<T>(dcx{d.x, sg * d.y});
    }
  } else if (L.kind == 3) {
    for (int idx = 0; idx < 4; ++idx) {
      dcx d = diag_entry(g, g.q[0], idx >> 1, idx & 1, a);
      o[idx ^ f] = to_cx<T>(dcx{d.x, sg * d.y});
    }
  } else {  // two-qubit non-diagonal: CNOT [out_c, out_t, in_c, in_t]
    for (int i = 0; i < 16; ++i) {
      const int oc = (i >> 3) & 1, ot = (i >> 2) & 1, ic = (i >> 1) & 1, it = i & 1;
      double v = 0;
      if (g.op == TQ_CNOT) v = (oc == ic) && (ot == (ic ? 1 - it : it)) ? 1.0 : 0.0;
      o[i ^ f] = to_cx<T>(dcx{v, 0.0});
    }
  }
}

template <typename T>
__global__ void tn_leaf_build_kernel(const DevLeaf* __restrict__ lv, int n_leaves, const tq_gate* __restrict__ gates,
                                     const double* __restrict__ cv, const T* __restrict__ params,
                                     typename Cx<T>::type* __restrict__ out) {
  const int li = blockIdx.x * blockDim.x + threadIdx.x;
  if (li < n_leaves) tn_leaf_build_one<T>(lv, li, gates, cv, params, out);
}

// The leaves of many networks in one launch: network blockIdx.y, its leaves over grid x
// (blocks past a network's leaf count do nothing).
struct DevLeafItem {
  const DevLeaf* lv;
  const tq_gate* gates;
  const double* cv;
  const void* params;
  void* out;
  int32_t n_leaves, pad;
};
static_assert(sizeof(DevLeafItem) == 48, "DevLeafItem layout");

template <typename T>
__global__ void tn_leaf_build_multi_kernel(const DevLeafItem* __restrict__ items) {
  const DevLeafItem it = items[blockIdx.y];
  const int li = blockIdx.x * blockDim.x + threadIdx.x;
  if (li < it.n_leaves)
    tn_leaf_build_one<T>(it.lv, li, it.gates, it.cv, (const T*)it.params, (typename Cx<T>::type*)it.out);
}

// d(leaf)/d(angle j) for the gate leaf kinds (conjugated for bra copies): the entries of
// dU/da_j in the leaf's own layout (2x2 [out, in]; diagonal over the wire(s)).
__device__ inline int leaf_derivative(const DevLeaf& L, const tq_gate& g, const double* a, int j, dcx (&d)[16]) {
  if (L.kind != 1 && L.kind != 2 && L.kind != 3) return 0;
  if (j >= gate_n_angles_dev(g.op)) return 0;
  dcx m[kAdjMatStride];
  gate_and_derivs(g.op, a, m);
  const double sg = L.conj ? -1.0 : 1.0;
  const int n = L.kind == 2 ? 2 : 4;
  for (int i = 0; i < n; ++i) d[i] = dcx{m[4 + 4 * j + i].x, sg * m[4 + 4 * j + i].y};
  return n;
}

// grad[p] = Re sum over (leaf, angle) entries of p: pscale * sum_x env[x] * dleaf[x].
// One work-group per parameter: thread t takes entries t, t + 256, ... (a parameter such as a
// QAOA angle has one entry per gate copy), then a fixed-order tree over the group.
constexpr int kPgThreads = 256;
template <typename T>
__device__ __forceinline__ void tn_param_grad_one(const DevLeaf* __restrict__ lv, const tq_gate* __restrict__ gates,
                                                  const T* __restrict__ params, const int32_t* __restrict__ pptr,
                                                  const int32_t* __restrict__ pent,
                                                  const typename Cx<T>::type* __restrict__ env, int p,
                                                  T* __restrict__ grad) {
  double acc = 0.0;
  for (int e = pptr[p] + threadIdx.x; e < pptr[p + 1]; e += kPgThreads) {
    const int li = pent[2 * e], j = pent[2 * e + 1];
    const DevLeaf L = lv[li];
    const tq_gate& g = gates[L.gate];
    double a[3];
    gate_angles(g, params, a);
    dcx d[16];
    const int n = leaf_derivative(L, g, a, j, d);
    const typename Cx<T>::type* E = env + L.off;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += (double)E[i ^ L.flip].x * d[i].x - (double)E[i ^ L.flip].y * d[i].y;
    acc += g.pscale[j] * s;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  __shared__ double red[kPgThreads / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) grad[p] = (T)((red[0] + red[1]) + (red[2] + red[3]));
}

template <typename T>
__global__ void __launch_bounds__(kPgThreads)
    tn_param_grad_kernel(const DevLeaf* __restrict__ lv, const tq_gate* __restrict__ gates,
                         const T* __restrict__ params, const int32_t* __restrict__ pptr,
                         const int32_t* __restrict__ pent, const typename Cx<T>::type* __restrict__ env,
                         int n_params, T* __restrict__ grad) {
  (void)n_params;
  tn_param_grad_one<T>(lv, gates, params, pptr, pent, env, (int)blockIdx.x, grad);
}

// The parameter gradients of many networks in one launch: network blockIdx.y, parameter
// blockIdx.x (groups past a network's parameter count return together, before any barrier).
struct DevPgItem {
  const DevLeaf* lv;
  const tq_gate* gates;
  const void* params;
  const int32_t* pptr;
  const int32_t* pent;
  const void* env;
  void* grad;
  int32_t n_params, pad;
};
static_assert(sizeof(DevPgItem) == 64, "DevPgItem layout");

template <typename T>
__global__ void __launch_bounds__(kPgThreads) tn_param_grad_multi_kernel(const DevPgItem* __restrict__ items) {
  const DevPgItem it = items[blockIdx.y];
  if ((int)blockIdx.x >= it.n_params) return;
  tn_param_grad_one<T>(it.lv, it.gates, (const T*)it.params, it.pptr, it.pent,
                       (const typename Cx<T>::type*)it.env, (int)blockIdx.x, (T*)it.grad);
}

// ---------------------------------------------------------------------------------------
// Host planning
// ---------------------------------------------------------------------------------------
static int pos_of(const std::vector<int>& inds, int id) {  // bit position from LSB
  for (size_t i = 0; i < inds.size(); ++i)
    if (inds[i] == id) return (int)(inds.size() - 1 - i);
  return -1;
}

// Build a pairwise contraction of tensors with index lists xi, yi into zi (order given).
static TnExec make_exec(const std::vector<int>& xi, const std::vector<int>& yi, const std::vector<int>& zi, bool allow_gemm,
                        int csz) {
  TnExec ex;
  DevTnStep& d = ex.dev;
  std::memset(&d, 0xff, sizeof d);
  d.zr = (int)zi.size();
  std::set<int> zs(zi.begin(), zi.end());
  for (int i = 0; i < d.zr; ++i) {
    const int id = zi[d.zr - 1 - i];  // output bit i from LSB
    const int px = pos_of(xi, id), py = pos_of(yi, id);
    d.xo[i] = px >= 0 ? (uint8_t)px : kNone;
    d.yo[i] = py >= 0 ? (uint8_t)py : kNone;
  }
  // summed bit j of the assignment counter: X's summed indices from its least significant
  // up, then Y's own ones likewise, so that the low counter bits (spread over the lanes of an
  // output) are the operands' low address bits
  std::vector<int> summed;
  for (auto it = xi.rbegin(); it != xi.rend(); ++it)
    if (!zs.count(*it)) summed.push_back(*it);
  for (auto it = yi.rbegin(); it != yi.rend(); ++it)
    if (!zs.count(*it) && std::find(summed.begin(), summed.end(), *it) == summed.end()) summed.push_back(*it);
  d.ks = (int)summed.size();
  for (int j = 0; j < d.ks; ++j) {
    const int px = pos_of(xi, summed[j]), py = pos_of(yi, summed[j]);
    d.xs[j] = px >= 0 ? (uint8_t)px : kNone;
    d.ys[j] = py >= 0 ? (uint8_t)py : kNone;
  }
  ex.flops = (int64_t(8) << d.zr) << d.ks;
  // GEMM eligibility: every Z index in exactly one of (X and Y) -> batch, or X only (M), or
  // Y only (N); every summed index in both (K); no broadcast.
  std::vector<int> bI, mI, nI, kI;
  bool ok = allow_gemm;  // FP32 MFMA for complex64, FP64 MFMA for complex128
  for (int id : zi) {
    const bool inx = pos_of(xi, id) >= 0, iny = pos_of(yi, id) >= 0;
    if (inx && iny) bI.push_back(id);
    else if (inx) mI.push_back(id);
    else if (iny) nI.push_back(id);
    else ok = false;
  }
  for (int id : summed) {
    if (pos_of(xi, id) < 0 || pos_of(yi, id) < 0) ok = false;
    kI.push_back(id);
  }
  // Z must already be [b][m][n] in the order given: check zi == b + m + n
  std::vector<int> want;
  want.insert(want.end(), bI.begin(), bI.end());
  want.insert(want.end(), mI.begin(), mI.end());
  want.insert(want.end(), nI.begin(), nI.end());
  if (want != zi) ok = false;
  if (ok && mI.size() >= 6 && nI.size() >= 5 && kI.size() >= 3 && (mI.size() + nI.size() + kI.size()) >= 18) {
    ex.method = 1;
    ex.B = int64_t(1) << bI.size();
    ex.M = int64_t(1) << mI.size();
    ex.N = int64_t(1) << nI.size();
    ex.K = int64_t(1) << kI.size();
    // permuted X: [b][m][k], permuted Y: [b][k][n]
    std::vector<int> xp, yp;
    xp.insert(xp.end(), bI.begin(), bI.end());
    xp.insert(xp.end(), mI.begin(), mI.end());
    xp.insert(xp.end(), kI.begin(), kI.end());
    yp.insert(yp.end(), bI.begin(), bI.end());
    yp.insert(yp.end(), kI.begin(), kI.end());
    yp.insert(yp.end(), nI.begin(), nI.end());
    ex.permx = xp != xi;
    ex.permy = yp != yi;
    ex.px.assign(kTnMaxBits, 0);
    ex.py.assign(kTnMaxBits, 0);
    for (size_t q = 0; q < xp.size(); ++q) ex.px[q] = (uint8_t)pos_of(xi, xp[xp.size() - 1 - q]);
    for (size_t q = 0; q < yp.size(); ++q) ex.py[q] = (uint8_t)pos_of(yi, yp[yp.size() - 1 - q]);
  }
  return ex;
}

}  // namespace tq

static tq_status runnable(const tq_tn_plan* p) {
  if (p->host_only) return tq::fail(TQ_EINVAL, "the plan was built without a context: it can be queried but not run");
  return TQ_OK;
}

tq_tn_plan::~tq_tn_plan() {
  void* p[] = {d_fwd, d_bwd, d_perm, d_bperm, d_gather, d_ffused, d_bfused, d_leaf_env};
  for (void* x : p)
    if (x) (void)hipFree(x);
}

using namespace tq;

extern "C" {

tq_status tq_tn_plan_create(tq_ctx* ctx, const tq_tn_desc* d, tq_tn_plan** out) {
  if (!d || !out) return fail(TQ_EINVAL, "null argument");
  *out = nullptr;
  if (d->dtype != TQ_C64 && d->dtype != TQ_C128) return fail(TQ_EINVAL, "unknown dtype");
  const int L = d->n_leaves;
  if (L < 1 || !d->leaf_rank || !d->leaf_inds) return fail(TQ_EINVAL, "no leaves");
  if (L > 1 && !d->pairs) return fail(TQ_EINVAL, "null tree");
  if (d->n_sliced < 0 || d->n_sliced > 24 || (d->n_sliced && !d->sliced)) return fail(TQ_EINVAL, "bad sliced list");
  if (d->n_out < 0 || (d->n_out && !d->out_inds)) return fail(TQ_EINVAL, "bad output list");
  auto p = std::make_unique<tq_tn_plan>();
  p->dtype = d->dtype;
  p->n_leaves = L;
  const int csz = d->dtype == TQ_C64 ? 8 : 16;
  std::set<int> sl(d->sliced, d->sliced + d->n_sliced);
  if ((int)sl.size() != d->n_sliced) return fail(TQ_EINVAL, "duplicate sliced index");
  p->sliced.assign(d->sliced, d->sliced + d->n_sliced);
  p->out_inds.assign(d->out_inds, d->out_inds + d->n_out);
  for (int id : p->out_inds)
    if (sl.count(id)) return fail(TQ_EINVAL, "an output index cannot be sliced");
  // leaves
  int64_t off = 0, ii = 0;
  std::map<int, int> count;
  for (int l = 0; l < L; ++l) {
    TnTensorInfo t;
    const int r = d->leaf_rank[l];
    if (r < 0 || r > 30) return fail(TQ_EINVAL, "leaf rank out of range");
    std::vector<int> full(d->leaf_inds + ii, d->leaf_inds + ii + r);
    ii += r;
    std::set<int> u(full.begin(), full.end());
    if ((int)u.size() != r) return fail(TQ_EINVAL, "leaf " + std::to_string(l) + " repeats an index");
    for (int id : full) {
      if (id < 0) return fail(TQ_EINVAL, "negative index id");
      count[id]++;
    }
    p->leaf_off.push_back(off);
    off += int64_t(1) << r;
    for (int q = 0; q < r; ++q) {
      if (sl.count(full[q])) {
        t.sdep = true;
      } else {
        t.inds.push_back(full[q]);
      }
    }
    for (size_t si = 0; si < p->sliced.size(); ++si)
      for (int q = 0; q < r; ++q)
        if (full[q] == p->sliced[si]) {
          t.sliced_pos.push_back(r - 1 - q);
          t.sliced_bits.push_back((int)si);
        }
    t.rank = (int)t.inds.size();
    t.leaf = l;
    p->t.push_back(t);
  }
  p->leaf_elems = off;
  // tree
  std::vector<char> used(2 * L, 0);
  std::map<int, int> live(count);  // index -> live holders
  for (int id : p->out_inds) live[id] += 1 << 20;  // outputs always kept
  for (int s = 0; s < L - 1; ++s) {
    const int a = d->pairs[2 * s], b = d->pairs[2 * s + 1];
    if (a < 0 || b < 0 || a >= L + s || b >= L + s || a == b || used[a] || used[b])
      return fail(TQ_EINVAL, "tree step " + std::to_string(s) + " uses an invalid or consumed id");
    used[a] = used[b] = 1;
    const TnTensorInfo &A = p->t[a], &B = p->t[b];
    // kept indices: appear in other live tensors or the output (counts over full leaves;
    // sliced ids are never in any tensor's index list)
    std::vector<int> bI, mI, nI;
    for (int id : A.inds) live[id]--;
    for (int id : B.inds) live[id]--;
    for (int id : A.inds) {
      const bool inB = std::find(B.inds.begin(), B.inds.end(), id) != B.inds.end();
      if (live[id] > 0) (inB ? bI : mI).push_back(id);
    }
    for (int id : B.inds) {
      const bool inA = std::find(A.inds.begin(), A.inds.end(), id) != A.inds.end();
      if (!inA && live[id] > 0) nI.push_back(id);
    }
    TnTensorInfo C;
    // index order of the result: [b][m][n] when the step can run as a GEMM (its output
    // layout); otherwise the larger operand's kept indices, in that operand's order, as the
    // low bits, so that the lanes of the direct kernel read the larger operand and write the
    // result at consecutive addresses (the other operand's indices go on top)
    int n_summed_both = 0;
    bool one_sided_sum = false;
    for (int id : A.inds)
      if (live[id] <= 0) {
        if (std::find(B.inds.begin(), B.inds.end(), id) != B.inds.end()) ++n_summed_both;
        else one_sided_sum = true;
      }
    for (int id : B.inds)
      if (live[id] <= 0 && std::find(A.inds.begin(), A.inds.end(), id) == A.inds.end()) one_sided_sum = true;
    const bool gemm_like = !one_sided_sum && mI.size() >= 6 && nI.size() >= 5 && n_summed_both >= 3 &&
                           mI.size() + nI.size() + n_summed_both >= 18;
    if (gemm_like) {
      C.inds = bI;
      C.inds.insert(C.inds.end(), mI.begin(), mI.end());
      C.inds.insert(C.inds.end(), nI.begin(), nI.end());
    } else {
      const TnTensorInfo& big = A.rank >= B.rank ? A : B;
      const TnTensorInfo& other = A.rank >= B.rank ? B : A;
      for (int id : other.inds)
        if (live[id] > 0 && std::find(big.inds.begin(), big.inds.end(), id) == big.inds.end()) C.inds.push_back(id);
      for (int id : big.inds)
        if (live[id] > 0) C.inds.push_back(id);
    }
    for (int id : C.inds) live[id]++;
    C.rank = (int)C.inds.size();
    if (C.rank > 34) return fail(TQ_ENOTSUP, "intermediate of rank " + std::to_string(C.rank) + " (slice more)");
    C.sdep = A.sdep || B.sdep;
    p->t.push_back(C);
    p->pairs.push_back({a, b});
  }
  p->root = L == 1 ? 0 : 2 * L - 2;
  // the result's open indices must equal out_inds as a set
  {
    std::set<int> got(p->t[p->root].inds.begin(), p->t[p->root].inds.end());
    std::set<int> want(p->out_inds.begin(), p->out_inds.end());
    if (got != want) return fail(TQ_EINVAL, "the tree's result indices differ from out_inds");
  }
  // forward execs (last step writes the output order requested)
  p->n_slices = int64_t(1) << p->sliced.size();
  int64_t per_slice = 0, shared = 0, max_el = 0, perm = 0;
  for (size_t s = 0; s < p->pairs.size(); ++s) {
    const int a = p->pairs[s].first, b = p->pairs[s].second, c = L + (int)s;
    std::vector<int> zi = p->t[c].inds;
    if (c == p->root && !p->out_inds.empty()) zi = p->out_inds;
    TnExec ex = make_exec(p->t[a].inds, p->t[b].inds, zi, true, csz);
    if (c == p->root) p->t[c].inds = zi;
    ex.x = a;
    ex.y = b;
    ex.z = c;
    if (ex.method == 1) {
      p->n_gemm++;
      p->gemm_flops += ex.flops;
      if (ex.permx) perm = std::max<int64_t>(perm, int64_t(1) << p->t[a].rank);
      if (ex.permy) perm = std::max<int64_t>(perm, int64_t(1) << p->t[b].rank);
    } else {
      p->n_direct++;
    }
    p->flops += ex.flops;
    p->fwd.push_back(ex);
    const int64_t sz = int64_t(1) << p->t[c].rank;
    max_el = std::max(max_el, sz);
    (p->t[c].sdep ? per_slice : shared) += sz;
  }
  for (auto& t : p->t)
    if (t.leaf >= 0 && t.sdep) per_slice += int64_t(1) << t.rank;
  p->flops *= p->n_slices;
  p->gemm_flops *= p->n_slices;
  p->max_elems = max_el;
  p->perm_elems = 2 * perm;
  // slice group: G copies of the slice-dependent tensors within the memory budget
  const int64_t budget = d->mem_budget > 0 ? d->mem_budget : (int64_t(4) << 30);
  int64_t G = d->slice_group > 0 ? d->slice_group : p->n_slices;
  G = std::min(G, p->n_slices);
  while (G > 1 && (shared + G * (per_slice + p->perm_elems)) * 2 * csz > budget) G >>= 1;
  p->G = std::max<int64_t>(G, 1);
  // store policy (Sec. 4.1 keeps the forward's intermediates for the backward pass): the
  // reverse pass can reuse what tq_tn_contract left in the workspace only when every slice's
  // intermediates are there at once, i.e. all slices run as one group within the budget
  if (d->store_policy < 0 || d->store_policy > 2) return fail(TQ_EINVAL, "store_policy must be 0, 1 or 2");
  const bool one_group = p->G >= p->n_slices;
  if (d->store_policy == TQ_TN_STORE && !one_group)
    return fail(TQ_ENOTSUP, "store policy: the memory budget cannot hold the intermediates of all " +
                                std::to_string(p->n_slices) + " slices at once (use recompute or auto)");
  p->store = d->store_policy != TQ_TN_RECOMPUTE && one_group;
  // workspace offsets (complex elements): shared tensors once, slice tensors G copies
  int64_t w = 0;
  for (auto& t : p->t) {
    if (t.leaf >= 0 && !t.sdep) continue;  // read from the leaf buffer
    t.off = w;
    w += (t.sdep ? p->G : 1) * (int64_t(1) << t.rank);
  }
  p->perm_off = w;
  w += p->G * p->perm_elems;
  p->split_off = w;  // shared by every direct step (they run one after another)
  p->split_elems = int64_t(1) << 18;
  w += p->split_elems;
  w += p->G;  // root per-slice values (if the root is shared, copies are still G)
  p->ws_fwd = w + (int64_t(1) << p->t[p->root].rank) * p->G;
  // reverse pass: environments of every tensor, G copies each
  p->env_off.assign(p->t.size(), 0);
  int64_t e = p->ws_fwd;
  for (size_t i = 0; i < p->t.size(); ++i) {
    p->env_off[i] = e;
    e += p->G * (int64_t(1) << p->t[i].rank);
  }
  p->ws_bwd = e;
  // reverse execs: D_x = contract(D_z, y), D_y = contract(D_z, x). The environment of an
  // intermediate is laid out with the indices it shares with its parent's environment as the
  // low bits, in the parent's order (so a reverse step reads D_z and writes D_x at matching
  // addresses); leaves and the root keep their own layout.
  std::vector<std::vector<int>> elay(p->t.size());
  for (size_t i = 0; i < p->t.size(); ++i) elay[i] = p->t[i].inds;
  for (size_t s = p->fwd.size(); s-- > 0;) {
    const TnExec& f = p->fwd[s];
    for (int child : {f.x, f.y}) {
      if (p->t[child].leaf >= 0) continue;
      std::vector<int> lay;
      for (int id : p->t[child].inds)
        if (std::find(elay[f.z].begin(), elay[f.z].end(), id) == elay[f.z].end()) lay.push_back(id);
      for (int id : elay[f.z])
        if (std::find(p->t[child].inds.begin(), p->t[child].inds.end(), id) != p->t[child].inds.end())
          lay.push_back(id);
      elay[child] = lay;
    }
    TnExec ex1 = make_exec(elay[f.z], p->t[f.y].inds, elay[f.x], false, csz);
    ex1.x = f.z;
    ex1.y = f.y;
    ex1.z = f.x;
    TnExec ex2 = make_exec(elay[f.z], p->t[f.x].inds, elay[f.y], false, csz);
    ex2.x = f.z;
    ex2.y = f.x;
    ex2.z = f.y;
    p->bwd.push_back(ex1);
    p->bwd.push_back(ex2);
  }
  // every sliced index must occur in some leaf
  for (int si : p->sliced)
    if (!count.count(si)) return fail(TQ_EINVAL, "sliced index " + std::to_string(si) + " is in no leaf");
  // gather tables of the sliced leaves
  std::vector<uint8_t> gt;
  for (size_t i = 0; i < p->t.size(); ++i) {
    TnTensorInfo& t = p->t[i];
    if (t.leaf < 0 || !t.sdep) continue;
    t.gather = (int)p->sliced_leaves.size();
    p->sliced_leaves.push_back((int)i);
    const int rf = t.rank + (int)t.sliced_pos.size();
    std::vector<uint8_t> row(3 * kTnMaxBits, 0);
    std::vector<char> is_sl(rf, 0);
    for (int q : t.sliced_pos) is_sl[q] = 1;
    int k = 0;
    for (int q = 0; q < rf; ++q)
      if (!is_sl[q]) row[k++] = (uint8_t)q;
    for (size_t q = 0; q < t.sliced_pos.size(); ++q) {
      row[kTnMaxBits + q] = (uint8_t)t.sliced_pos[q];
      row[2 * kTnMaxBits + q] = (uint8_t)t.sliced_bits[q];
    }
    gt.insert(gt.end(), row.begin(), row.end());
  }
  // execution segments (the workspace layout is final here)
  std::vector<DevFused> ff, bf;
  {
    auto small = [](const TnExec& ex) {
      return ex.method == 0 && ex.dev.zr <= kTnFusedMaxOut && ex.dev.zr + ex.dev.ks <= kTnFusedMaxWork;
    };
    auto operand = [&](int id, int64_t* o, int64_t* st, bool* leaf) {
      const TnTensorInfo& t = p->t[id];
      if (t.leaf >= 0 && !t.sdep) {
        *o = p->leaf_off[t.leaf];
        *st = 0;
        *leaf = true;
      } else {
        *o = t.off;
        *st = t.sdep ? (int64_t(1) << t.rank) : 0;
        *leaf = false;
      }
    };
    for (size_t k = 0; k < p->fwd.size(); ++k) {
      const TnExec& ex = p->fwd[k];
      const int shared = p->t[ex.z].sdep ? 0 : 1;
      if (small(ex)) {
        if (p->fseg.empty() || !p->fseg.back().fused || p->fseg.back().shared != shared ||
            p->fseg.back().count == kTnRunCap) {
          tq_tn_plan::Seg sg;
          sg.fused = 1;
          sg.first = (int)k;
          sg.list = (int64_t)ff.size();
          sg.shared = shared;
          p->fseg.push_back(sg);
        }
        p->fseg.back().count++;
        DevFused f{};
        bool lx, ly, lz;
        f.step = (int32_t)k;
        operand(ex.x, &f.xo, &f.xs, &lx);
        operand(ex.y, &f.yo, &f.ys, &ly);
        operand(ex.z, &f.zo, &f.zs, &lz);
        f.flags = (lx ? 1 : 0) | (ly ? 2 : 0);
        ff.push_back(f);
      } else {
        tq_tn_plan::Seg sg;
        sg.first = (int)k;
        sg.count = 1;
        sg.shared = shared;
        p->fseg.push_back(sg);
      }
    }
    for (size_t k = 0; k < p->bwd.size(); ++k) {
      const TnExec& ex = p->bwd[k];
      if (small(ex)) {
        if (p->bseg.empty() || !p->bseg.back().fused || p->bseg.back().count == kTnRunCap) {
          tq_tn_plan::Seg sg;
          sg.fused = 1;
          sg.first = (int)k;
          sg.list = (int64_t)bf.size();
          p->bseg.push_back(sg);
        }
        p->bseg.back().count++;
        DevFused f{};
        bool ly;
        f.step = (int32_t)k;
        f.xo = p->env_off[ex.x];
        f.xs = int64_t(1) << p->t[ex.x].rank;
        operand(ex.y, &f.yo, &f.ys, &ly);
        f.zo = p->env_off[ex.z];
        f.zs = int64_t(1) << p->t[ex.z].rank;
        f.flags = ly ? 2 : 0;
        bf.push_back(f);
      } else {
        tq_tn_plan::Seg sg;
        sg.first = (int)k;
        sg.count = 1;
        p->bseg.push_back(sg);
      }
    }
  }
  // order each fused run by dependency level and mark the levels (a topological order: a
  // step's operands come from leaves, earlier segments or lower levels of its run)
  auto levelize = [](std::vector<DevFused>& lst, const tq_tn_plan::Seg& sg, const std::vector<TnExec>& ex,
                     bool reverse) {
    std::map<int, int> made;  // tensor (or environment slot) -> level in this run
    std::vector<std::pair<int, int>> order;  // (level, position in the run)
    for (int i = 0; i < sg.count; ++i) {
      const TnExec& e = ex[lst[sg.list + i].step];
      int l = 0;
      auto it = made.find(e.x);
      if (it != made.end()) l = std::max(l, it->second);
      if (!reverse) {  // the reverse pass reads forward values as its y operands
        it = made.find(e.y);
        if (it != made.end()) l = std::max(l, it->second);
      }
      made[e.z] = l + 1;
      order.emplace_back(l + 1, i);
    }
    std::stable_sort(order.begin(), order.end());
    std::vector<DevFused> run;
    for (auto& o : order) run.push_back(lst[sg.list + o.second]);
    for (size_t i = 0; i < run.size();) {
      size_t j = i;
      while (j < run.size() && order[j].first == order[i].first) ++j;
      int32_t r0 = 0;
      for (size_t k = i; k < j; ++k) {
        const DevTnStep& d = ex[run[k].step].dev;
        run[k].flags &= 0xff;
        run[k].r0 = r0;
        run[k].rn = tn_wave_rounds(d.zr, d.ks);
        run[k].lw = 0;
        r0 += run[k].rn;
      }
      run[i].flags |= (int32_t)((j - i) << 8);
      run[i].lw = r0;
      i = j;
    }
    std::copy(run.begin(), run.end(), lst.begin() + sg.list);
  };
  for (const auto& sg : p->fseg)
    if (sg.fused) levelize(ff, sg, p->fwd, false);
  for (const auto& sg : p->bseg)
    if (sg.fused) levelize(bf, sg, p->bwd, true);
  std::vector<int64_t> le;
  for (int l = 0; l < L; ++l) {
    const TnTensorInfo& t = p->t[l];
    if (t.sdep) continue;
    le.push_back(p->leaf_off[l]);
    le.push_back(p->env_off[l]);
    le.push_back(int64_t(1) << t.rank);
  }
  p->n_leaf_env = (int)(le.size() / 3);
  // device copies of the step tables (none for a host-only plan)
  p->host_only = !ctx;
  if (ctx) {
    std::vector<DevTnStep> fs, bs;
    std::vector<uint8_t> pt;
    for (auto& f : p->fwd) {
      fs.push_back(f.dev);
      std::vector<uint8_t> px = f.px, py = f.py;
      px.resize(kTnMaxBits, 0);
      py.resize(kTnMaxBits, 0);
      pt.insert(pt.end(), px.begin(), px.end());
      pt.insert(pt.end(), py.begin(), py.end());
    }
    for (auto& b : p->bwd) bs.push_back(b.dev);
    auto up = [](const void* src, size_t bytes, void** dst) -> tq_status {
      TQ_HIP(hipMalloc(dst, std::max<size_t>(bytes, 64)));
      if (bytes) TQ_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
      return TQ_OK;
    };
    TQ_TRY(up(fs.data(), fs.size() * sizeof(DevTnStep), &p->d_fwd));
    TQ_TRY(up(bs.data(), bs.size() * sizeof(DevTnStep), &p->d_bwd));
    TQ_TRY(up(pt.data(), pt.size(), &p->d_perm));
    TQ_TRY(up(gt.data(), gt.size(), &p->d_gather));
    TQ_TRY(up(ff.data(), ff.size() * sizeof(DevFused), &p->d_ffused));
    TQ_TRY(up(bf.data(), bf.size() * sizeof(DevFused), &p->d_bfused));
    TQ_TRY(up(le.data(), le.size() * sizeof(int64_t), &p->d_leaf_env));
  }
  *out = p.release();
  return TQ_OK;
}

void tq_tn_plan_destroy(tq_tn_plan* plan) { delete plan; }

int64_t tq_tn_leaf_elems(const tq_tn_plan* p) { return p ? p->leaf_elems : -1; }

int64_t tq_tn_leaf_offset(const tq_tn_plan* p, int32_t leaf) {
  if (!p || leaf < 0 || leaf >= p->n_leaves) return -1;
  return p->leaf_off[leaf];
}

int32_t tq_tn_plan_stores(const tq_tn_plan* p) { return p ? (p->store ? 1 : 0) : -1; }

tq_status tq_tn_plan_segments(const tq_tn_plan* p, int64_t out[4]) {
  if (!p || !out) return fail(TQ_EINVAL, "null argument");
  int64_t ff = 0, bf = 0;
  for (const auto& sg : p->fseg) ff += sg.fused;
  for (const auto& sg : p->bseg) bf += sg.fused;
  out[0] = (int64_t)p->fseg.size();
  out[1] = ff;
  out[2] = (int64_t)p->bseg.size();
  out[3] = bf;
  return TQ_OK;
}

int64_t tq_tn_workspace(const tq_tn_plan* p, int32_t backward) {
  if (!p) return -1;
  const int csz = p->dtype == TQ_C64 ? 8 : 16;
  return (backward ? p->ws_bwd : p->ws_fwd) * csz + 1024;
}

tq_status tq_tn_plan_info(const tq_tn_plan* p, int64_t out[8]) {
  if (!p || !out) return fail(TQ_EINVAL, "null argument");
  out[0] = (int64_t)p->fwd.size();
  out[1] = p->n_direct;
  out[2] = p->n_gemm;
  out[3] = p->n_slices;
  out[4] = p->G;
  out[5] = p->flops;
  out[6] = p->gemm_flops;
  out[7] = p->max_elems;
  return TQ_OK;
}

}  // extern "C"

namespace tq {

// ---- execution: see tn_exec below ----

}  // namespace tq

namespace tq {

static inline unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 4096));
}

template <typename T>
struct TnRun {
  using C = typename Cx<T>::type;
  const tq_tn_plan* p;
  const C* leaves;
  C* ws;
  hipStream_t st;
  int64_t s0 = 0;  // first slice of the group
  int64_t g = 1;   // slices in this group
  // forward storage of tensor i: pointer and per-copy stride (0 = shared by the group)
  C* tptr(int i, int64_t* stride) const {
    const TnTensorInfo& t = p->t[i];
    if (t.leaf >= 0 && !t.sdep) {
      *stride = 0;
      return const_cast<C*>(leaves) + p->leaf_off[t.leaf];
    }
    *stride = t.sdep ? (int64_t(1) << t.rank) : 0;
    return ws + t.off;
  }
  C* eptr(int i) const { return ws + p->env_off[i]; }  // environments: g copies, stride = size
  int64_t esz(int i) const { return int64_t(1) << p->t[i].rank; }
};

// Launch shape of a direct step: 2^tb lanes per output, enough lanes in total (about 2^16)
// to fill the machine, at most 256 per output; rb work-groups over the output rounds; a step
// with few outputs and many summed assignments also splits its summed range over 2^kb
// chunks of work-groups (up to about 2^17 lanes, within the plan's partial-sum region).
// Work-groups of one direct step at most: past that, a work-group takes several output
// rounds and builds its offset tables once for all of them (2048 measured best of 256 to
// 16384 on the 75 QAOA p = 4 networks; 256 starves the device of parallel work).
constexpr int64_t kTnMaxRoundBlocks = 2048;

static void direct_shape(const DevTnStep& h, int64_t copies, int64_t split_elems, int* tbp, int* kbp, unsigned* rbp) {
  const int zr = h.zr, ks = h.ks;
  int tb = std::max(0, 16 - zr);
  tb = std::min(tb, std::min(8, ks));
  const int64_t nz = int64_t(1) << zr;
  const int64_t gpb = 256 >> tb;
  const int kt = std::min(ks, kTnTabBits);
  int kb = 0;
  while (kb < ks - kt && (nz << (tb + kb)) * copies < (int64_t(1) << 17) && (nz << (kb + 1)) * copies <= split_elems)
    ++kb;
  // the wide form (kb = 0 only) takes kTnWideOpl outputs per lane and round
  const int64_t per = (kb == 0 && tn_wide_form(tb, ks)) ? gpb * kTnWideOpl : gpb;
  const int64_t rounds = (nz + per - 1) / per;
  *tbp = tb;
  *kbp = kb;
  *rbp = (unsigned)std::max<int64_t>(1, std::min<int64_t>(rounds, kTnMaxRoundBlocks));
}

// One large direct step over the device (shape from direct_shape).
template <typename T>
static tq_status tn_direct(TnRun<T>& R, const DevTnStep* dstep, const DevTnStep& h, const typename Cx<T>::type* x,
                           int64_t xs, const typename Cx<T>::type* y, int64_t ys, typename Cx<T>::type* z, int64_t zs,
                           int64_t copies) {
  using C = typename Cx<T>::type;
  int tb, kb;
  unsigned rb;
  direct_shape(h, copies, R.p->split_elems, &tb, &kb, &rb);
  const int64_t nz = int64_t(1) << h.zr;
  C* P = R.ws + R.p->split_off;
  const int64_t ps = nz << kb;
  for (int64_t c0 = 0; c0 < copies; c0 += 65535) {
    const int64_t cn = std::min<int64_t>(65535, copies - c0);
    hipLaunchKernelGGL(tn_direct_kernel<T>, dim3(rb << kb, (unsigned)cn), dim3(256), 0, R.st, dstep, x + xs * c0, xs,
                       y + ys * c0, ys, z + zs * c0, zs, tb, kb, (int)rb, P, ps);
    if (kb > 0)
      hipLaunchKernelGGL(tn_chunk_sum_kernel<T>, dim3(grid_for(nz), (unsigned)cn), dim3(256), 0, R.st, P, ps,
                         z + zs * c0, zs, nz, 1 << kb);
  }
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

// A run of small steps: one work-group per slice copy (grid x; copies <= 2^24).
template <typename T>
static tq_status tn_fused(TnRun<T>& R, const DevTnStep* steps, const void* list, int n, int64_t copies) {
  if (n > kTnRunCap) return fail(TQ_EINVAL, "fused run longer than the LDS staging holds");
  hipLaunchKernelGGL(tn_fused_kernel<T>, dim3((unsigned)copies), dim3(kTnFusedThreads), 0, R.st, steps,
                     (const DevFused*)list, n,
                     R.leaves, R.ws);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

template <typename T>
static tq_status tn_fwd_wide(TnRun<T>& R, const tq_tn_plan::Seg& sg);

template <typename T>
static tq_status tn_forward_group(TnRun<T>& R) {
  const tq_tn_plan* p = R.p;
  // sliced leaves: restrict each to the group's slices
  for (int li : p->sliced_leaves) {
    const TnTensorInfo& t = p->t[li];
    const uint8_t* tab = (const uint8_t*)p->d_gather + (size_t)t.gather * 3 * kTnMaxBits;
    const int64_t n = int64_t(1) << t.rank;
    hipLaunchKernelGGL(tn_slice_gather_kernel<T>, dim3(grid_for(n), (unsigned)R.g), dim3(256), 0, R.st,
                       R.leaves + p->leaf_off[t.leaf], R.ws + t.off, t.rank, tab, tab + kTnMaxBits,
                       tab + 2 * kTnMaxBits, (int)t.sliced_pos.size(), R.s0);
    TQ_HIP(hipGetLastError());
  }
  for (const tq_tn_plan::Seg& sg : p->fseg) {
    if (sg.fused) {
      TQ_TRY(tn_fused<T>(R, (const DevTnStep*)p->d_fwd, (const DevFused*)p->d_ffused + sg.list, sg.count,
                         sg.shared ? 1 : R.g));
      continue;
    }
    TQ_TRY(tn_fwd_wide<T>(R, sg));
  }
  return TQ_OK;
}

// One large forward step (a segment that is not a fused run).
template <typename T>
static tq_status tn_fwd_wide(TnRun<T>& R, const tq_tn_plan::Seg& sg) {
  using C = typename Cx<T>::type;
  const tq_tn_plan* p = R.p;
  {
    const size_t s = (size_t)sg.first;
    const TnExec& ex = p->fwd[s];
    int64_t xs, ys, zs;
    const C* x = R.tptr(ex.x, &xs);
    const C* y = R.tptr(ex.y, &ys);
    C* z = R.tptr(ex.z, &zs);
    const int64_t copies = p->t[ex.z].sdep ? R.g : 1;
    if (ex.method == 1) {
      {
        // permute X -> [b][m][k], Y -> [b][k][n] into the group's scratch, then GEMM per copy
        C* pbuf = R.ws + p->perm_off;
        const int64_t half = p->perm_elems / 2;
        const uint8_t* perm = (const uint8_t*)p->d_perm + s * 2 * kTnMaxBits;
        const C* xa = x;
        const C* ya = y;
        int64_t xas = xs, yas = ys;
        if (ex.permx) {
          const int r = p->t[ex.x].rank;
          const int64_t cx = xs ? copies : 1;
          hipLaunchKernelGGL(tn_permute_kernel<T>, dim3(grid_for(int64_t(1) << r), (unsigned)cx), dim3(256), 0, R.st,
                             x, xs, pbuf, p->perm_elems, perm, r);
          xa = pbuf;
          xas = xs ? p->perm_elems : 0;
        }
        if (ex.permy) {
          const int r = p->t[ex.y].rank;
          const int64_t cy = ys ? copies : 1;
          hipLaunchKernelGGL(tn_permute_kernel<T>, dim3(grid_for(int64_t(1) << r), (unsigned)cy), dim3(256), 0, R.st,
                             y, ys, pbuf + half, p->perm_elems, perm + kTnMaxBits, r);
          ya = pbuf + half;
          yas = ys ? p->perm_elems : 0;
        }
        TQ_HIP(hipGetLastError());
        for (int64_t c = 0; c < copies; ++c) {
          const dim3 grid((unsigned)(ex.N / 32), (unsigned)(ex.M / 64), (unsigned)ex.B);
          if constexpr (sizeof(T) == 4) {
            if (ex.M % 128 == 0 && ex.N % 64 == 0 && ex.K % 16 == 0)  // the large tile
              hipLaunchKernelGGL(tn_cgemm_mfma128_kernel, dim3((unsigned)(ex.N / 64), (unsigned)(ex.M / 128),
                                 (unsigned)ex.B), dim3(256), 0, R.st, (const float2*)(xa + xas * c), ex.M * ex.K,
                                 (const float2*)(ya + yas * c), ex.K * ex.N, (float2*)(z + zs * c), ex.M * ex.N,
                                 (int)ex.M, (int)ex.N, (int)ex.K);
            else
              hipLaunchKernelGGL(tn_cgemm_mfma_kernel, grid, dim3(256), 0, R.st, (const float2*)(xa + xas * c),
                                 ex.M * ex.K, (const float2*)(ya + yas * c), ex.K * ex.N, (float2*)(z + zs * c),
                                 ex.M * ex.N, (int)ex.M, (int)ex.N, (int)ex.K);
          } else {
            if (ex.M % 128 == 0 && ex.N % 64 == 0)  // the large tile
              hipLaunchKernelGGL(tn_zgemm_mfma128_kernel, dim3((unsigned)(ex.N / 64), (unsigned)(ex.M / 128),
                                 (unsigned)ex.B), dim3(256), 0, R.st, (const double2*)(xa + xas * c), ex.M * ex.K,
                                 (const double2*)(ya + yas * c), ex.K * ex.N, (double2*)(z + zs * c), ex.M * ex.N,
                                 (int)ex.M, (int)ex.N, (int)ex.K);
            else
              hipLaunchKernelGGL(tn_zgemm_mfma_kernel, grid, dim3(256), 0, R.st, (const double2*)(xa + xas * c),
                                 ex.M * ex.K, (const double2*)(ya + yas * c), ex.K * ex.N, (double2*)(z + zs * c),
                                 ex.M * ex.N, (int)ex.M, (int)ex.N, (int)ex.K);
          }
        }
        TQ_HIP(hipGetLastError());
        return TQ_OK;
      }
    }
    TQ_TRY(tn_direct<T>(R, (const DevTnStep*)p->d_fwd + s, ex.dev, x, xs, y, ys, z, zs, copies));
  }
  return TQ_OK;
}

template <typename T>
static tq_status tn_contract_t(tq_ctx* ctx, const tq_tn_plan* p, const void* d_leaves, void* d_out, void* d_work,
                               int64_t work_bytes, hipStream_t stream) {
  using C = typename Cx<T>::type;
  (void)ctx;
  if (work_bytes < tq_tn_workspace(p, 0)) return fail(TQ_EWORKSPACE, "tn workspace too small");
  TnRun<T> R{p, (const C*)d_leaves, (C*)d_work, stream};
  const int64_t nout = int64_t(1) << p->t[p->root].rank;
  if (p->fwd.empty()) {  // a single leaf
    hipLaunchKernelGGL(tn_sum_copies_kernel<T>, dim3(grid_for(nout)), dim3(256), 0, stream, (const C*)d_leaves, 0, 1,
                       (C*)d_out, nout, 0);
    TQ_HIP(hipGetLastError());
    return TQ_OK;
  }
  for (int64_t s0 = 0; s0 < p->n_slices; s0 += p->G) {
    R.s0 = s0;
    R.g = std::min<int64_t>(p->G, p->n_slices - s0);
    TQ_TRY(tn_forward_group<T>(R));
    int64_t rs;
    const C* root = R.tptr(p->root, &rs);
    hipLaunchKernelGGL(tn_sum_copies_kernel<T>, dim3(grid_for(nout)), dim3(256), 0, stream, root, rs, (int)R.g,
                       (C*)d_out, nout, s0 > 0 ? 1 : 0);
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}

template <typename T>
static tq_status tn_backward_t(tq_ctx* ctx, const tq_tn_plan* p, const void* d_leaves, const void* d_grad_out,
                               void* d_grad, void* d_work, int64_t work_bytes, hipStream_t stream) {
  using C = typename Cx<T>::type;
  (void)ctx;
  if (work_bytes < tq_tn_workspace(p, 1)) return fail(TQ_EWORKSPACE, "tn workspace too small for the reverse pass");
  TnRun<T> R{p, (const C*)d_leaves, (C*)d_work, stream};
  C* grad = (C*)d_grad;
  hipLaunchKernelGGL(tn_fill_kernel<T>, dim3(grid_for(p->leaf_elems)), dim3(256), 0, stream, grad, p->leaf_elems,
                     C{0, 0});
  TQ_HIP(hipGetLastError());
  const int64_t nout = int64_t(1) << p->t[p->root].rank;
  if (p->fwd.empty()) {
    hipLaunchKernelGGL(tn_sum_copies_kernel<T>, dim3(grid_for(nout)), dim3(256), 0, stream, (const C*)d_grad_out, 0, 1,
                       grad, nout, 0);
    TQ_HIP(hipGetLastError());
    return TQ_OK;
  }
  for (int64_t s0 = 0; s0 < p->n_slices; s0 += p->G) {
    R.s0 = s0;
    R.g = std::min<int64_t>(p->G, p->n_slices - s0);
    // store policy: the intermediates of the preceding tq_tn_contract are still in the
    // workspace (one group holds every slice); recompute policy: rebuild them here
    if (!p->store) TQ_TRY(tn_forward_group<T>(R));
    // environment of the result: the upstream value, one copy per slice
    hipLaunchKernelGGL(tn_broadcast_kernel<T>, dim3(grid_for(nout), (unsigned)R.g), dim3(256), 0, stream,
                       (const C*)d_grad_out, R.eptr(p->root), nout);
    TQ_HIP(hipGetLastError());
    for (const tq_tn_plan::Seg& sg : p->bseg) {
      if (sg.fused) {
        TQ_TRY(tn_fused<T>(R, (const DevTnStep*)p->d_bwd, (const DevFused*)p->d_bfused + sg.list, sg.count, R.g));
        continue;
      }
      const size_t k = (size_t)sg.first;
      const TnExec& ex = p->bwd[k];
      int64_t ys;
      const C* y = R.tptr(ex.y, &ys);
      TQ_TRY(tn_direct<T>(R, (const DevTnStep*)p->d_bwd + k, ex.dev, R.eptr(ex.x), R.esz(ex.x), y, ys, R.eptr(ex.z),
                          R.esz(ex.z), R.g));
    }
    // leaf environments -> gradient buffer (sum over the group's slices, in order)
    if (p->n_leaf_env > 0) {
      hipLaunchKernelGGL(tn_leaf_env_kernel<T>, dim3((unsigned)p->n_leaf_env), dim3(256), 0, stream,
                         (const int64_t*)p->d_leaf_env, (const C*)R.ws, (int)R.g, grad);
      TQ_HIP(hipGetLastError());
    }
    for (int li : p->sliced_leaves) {
      const TnTensorInfo& t = p->t[li];
      const int64_t n = int64_t(1) << t.rank;
      const uint8_t* tab = (const uint8_t*)p->d_gather + (size_t)t.gather * 3 * kTnMaxBits;
      hipLaunchKernelGGL(tn_slice_scatter_kernel<T>, dim3(grid_for(n)), dim3(256), 0, stream, R.eptr(li), n,
                         (int)R.g, grad + p->leaf_off[t.leaf], t.rank, tab, tab + kTnMaxBits, tab + 2 * kTnMaxBits,
                         (int)t.sliced_pos.size(), s0);
    }
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}

// host tables of a circuit network's leaves
static tq_status leaf_table(tq_ctx* ctx, const tq_tn_plan* p, const tq_gate* gates, int32_t n_gates,
                            const tq_tn_leaf* lv, int32_t n_const, std::vector<DevLeaf>& out) {
  (void)ctx;
  out.resize(p->n_leaves);
  for (int l = 0; l < p->n_leaves; ++l) {
    const tq_tn_leaf& x = lv[l];
    const int rank = (int)p->t[l].inds.size() + (int)p->t[l].sliced_pos.size();
    DevLeaf d{x.kind, x.gate, x.conj, x.const_off, p->leaf_off[l], x.flip, 0};
    static const int want_rank[5] = {-1, 2, 1, 2, 4};
    if (x.kind < 0 || x.kind > 4) return fail(TQ_EINVAL, "leaf " + std::to_string(l) + ": unknown kind");
    if (x.flip >= (1 << std::min(rank, 15)))
      return fail(TQ_EINVAL, "leaf " + std::to_string(l) + ": flip mask beyond the leaf's rank");
    if (x.kind == 0) {
      if (x.const_off < 0 || x.const_off + (1 << rank) > n_const)
        return fail(TQ_EINVAL, "leaf " + std::to_string(l) + ": constant values out of range");
      d.gate = 1 << rank;  // entry count for constants
    } else {
      if (x.gate < 0 || x.gate >= n_gates) return fail(TQ_EINVAL, "leaf " + std::to_string(l) + ": bad gate index");
      if (rank != want_rank[x.kind]) return fail(TQ_EINVAL, "leaf " + std::to_string(l) + ": rank does not fit kind");
    }
    out[l] = d;
  }
  return TQ_OK;
}

// Checks one network's leaf-build arguments and, when `it` is given, fills its launch record
// (the device tables come from the context's content-keyed cache).
static tq_status leaf_build_item(tq_ctx* ctx, const tq_tn_plan* plan, const tq_gate* gates, int32_t n_gates,
                                 const tq_tn_leaf* leaves, const double* const_vals, int32_t n_const,
                                 const void* d_params, void* d_leaves, DevLeafItem* it) {
  if (!plan || !leaves || !d_leaves) return fail(TQ_EINVAL, "null argument");
  TQ_TRY(runnable(plan));
  if (n_gates > 0 && (!gates || !d_params)) return fail(TQ_EINVAL, "null gates or params");
  if (n_const > 0 && !const_vals) return fail(TQ_EINVAL, "null constant values");
  TQ_TRY(validate_gates(gates, n_gates, 1 << 30, 0x7fffffff));
  std::vector<DevLeaf> dl;
  TQ_TRY(leaf_table(ctx, plan, gates, n_gates, leaves, n_const, dl));
  if (!it) return TQ_OK;
  void *dlv, *dg, *dc;
  TQ_TRY(cached_table(ctx, dl.data(), dl.size() * sizeof(DevLeaf), &dlv));
  TQ_TRY(cached_table(ctx, gates, (size_t)n_gates * sizeof(tq_gate), &dg));
  TQ_TRY(cached_table(ctx, const_vals, (size_t)n_const * 2 * sizeof(double), &dc));
  *it = DevLeafItem{(const DevLeaf*)dlv, (const tq_gate*)dg, (const double*)dc, d_params, d_leaves, plan->n_leaves, 0};
  return TQ_OK;
}

// The same for one network's parameter gradient: the parameter -> (leaf, angle) lists, in
// leaf order.
static tq_status param_grad_item(tq_ctx* ctx, const tq_tn_plan* plan, const tq_gate* gates, int32_t n_gates,
                                 const tq_tn_leaf* leaves, const void* d_params, int32_t n_params,
                                 const void* d_grad_leaves, void* d_grad_params, DevPgItem* it) {
  if (!plan || !leaves || !d_grad_leaves || !d_grad_params) return fail(TQ_EINVAL, "null argument");
  TQ_TRY(runnable(plan));
  if (n_params < 0) return fail(TQ_EINVAL, "negative n_params");
  TQ_TRY(validate_gates(gates, n_gates, 1 << 30, n_params));
  std::vector<DevLeaf> dl;
  TQ_TRY(leaf_table(ctx, plan, gates, n_gates, leaves, 1 << 30, dl));
  if (!it) return TQ_OK;
  std::vector<std::vector<std::pair<int, int>>> by(n_params);
  for (int l = 0; l < plan->n_leaves; ++l) {
    if (leaves[l].kind == 0) continue;
    const tq_gate& g = gates[leaves[l].gate];
    for (int j = 0; j < gate_n_angles(g.op); ++j)
      if (g.pidx[j] >= 0) by[g.pidx[j]].push_back({l, j});
  }
  std::vector<int32_t> ptr(1, 0), ent;
  for (int q = 0; q < n_params; ++q) {
    for (auto& e : by[q]) {
      ent.push_back(e.first);
      ent.push_back(e.second);
    }
    ptr.push_back((int32_t)(ent.size() / 2));
  }
  void *dlv, *dg, *dp, *de;
  TQ_TRY(cached_table(ctx, dl.data(), dl.size() * sizeof(DevLeaf), &dlv));
  TQ_TRY(cached_table(ctx, gates, (size_t)n_gates * sizeof(tq_gate), &dg));
  TQ_TRY(cached_table(ctx, ptr.data(), ptr.size() * sizeof(int32_t), &dp));
  TQ_TRY(cached_table(ctx, ent.data(), std::max<size_t>(ent.size(), 1) * sizeof(int32_t), &de));
  *it = DevPgItem{(const DevLeaf*)dlv, (const tq_gate*)dg, d_params, (const int32_t*)dp, (const int32_t*)de,
                  d_grad_leaves, d_grad_params, n_params, 0};
  return TQ_OK;
}

}  // namespace tq

extern "C" {

tq_status tq_tn_contract(tq_ctx* ctx, const tq_tn_plan* plan, const void* d_leaves, void* d_out, void* d_work,
                         int64_t work_bytes, void* stream) {
  if (!ctx || !plan || !d_leaves || !d_out || !d_work) return fail(TQ_EINVAL, "null argument");
  TQ_TRY(runnable(plan));
  if (plan->dtype == TQ_C64)
    return tn_contract_t<float>(ctx, plan, d_leaves, d_out, d_work, work_bytes, (hipStream_t)stream);
  return tn_contract_t<double>(ctx, plan, d_leaves, d_out, d_work, work_bytes, (hipStream_t)stream);
}

tq_status tq_tn_backward(tq_ctx* ctx, const tq_tn_plan* plan, const void* d_leaves, const void* d_grad_out,
                         void* d_grad_leaves, void* d_work, int64_t work_bytes, void* stream) {
  if (!ctx || !plan || !d_leaves || !d_grad_out || !d_grad_leaves || !d_work) return fail(TQ_EINVAL, "null argument");
  TQ_TRY(runnable(plan));
  if (plan->dtype == TQ_C64)
    return tn_backward_t<float>(ctx, plan, d_leaves, d_grad_out, d_grad_leaves, d_work, work_bytes,
                                (hipStream_t)stream);
  return tn_backward_t<double>(ctx, plan, d_leaves, d_grad_out, d_grad_leaves, d_work, work_bytes,
                               (hipStream_t)stream);
}

}  // extern "C"

namespace tq {

// One large reverse step (a segment that is not a fused run).
template <typename T>
static tq_status tn_bwd_wide(TnRun<T>& R, const tq_tn_plan::Seg& sg) {
  using C = typename Cx<T>::type;
  const tq_tn_plan* p = R.p;
  const size_t k = (size_t)sg.first;
  const TnExec& ex = p->bwd[k];
  int64_t ys;
  const C* y = R.tptr(ex.y, &ys);
  return tn_direct<T>(R, (const DevTnStep*)p->d_bwd + k, ex.dev, R.eptr(ex.x), R.esz(ex.x), y, ys, R.eptr(ex.z),
                      R.esz(ex.z), R.g);
}

// Many unsliced networks in rounds: in round r every network runs its r-th segment; the
// fused runs of a round share one launch (one work-group per network), large steps launch
// on their own. Item tables of every round are built first and uploaded in one copy.
template <typename T>
static tq_status tn_batch_t(tq_ctx* ctx, const std::vector<const tq_tn_plan*>& P, const std::vector<const void*>& L,
                            const std::vector<const void*>& G, const std::vector<void*>& O,
                            const std::vector<void*>& Wk, int mode, hipStream_t stream) {
  using C = typename Cx<T>::type;
  const size_t n = P.size();
  std::vector<TnRun<T>> R;
  for (size_t i = 0; i < n; ++i) R.push_back(TnRun<T>{P[i], (const C*)L[i], (C*)Wk[i], stream});
  std::vector<unsigned char> blob;
  auto put = [&](const void* x, size_t bytes) {
    const size_t off = blob.size();
    blob.insert(blob.end(), (const unsigned char*)x, (const unsigned char*)x + bytes);
    return off;
  };
  // per round: the fused runs (one launch), and the plain direct steps of every network
  // (one multi-network launch, up to kTnMultiMaxItems per launch; the rest launch alone)
  struct DirectRound {  // one multi-network launch: kind 0 direct steps, 1 chunk sums
    size_t first_off = 0, items_off = 0;
    int count = 0, kind = 0;
    int64_t blocks = 0;
  };
  std::vector<std::vector<char>> fdone, bdone;  // [round][network]: run by a multi launch
  bool bad_run = false;                         // a fused run longer than the LDS staging holds
  auto rounds = [&](bool fwd, std::vector<std::pair<size_t, int>>& tab, std::vector<std::vector<DirectRound>>& dtab,
                    std::vector<std::vector<char>>& done) {
    size_t rmax = 0;
    for (size_t i = 0; i < n; ++i) rmax = std::max(rmax, (fwd ? P[i]->fseg : P[i]->bseg).size());
    for (size_t r = 0; r < rmax; ++r) {
      const size_t off = blob.size();
      int cnt = 0;
      for (size_t i = 0; i < n; ++i) {
        const auto& segs = fwd ? P[i]->fseg : P[i]->bseg;
        if (r >= segs.size() || !segs[r].fused) continue;
        DevFusedItem it{};
        it.steps = (const DevTnStep*)(fwd ? P[i]->d_fwd : P[i]->d_bwd);
        it.list = (const DevFused*)(fwd ? P[i]->d_ffused : P[i]->d_bfused) + segs[r].list;
        it.leaves = L[i];
        it.ws = Wk[i];
        it.n = segs[r].count;
        if (it.n > kTnRunCap) bad_run = true;
        put(&it, sizeof it);
        ++cnt;
      }
      tab.push_back({off, cnt});
      // direct steps of this round
      std::vector<DevDirectItem> items;
      std::vector<DevChunkItem> chunks;
      std::vector<char> dn(n, 0);
      for (size_t i = 0; i < n; ++i) {
        const auto& segs = fwd ? P[i]->fseg : P[i]->bseg;
        if (r >= segs.size() || segs[r].fused) continue;
        const size_t k = (size_t)segs[r].first;
        const TnExec& ex = fwd ? P[i]->fwd[k] : P[i]->bwd[k];
        if (ex.method != 0) continue;
        int tb, kb;
        unsigned rb;
        direct_shape(ex.dev, 1, P[i]->split_elems, &tb, &kb, &rb);
        DevDirectItem d{};
        d.st = (const DevTnStep*)(fwd ? P[i]->d_fwd : P[i]->d_bwd) + k;
        int64_t st;
        if (fwd) {
          d.x = R[i].tptr(ex.x, &st);
          d.y = R[i].tptr(ex.y, &st);
          d.z = R[i].tptr(ex.z, &st);
        } else {
          d.x = R[i].eptr(ex.x);
          d.y = R[i].tptr(ex.y, &st);
          d.z = R[i].eptr(ex.z);
        }
        d.P = R[i].ws + P[i]->split_off;
        d.tb = tb;
        d.rb = (int32_t)rb;
        d.kb = kb;
        items.push_back(d);
        if (kb > 0) {
          DevChunkItem ci{};
          ci.P = d.P;
          ci.z = d.z;
          ci.nz = int64_t(1) << ex.dev.zr;
          ci.nchunks = 1 << kb;
          chunks.push_back(ci);
        }
        dn[i] = 1;
      }
      std::vector<DirectRound> drs;
      auto pack = [&](auto& vec, auto blocks_of, int kind) {
        using Item = typename std::decay<decltype(vec[0])>::type;
        for (size_t a = 0; a < vec.size(); a += kTnMultiMaxItems) {
          const size_t b = std::min(vec.size(), a + (size_t)kTnMultiMaxItems);
          DirectRound dr;
          std::vector<int32_t> first;
          int64_t blocks = 0;
          for (size_t j = a; j < b; ++j) {
            first.push_back((int32_t)blocks);
            blocks += blocks_of(vec[j]);
          }
          first.push_back((int32_t)blocks);
          dr.first_off = put(first.data(), first.size() * sizeof(int32_t));
          while (blob.size() % 16) blob.push_back(0);
          dr.items_off = put(vec.data() + a, (b - a) * sizeof(Item));
          dr.count = (int)(b - a);
          dr.blocks = blocks;
          dr.kind = kind;
          drs.push_back(dr);
        }
      };
      pack(items, [](const DevDirectItem& d) { return (int64_t)d.rb << d.kb; }, 0);
      pack(chunks, [](const DevChunkItem& c) { return (int64_t)grid_for(c.nz); }, 1);
      dtab.push_back(drs);
      done.push_back(dn);
    }
  };
  std::vector<std::pair<size_t, int>> ftab, btab;
  std::vector<std::vector<DirectRound>> fdt, bdt;
  rounds(true, ftab, fdt, fdone);
  size_t head_off = 0, tail_off = 0;
  if (mode == 0) {
    tail_off = blob.size();
    for (size_t i = 0; i < n; ++i) {
      DevCopyItem c{(const C*)Wk[i] + P[i]->t[P[i]->root].off, O[i], int64_t(1) << P[i]->t[P[i]->root].rank};
      put(&c, sizeof c);
    }
  } else {
    head_off = blob.size();
    for (size_t i = 0; i < n; ++i) {
      DevCopyItem c{G[i], (C*)Wk[i] + P[i]->env_off[P[i]->root], int64_t(1) << P[i]->t[P[i]->root].rank};
      put(&c, sizeof c);
    }
    rounds(false, btab, bdt, bdone);
    tail_off = blob.size();
    for (size_t i = 0; i < n; ++i) {
      DevEnvItem e{(const int64_t*)P[i]->d_leaf_env, Wk[i], O[i], P[i]->n_leaf_env, 0};
      put(&e, sizeof e);
    }
  }
  if (bad_run) return fail(TQ_EINVAL, "fused run longer than the LDS staging holds");
  if (!ctx->side) {
    TQ_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    TQ_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    TQ_HIP(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  }
  void* dev;
  TQ_TRY(stage_upload(ctx, S_TNB, blob.data(), blob.size(), stream, &dev));
  const unsigned char* db = (const unsigned char*)dev;
  auto run_rounds = [&](bool fwd, const std::vector<std::pair<size_t, int>>& tab,
                        const std::vector<std::vector<DirectRound>>& dtab,
                        const std::vector<std::vector<char>>& done) -> tq_status {
    for (size_t r = 0; r < tab.size(); ++r) {
      // the fused runs and the direct steps of a round belong to different networks: when a
      // round has both, the direct launches go to the context's second stream (forked from and
      // joined back into the caller's stream), so the latency-bound runs on a few CUs overlap
      // the bandwidth-bound steps
      const bool fork = tab[r].second > 0 && !dtab[r].empty();
      hipStream_t ds = stream;
      if (fork) {
        TQ_HIP(hipEventRecord(ctx->ev_fork, stream));
        TQ_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
        ds = ctx->side;
      }
      for (const DirectRound& dr : dtab[r]) {  // direct launches first, then their chunk sums
        if (dr.kind == 0)
          hipLaunchKernelGGL(tn_direct_multi_kernel<T>, dim3((unsigned)dr.blocks), dim3(256), 0, ds,
                             (const int32_t*)(db + dr.first_off), (const DevDirectItem*)(db + dr.items_off), dr.count);
        else
          hipLaunchKernelGGL(tn_chunk_sum_multi_kernel<T>, dim3((unsigned)dr.blocks), dim3(256), 0, ds,
                             (const int32_t*)(db + dr.first_off), (const DevChunkItem*)(db + dr.items_off), dr.count);
        TQ_HIP(hipGetLastError());
      }
      if (tab[r].second > 0) {
        hipLaunchKernelGGL(tn_fused_multi_kernel<T>, dim3((unsigned)tab[r].second), dim3(kTnFusedThreads), 0, stream,
                           (const DevFusedItem*)(db + tab[r].first));
        TQ_HIP(hipGetLastError());
      }
      if (fork) {
        TQ_HIP(hipEventRecord(ctx->ev_join, ctx->side));
        TQ_HIP(hipStreamWaitEvent(stream, ctx->ev_join, 0));
      }
      for (size_t i = 0; i < n; ++i) {
        const auto& segs = fwd ? P[i]->fseg : P[i]->bseg;
        if (r < segs.size() && !segs[r].fused && !done[r][i])
          TQ_TRY(fwd ? tn_fwd_wide<T>(R[i], segs[r]) : tn_bwd_wide<T>(R[i], segs[r]));
      }
    }
    return TQ_OK;
  };
  TQ_TRY(run_rounds(true, ftab, fdt, fdone));
  if (mode == 0) {
    hipLaunchKernelGGL(tn_copy_multi_kernel<T>, dim3((unsigned)n), dim3(256), 0, stream,
                       (const DevCopyItem*)(db + tail_off));
    TQ_HIP(hipGetLastError());
    return TQ_OK;
  }
  hipLaunchKernelGGL(tn_copy_multi_kernel<T>, dim3((unsigned)n), dim3(256), 0, stream,
                     (const DevCopyItem*)(db + head_off));
  TQ_HIP(hipGetLastError());
  TQ_TRY(run_rounds(false, btab, bdt, bdone));
  hipLaunchKernelGGL(tn_env_multi_kernel<T>, dim3((unsigned)n), dim3(256), 0, stream,
                     (const DevEnvItem*)(db + tail_off));
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

// Shared driver of the batched calls: unsliced plans in rounds, the rest one by one.
static tq_status tn_batch(tq_ctx* ctx, int32_t n, const tq_tn_plan* const* plans, const void* const* d_leaves,
                          const void* const* d_gout, void* const* d_out, void* const* d_work,
                          const int64_t* work_bytes, int mode, hipStream_t stream) {
  if (!ctx || n < 0 || (n > 0 && (!plans || !d_leaves || !d_out || !d_work || !work_bytes)))
    return fail(TQ_EINVAL, "null argument");
  if (mode == 1 && n > 0 && !d_gout) return fail(TQ_EINVAL, "null upstream values");
  std::vector<const tq_tn_plan*> P[2];
  std::vector<const void*> L[2], G[2];
  std::vector<void*> O[2], Wk[2];
  std::vector<int> rest;
  for (int i = 0; i < n; ++i) {
    const tq_tn_plan* p = plans[i];
    if (!p || !d_leaves[i] || !d_out[i] || !d_work[i] || (mode == 1 && !d_gout[i]))
      return fail(TQ_EINVAL, "null plan or buffer for network " + std::to_string(i));
    TQ_TRY(runnable(p));
    if (work_bytes[i] < tq_tn_workspace(p, mode))
      return fail(TQ_EWORKSPACE, "workspace too small for network " + std::to_string(i));
    if (p->n_slices != 1 || p->fwd.empty()) {
      rest.push_back(i);
      continue;
    }
    const int k = p->dtype == TQ_C64 ? 0 : 1;
    P[k].push_back(p);
    L[k].push_back(d_leaves[i]);
    G[k].push_back(mode == 1 ? d_gout[i] : nullptr);
    O[k].push_back(d_out[i]);
    Wk[k].push_back(d_work[i]);
  }
  // the other (sliced) networks run one by one, spread over the context's stream pool (forked
  // from the caller's stream before the rounds start and joined back at the end), so their
  // many small launches overlap each other and the rounds
  constexpr int kPool = 4;
  const int np = (int)std::min<size_t>(rest.size(), kPool);
  if (np > 0) {
    if (!ctx->ev_fork) TQ_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    for (int k = 0; k < np; ++k)
      if (!ctx->pool[k]) {
        TQ_HIP(hipStreamCreateWithFlags(&ctx->pool[k], hipStreamNonBlocking));
        TQ_HIP(hipEventCreateWithFlags(&ctx->pool_done[k], hipEventDisableTiming));
      }
    TQ_HIP(hipEventRecord(ctx->ev_fork, stream));
    for (int k = 0; k < np; ++k) TQ_HIP(hipStreamWaitEvent(ctx->pool[k], ctx->ev_fork, 0));
  }
  tq_status st = TQ_OK;
  for (size_t k = 0; k < rest.size() && st == TQ_OK; ++k) {
    const int i = rest[k];
    hipStream_t s = ctx->pool[k % kPool];
    st = mode == 0 ? tq_tn_contract(ctx, plans[i], d_leaves[i], d_out[i], d_work[i], work_bytes[i], s)
                   : tq_tn_backward(ctx, plans[i], d_leaves[i], d_gout[i], d_out[i], d_work[i], work_bytes[i], s);
  }
  if (st == TQ_OK && !P[0].empty()) st = tn_batch_t<float>(ctx, P[0], L[0], G[0], O[0], Wk[0], mode, stream);
  if (st == TQ_OK && !P[1].empty()) st = tn_batch_t<double>(ctx, P[1], L[1], G[1], O[1], Wk[1], mode, stream);
  for (int k = 0; k < np; ++k) {  // join, also after an error, so no pool work outlives the call's order
    TQ_HIP(hipEventRecord(ctx->pool_done[k], ctx->pool[k]));
    TQ_HIP(hipStreamWaitEvent(stream, ctx->pool_done[k], 0));
  }
  return st;
}

}  // namespace tq

extern "C" {

tq_status tq_tn_contract_batch(tq_ctx* ctx, int32_t n, const tq_tn_plan* const* plans, const void* const* d_leaves,
                               void* const* d_out, void* const* d_work, const int64_t* work_bytes, void* stream) {
  return tn_batch(ctx, n, plans, d_leaves, nullptr, d_out, d_work, work_bytes, 0, (hipStream_t)stream);
}

tq_status tq_tn_backward_batch(tq_ctx* ctx, int32_t n, const tq_tn_plan* const* plans, const void* const* d_leaves,
                               const void* const* d_grad_out, void* const* d_grad_leaves, void* const* d_work,
                               const int64_t* work_bytes, void* stream) {
  return tn_batch(ctx, n, plans, d_leaves, d_grad_out, d_grad_leaves, d_work, work_bytes, 1, (hipStream_t)stream);
}

tq_status tq_tn_build_leaves(tq_ctx* ctx, const tq_tn_plan* plan, const tq_gate* gates, int32_t n_gates,
                             const tq_tn_leaf* leaves, const double* const_vals, int32_t n_const, const void* d_params,
                             void* d_leaves, void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null argument");
  DevLeafItem it{};
  TQ_TRY(leaf_build_item(ctx, plan, gates, n_gates, leaves, const_vals, n_const, d_params, d_leaves, &it));
  const int nl = it.n_leaves;
  if (plan->dtype == TQ_C64)
    hipLaunchKernelGGL(tn_leaf_build_kernel<float>, dim3((nl + 127) / 128), dim3(128), 0, (hipStream_t)stream,
                       it.lv, nl, it.gates, it.cv, (const float*)d_params, (float2*)d_leaves);
  else
    hipLaunchKernelGGL(tn_leaf_build_kernel<double>, dim3((nl + 127) / 128), dim3(128), 0, (hipStream_t)stream,
                       it.lv, nl, it.gates, it.cv, (const double*)d_params, (double2*)d_leaves);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

tq_status tq_tn_param_grad(tq_ctx* ctx, const tq_tn_plan* plan, const tq_gate* gates, int32_t n_gates,
                           const tq_tn_leaf* leaves, const void* d_params, int32_t n_params,
                           const void* d_grad_leaves, void* d_grad_params, void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null argument");
  DevPgItem it{};
  TQ_TRY(param_grad_item(ctx, plan, gates, n_gates, leaves, d_params, n_params, d_grad_leaves, d_grad_params, &it));
  if (n_params == 0) return TQ_OK;
  if (plan->dtype == TQ_C64)
    hipLaunchKernelGGL(tn_param_grad_kernel<float>, dim3(n_params), dim3(kPgThreads), 0, (hipStream_t)stream,
                       it.lv, it.gates, (const float*)d_params, it.pptr, it.pent, (const float2*)d_grad_leaves,
                       n_params, (float*)d_grad_params);
  else
    hipLaunchKernelGGL(tn_param_grad_kernel<double>, dim3(n_params), dim3(kPgThreads), 0, (hipStream_t)stream,
                       it.lv, it.gates, (const double*)d_params, it.pptr, it.pent, (const double2*)d_grad_leaves,
                       n_params, (double*)d_grad_params);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

// The batched leaf calls gather each network's device tables from the context's table cache
// and launch once per chunk of networks. A chunk looks up at most 4 * kTnLeafChunk tables,
// well under half the cache's entry bound, so the cache's least-recently-used eviction never
// frees a table of the chunk being gathered; it synchronises the device before freeing, so
// earlier chunks' launches have finished by then.
constexpr int kTnLeafChunk = 256;

tq_status tq_tn_build_leaves_batch(tq_ctx* ctx, int32_t n, const tq_tn_plan* const* plans,
                                   const tq_gate* const* gates, const int32_t* n_gates,
                                   const tq_tn_leaf* const* leaves, const double* const* const_vals,
                                   const int32_t* n_const, const void* const* d_params, void* const* d_leaves,
                                   void* stream) {
  if (!ctx || n < 0 || (n > 0 && (!plans || !gates || !n_gates || !leaves || !const_vals || !n_const || !d_params ||
                                  !d_leaves)))
    return fail(TQ_EINVAL, "null argument");
  for (int i = 0; i < n; ++i) {  // every network is checked before anything is launched
    if (!plans[i]) return fail(TQ_EINVAL, "null plan for network " + std::to_string(i));
    if (plans[i]->dtype != plans[0]->dtype)
      return fail(TQ_EINVAL, "network " + std::to_string(i) + ": every network of a batch must have the same dtype");
    const tq_status st = leaf_build_item(ctx, plans[i], gates[i], n_gates[i], leaves[i], const_vals[i], n_const[i],
                                         d_params[i], d_leaves[i], nullptr);
    if (st != TQ_OK) return fail(st, "network " + std::to_string(i) + ": " + tq_last_error());
  }
  for (int c0 = 0; c0 < n; c0 += kTnLeafChunk) {
    const int cn = std::min(kTnLeafChunk, n - c0);
    std::vector<DevLeafItem> items((size_t)cn);
    int blocks = 0;
    for (int k = 0; k < cn; ++k) {
      const int i = c0 + k;
      TQ_TRY(leaf_build_item(ctx, plans[i], gates[i], n_gates[i], leaves[i], const_vals[i], n_const[i], d_params[i],
                             d_leaves[i], &items[(size_t)k]));
      blocks = std::max(blocks, (items[(size_t)k].n_leaves + 127) / 128);
    }
    if (blocks == 0) continue;
    void* dev;
    TQ_TRY(stage_upload(ctx, S_TNB, items.data(), items.size() * sizeof(DevLeafItem), (hipStream_t)stream, &dev));
    if (plans[0]->dtype == TQ_C64)
      hipLaunchKernelGGL(tn_leaf_build_multi_kernel<float>, dim3((unsigned)blocks, (unsigned)cn), dim3(128), 0,
                         (hipStream_t)stream, (const DevLeafItem*)dev);
    else
      hipLaunchKernelGGL(tn_leaf_build_multi_kernel<double>, dim3((unsigned)blocks, (unsigned)cn), dim3(128), 0,
                         (hipStream_t)stream, (const DevLeafItem*)dev);
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}

tq_status tq_tn_param_grad_batch(tq_ctx* ctx, int32_t n, const tq_tn_plan* const* plans,
                                 const tq_gate* const* gates, const int32_t* n_gates, const tq_tn_leaf* const* leaves,
                                 const void* const* d_params, const int32_t* n_params,
                                 const void* const* d_grad_leaves, void* const* d_grad_params, void* stream) {
  if (!ctx || n < 0 || (n > 0 && (!plans || !gates || !n_gates || !leaves || !d_params || !n_params ||
                                  !d_grad_leaves || !d_grad_params)))
    return fail(TQ_EINVAL, "null argument");
  for (int i = 0; i < n; ++i) {  // every network is checked before anything is launched
    if (!plans[i]) return fail(TQ_EINVAL, "null plan for network " + std::to_string(i));
    if (plans[i]->dtype != plans[0]->dtype)
      return fail(TQ_EINVAL, "network " + std::to_string(i) + ": every network of a batch must have the same dtype");
    const tq_status st = param_grad_item(ctx, plans[i], gates[i], n_gates[i], leaves[i], d_params[i], n_params[i],
                                         d_grad_leaves[i], d_grad_params[i], nullptr);
    if (st != TQ_OK) return fail(st, "network " + std::to_string(i) + ": " + tq_last_error());
  }
  for (int c0 = 0; c0 < n; c0 += kTnLeafChunk) {
    const int cn = std::min(kTnLeafChunk, n - c0);
    std::vector<DevPgItem> items((size_t)cn);
    int blocks = 0;
    for (int k = 0; k < cn; ++k) {
      const int i = c0 + k;
      TQ_TRY(param_grad_item(ctx, plans[i], gates[i], n_gates[i], leaves[i], d_params[i], n_params[i],
                             d_grad_leaves[i], d_grad_params[i], &items[(size_t)k]));
      blocks = std::max(blocks, n_params[i]);
    }
    if (blocks == 0) continue;
    void* dev;
    TQ_TRY(stage_upload(ctx, S_TNB, items.data(), items.size() * sizeof(DevPgItem), (hipStream_t)stream, &dev));
    if (plans[0]->dtype == TQ_C64)
      hipLaunchKernelGGL(tn_param_grad_multi_kernel<float>, dim3((unsigned)blocks, (unsigned)cn), dim3(kPgThreads), 0,
                         (hipStream_t)stream, (const DevPgItem*)dev);
    else
      hipLaunchKernelGGL(tn_param_grad_multi_kernel<double>, dim3((unsigned)blocks, (unsigned)cn), dim3(kPgThreads),
                         0, (hipStream_t)stream, (const DevPgItem*)dev);
    TQ_HIP(hipGetLastError());
  }
  return TQ_OK;
}

}  // extern "C"
