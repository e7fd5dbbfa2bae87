// Measurements beyond Z strings (the paper's Sec. 5.1.1: expectation values and
// probabilities of the final state):
//
// * Pauli strings with X, Y and Z factors. For P = (x-mask f, z-mask m, nY factors Y),
//   P|x> = i^nY (-1)^{|x & m|} |x ^ f> with m covering the Y and Z positions, so
//   <psi|P|psi> = i^nY sum_x (-1)^{|x & m|} conj(psi_{x^f}) psi_x. Taking x and x ^ f together
//   (x with the highest bit h of f cleared), the pair gives 2 s Re A (nY even) or
//   2 s Im A (nY odd), with A = conj(psi_{x^f}) psi_x, s = +-(-1)^{|x & m|} by nY mod 4.
//   Each amplitude is read once per distinct flip mask f; terms sharing f share the reads.
// * Marginal probabilities of chosen qubits: P(y) = sum over the other qubits of |psi|^2.
//   Each work-group sums one outcome over a segment of the other qubits' values, so every
//   sum is a fixed-order tree (no atomics) and results repeat bitwise.
#include <algorithm>
#include <map>

#include "sv_device.h"

namespace tq {

constexpr int kObsThreads = 256;
constexpr int kPauliTerms = 8;  // terms sharing one flip mask per launch

struct PauliGroup {
  uint64_t f;                   // flip mask over bit positions (0: diagonal terms)
  int h;                        // highest set bit of f (-1 for f = 0)
  int nk;                       // terms in this launch
  uint64_t m[kPauliTerms];      // sign masks over bit positions
  int32_t cls[kPauliTerms];     // nY mod 4
  int32_t slot[kPauliTerms];    // column of the per-term value table
};

// Fixed-order sum over the 256 threads of a work-group (butterflies within waves, then the
// four wave totals in order); every thread gets the total.
__device__ __forceinline__ double group_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// partial[c][k][block] = the block's share of term k's value for circuit c.
template <typename T>
__global__ void __launch_bounds__(kObsThreads)
    pauli_partial_kernel(const typename Cx<T>::type* __restrict__ st, BatchMap smap, int n, PauliGroup g,
                         double* __restrict__ partial) {
  using C = typename Cx<T>::type;
  const C* s = st + smap.at(blockIdx.y);
  const int64_t total = g.f ? (int64_t(1) << (n - 1)) : (int64_t(1) << n);
  double acc[kPauliTerms];
#pragma unroll
  for (int k = 0; k < kPauliTerms; ++k) acc[k] = 0.0;
  const int64_t lo = g.h > 0 ? ((int64_t(1) << g.h) - 1) : 0;
  for (int64_t i = (int64_t)blockIdx.x * kObsThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kObsThreads) {
    const uint64_t x = g.f ? (uint64_t)(((i & ~lo) << 1) | (i & lo)) : (uint64_t)i;
    const C a = s[x];
    if (g.f == 0) {
      const double p = (double)a.x * a.x + (double)a.y * a.y;
#pragma unroll
      for (int k = 0; k < kPauliTerms; ++k)
        if (k < g.nk) acc[k] += (__popcll(x & g.m[k]) & 1) ? -p : p;
      continue;
    }
    const C b = s[x ^ g.f];
    // A = conj(b) * a
    const double re = (double)b.x * a.x + (double)b.y * a.y;
    const double im = (double)b.x * a.y - (double)b.y * a.x;
#pragma unroll
    for (int k = 0; k < kPauliTerms; ++k) {
      if (k < g.nk) {
        const int c = g.cls[k];
        double v = (c & 1) ? 2.0 * im : 2.0 * re;
        const bool neg = (c == 1 || c == 2) != (bool)(__popcll(x & g.m[k]) & 1);
        acc[k] += neg ? -v : v;
      }
    }
  }
  __shared__ double red[kObsThreads / 64];
  for (int k = 0; k < g.nk; ++k) {
    const double t = group_sum(acc[k], red);
    if (threadIdx.x == 0) partial[((int64_t)blockIdx.y * kPauliTerms + k) * gridDim.x + blockIdx.x] = t;
  }
}

// value[c][slot_k] = sum over blocks (in order) of the partials of term k.
__global__ void __launch_bounds__(kObsThreads)
    pauli_sum_kernel(const double* __restrict__ partial, int nb, PauliGroup g, double* __restrict__ value,
                     int n_slots) {
  __shared__ double red[kObsThreads / 64];
  for (int k = 0; k < g.nk; ++k) {
    double x = 0.0;
    for (int b = threadIdx.x; b < nb; b += kObsThreads)
      x += partial[((int64_t)blockIdx.x * kPauliTerms + k) * nb + b];
    const double t = group_sum(x, red);
    if (threadIdx.x == 0) value[(int64_t)blockIdx.x * n_slots + g.slot[k]] = t;
  }
}

// out[row(c)][o] = sum over terms (in order) of coeff_k * value[c][k].
template <typename T>
__global__ void pauli_combine_kernel(const double* __restrict__ value, int n_terms, int stride,
                                     const double* __restrict__ coeff, const int32_t* __restrict__ obs, int n_obs,
                                     T* __restrict__ out, BatchMap rows, int cn) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cn) return;
  for (int o = 0; o < n_obs; ++o) {
    double acc = 0.0;
    for (int k = 0; k < n_terms; ++k)
      if (obs[k] == o) acc += coeff[k] * value[(int64_t)c * stride + k];
    out[rows.at(c) * n_obs + o] = (T)acc;
  }
}

// ---- marginal probabilities ---------------------------------------------------------------

struct ProbDesc {
  int n, k;                 // register size, selected qubits
  int seg_bits;             // the other qubits' values are split into 2^seg_bits segments
  int64_t ysel[4][256];     // deposit of outcome bits (8 per table) into the selected positions
  int64_t rdep[4][256];     // deposit of the other qubits' values (8 bits per table)
};

// Block (y * S + seg, c): sum of |psi|^2 over the rest values of segment seg for outcome y.
template <typename T>
__global__ void __launch_bounds__(kObsThreads)
    probs_partial_kernel(const typename Cx<T>::type* __restrict__ st, BatchMap smap, const ProbDesc* __restrict__ d,
                         double* __restrict__ partial) {
  using C = typename Cx<T>::type;
  __shared__ int64_t tab[4][256];
  __shared__ double red[kObsThreads / 64];
  for (int i = threadIdx.x; i < 4 * 256; i += kObsThreads) tab[i >> 8][i & 255] = d->rdep[i >> 8][i & 255];
  __syncthreads();
  const C* s = st + smap.at(blockIdx.y);
  const int S = 1 << d->seg_bits;
  const int64_t y = blockIdx.x >> d->seg_bits;
  const int seg = blockIdx.x & (S - 1);
  const int64_t base = d->ysel[0][y & 255] | d->ysel[1][(y >> 8) & 255] | d->ysel[2][(y >> 16) & 255] |
                       d->ysel[3][(y >> 24) & 255];
  const int rbits = d->n - d->k;
  const int64_t per = (int64_t(1) << rbits) >> d->seg_bits;
  const int64_t r0 = (int64_t)seg * per;
  double acc = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r0 + per; r += kObsThreads) {
    const int64_t x = base | tab[0][r & 255] | tab[1][(r >> 8) & 255] | tab[2][(r >> 16) & 255] | tab[3][(r >> 24) & 255];
    const C a = s[x];
    acc += (double)a.x * a.x + (double)a.y * a.y;
  }
  const double t = group_sum(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

template <typename T>
__global__ void probs_final_kernel(const double* __restrict__ partial, int64_t n_out, int seg_bits,
                                   T* __restrict__ out, BatchMap rows) {
  const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= n_out) return;
  const int S = 1 << seg_bits;
  const double* p = partial + ((int64_t)blockIdx.y * n_out + y) * S;
  double acc = 0.0;
  for (int s = 0; s < S; ++s) acc += p[s];
  out[rows.at(blockIdx.y) * n_out + y] = (T)acc;
}

template <typename T>
static tq_status pauli_t(tq_ctx* ctx, const tq_batch* batch, const void* d_states, const tq_pauli_term* terms,
                         int n_terms, int n_obs, void* d_out, hipStream_t stream) {
  using C = typename Cx<T>::type;
  std::vector<Group> groups;
  TQ_TRY(group_batch(batch, nullptr, groups));
  if (n_obs < 1) return fail(TQ_EINVAL, "n_obs must be >= 1");
  if (n_terms < 0 || (n_terms > 0 && !terms)) return fail(TQ_EINVAL, "bad terms");
  if (!groups.empty() && (!d_states || !d_out)) return fail(TQ_EINVAL, "null device pointer");
  for (int k = 0; k < n_terms; ++k)
    if (terms[k].obs < 0 || terms[k].obs >= n_obs) return fail(TQ_EINVAL, "term obs index out of range");
  std::map<int, std::vector<int>> by_n;
  for (const Group& gr : groups) {
    for (int k = 0; k < n_terms; ++k)
      if (gr.n < 64 && ((terms[k].x_mask | terms[k].z_mask) >> gr.n) != 0)
        return fail(TQ_EINVAL, "term names a qubit >= n");
    for (int i : gr.members) by_n[gr.n].push_back(i);
  }
  std::vector<double> cf(std::max(n_terms, 1));
  std::vector<int32_t> ob(std::max(n_terms, 1));
  for (int k = 0; k < n_terms; ++k) cf[k] = terms[k].coeff, ob[k] = terms[k].obs;
  void *dcf, *dob;
  TQ_TRY(cached_table(ctx, cf.data(), cf.size() * sizeof(double), &dcf));
  TQ_TRY(cached_table(ctx, ob.data(), ob.size() * sizeof(int32_t), &dob));
  for (auto& kv : by_n) {
    const int n = kv.first;
    std::vector<int>& mem = kv.second;
    std::sort(mem.begin(), mem.end());
    // terms in position space, grouped by flip mask (first appearance order)
    std::vector<PauliGroup> launches;
    std::map<uint64_t, int> open;
    for (int k = 0; k < n_terms; ++k) {
      uint64_t f = 0, m = 0;
      int ny = 0;
      for (int q = 0; q < n; ++q) {
        const bool xb = (terms[k].x_mask >> q) & 1ull, zb = (terms[k].z_mask >> q) & 1ull;
        const uint64_t bit = 1ull << (n - 1 - q);
        if (xb) f |= bit;
        if (zb) m |= bit;
        if (xb && zb) ++ny;
      }
      auto it = open.find(f);
      if (it == open.end() || launches[it->second].nk == kPauliTerms) {
        PauliGroup g{};
        g.f = f;
        g.h = f ? 63 - __builtin_clzll(f) : -1;
        launches.push_back(g);
        open[f] = (int)launches.size() - 1;
        it = open.find(f);
      }
      PauliGroup& g = launches[it->second];
      g.m[g.nk] = m;
      g.cls[g.nk] = ny & 3;
      g.slot[g.nk] = k;
      ++g.nk;
    }
    BatchMap smap, rows;
    TQ_TRY(member_map(ctx, S_MISC, batch->state_off, mem, stream, &smap));
    std::vector<int64_t> rr(mem.begin(), mem.end());
    std::vector<int> ident(mem.size());
    for (size_t i = 0; i < mem.size(); ++i) ident[i] = (int)i;
    TQ_TRY(member_map(ctx, S_MISC, rr.data(), ident, stream, &rows));
    for (size_t c0 = 0; c0 < mem.size(); c0 += 65535) {
      const int cn = (int)std::min<size_t>(65535, mem.size() - c0);
      const int64_t pairs = int64_t(1) << (n > 1 ? n - 1 : 0);
      const int nb = (int)std::max<int64_t>(1, std::min<int64_t>((pairs + kObsThreads - 1) / kObsThreads,
                                                                 std::max(1, 1024 / cn)));
      void* work;
      const size_t vals = (size_t)cn * std::max(n_terms, 1);
      TQ_TRY(scratch(ctx, S_PARTIAL, (vals + (size_t)cn * kPauliTerms * nb) * sizeof(double), &work));
      double* value = (double*)work;
      double* partial = value + vals;
      const BatchMap sm = smap.shifted((int)c0), rm = rows.shifted((int)c0);
      for (const PauliGroup& g : launches) {
        hipLaunchKernelGGL(pauli_partial_kernel<T>, dim3((unsigned)nb, (unsigned)cn), dim3(kObsThreads), 0, stream,
                           (const C*)d_states, sm, n, g, partial);
        hipLaunchKernelGGL(pauli_sum_kernel, dim3((unsigned)cn), dim3(kObsThreads), 0, stream, partial, nb, g, value,
                           std::max(n_terms, 1));
      }
      hipLaunchKernelGGL(pauli_combine_kernel<T>, dim3((unsigned)((cn + 63) / 64)), dim3(64), 0, stream, value,
                         n_terms, std::max(n_terms, 1), (const double*)dcf, (const int32_t*)dob, n_obs, (T*)d_out, rm,
                         cn);
      TQ_HIP(hipGetLastError());
    }
  }
  return TQ_OK;
}

template <typename T>
static tq_status probs_t(tq_ctx* ctx, const tq_batch* batch, const void* d_states, const int32_t* qubits, int k,
                         void* d_out, hipStream_t stream) {
  using C = typename Cx<T>::type;
  std::vector<Group> groups;
  TQ_TRY(group_batch(batch, nullptr, groups));
  if (k < 1 || k > 24 || !qubits) return fail(TQ_EINVAL, "select 1..24 qubits");
  for (const Group& gr : groups)
    if (gr.n - k > 32) return fail(TQ_ENOTSUP, "more than 32 unselected qubits");
  if (!groups.empty() && (!d_states || !d_out)) return fail(TQ_EINVAL, "null device pointer");
  std::map<int, std::vector<int>> by_n;
  for (const Group& gr : groups) {
    for (int i = 0; i < k; ++i) {
      if (qubits[i] < 0 || qubits[i] >= gr.n) return fail(TQ_EINVAL, "selected qubit outside the register");
      for (int j = 0; j < i; ++j)
        if (qubits[j] == qubits[i]) return fail(TQ_EINVAL, "duplicate selected qubit");
    }
    for (int i : gr.members) by_n[gr.n].push_back(i);
  }
  for (auto& kv : by_n) {
    const int n = kv.first;
    std::vector<int>& mem = kv.second;
    std::sort(mem.begin(), mem.end());
    ProbDesc d{};
    d.n = n;
    d.k = k;
    // outcome bit j (from the least significant) is the listed qubit k-1-j, at position
    // n-1-qubit; the other qubits' values fill the remaining positions in increasing order
    std::vector<int> ypos(k), rpos;
    for (int j = 0; j < k; ++j) ypos[j] = n - 1 - qubits[k - 1 - j];
    for (int p = 0; p < n; ++p)
      if (std::find(ypos.begin(), ypos.end(), p) == ypos.end()) rpos.push_back(p);
    for (int t = 0; t < 4; ++t)
      for (int v = 0; v < 256; ++v) {
        int64_t a = 0, b = 0;
        for (int bit = 0; bit < 8; ++bit) {
          const int j = t * 8 + bit;
          if (!((v >> bit) & 1)) continue;
          if (j < k) a |= int64_t(1) << ypos[j];
          if (j < (int)rpos.size()) b |= int64_t(1) << rpos[j];
        }
        d.ysel[t][v] = a;
        d.rdep[t][v] = b;
      }
    const int rbits = n - k;
    for (size_t c0 = 0; c0 < mem.size(); c0 += 65535) {
      const int cn = (int)std::min<size_t>(65535, mem.size() - c0);
      const int64_t n_out = int64_t(1) << k;
      int sb = 0;  // segments: enough blocks to fill the device, each at least 256 values
      while (sb < rbits - 8 && (n_out << sb) * cn < 1024) ++sb;
      d.seg_bits = sb;
      void* work;
      TQ_TRY(scratch(ctx, S_PARTIAL, (size_t)cn * (n_out << sb) * sizeof(double), &work));
      void* dd;
      TQ_TRY(cached_table(ctx, &d, sizeof d, &dd));
      BatchMap smap, rows;
      std::vector<int> part(mem.begin() + c0, mem.begin() + c0 + cn);
      TQ_TRY(member_map(ctx, S_MISC, batch->state_off, part, stream, &smap));
      std::vector<int64_t> rr(part.begin(), part.end());
      std::vector<int> ident(part.size());
      for (size_t i = 0; i < part.size(); ++i) ident[i] = (int)i;
      TQ_TRY(member_map(ctx, S_MISC, rr.data(), ident, stream, &rows));
      if ((n_out << sb) > 0x7fffffff) return fail(TQ_ENOTSUP, "too many outcomes");
      hipLaunchKernelGGL(probs_partial_kernel<T>, dim3((unsigned)(n_out << sb), (unsigned)cn), dim3(kObsThreads), 0,
                         stream, (const C*)d_states, smap, (const ProbDesc*)dd, (double*)work);
      hipLaunchKernelGGL(probs_final_kernel<T>, dim3((unsigned)((n_out + 255) / 256), (unsigned)cn), dim3(256), 0,
                         stream, (const double*)work, n_out, sb, (T*)d_out, rows);
      TQ_HIP(hipGetLastError());
    }
  }
  return TQ_OK;
}

}  // namespace tq

using namespace tq;

extern "C" tq_status tq_expval_pauli(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const void* d_states,
                                     const tq_pauli_term* terms, int32_t n_terms, int32_t n_obs, void* d_out,
                                     void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null context");
  if (dt == TQ_C64) return pauli_t<float>(ctx, batch, d_states, terms, n_terms, n_obs, d_out, (hipStream_t)stream);
  if (dt == TQ_C128) return pauli_t<double>(ctx, batch, d_states, terms, n_terms, n_obs, d_out, (hipStream_t)stream);
  return fail(TQ_EINVAL, "unknown dtype");
}

extern "C" tq_status tq_probs(tq_ctx* ctx, tq_dtype dt, const tq_batch* batch, const void* d_states,
                              const int32_t* qubits, int32_t n_sel, void* d_out, void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null context");
  if (dt == TQ_C64) return probs_t<float>(ctx, batch, d_states, qubits, n_sel, d_out, (hipStream_t)stream);
  if (dt == TQ_C128) return probs_t<double>(ctx, batch, d_states, qubits, n_sel, d_out, (hipStream_t)stream);
  return fail(TQ_EINVAL, "unknown dtype");
}

// Pauli decomposition of a Hermitian matrix on k qubits: H = sum_P c_P P with
// c_P = Tr(P H) / 2^k, real for Hermitian H (host only).
extern "C" int32_t tq_pauli_decompose(const double* herm, int32_t k, const int32_t* qubits, double tol, int32_t obs,
                                      tq_pauli_term* out, int32_t cap) {
  if (!herm || !qubits || k < 1 || k > 6) {
    fail(TQ_EINVAL, "tq_pauli_decompose: 1..6 qubits and a matrix are required");
    return -1;
  }
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < i; ++j)
      if (qubits[i] == qubits[j] || qubits[i] < 0 || qubits[i] > 63) {
        fail(TQ_EINVAL, "tq_pauli_decompose: qubits must be distinct and in 0..63");
        return -1;
      }
  const int dim = 1 << k;
  int count = 0;
  // string s: digit j (base 4) is the factor on qubits[j]: 0 I, 1 X, 2 Y, 3 Z; the matrix
  // index has qubits[0] as its most significant bit
  for (int s = 0; s < (1 << (2 * k)); ++s) {
    double re = 0.0, im = 0.0;
    // Tr(P H) = sum_{a,b} P[a][b] H[b][a]; P[a][b] = prod_j p_j[a_j][b_j]
    for (int a = 0; a < dim; ++a) {
      int b = 0;
      double pr = 1.0, pi = 0.0;  // P[a][b] for the unique b with a nonzero entry
      for (int j = 0; j < k; ++j) {
        const int d = (s >> (2 * j)) & 3;
        const int bit = k - 1 - j;
        const int aj = (a >> bit) & 1;
        int bj = aj;
        double fr = 1.0, fi = 0.0;
        if (d == 1) bj = 1 - aj;                                  // X
        else if (d == 2) { bj = 1 - aj; fr = 0.0; fi = aj ? 1.0 : -1.0; }  // Y: [[0,-i],[i,0]]
        else if (d == 3) fr = aj ? -1.0 : 1.0;                     // Z
        b |= bj << bit;
        const double nr = pr * fr - pi * fi, ni = pr * fi + pi * fr;
        pr = nr;
        pi = ni;
      }
      const double hr = herm[2 * (b * dim + a)], hi = herm[2 * (b * dim + a) + 1];
      re += pr * hr - pi * hi;
      im += pr * hi + pi * hr;
    }
    (void)im;  // zero for a Hermitian H
    const double c = re / dim;
    if (std::abs(c) <= tol) continue;
    if (out && count < cap) {
      tq_pauli_term t{};
      for (int j = 0; j < k; ++j) {
        const int d = (s >> (2 * j)) & 3;
        const uint64_t bit = 1ull << qubits[j];
        if (d == 1 || d == 2) t.x_mask |= bit;
        if (d == 2 || d == 3) t.z_mask |= bit;
      }
      t.coeff = c;
      t.obs = obs;
      out[count] = t;
    }
    ++count;
  }
  if (out && count > cap) {
    fail(TQ_ESIZE, "tq_pauli_decompose: capacity " + std::to_string(cap) + " < " + std::to_string(count));
    return -1;
  }
  return count;
}
