// Attainable-peak probes: the rates that the roofline fractions of the simulator's kernels
// are also quoted against, measured on the device at hand instead of taken from its
// datasheet. Five fixed kernels, each doing a known amount of work:
//   stream copy  - reads one half of a buffer and writes the other half (one 16-byte vector
//                  per thread: the fastest of 1, 2, 4 and 8 vectors per thread, and of plain
//                  and non-temporal accesses, on multi-GiB buffers),
//   stream read  - reads the whole buffer (4 vectors per thread) and writes nothing,
//   FP32 FMA     - independent non-packed v_fma_f32 chains (the instruction form the state
//                  kernels compile to: packed FP32 is disabled in this library's build),
//   FP32 MFMA    - independent 16x16x4 FP32 matrix-core accumulations,
//   FP64 MFMA    - the same with 16x16x4 FP64.
// The caller times one launch with events on the same stream and divides the reported work
// by the elapsed time.
#include "sv_device.h"

namespace tq {

constexpr int kPeakThreads = 256;
constexpr int kPeakBlocks = 2048;  // 8 blocks of 4 waves per CU on 256 CUs
constexpr int kPeakChains = 8;     // independent accumulators per thread / wave
constexpr int kReadPerThread = 4;  // 16-byte vectors per thread of the read probe

__global__ __launch_bounds__(kPeakThreads) void peak_copy_kernel(const float4* __restrict__ src,
                                                                 float4* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * kPeakThreads + threadIdx.x;
  dst[i] = src[i];
}

// Sums the vectors; the store happens only for a sum no finite buffer of zeros produces, so
// nothing is written in practice, yet the loads cannot be removed.
__global__ __launch_bounds__(kPeakThreads) void peak_read_kernel(const float4* __restrict__ src,
                                                                 float* __restrict__ sink) {
  const int64_t base = (int64_t)blockIdx.x * (kPeakThreads * kReadPerThread) + threadIdx.x;
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kReadPerThread; ++k) {
    const float4 v = src[base + k * kPeakThreads];
    s += (v.x + v.y) + (v.z + v.w);
  }
  if (s == -1.0f) sink[0] = s;
}

// a <- a * x + y on kPeakChains chains; x < 1 keeps every chain bounded.
__global__ __launch_bounds__(kPeakThreads) void peak_fma_kernel(float* __restrict__ out, int32_t iters, float x,
                                                                float y) {
  const int t = blockIdx.x * kPeakThreads + threadIdx.x;
  float a[kPeakChains];
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) a[c] = (float)(t & 7) + 0.25f * c;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) a[c] = __builtin_fmaf(a[c], x, y);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) s += a[c];
  out[t] = s;
}

__global__ __launch_bounds__(kPeakThreads) void peak_mfma_f32_kernel(float* __restrict__ out, int32_t iters,
                                                                     float x) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const int t = blockIdx.x * kPeakThreads + threadIdx.x;
  const int l = threadIdx.x & 63;  // lane: supplies A[l % 16][l / 16] and B[l / 16][l % 16]
  const float a = x * (float)(l & 15), b = x * (float)(l >> 4);
  f4 acc[kPeakChains];
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) acc[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[t] = s;
}

__global__ __launch_bounds__(kPeakThreads) void peak_mfma_f64_kernel(double* __restrict__ out, int32_t iters,
                                                                     double x) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int t = blockIdx.x * kPeakThreads + threadIdx.x;
  const int l = threadIdx.x & 63;
  const double a = x * (double)(l & 15), b = x * (double)(l >> 4);
  d4 acc[kPeakChains];
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[t] = s;
}

}  // namespace tq

extern "C" tq_status tq_peak_probe(int32_t kind, void* d_buf, uint64_t bytes, int32_t iters, double* work,
                                   void* stream) {
  using namespace tq;
  if (!d_buf || !work) return fail(TQ_EINVAL, "null pointer");
  const hipStream_t s = (hipStream_t)stream;
  const uint64_t threads = (uint64_t)kPeakBlocks * kPeakThreads;
  if (kind == 0 || kind == 4) {
    const uint64_t chunk = 2ull * 16 * kPeakThreads * kReadPerThread;  // 32 KiB
    if (bytes == 0 || bytes % chunk != 0)
      return fail(TQ_ESIZE, "stream probe: the buffer size must be a positive multiple of 32 KiB");
    if (bytes / chunk > (1ull << 28)) return fail(TQ_ESIZE, "stream probe: buffer too large");
    if (kind == 0) {
      const uint64_t half = bytes / 2;
      const float4* src = (const float4*)d_buf;
      float4* dst = (float4*)((char*)d_buf + half);
      hipLaunchKernelGGL(peak_copy_kernel, dim3((unsigned)(half / (16 * kPeakThreads))), dim3(kPeakThreads), 0, s,
                         src, dst);
    } else {
      hipLaunchKernelGGL(peak_read_kernel, dim3((unsigned)(bytes / (16 * kPeakThreads * kReadPerThread))),
                         dim3(kPeakThreads), 0, s, (const float4*)d_buf, (float*)d_buf);
    }
    TQ_HIP(hipGetLastError());
    *work = (double)bytes;  // copy: half read + half written; read: all of it
    return TQ_OK;
  }
  if (kind < 1 || kind > 3)
    return fail(TQ_EINVAL, "kind must be 0 (copy), 1 (FP32 FMA), 2 (FP32 MFMA), 3 (FP64 MFMA) or 4 (read)");
  if (iters < 1) return fail(TQ_EINVAL, "iters must be positive");
  const uint64_t need = threads * (kind == 3 ? 8 : 4);
  if (bytes < need) return fail(TQ_ESIZE, "compute probe: the buffer must hold one value per thread (" +
                                              std::to_string(need) + " bytes)");
  if (kind == 1) {
    hipLaunchKernelGGL(peak_fma_kernel, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, (float*)d_buf, iters,
                       0.999f, 1e-3f);
    *work = (double)threads * iters * kPeakChains * 2.0;
  } else if (kind == 2) {
    hipLaunchKernelGGL(peak_mfma_f32_kernel, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, (float*)d_buf, iters,
                       1e-3f);
    *work = (double)(threads / 64) * iters * kPeakChains * (16.0 * 16 * 4 * 2);
  } else {
    hipLaunchKernelGGL(peak_mfma_f64_kernel, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, (double*)d_buf, iters,
                       1e-3);
    *work = (double)(threads / 64) * iters * kPeakChains * (16.0 * 16 * 4 * 2);
  }
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}
