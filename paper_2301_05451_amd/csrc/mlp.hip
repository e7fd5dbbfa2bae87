// Cost-model MLP: x -> tanh(W_1 x + b_1) -> ... -> tanh(W_{L-1} h + b_{L-1}) -> W_L h + b_L
// (one scalar output), float32. It predicts the runtime of a contraction tree from the
// tree's features, so candidate trees can be ranked by predicted time instead of FLOPs
// (Sec. 3.2.2 ranks them by the FLOP count; for the small pairwise steps that dominate
// these networks runtime and FLOPs disagree, which Sec. 6.6 observes).
//
// Parameters are packed layer by layer: W_l [out][in] row-major, then b_l [out].
// Training minimises the mean squared error over the batch with Adam. Every reduction over
// the batch is a per-thread loop in a fixed order, so repeated runs are bitwise equal.
// The layers are small (tens of neurons), so these are plain VALU kernels: one thread per
// (sample, neuron) or per weight.
#include <algorithm>
#include <cmath>

#include "tq_internal.h"

namespace tq {
namespace {

constexpr int kMlpMaxLayers = 8;
constexpr int kThreads = 256;

struct MlpShape {
  int L = 0;
  int sizes[kMlpMaxLayers + 1] = {0};
  int64_t woff[kMlpMaxLayers] = {0};  // offset of W_l in the packed parameters
  int64_t boff[kMlpMaxLayers] = {0};  // offset of b_l
  int64_t nparams = 0;
  int64_t act_off[kMlpMaxLayers + 1] = {0};  // workspace offsets (floats) of layer outputs h_1..h_L
  int64_t delta_off[2] = {0, 0};             // two ping-pong delta buffers
  int64_t loss_off = 0, grad_off = 0, floats = 0;
  int maxw = 0;
};

tq_status shape_of(const tq_mlp_desc* d, int64_t batch, MlpShape* s) {
  if (!d) return fail(TQ_EINVAL, "null MLP descriptor");
  if (d->n_layers < 1 || d->n_layers > kMlpMaxLayers) return fail(TQ_EINVAL, "n_layers must be in 1..8");
  if (batch < 0) return fail(TQ_EINVAL, "negative batch");
  s->L = d->n_layers;
  for (int l = 0; l <= s->L; ++l) {
    if (d->sizes[l] < 1 || d->sizes[l] > 4096) return fail(TQ_EINVAL, "layer sizes must be in 1..4096");
    s->sizes[l] = d->sizes[l];
    s->maxw = std::max(s->maxw, d->sizes[l]);
  }
  if (s->sizes[s->L] != 1) return fail(TQ_EINVAL, "the last layer must have one output");
  int64_t p = 0;
  for (int l = 0; l < s->L; ++l) {
    s->woff[l] = p;
    p += (int64_t)s->sizes[l + 1] * s->sizes[l];
    s->boff[l] = p;
    p += s->sizes[l + 1];
  }
  s->nparams = p;
  int64_t w = 0;
  for (int l = 1; l <= s->L; ++l) {
    s->act_off[l] = w;
    w += batch * s->sizes[l];
  }
  s->delta_off[0] = w;
  w += batch * s->maxw;
  s->delta_off[1] = w;
  w += batch * s->maxw;
  s->loss_off = w;
  w += 64;
  s->grad_off = w;
  w += p;
  s->floats = w;
  return TQ_OK;
}

// h_out[b][j] = act(b_j + sum_i W[j][i] h_in[b][i])
__global__ void __launch_bounds__(kThreads)
    mlp_fwd_kernel(const float* __restrict__ W, const float* __restrict__ bias, const float* __restrict__ hin,
                   float* __restrict__ hout, int nin, int nout, int batch, int use_tanh) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)batch * nout) return;
  const int b = (int)(gid / nout), j = (int)(gid % nout);
  const float* w = W + (int64_t)j * nin;
  const float* x = hin + (int64_t)b * nin;
  float z = bias[j];
  for (int i = 0; i < nin; ++i) z = fmaf(w[i], x[i], z);
  hout[gid] = use_tanh ? tanhf(z) : z;
}

// One work-group: residuals r_b = yhat_b - y_b, delta_b = 2 r_b / B, loss = mean r_b^2
// (per-thread strided sums, then a fixed tree).
__global__ void __launch_bounds__(kThreads)
    mlp_loss_kernel(const float* __restrict__ yhat, const float* __restrict__ y, float* __restrict__ delta,
                    float* __restrict__ loss, int batch) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  const float scale = 2.0f / (float)batch;
  for (int b = threadIdx.x; b < batch; b += kThreads) {
    const float r = yhat[b] - y[b];
    delta[b] = scale * r;
    acc += (double)r * (double)r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = (float)(red[0] / (double)batch);
}

// delta_in[b][i] = (sum_j W[j][i] delta_out[b][j]) * (1 - h_in[b][i]^2)   (tanh')
__global__ void __launch_bounds__(kThreads)
    mlp_bwd_kernel(const float* __restrict__ W, const float* __restrict__ dout, const float* __restrict__ hin,
                   float* __restrict__ din, int nin, int nout, int batch) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)batch * nin) return;
  const int b = (int)(gid / nin), i = (int)(gid % nin);
  const float* d = dout + (int64_t)b * nout;
  float s = 0.f;
  for (int j = 0; j < nout; ++j) s = fmaf(W[(int64_t)j * nin + i], d[j], s);
  const float h = hin[gid];
  din[gid] = s * (1.f - h * h);
}

// gW[j][i] = sum_b delta[b][j] h_in[b][i] (i < nin); gb[j] = sum_b delta[b][j] (i == nin).
__global__ void __launch_bounds__(kThreads)
    mlp_wgrad_kernel(const float* __restrict__ delta, const float* __restrict__ hin, float* __restrict__ gW,
                     float* __restrict__ gb, int nin, int nout, int batch) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nout * (nin + 1)) return;
  const int j = (int)(gid / (nin + 1)), i = (int)(gid % (nin + 1));
  float s = 0.f;
  if (i < nin) {
    for (int b = 0; b < batch; ++b) s = fmaf(delta[(int64_t)b * nout + j], hin[(int64_t)b * nin + i], s);
    gW[(int64_t)j * nin + i] = s;
  } else {
    for (int b = 0; b < batch; ++b) s += delta[(int64_t)b * nout + j];
    gb[j] = s;
  }
}

// Adam (Kingma and Ba) with bias correction; c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void __launch_bounds__(kThreads)
    mlp_adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                    int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kThreads - 1) / kThreads); }

// Forward through every layer; the output layer writes `last` if given, else the
// workspace's h_L.
tq_status enqueue_forward(const MlpShape& s, const float* params, const float* x, int batch, float* ws,
                          float* last, hipStream_t stream) {
  const float* hin = x;
  for (int l = 0; l < s.L; ++l) {
    float* hout = (l == s.L - 1 && last) ? last : ws + s.act_off[l + 1];
    const int nin = s.sizes[l], nout = s.sizes[l + 1];
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(blocks_for((int64_t)batch * nout)), dim3(kThreads), 0, stream,
                       params + s.woff[l], params + s.boff[l], hin, hout, nin, nout, batch, l < s.L - 1 ? 1 : 0);
    TQ_HIP(hipGetLastError());
    hin = hout;
  }
  return TQ_OK;
}

}  // namespace
}  // namespace tq

using namespace tq;

extern "C" {

int64_t tq_mlp_param_count(const tq_mlp_desc* desc) {
  MlpShape s;
  if (shape_of(desc, 0, &s) != TQ_OK) return -1;
  return s.nparams;
}

int64_t tq_mlp_workspace(const tq_mlp_desc* desc, int32_t batch) {
  MlpShape s;
  if (shape_of(desc, batch, &s) != TQ_OK) return -1;
  return s.floats * (int64_t)sizeof(float) + 256;
}

tq_status tq_mlp_forward(tq_ctx* ctx, const tq_mlp_desc* desc, const float* d_params, const float* d_x, int32_t batch,
                         float* d_y, void* d_work, int64_t work_bytes, void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null context");
  MlpShape s;
  TQ_TRY(shape_of(desc, batch, &s));
  if (batch == 0) return TQ_OK;
  if (!d_params || !d_x || !d_y || !d_work) return fail(TQ_EINVAL, "null device pointer");
  if (work_bytes < s.floats * (int64_t)sizeof(float)) return fail(TQ_EWORKSPACE, "MLP workspace too small");
  hipStream_t st = (hipStream_t)stream;
  float* ws = (float*)d_work;
  return enqueue_forward(s, d_params, d_x, batch, ws, d_y, st);
}

tq_status tq_mlp_train_step(tq_ctx* ctx, const tq_mlp_desc* desc, float* d_params, float* d_m, float* d_v, int32_t t,
                            float lr, float beta1, float beta2, float eps, const float* d_x, const float* d_y,
                            int32_t batch, float* d_loss, float* d_grad, void* d_work, int64_t work_bytes,
                            void* stream) {
  if (!ctx) return fail(TQ_EINVAL, "null context");
  MlpShape s;
  TQ_TRY(shape_of(desc, batch, &s));
  if (batch < 1) return fail(TQ_EINVAL, "training needs batch >= 1");
  if (t < 1) return fail(TQ_EINVAL, "Adam step t is 1-based");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
    return fail(TQ_EINVAL, "bad Adam hyper-parameters");
  if (!d_params || !d_m || !d_v || !d_x || !d_y || !d_work) return fail(TQ_EINVAL, "null device pointer");
  if (work_bytes < s.floats * (int64_t)sizeof(float)) return fail(TQ_EWORKSPACE, "MLP workspace too small");
  hipStream_t st = (hipStream_t)stream;
  float* ws = (float*)d_work;
  float* grad = d_grad ? d_grad : ws + s.grad_off;
  TQ_TRY(enqueue_forward(s, d_params, d_x, batch, ws, nullptr, st));
  float* dcur = ws + s.delta_off[0];
  float* dnext = ws + s.delta_off[1];
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(kThreads), 0, st, ws + s.act_off[s.L], d_y, dcur,
                     d_loss ? d_loss : ws + s.loss_off, batch);
  TQ_HIP(hipGetLastError());
  for (int l = s.L - 1; l >= 0; --l) {
    const int nin = s.sizes[l], nout = s.sizes[l + 1];
    const float* hin = l == 0 ? d_x : ws + s.act_off[l];
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3(blocks_for((int64_t)nout * (nin + 1))), dim3(kThreads), 0, st, dcur,
                       hin, grad + s.woff[l], grad + s.boff[l], nin, nout, batch);
    TQ_HIP(hipGetLastError());
    if (l > 0) {
      hipLaunchKernelGGL(mlp_bwd_kernel, dim3(blocks_for((int64_t)batch * nin)), dim3(kThreads), 0, st,
                         d_params + s.woff[l], dcur, hin, dnext, nin, nout, batch);
      TQ_HIP(hipGetLastError());
      std::swap(dcur, dnext);
    }
  }
  const double c1 = 1.0 - std::pow((double)beta1, (double)t);
  const double c2 = 1.0 - std::pow((double)beta2, (double)t);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(blocks_for(s.nparams)), dim3(kThreads), 0, st, d_params, grad, d_m, d_v,
                     s.nparams, lr, beta1, beta2, eps, (float)c1, (float)c2);
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

}  // extern "C"
