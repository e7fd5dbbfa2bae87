// Parameter updates of a hybrid quantum-classical training loop (Sec. 4: the VQC cost is
// minimised by gradient steps on the circuit parameters), on the device so a training step
// never leaves the GPU: plain gradient descent, or Adam (Kingma and Ba) with bias correction.
#include "sv_device.h"

namespace tq {

template <typename T>
__global__ void sgd_kernel(T* __restrict__ p, const T* __restrict__ g, double lr, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (T)((double)p[i] - lr * (double)g[i]);
}

// c1 = 1 - beta1^t, c2 = 1 - beta2^t (bias corrections of step t).
template <typename T>
__global__ void adam_kernel(T* __restrict__ p, const T* __restrict__ g, T* __restrict__ m, T* __restrict__ v,
                            double lr, double b1, double b2, double eps, double c1, double c2, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double gi = (double)g[i];
    const double mi = b1 * (double)m[i] + (1.0 - b1) * gi;
    const double vi = b2 * (double)v[i] + (1.0 - b2) * gi * gi;
    m[i] = (T)mi;
    v[i] = (T)vi;
    p[i] = (T)((double)p[i] - lr * (mi / c1) / (sqrt(vi / c2) + eps));
  }
}

template <typename T>
static tq_status step_t(int kind, void* d_params, const void* d_grad, void* d_m, void* d_v, int32_t t, double lr,
                        double b1, double b2, double eps, int64_t n, hipStream_t s) {
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  if (kind == 0) {
    hipLaunchKernelGGL(sgd_kernel<T>, dim3(blocks), dim3(256), 0, s, (T*)d_params, (const T*)d_grad, lr, n);
  } else {
    const double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
    hipLaunchKernelGGL(adam_kernel<T>, dim3(blocks), dim3(256), 0, s, (T*)d_params, (const T*)d_grad, (T*)d_m,
                       (T*)d_v, lr, b1, b2, eps, c1, c2, n);
  }
  TQ_HIP(hipGetLastError());
  return TQ_OK;
}

}  // namespace tq

extern "C" tq_status tq_optimizer_step(tq_dtype dt, int32_t kind, void* d_params, const void* d_grad, void* d_m,
                                       void* d_v, int32_t t, double lr, double beta1, double beta2, double eps,
                                       int64_t n, void* stream) {
  using namespace tq;
  if (dt != TQ_C64 && dt != TQ_C128) return fail(TQ_EINVAL, "unknown dtype");
  if (kind != 0 && kind != 1) return fail(TQ_EINVAL, "kind must be 0 (gradient descent) or 1 (Adam)");
  if (n < 0) return fail(TQ_EINVAL, "negative parameter count");
  if (n == 0) return TQ_OK;
  if (!d_params || !d_grad || (kind == 1 && (!d_m || !d_v))) return fail(TQ_EINVAL, "null device pointer");
  if (kind == 1 && (t < 1 || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0)))
    return fail(TQ_EINVAL, "bad Adam step or hyper-parameters");
  if (dt == TQ_C64)
    return step_t<float>(kind, d_params, d_grad, d_m, d_v, t, lr, beta1, beta2, eps, n, (hipStream_t)stream);
  return step_t<double>(kind, d_params, d_grad, d_m, d_v, t, lr, beta1, beta2, eps, n, (hipStream_t)stream);
}
