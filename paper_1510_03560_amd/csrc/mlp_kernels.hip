// HIP kernels of the learned activation proposal: a 12-64-64-1 perceptron
// with ReLU hidden layers and a logistic output, its binary cross-entropy
// gradient and the Adam update (Kingma and Ba 2015).  The network is tiny
// (5081 parameters), so every kernel keeps its parameters in LDS and uses
// plain FP32 FMA-free arithmetic (the library is compiled without
// contraction); the gradient sums run over the samples in order, one thread
// per parameter, so training does not depend on scheduling.

#include <hip/hip_runtime.h>

#include <cmath>

#include "lbm.h"
#include "lbm_mlp.h"

namespace lbm_mlp {
namespace {

constexpr int kIn = LBM_MLP_IN;
constexpr int kHid = LBM_MLP_HIDDEN;
constexpr int kN = LBM_MLP_NPARAMS;
// offsets into the parameter vector
constexpr int kMean = 0;
constexpr int kIstd = kMean + kIn;
constexpr int kW1 = kIstd + kIn;        // [kHid][kIn]
constexpr int kB1 = kW1 + kHid * kIn;
constexpr int kW2 = kB1 + kHid;         // [kHid][kHid]
constexpr int kB2 = kW2 + kHid * kHid;
constexpr int kW3 = kB2 + kHid;
constexpr int kB3 = kW3 + kHid;
static_assert(kB3 + 1 == kN, "parameter layout");
constexpr int kScratch = 1 + 2 * kHid;  // per sample: dz, dh2[64], dh1[64]

__global__ void __launch_bounds__(256) k_forward(const float* __restrict__ P, const float* __restrict__ x, int n,
                                                 float* __restrict__ logits, float* __restrict__ h1o,
                                                 float* __restrict__ h2o) {
  __shared__ float sp[kN];
  for (int i = threadIdx.x; i < kN; i += blockDim.x) sp[i] = P[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float xn[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i) xn[i] = (x[(size_t)s * kIn + i] - sp[kMean + i]) * sp[kIstd + i];
  float h1[kHid];
#pragma unroll
  for (int j = 0; j < kHid; ++j) {
    float acc = sp[kB1 + j];
#pragma unroll
    for (int i = 0; i < kIn; ++i) acc = acc + sp[kW1 + j * kIn + i] * xn[i];
    h1[j] = acc > 0.0f ? acc : 0.0f;
    if (h1o) h1o[(size_t)s * kHid + j] = h1[j];
  }
  float z = sp[kB3];
#pragma unroll 4
  for (int j = 0; j < kHid; ++j) {
    float acc = sp[kB2 + j];
#pragma unroll
    for (int k = 0; k < kHid; ++k) acc = acc + sp[kW2 + j * kHid + k] * h1[k];
    const float h2 = acc > 0.0f ? acc : 0.0f;
    if (h2o) h2o[(size_t)s * kHid + j] = h2;
    z = z + sp[kW3 + j] * h2;
  }
  logits[s] = z;
}

// Backward, per sample: dz = (sigma(z) - y) / n, dh2 = dz w3 [h2 > 0],
// dh1 = W2^T dh2 [h1 > 0].
__global__ void __launch_bounds__(256) k_backward_sample(const float* __restrict__ P, const float* __restrict__ y,
                                                         int n, const float* __restrict__ logits,
                                                         const float* __restrict__ h1,
                                                         const float* __restrict__ h2, float* __restrict__ scr) {
  __shared__ float sp[kN];
  for (int i = threadIdx.x; i < kN; i += blockDim.x) sp[i] = P[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float z = logits[s];
  const float sig = 1.0f / (1.0f + expf(-z));
  const float dz = (sig - y[s]) / (float)n;
  float* o = scr + (size_t)s * kScratch;
  o[0] = dz;
  float dh2[kHid];
#pragma unroll
  for (int j = 0; j < kHid; ++j) {
    dh2[j] = h2[(size_t)s * kHid + j] > 0.0f ? dz * sp[kW3 + j] : 0.0f;
    o[1 + j] = dh2[j];
  }
#pragma unroll 4
  for (int k = 0; k < kHid; ++k) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < kHid; ++j) acc = acc + sp[kW2 + j * kHid + k] * dh2[j];
    o[1 + kHid + k] = h1[(size_t)s * kHid + k] > 0.0f ? acc : 0.0f;
  }
}

// Backward, per parameter: the sum over samples in order.  Thread kN adds up
// the mean loss.
__global__ void __launch_bounds__(256) k_backward_param(const float* __restrict__ P, const float* __restrict__ x,
                                                        const float* __restrict__ y, int n,
                                                        const float* __restrict__ logits,
                                                        const float* __restrict__ h1,
                                                        const float* __restrict__ h2,
                                                        const float* __restrict__ scr, float* __restrict__ grad,
                                                        float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kN) return;
  if (p == kN) {
    if (loss) {
      float acc = 0.0f;
      for (int s = 0; s < n; ++s) {
        const float z = logits[s];
        // max(z, 0) - z y + log(1 + e^-|z|)
        acc = acc + ((z > 0.0f ? z : 0.0f) - z * y[s] + log1pf(expf(-fabsf(z))));
      }
      loss[0] = n > 0 ? acc / (float)n : 0.0f;
    }
    return;
  }
  float acc = 0.0f;
  if (p < kW1) {
    acc = 0.0f;  // standardisation constants are not trained
  } else if (p < kB1) {
    const int j = (p - kW1) / kIn, i = (p - kW1) % kIn;
    const float mu = P[kMean + i], is = P[kIstd + i];
    for (int s = 0; s < n; ++s) acc = acc + scr[(size_t)s * kScratch + 1 + kHid + j] * ((x[(size_t)s * kIn + i] - mu) * is);
  } else if (p < kW2) {
    const int j = p - kB1;
    for (int s = 0; s < n; ++s) acc = acc + scr[(size_t)s * kScratch + 1 + kHid + j];
  } else if (p < kB2) {
    const int j = (p - kW2) / kHid, k = (p - kW2) % kHid;
    for (int s = 0; s < n; ++s) acc = acc + scr[(size_t)s * kScratch + 1 + j] * h1[(size_t)s * kHid + k];
  } else if (p < kW3) {
    const int j = p - kB2;
    for (int s = 0; s < n; ++s) acc = acc + scr[(size_t)s * kScratch + 1 + j];
  } else if (p < kB3) {
    const int j = p - kW3;
    for (int s = 0; s < n; ++s) acc = acc + scr[(size_t)s * kScratch] * h2[(size_t)s * kHid + j];
  } else {
    for (int s = 0; s < n; ++s) acc = acc + scr[(size_t)s * kScratch];
  }
  grad[p] = acc;
}

__global__ void k_adam(float* __restrict__ P, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float c1, float c2, float lr, float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kW1 || p >= kN) return;
  const float gi = g[p];
  const float mi = b1 * m[p] + (1.0f - b1) * gi;
  const float vi = b2 * v[p] + (1.0f - b2) * (gi * gi);
  m[p] = mi;
  v[p] = vi;
  P[p] = P[p] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

int status(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EHIP; }

}  // namespace
}  // namespace lbm_mlp

using namespace lbm_mlp;

extern "C" int lbm_mlp_forward(const float* params, const float* x, int32_t n, float* logits, float* h1, float* h2,
                               void* stream) {
  if (!params || n < 0 || (n > 0 && (!x || !logits))) return LBM_EINVAL;
  if (n == 0) return LBM_OK;
  hipLaunchKernelGGL(k_forward, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, x, n, logits, h1,
                     h2);
  return status(hipGetLastError());
}

extern "C" int lbm_mlp_backward(const float* params, const float* x, const float* y, int32_t n, const float* logits,
                                const float* h1, const float* h2, float* scratch, float* grad, float* loss,
                                void* stream) {
  if (!params || !grad || n < 0 || (n > 0 && (!x || !y || !logits || !h1 || !h2 || !scratch))) return LBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (n > 0)
    hipLaunchKernelGGL(k_backward_sample, dim3((n + 255) / 256), dim3(256), 0, st, params, y, n, logits, h1, h2,
                       scratch);
  hipLaunchKernelGGL(k_backward_param, dim3((kN + 1 + 255) / 256), dim3(256), 0, st, params, x, y, n, logits, h1, h2,
                     scratch, grad, loss);
  return status(hipGetLastError());
}

extern "C" int lbm_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t t, float lr, float beta1,
                            float beta2, float eps, void* stream) {
  if (!params || !grad || !m || !v || t < 1) return LBM_EINVAL;
  const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((kN + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grad, m, v, c1, c2,
                     lr, beta1, beta2, eps);
  return status(hipGetLastError());
}
