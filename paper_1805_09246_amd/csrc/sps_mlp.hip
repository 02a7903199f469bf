// sps_mlp.hip -- learned cardinality estimator: training and batched inference kernels.
//
// Network (an addition to the paper's method): per-age live counts x_a of a host's union SLE
// (a < 10, each encoded by mlp_encode) -> 64 ReLU -> 64 ReLU -> 1, predicting the natural
// log of the host's cardinality.  Parameters are float32 in the order W1 (64 x 10), b1, W2 (64 x 64),
// b2, W3 (1 x 64), b3.  Loss: mean squared error over the batch.
//
// Layout on the GPU: one wave64 per sample, hidden unit j in lane j.  A wave keeps its
// parameter rows (and W2's column for back-propagation) in registers, broadcasts the other
// lanes' activations with v_readlane, and accumulates its samples' gradients in registers;
// every wave then writes one partial gradient, and a second kernel sums the partials in a
// fixed order (bitwise reproducible) before Adam.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sps_internal.h"

namespace sps {

namespace {
constexpr int kIn = SPS_MLP_IN;
constexpr int kH = SPS_MLP_HIDDEN;
constexpr int oW1 = 0;
constexpr int oB1 = oW1 + kH * kIn;
constexpr int oW2 = oB1 + kH;
constexpr int oB2 = oW2 + kH * kH;
constexpr int oW3 = oB2 + kH;
constexpr int oB3 = oW3 + kH;
constexpr int kP = oB3 + 1;
static_assert(kP == SPS_MLP_PARAMS, "parameter count");
static_assert(kH == 64, "one hidden unit per lane of a wave64");

__device__ __forceinline__ float bcast(float v, int k) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
}

__device__ __forceinline__ float round_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}
}  // namespace

// Partial gradients of the loss over samples idx[0..n) (or 0..n when idx is null).
// Features are counts out of etap cells; scale = 2 / (batch size) for the mean.
__global__ void __launch_bounds__(256) k_mlp_grad(const float* __restrict__ w,
                                                  const uint32_t* __restrict__ feat,
                                                  const float* __restrict__ target,
                                                  const uint32_t* __restrict__ idx, uint32_t n,
                                                  uint32_t etap, float scale,
                                                  float* __restrict__ partial,
                                                  float* __restrict__ partial_loss) {
  const int lane = (int)__lane_id();
  const uint32_t wave = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const uint32_t n_waves = gridDim.x * (blockDim.x / 64);
  float w1[kIn], w2row[kH], w2col[kH];
  for (int i = 0; i < kIn; ++i) w1[i] = w[oW1 + lane * kIn + i];
  for (int k = 0; k < kH; ++k) {
    w2row[k] = w[oW2 + lane * kH + k];
    w2col[k] = w[oW2 + k * kH + lane];
  }
  const float b1 = w[oB1 + lane], b2 = w[oB2 + lane], w3 = w[oW3 + lane], b3 = w[oB3];
  float g1[kIn], g2[kH];
  for (int i = 0; i < kIn; ++i) g1[i] = 0.f;
  for (int k = 0; k < kH; ++k) g2[k] = 0.f;
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, loss = 0.f;
  for (uint32_t s = wave; s < n; s += n_waves) {
    const uint32_t row = idx ? idx[s] : s;
    float x[kIn];
    for (int i = 0; i < kIn; ++i) x[i] = mlp_encode(feat[(uint64_t)row * kIn + i], etap);
    const float t = target[row];
    // forward
    float z1 = b1;
    for (int i = 0; i < kIn; ++i) z1 += w1[i] * x[i];
    const float h1 = fmaxf(z1, 0.f);
    float h1k[kH];
    for (int k = 0; k < kH; ++k) h1k[k] = bcast(h1, k);
    float z2 = b2;
    for (int k = 0; k < kH; ++k) z2 += w2row[k] * h1k[k];
    const float h2 = fmaxf(z2, 0.f);
    float y = w3 * h2;
    for (int o = 32; o > 0; o >>= 1) y += __shfl_xor(y, o, 64);
    y += b3;
    // backward
    const float d = y - t;
    loss += d * d;
    const float dy = scale * d;
    gw3 += dy * h2;
    gb3 += dy;
    const float dz2 = z2 > 0.f ? dy * w3 : 0.f;
    gb2 += dz2;
    for (int k = 0; k < kH; ++k) g2[k] += dz2 * h1k[k];
    float dh1 = 0.f;
    for (int j = 0; j < kH; ++j) dh1 += w2col[j] * bcast(dz2, j);
    const float dz1 = z1 > 0.f ? dh1 : 0.f;
    gb1 += dz1;
    for (int i = 0; i < kIn; ++i) g1[i] += dz1 * x[i];
  }
  float* p = partial + (uint64_t)wave * kP;
  for (int i = 0; i < kIn; ++i) p[oW1 + lane * kIn + i] = g1[i];
  p[oB1 + lane] = gb1;
  for (int k = 0; k < kH; ++k) p[oW2 + lane * kH + k] = g2[k];
  p[oB2 + lane] = gb2;
  p[oW3 + lane] = gw3;
  if (lane == 0) {
    p[oB3] = gb3;
    partial_loss[wave] = loss;
  }
}

// Sum the per-wave partials in wave order; grad[p] and loss (mean over n_samples).
__global__ void __launch_bounds__(256) k_mlp_reduce(const float* __restrict__ partial,
                                                    const float* __restrict__ partial_loss,
                                                    uint32_t n_waves, float inv_n,
                                                    float* __restrict__ grad,
                                                    float* __restrict__ loss) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < (uint32_t)kP) {
    float g = 0.f;
    for (uint32_t wv = 0; wv < n_waves; ++wv) g += partial[(uint64_t)wv * kP + p];
    grad[p] = g;
  }
  if (p == 0 && loss) {
    float l = 0.f;
    for (uint32_t wv = 0; wv < n_waves; ++wv) l += partial_loss[wv];
    *loss = l * inv_n;
  }
}

// Adam (Kingma & Ba 2015), bias-corrected, step counted from 1.  omb1 = 1 - beta1 and
// omb2 = 1 - beta2 come from the host in double precision (1 - 0.999f in float is off by
// 1.3e-5 relative).
__global__ void __launch_bounds__(256) k_mlp_adam(float* __restrict__ w, float* __restrict__ m,
                                                  float* __restrict__ v,
                                                  const float* __restrict__ grad, float lr,
                                                  float b1, float b2, float omb1, float omb2,
                                                  float eps, float c1, float c2) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (uint32_t)kP) return;
  const float g = grad[p];
  const float mp = b1 * m[p] + omb1 * g;
  const float vp = b2 * v[p] + omb2 * g * g;
  m[p] = mp;
  v[p] = vp;
  const float mh = mp / c1;
  const float vh = vp / c2;
  w[p] = w[p] - lr * mh / (sqrtf(vh) + eps);
}

// Batched inference: y[s] for every sample; bf16 != 0 rounds weights and activations to
// bfloat16 with float accumulation (the precision used inside scans).
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ w,
                                                     const uint32_t* __restrict__ feat,
                                                     uint32_t n, uint32_t etap, int bf16,
                                                     float* __restrict__ y_out) {
  const int lane = (int)__lane_id();
  const uint32_t wave = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const uint32_t n_waves = gridDim.x * (blockDim.x / 64);
  auto R = [bf16](float f) { return bf16 ? round_bf16(f) : f; };
  float w1[kIn], w2row[kH];
  for (int i = 0; i < kIn; ++i) w1[i] = R(w[oW1 + lane * kIn + i]);
  for (int k = 0; k < kH; ++k) w2row[k] = R(w[oW2 + lane * kH + k]);
  const float b1 = w[oB1 + lane], b2 = w[oB2 + lane], w3 = R(w[oW3 + lane]), b3 = w[oB3];
  for (uint32_t s = wave; s < n; s += n_waves) {
    float z1 = 0.f;
    for (int i = 0; i < kIn; ++i) z1 += w1[i] * R(mlp_encode(feat[(uint64_t)s * kIn + i], etap));
    const float h1 = R(fmaxf(z1 + b1, 0.f));
    float z2 = 0.f;
    for (int k = 0; k < kH; ++k) z2 += w2row[k] * bcast(h1, k);
    const float h2 = R(fmaxf(z2 + b2, 0.f));
    float y = w3 * h2;
    for (int o = 32; o > 0; o >>= 1) y += __shfl_xor(y, o, 64);
    if (lane == 0) y_out[s] = y + b3;
  }
}

uint32_t mlp_grad_waves(uint32_t n) {
  uint32_t w = (n + 15) / 16;
  if (w > 1024) w = 1024;
  if (w < 4) w = 4;
  return (w + 3) / 4 * 4;
}

hipError_t launch_mlp_grad(const float* w, const uint32_t* feat, const float* target,
                           const uint32_t* idx, uint32_t n, uint32_t etap, float* partial,
                           float* partial_loss, float* grad, float* loss, hipStream_t st) {
  const uint32_t waves = mlp_grad_waves(n);
  {
    ProfScope ps(SPS_STAGE_MLP, st);
    hipLaunchKernelGGL(k_mlp_grad, dim3(waves / 4), dim3(256), 0, st, w, feat, target, idx, n,
                       etap, 2.f / (float)n, partial, partial_loss);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kP + 255) / 256), dim3(256), 0, st, partial,
                       partial_loss, waves, 1.f / (float)n, grad, loss);
  }
  return hipGetLastError();
}

// Workspace of the allocation-free gradient call: the per-wave partial gradients (kP floats
// per wave) and then the per-wave losses of a batch of at most kMlpNoAllocMaxN samples.  Each
// device holds its own copy for the life of the process; calls on one device share it.
constexpr uint32_t kMlpNoAllocWaves = (kMlpNoAllocMaxN + 15) / 16;
static_assert(kMlpNoAllocWaves % 4 == 0, "whole blocks of four waves");
static __device__ __align__(256) float scratch[(uint64_t)kMlpNoAllocWaves * (kP + 1)];

// Device address of this device's copy of `scratch`, looked up once per device with that
// device current (the host-side name of the array is not a device address).
hipError_t mlp_scratch(float** out, uint64_t* floats) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static float* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<float*>(p);
  }
  *out = addr[dev];
  *floats = (uint64_t)kMlpNoAllocWaves * (kP + 1);
  return hipSuccess;
}

hipError_t launch_mlp_adam(float* w, float* m, float* v, const float* grad, uint32_t step,
                           float lr, double b1, double b2, float eps, hipStream_t st) {
  const float c1 = (float)(1.0 - pow(b1, (double)step));
  const float c2 = (float)(1.0 - pow(b2, (double)step));
  const float omb1 = (float)(1.0 - b1), omb2 = (float)(1.0 - b2);
  ProfScope ps(SPS_STAGE_MLP, st, ProfScope::kKernel);
  launch_k(ps, k_mlp_adam, dim3((kP + 255) / 256), dim3(256), 0, st, w, m, v, grad, lr,
                     (float)b1, (float)b2, omb1, omb2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* w, const uint32_t* feat, uint32_t n, uint32_t etap,
                              int bf16, float* y, int n_cu, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint32_t blocks = (n + 3) / 4;
  if (blocks > (uint32_t)n_cu * 8) blocks = (uint32_t)n_cu * 8;
  ProfScope ps(SPS_STAGE_MLP, st, ProfScope::kKernel);
  launch_k(ps, k_mlp_forward, dim3(blocks), dim3(256), 0, st, w, feat, n, etap, bf16, y);
  return hipGetLastError();
}

}  // namespace sps
