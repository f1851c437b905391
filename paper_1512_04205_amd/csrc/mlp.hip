// Learned background-mode selector: a 6-64-64-1 GELU network over per-mode features,
// trained with binary cross-entropy and Adam on selections the method itself makes
// (sparse coding), used in place of sparse coding when it is confident.  The paper
// proposes learning the background amplitude profile (Section 2.2, "DMD for
// Foreground/Background Separation", its last paragraph); the network and features are this library's choice.
//
// Layout: one flat float32 parameter vector, W1 (64 x 6 row-major), b1, W2 (64 x 64),
// b2, w3 (64), b3 (4673 numbers).  A wave evaluates one sample with lane i holding
// hidden unit i of both layers, so each layer is 64 lane-local dot products with the
// previous layer's activations broadcast from LDS, and the backward pass needs only the
// transpose read of W2 from LDS.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "cdmd.h"
#include "kernels.hpp"

namespace cdmd {
namespace k {

namespace {

constexpr int MH = 64, MF = 6;
constexpr int O_W1 = 0, O_B1 = 384, O_W2 = 448, O_B2 = 4544, O_W3 = 4608, O_B3 = 4672;
constexpr int MP = 4673;
constexpr int W2S = 65;   // LDS row stride of W2 (conflict-free row and column reads)
constexpr int SPW = 8;    // samples per wave in the gradient kernel

__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.7071067811865476f));
}
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.7071067811865476f)) + x * expf(-0.5f * x * x) * 0.3989422804014327f;
}
__device__ __forceinline__ float wsum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return __shfl(v, 0, 64);
}
__device__ __forceinline__ float bf16r(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

struct Net {
  float* W2;   // [64][W2S]
  float* W1;   // [64][6]
  float* b1;
  float* b2;
  float* w3;
  float b3;
};

// Stage the parameters into LDS; with round_bf16 the hidden and output layers' weights
// are rounded to bfloat16 (the input layer stays float32: it carries the features'
// standardisation, whose large, cancelling terms bfloat16 would not hold).
__device__ void stage(const float* __restrict__ th, float* lds, bool round_bf16, Net& net) {
  net.W2 = lds;
  net.W1 = lds + MH * W2S;
  net.b1 = net.W1 + MH * MF;
  net.b2 = net.b1 + MH;
  net.w3 = net.b2 + MH;
  for (int e = threadIdx.x; e < MH * MH; e += blockDim.x) {
    const float v = th[O_W2 + e];
    net.W2[(e / MH) * W2S + (e % MH)] = round_bf16 ? bf16r(v) : v;
  }
  for (int e = threadIdx.x; e < MH * MF; e += blockDim.x) net.W1[e] = th[O_W1 + e];
  for (int e = threadIdx.x; e < MH; e += blockDim.x) {
    net.b1[e] = th[O_B1 + e];
    net.b2[e] = th[O_B2 + e];
    net.w3[e] = round_bf16 ? bf16r(th[O_W3 + e]) : th[O_W3 + e];
  }
  net.b3 = th[O_B3];
  __syncthreads();
}

constexpr int kLdsFloats = MH * W2S + MH * MF + 3 * MH;

// Per-wave gradient of the mean loss over the batch (sum of per-sample terms / nb).
// Sample q of the batch is row idx[q] of X (or q when idx is null); rows outside
// [0, nsamp) contribute nothing.  Each wave writes
// its partial gradient to part[(block * 4 + wave) * MP ...] and its partial loss.
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ th, const float* __restrict__ X,
                                                  const float* __restrict__ y, const int32_t* __restrict__ idx,
                                                  int nb, int64_t nsamp, float* __restrict__ part,
                                                  float* __restrict__ lpart) {
  __shared__ float lds[kLdsFloats];
  __shared__ float sh1[4][MH], sd2[4][MH];
  Net net;
  stage(th, lds, false, net);
  const int w = threadIdx.x >> 6, i = threadIdx.x & 63;
  float gW2[MH];
#pragma unroll
  for (int j = 0; j < MH; ++j) gW2[j] = 0.f;
  float gW1[MF] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, ls = 0.f;
  const float inv = 1.0f / (float)nb;
  const int q0 = (blockIdx.x * 4 + w) * SPW;
  for (int u = 0; u < SPW; ++u) {
    const int q = q0 + u;
    if (q >= nb) break;  // uniform over the wave
    const int64_t row = idx ? (int64_t)idx[q] : (int64_t)q;
    if (row < 0 || row >= nsamp) continue;  // caller index out of range: no contribution
    float x[MF];
#pragma unroll
    for (int f = 0; f < MF; ++f) x[f] = X[row * MF + f];
    const float yt = y[row];
    float a1 = net.b1[i];
#pragma unroll
    for (int f = 0; f < MF; ++f) a1 += net.W1[i * MF + f] * x[f];
    const float h1 = gelu(a1);
    sh1[w][i] = h1;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    float a2 = net.b2[i];
#pragma unroll 16
    for (int j = 0; j < MH; ++j) a2 += net.W2[i * W2S + j] * sh1[w][j];
    const float h2 = gelu(a2);
    const float z = wsum(net.w3[i] * h2) + net.b3;
    // d loss / d z of the mean binary cross-entropy with logits
    const float sg = 1.0f / (1.0f + expf(-z));
    const float dz = (sg - yt) * inv;
    ls += (fmaxf(z, 0.f) - z * yt + log1pf(expf(-fabsf(z)))) * inv;
    gw3 += dz * h2;
    gb3 += dz;
    const float d2 = dz * net.w3[i] * gelu_grad(a2);
    gb2 += d2;
    sd2[w][i] = d2;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < MH; ++j) gW2[j] += d2 * sh1[w][j];
    float s = 0.f;
#pragma unroll 16
    for (int r = 0; r < MH; ++r) s += net.W2[r * W2S + i] * sd2[w][r];
    const float d1 = s * gelu_grad(a1);
    gb1 += d1;
#pragma unroll
    for (int f = 0; f < MF; ++f) gW1[f] += d1 * x[f];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  float* g = part + (int64_t)(blockIdx.x * 4 + w) * MP;
#pragma unroll
  for (int j = 0; j < MH; ++j) g[O_W2 + i * MH + j] = gW2[j];
#pragma unroll
  for (int f = 0; f < MF; ++f) g[O_W1 + i * MF + f] = gW1[f];
  g[O_B1 + i] = gb1;
  g[O_B2 + i] = gb2;
  g[O_W3 + i] = gw3;
  if (i == 0) {
    g[O_B3] = gb3;
    lpart[blockIdx.x * 4 + w] = ls;
  }
}

// Sum the per-wave partials in order (float64); then either store the gradient or apply
// one Adam step (bias-corrected, step number t >= 1).
__global__ __launch_bounds__(256) void k_mlp_update(const float* __restrict__ part, const float* __restrict__ lpart,
                                                    int nparts, float* __restrict__ th, float* __restrict__ am,
                                                    float* __restrict__ av, float lr, int64_t t, float* __restrict__ grad,
                                                    float* __restrict__ loss) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0 && loss) {
    double l = 0.0;
    for (int q = 0; q < nparts; ++q) l += (double)lpart[q];
    *loss = (float)l;
  }
  if (e >= MP) return;
  double gs = 0.0;
  for (int q = 0; q < nparts; ++q) gs += (double)part[(int64_t)q * MP + e];
  const float g = (float)gs;
  if (grad) grad[e] = g;
  if (am) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float m1 = b1 * am[e] + (1.0f - b1) * g;
    const float v1 = b2 * av[e] + (1.0f - b2) * g * g;
    am[e] = m1;
    av[e] = v1;
    const double c1 = 1.0 - pow(0.9, (double)t), c2 = 1.0 - pow(0.999, (double)t);
    const float mh = (float)(m1 / c1), vh = (float)(v1 / c2);
    th[e] -= lr * mh / (sqrtf(vh) + 1e-8f);
  }
}

// Logits of n samples; with round_bf16 the hidden activations and the weights after the
// input layer are rounded to bfloat16 (float32 accumulation; the input layer in float32).
// One wave per sample.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ th, const float* __restrict__ X,
                                                     int n, int round_bf16, float* __restrict__ logits) {
  __shared__ float lds[kLdsFloats];
  __shared__ float sh1[4][MH];
  Net net;
  stage(th, lds, round_bf16 != 0, net);
  const int w = threadIdx.x >> 6, i = threadIdx.x & 63;
  for (int q = blockIdx.x * 4 + w; q < n; q += gridDim.x * 4) {
    float a1 = net.b1[i];
#pragma unroll
    for (int f = 0; f < MF; ++f) {
      a1 += net.W1[i * MF + f] * X[(int64_t)q * MF + f];
    }
    float h1 = gelu(a1);
    if (round_bf16) h1 = bf16r(h1);
    sh1[w][i] = h1;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    float a2 = net.b2[i];
#pragma unroll 16
    for (int j = 0; j < MH; ++j) a2 += net.W2[i * W2S + j] * sh1[w][j];
    float h2 = gelu(a2);
    if (round_bf16) h2 = bf16r(h2);
    const float z = wsum(net.w3[i] * h2) + net.b3;
    if (i == 0) logits[q] = z;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Features of k modes (one wave per mode): |lambda|, |arg lambda|,
// log(|b| ||phi|| / ||x_1||), ||phi|| / max_i ||phi_i||,
// (1/m) sum_t |b|^2 |lambda|^2t ||phi||^2 / ||x_1||^2 (lanes over t), j / k.
// in: lam[2k], b[2k], phin[k] (float64).
__global__ __launch_bounds__(256) void k_mode_features(const double* __restrict__ lam, const double* __restrict__ b,
                                                       const double* __restrict__ phin, double x1n2, int64_t m, int k,
                                                       float* __restrict__ F) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + w;
  if (j >= k) return;  // uniform over the wave
  const double lr = lam[2 * j], li = lam[2 * j + 1];
  const double a = hypot(lr, li);
  const double bm = hypot(b[2 * j], b[2 * j + 1]);
  const double pn = phin[j];
  double pmax = 0.0;
  for (int i = l; i < k; i += 64) pmax = fmax(pmax, phin[i]);
  double s = 0.0;
  const double la2 = a > 0.0 ? 2.0 * log(a) : -INFINITY;
  for (int64_t t = l; t < m; t += 64) s += t == 0 ? 1.0 : exp((double)t * la2);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o, 64);
    pmax = fmax(pmax, __shfl_xor(pmax, o, 64));
  }
  if (l == 0) {
    float* f = F + (int64_t)j * MF;
    const double rel = bm * pn / sqrt(x1n2);
    f[0] = (float)a;
    f[1] = (float)fabs(atan2(li, lr));
    f[2] = (float)log(rel > 1e-300 ? rel : 1e-300);
    f[3] = (float)(pmax > 0.0 ? pn / pmax : 0.0);
    f[4] = (float)(bm * bm * pn * pn / x1n2 * (s / (double)m));
    f[5] = (float)((double)j / (double)k);
  }
}

}  // namespace

int mlp_nparts(int batch) { return ((batch + 4 * SPW - 1) / (4 * SPW)) * 4; }

hipError_t mlp_grad(const float* th, const float* X, const float* y, const int32_t* idx, int nb, float* part,
                    float* lpart, float* grad, float* loss, hipStream_t stream) {
  const int blocks = (nb + 4 * SPW - 1) / (4 * SPW);
  hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(256), 0, stream, th, X, y, idx, nb, (int64_t)nb, part,
                     lpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_update, dim3((MP + 255) / 256), dim3(256), 0, stream, part, lpart, blocks * 4,
                     (float*)nullptr, (float*)nullptr, (float*)nullptr, 0.f, (int64_t)0, grad, loss);
  return hipGetLastError();
}

hipError_t mlp_train(float* th, float* am, float* av, const float* X, const float* y, int64_t nsamp,
                     const int32_t* idx, int batch, int steps, float lr, int64_t t0, float* part, float* lpart,
                     float* losses, hipStream_t stream) {
  const int blocks = (batch + 4 * SPW - 1) / (4 * SPW);
  for (int s = 0; s < steps; ++s) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(256), 0, stream, th, X, y, idx + (int64_t)s * batch, batch,
                       nsamp, part, lpart);
    hipLaunchKernelGGL(k_mlp_update, dim3((MP + 255) / 256), dim3(256), 0, stream, part, lpart, blocks * 4, th, am,
                       av, lr, t0 + s + 1, (float*)nullptr, losses ? losses + s : (float*)nullptr);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free training call: the per-wave partial gradients and
// losses of one batch of at most CDMD_MLP_NOALLOC_MAX_BATCH samples (2.4 MB).  Every
// device the library runs on holds its own copy until the process ends.  k_mlp_grad
// writes every partial of a launch before k_mlp_update reads them, so nothing needs
// clearing between calls.
namespace {
constexpr int kNoAllocParts = ((CDMD_MLP_NOALLOC_MAX_BATCH + 4 * SPW - 1) / (4 * SPW)) * 4;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) float scratch[(size_t)kNoAllocParts * MP + kNoAllocParts];

// The device address of `scratch` on the current device, looked up once per device with
// that device current (host code must not use the symbol itself as an address).
static hipError_t scratch_ptr(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t mlp_train_noalloc(float* th, float* am, float* av, const float* X, const float* y, int64_t nsamp,
                             const int32_t* idx, int batch, int steps, float lr, int64_t t0, float* losses,
                             hipStream_t stream) {
  if (batch < 1 || batch > CDMD_MLP_NOALLOC_MAX_BATCH || mlp_nparts(batch) > kNoAllocParts)
    return hipErrorInvalidValue;
  float* base = nullptr;
  const hipError_t e = scratch_ptr(&base);
  if (e != hipSuccess) return e;
  return mlp_train(th, am, av, X, y, nsamp, idx, batch, steps, lr, t0, base, base + (size_t)kNoAllocParts * MP,
                   losses, stream);
}

hipError_t mlp_forward(const float* th, const float* X, int n, int round_bf16, float* logits, hipStream_t stream) {
  int blocks = (n + 3) / 4;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(256), 0, stream, th, X, n, round_bf16, logits);
  return hipGetLastError();
}

hipError_t mode_features(const double* lam, const double* b, const double* phin, double x1n2, int64_t m, int k,
                         float* F, hipStream_t stream) {
  hipLaunchKernelGGL(k_mode_features, dim3((k + 3) / 4), dim3(256), 0, stream, lam, b, phin, x1n2, m, k, F);
  return hipGetLastError();
}

}  // namespace k
}  // namespace cdmd
