// bs32_mlp.hip -- training kernels of the learned step-size proposer.
//
// Forward and backward of the 9 -> 64 -> 64 -> 1 tanh network (on standardized
// features; the standardization is not trained) over a tile of 64 samples per workgroup (activations staged in LDS), the asymmetric squared
// loss (overshoot weighted: a rejected step costs three evaluations), and an
// Adam update of FP32 master weights that also refreshes their BF16 copy (the
// weights every forward pass reads).  All sums have a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>

#include "bs32_internal.hpp"
#include "bs32_mlp.hpp"

namespace bs32 {

constexpr int kTile = 64;

__device__ __forceinline__ float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
  u += 0x7fffu + ((u >> 16) & 1u);                  // round to nearest, ties to even
  return __uint_as_float(u & 0xffff0000u);
}

// gradient of (1/n) sum_s w_s (y_s - label_s)^2 over the samples of one tile;
// w_s = over_w when the prediction overshoots the label, 1 otherwise
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ W, const float* __restrict__ X,
                                                  const float* __restrict__ Y, const int* __restrict__ idx, int nb,
                                                  float inv_n, float over_w, float* __restrict__ part,
                                                  double* __restrict__ loss_part) {
  __shared__ float sx[kTile][kMlpIn];
  __shared__ float sh1[kTile][kMlpHid];
  __shared__ float sh2[kTile][kMlpHid];
  __shared__ float sdy[kTile];
  const int t = threadIdx.x;
  const int base = blockIdx.x * kTile;
  const int ns = min(kTile, nb - base);
  float* g = part + (size_t)blockIdx.x * kMlpNet;
  for (int e = t; e < kTile * kMlpIn; e += blockDim.x) {
    const int s = e / kMlpIn, k = e % kMlpIn;
    float v = 0.f;
    if (s < ns) {
      const long long q = idx ? idx[base + s] : base + s;
      v = X[q * kMlpIn + k];
    }
    sx[s][k] = v;
  }
  __syncthreads();
  for (int e = t; e < kTile * kMlpHid; e += blockDim.x) {
    const int s = e / kMlpHid, j = e % kMlpHid;
    float z = W[kMlpB1 + j];
    for (int k = 0; k < kMlpIn; ++k) z = fmaf(W[kMlpW1 + j * kMlpIn + k], sx[s][k], z);
    sh1[s][j] = tanhf(z);
  }
  __syncthreads();
  for (int e = t; e < kTile * kMlpHid; e += blockDim.x) {
    const int s = e / kMlpHid, j = e % kMlpHid;
    float z = W[kMlpB2 + j];
    for (int k = 0; k < kMlpHid; ++k) z = fmaf(W[kMlpW2 + j * kMlpHid + k], sh1[s][k], z);
    sh2[s][j] = tanhf(z);
  }
  __syncthreads();
  double loss = 0.0;
  if (t < kTile) {
    float y = W[kMlpB3];
    for (int j = 0; j < kMlpHid; ++j) y = fmaf(W[kMlpW3 + j], sh2[t][j], y);
    float dy = 0.f;
    if (t < ns) {
      const long long q = idx ? idx[base + t] : base + t;
      const float r = y - Y[q];
      const float w = r > 0.f ? over_w : 1.f;
      loss = (double)w * (double)r * (double)r;
      dy = 2.f * w * r * inv_n;
    }
    sdy[t] = dy;
  }
  if (t < 64) {  // wave 0 holds every sample of the tile
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off, 64);
    if (t == 0) loss_part[blockIdx.x] = loss;
  }
  __syncthreads();
  if (t < kMlpHid) {
    float acc = 0.f;
    for (int s = 0; s < kTile; ++s) acc = fmaf(sdy[s], sh2[s][t], acc);
    g[kMlpW3 + t] = acc;
  } else if (t == kMlpHid) {
    float acc = 0.f;
    for (int s = 0; s < kTile; ++s) acc += sdy[s];
    g[kMlpB3] = acc;
  }
  __syncthreads();
  // back through layer 2's tanh (in place: sh2 becomes dL/dz2)
  for (int e = t; e < kTile * kMlpHid; e += blockDim.x) {
    const int s = e / kMlpHid, j = e % kMlpHid;
    const float h = sh2[s][j];
    sh2[s][j] = sdy[s] * W[kMlpW3 + j] * (1.f - h * h);
  }
  __syncthreads();
  for (int e = t; e < kMlpHid * kMlpHid; e += blockDim.x) {
    const int j = e / kMlpHid, k = e % kMlpHid;
    float acc = 0.f;
    for (int s = 0; s < kTile; ++s) acc = fmaf(sh2[s][j], sh1[s][k], acc);
    g[kMlpW2 + e] = acc;
  }
  if (t < kMlpHid) {
    float acc = 0.f;
    for (int s = 0; s < kTile; ++s) acc += sh2[s][t];
    g[kMlpB2 + t] = acc;
  }
  __syncthreads();
  // back through layer 1's tanh (in place: sh1 becomes dL/dz1; each thread owns its element)
  for (int e = t; e < kTile * kMlpHid; e += blockDim.x) {
    const int s = e / kMlpHid, k = e % kMlpHid;
    float acc = 0.f;
    for (int j = 0; j < kMlpHid; ++j) acc = fmaf(sh2[s][j], W[kMlpW2 + j * kMlpHid + k], acc);
    const float h = sh1[s][k];
    sh1[s][k] = acc * (1.f - h * h);
  }
  __syncthreads();
  for (int e = t; e < kMlpHid * kMlpIn; e += blockDim.x) {
    const int j = e / kMlpIn, k = e % kMlpIn;
    float acc = 0.f;
    for (int s = 0; s < kTile; ++s) acc = fmaf(sh1[s][j], sx[s][k], acc);
    g[kMlpW1 + e] = acc;
  }
  if (t < kMlpHid) {
    float acc = 0.f;
    for (int s = 0; s < kTile; ++s) acc += sh1[s][t];
    g[kMlpB1 + t] = acc;
  }
}

// parameter-wise sum of the tile gradients (FP64, tile order) -> out
__global__ void k_mlp_reduce(const float* __restrict__ part, int nparts, double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpNet) return;
  double g = 0.0;
  for (int q = 0; q < nparts; ++q) g += (double)part[(size_t)q * kMlpNet + p];
  out[p] = g;
}

// Adam on the FP32 master weights from the summed tile gradients; refreshes the BF16 copy
__global__ void k_mlp_adam(float* __restrict__ master, float* __restrict__ m1, float* __restrict__ m2,
                           float* __restrict__ wq, const float* __restrict__ part, int nparts, float lr, float beta1,
                           float beta2, float eps, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpNet) return;
  double g = 0.0;
  for (int q = 0; q < nparts; ++q) g += (double)part[(size_t)q * kMlpNet + p];
  const float gf = (float)g;
  const float a = beta1 * m1[p] + (1.f - beta1) * gf;
  const float b = beta2 * m2[p] + (1.f - beta2) * gf * gf;
  m1[p] = a;
  m2[p] = b;
  const float w = master[p] - lr * (a / bc1) / (sqrtf(b / bc2) + eps);
  master[p] = w;
  wq[p] = bf16_round(w);
}

// dst = src with the first n_round values rounded to BF16 (the rest copied)
__global__ void k_bf16_copy(const float* __restrict__ src, float* __restrict__ dst, int n_round, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dst[p] = p < n_round ? bf16_round(src[p]) : src[p];
}

hipError_t launch_mlp_grad(const float* W, const float* X, const float* Y, const int* idx, int nb, float inv_n,
                           float over_w, float* part, double* loss_part, hipStream_t s) {
  const int tiles = (nb + kTile - 1) / kTile;
  if (tiles <= 0) return hipSuccess;
  k_mlp_grad<<<tiles, 256, 0, s>>>(W, X, Y, idx, nb, inv_n, over_w, part, loss_part);
  return hipGetLastError();
}
hipError_t launch_mlp_reduce(const float* part, int nparts, double* out, hipStream_t s) {
  k_mlp_reduce<<<(kMlpNet + 255) / 256, 256, 0, s>>>(part, nparts, out);
  return hipGetLastError();
}
hipError_t launch_mlp_adam(float* master, float* m1, float* m2, float* wq, const float* part, int nparts, float lr,
                           float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t s) {
  k_mlp_adam<<<(kMlpNet + 255) / 256, 256, 0, s>>>(master, m1, m2, wq, part, nparts, lr, beta1, beta2, eps, bc1,
                                                      bc2);
  return hipGetLastError();
}
hipError_t launch_bf16_copy(const float* src, float* dst, int n_round, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_bf16_copy<<<(n + 255) / 256, 256, 0, s>>>(src, dst, n_round, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Allocation-free gradient (bs32_mlp_grad_noalloc): the same kernels as
// bs32_mlp_grad, with every intermediate buffer in one file-scope device array.
// Layout: standardized features [kNaMaxSamples][9] FP32 | BF16 copy of the
// weights [kMlpParams] FP32 | tile gradients [kNaMaxSamples/64][kMlpNet] FP32 |
// tile losses [kNaMaxSamples/64] FP64.  Every kernel below writes each byte it
// later reads, so nothing needs clearing between calls.
// ---------------------------------------------------------------------------
constexpr size_t kNaX = (size_t)kNaMaxSamples * kMlpIn * sizeof(float);
constexpr size_t kNaWq = ((size_t)kMlpParams * sizeof(float) + 255) / 256 * 256;
constexpr size_t kNaPart = (size_t)(kNaMaxSamples / kTile) * kMlpNet * sizeof(float);
constexpr size_t kNaLoss = (size_t)(kNaMaxSamples / kTile) * sizeof(double);
constexpr size_t kNaBytes = kNaX + kNaWq + kNaPart + kNaLoss;
static_assert(kNaX % 256 == 0 && kNaPart % 256 == 0, "scratch sections stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

// the array's address on each device (host code never uses its name for memory)
constexpr int kNaMaxDevices = 64;
static void* g_scratch_dev[kNaMaxDevices] = {};
static std::mutex g_scratch_mu;

hipError_t noalloc_bind(int device) {
  if (device < 0 || device >= kNaMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));  // the current device's copy
  if (e != hipSuccess) return e;
  g_scratch_dev[device] = ptr;
  return hipSuccess;
}

// FP32 standardization of raw features, the same two roundings as bs32_mlp_grad's host loop
__global__ void k_na_standardize(const float* __restrict__ W, const float* __restrict__ F, int n,
                                 float* __restrict__ X) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * kMlpIn) return;
  const int k = e % kMlpIn;
  X[e] = (F[e] - W[kMlpMu + k]) * W[kMlpInvSd + k];
}

// the untrained standardization gets a zero gradient; the loss is the tile losses
// summed in tile order, over n
__global__ void k_na_finish(const double* __restrict__ lp, int tiles, int n, double* __restrict__ grad,
                            double* __restrict__ loss) {
  const int t = threadIdx.x;
  if (t < kMlpParams - kMlpNet) grad[kMlpNet + t] = 0.0;
  if (t == 0 && loss) {
    double L = 0.0;
    for (int q = 0; q < tiles; ++q) L += lp[q];
    *loss = L / (double)n;
  }
}

hipError_t launch_mlp_grad_noalloc(int device, const float* W, const float* F, const float* Y, int n, double* grad,
                                   double* loss, hipStream_t s) {
  if (device < 0 || device >= kNaMaxDevices || !g_scratch_dev[device]) return hipErrorNotInitialized;
  if (n < 1 || n > kNaMaxSamples) return hipErrorInvalidValue;
  unsigned char* base = (unsigned char*)g_scratch_dev[device];
  float* X = (float*)base;
  float* wq = (float*)(base + kNaX);
  float* part = (float*)(base + kNaX + kNaWq);
  double* lp = (double*)(base + kNaX + kNaWq + kNaPart);
  const int tiles = (n + kTile - 1) / kTile;
  k_na_standardize<<<(n * kMlpIn + 255) / 256, 256, 0, s>>>(W, F, n, X);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_bf16_copy(W, wq, kMlpNet, kMlpParams, s);
  if (e == hipSuccess) e = launch_mlp_grad(wq, X, Y, nullptr, n, 1.0f / (float)n, kMlpOverW, part, lp, s);
  if (e == hipSuccess) e = launch_mlp_reduce(part, tiles, grad, s);
  if (e == hipSuccess) {
    k_na_finish<<<1, 64, 0, s>>>(lp, tiles, n, grad, loss);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace bs32
