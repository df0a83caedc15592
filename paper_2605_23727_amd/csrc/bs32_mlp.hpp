// bs32_mlp.hpp -- the learned step-size proposer: a 9 -> 64 -> 64 -> 1 tanh
// network with BF16-valued weights and FP32 accumulation.  One device routine
// evaluates it for one workgroup; the controller (inference) and the training
// kernels both use it, so the two see the same arithmetic.
#pragma once
#include <hip/hip_runtime.h>

namespace bs32 {

constexpr int kMlpIn = 9;
constexpr int kMlpHid = 64;
// parameter vector: W1[64][9], b1[64], W2[64][64], b2[64], w3[64], b3 (the network,
// BF16 values), then mu[9], inv_sd[9] (feature standardization, FP32 values)
constexpr int kMlpW1 = 0;
constexpr int kMlpB1 = kMlpW1 + kMlpHid * kMlpIn;
constexpr int kMlpW2 = kMlpB1 + kMlpHid;
constexpr int kMlpB2 = kMlpW2 + kMlpHid * kMlpHid;
constexpr int kMlpW3 = kMlpB2 + kMlpHid;
constexpr int kMlpB3 = kMlpW3 + kMlpHid;
constexpr int kMlpNet = kMlpB3 + 1;  // 4865 network weights
constexpr int kMlpMu = kMlpNet;
constexpr int kMlpInvSd = kMlpMu + kMlpIn;
constexpr int kMlpParams = kMlpInvSd + kMlpIn;  // 4883

// Features of the proposal after attempt n (most recent first):
//   f[0..3] = log h_n, log h_{n-1}, log h_{n-2}, log h_{n-3}     (attempted steps)
//   f[4..7] = log(max(E, 1e-30 Rel) / Rel) of the same attempts
//   f[8]    = log max_k |K1_k| / max(|X^n_k|, Ab/Rel)           (weighted size of f(t_n, X^n))
// The network reads x_k = (f_k - mu_k) * inv_sd_k (FP32).
// Output: delta = log(h_{n+1} / h_n).  Guards: the proposal is used only when
// every |x_k| <= kMlpXMax (the features lie where the network was trained) and
// delta lies inside [log 0.2, log 5] and within log 2 of the classical rule's
// own step ratio; otherwise the classical rule decides.
constexpr double kMlpDeltaMin = -1.6094379124341003;  // log 0.2
constexpr double kMlpDeltaMax = 1.6094379124341003;   // log 5
constexpr double kMlpTrust = 0.6931471805599453;      // log 2
constexpr float kMlpXMax = 4.0f;
constexpr float kMlpOverW = 4.0f;  // loss weight of an overshooting proposal (a rejection costs 3 RHS)

// Forward pass of one sample by one workgroup (blockDim >= 64): feat[9] in LDS,
// h1/h2 scratch [64] in LDS; returns the output on every thread (NaN when a
// standardized feature lies outside [-kMlpXMax, kMlpXMax]).
__device__ inline float mlp_forward_wg(const float* __restrict__ W, const float* feat, float* h1, float* h2,
                                       float* red) {
  const int t = threadIdx.x;
  if (t < kMlpHid) {
    float z = W[kMlpB1 + t];
    for (int k = 0; k < kMlpIn; ++k) {
      const float x = (feat[k] - W[kMlpMu + k]) * W[kMlpInvSd + k];
      z = fmaf(W[kMlpW1 + t * kMlpIn + k], x, z);
    }
    h1[t] = tanhf(z);
  }
  __syncthreads();
  if (t < kMlpHid) {
    float z = W[kMlpB2 + t];
    for (int k = 0; k < kMlpHid; ++k) z = fmaf(W[kMlpW2 + t * kMlpHid + k], h1[k], z);
    h2[t] = tanhf(z);
  }
  __syncthreads();
  if (t == 0) {
    float y = W[kMlpB3];
    for (int k = 0; k < kMlpHid; ++k) y = fmaf(W[kMlpW3 + k], h2[k], y);
    for (int k = 0; k < kMlpIn; ++k) {  // outside the trained region: no proposal
      const float x = (feat[k] - W[kMlpMu + k]) * W[kMlpInvSd + k];
      if (!(fabsf(x) <= kMlpXMax)) y = __builtin_nanf("");
    }
    red[0] = y;
  }
  __syncthreads();
  return red[0];
}

}  // namespace bs32
