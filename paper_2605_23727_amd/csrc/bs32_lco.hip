// bs32_lco.hip -- analytic solution of the coupled linear oscillators (paper
// Benchmark 1, eq. (LCO), uniform weights M_ij = 1/N) and the real local error
// of eq. (LCO-Local-Error): diagnostics of the solver's accuracy, not steps of it.
//
// With the means m = (1/N) sum_j X_j1 and w = (1/N) sum_j X_j2 the coupling of
// agent i is m - X_i1, so the means turn as an undamped oscillator (m' = w,
// w' = -m) and the deviations d_i = X_i1 - m, e_i = X_i2 - w move as a damped one
// (d' = e - d, e' = -d).  That matrix has trace -1 and determinant 1, so its
// exponential is e^{-h/2} (cos(wh) I + sin(wh)/w (B + I/2)) with w = sqrt(3)/2.
//
// One workgroup per state: the two means by a fixed-order block reduction, then
// the flow of every agent (and, for the local error, the largest scaled
// deviation from the next recorded state).  States are agent-major FP64 (2N
// values each), as the solver's public interface holds them.
#include "bs32_internal.hpp"

namespace bs32 {
namespace {

constexpr int kLcoThreads = 256;
constexpr double kLcoOmega = 0.86602540378443864676;  // sqrt(3) / 2

// means of the two components of one state (every thread receives them)
__device__ void lco_means(const double* __restrict__ X, long long n, double* m, double* w) {
  __shared__ double s0[kLcoThreads], s1[kLcoThreads];
  const int tid = threadIdx.x;
  double a0 = 0.0, a1 = 0.0;
  for (long long i = tid; i < n; i += kLcoThreads) {
    a0 += X[2 * i];
    a1 += X[2 * i + 1];
  }
  s0[tid] = a0;
  s1[tid] = a1;
  __syncthreads();
  for (int off = kLcoThreads / 2; off > 0; off >>= 1) {
    if (tid < off) {
      s0[tid] += s0[tid + off];
      s1[tid] += s1[tid + off];
    }
    __syncthreads();
  }
  *m = s0[0] / (double)n;
  *w = s1[0] / (double)n;
  __syncthreads();  // the shared sums may be reused by the caller's next state
}

struct LcoStep {
  double c, s;          // cos h, sin h (mean rotation)
  double damp, co, so;  // e^{-h/2}, cos(w h), sin(w h) / w (deviation motion)
};

__device__ LcoStep lco_step(double h) {
  LcoStep q;
  q.c = cos(h);
  q.s = sin(h);
  q.damp = exp(-0.5 * h);
  q.co = cos(kLcoOmega * h);
  q.so = sin(kLcoOmega * h) / kLcoOmega;
  return q;
}

__device__ void lco_agent(const LcoStep& q, double m, double w, double x1, double x2, double* y1, double* y2) {
  const double mh = q.c * m + q.s * w;
  const double wh = q.c * w - q.s * m;
  const double d = x1 - m, e = x2 - w;
  // (B + I/2)(d, e) = (-d/2 + e, -d + e/2)
  const double dh = q.damp * (q.co * d + q.so * (e - 0.5 * d));
  const double eh = q.damp * (q.co * e + q.so * (0.5 * e - d));
  *y1 = mh + dh;
  *y2 = wh + eh;
}

// max that keeps a NaN (a non-finite state must not read as a small error)
__device__ double lco_nanmax(double a, double b) { return (a != a || b != b) ? NAN : fmax(a, b); }

__global__ __launch_bounds__(kLcoThreads) void k_lco_flow(const double* __restrict__ X, const double* __restrict__ h,
                                                          long long n, double* __restrict__ out) {
  const long long k = blockIdx.x;
  const double* x = X + k * 2 * n;
  double* y = out + k * 2 * n;
  double m, w;
  lco_means(x, n, &m, &w);
  const LcoStep q = lco_step(h[k]);
  for (long long i = threadIdx.x; i < n; i += kLcoThreads) lco_agent(q, m, w, x[2 * i], x[2 * i + 1], &y[2 * i], &y[2 * i + 1]);
}

__global__ __launch_bounds__(kLcoThreads) void k_lco_local_error(const double* __restrict__ states,
                                                                 const double* __restrict__ h, long long n,
                                                                 double delta, double* __restrict__ err) {
  __shared__ double sm[kLcoThreads];
  const long long k = blockIdx.x;
  const double* x = states + k * 2 * n;
  const double* xn = x + 2 * n;  // the next recorded state
  double m, w;
  lco_means(x, n, &m, &w);
  const LcoStep q = lco_step(h[k]);
  double r = 0.0;
  for (long long i = threadIdx.x; i < n; i += kLcoThreads) {
    double e1, e2;
    lco_agent(q, m, w, x[2 * i], x[2 * i + 1], &e1, &e2);
    r = lco_nanmax(r, fabs(xn[2 * i] - e1) / fmax(fabs(e1), delta));
    r = lco_nanmax(r, fabs(xn[2 * i + 1] - e2) / fmax(fabs(e2), delta));
  }
  const int tid = threadIdx.x;
  sm[tid] = r;
  __syncthreads();
  for (int off = kLcoThreads / 2; off > 0; off >>= 1) {
    if (tid < off) sm[tid] = lco_nanmax(sm[tid], sm[tid + off]);
    __syncthreads();
  }
  if (tid == 0) err[k] = sm[0];
}

}  // namespace

hipError_t launch_lco_flow(const double* X, const double* h, long long n, long long count, double* out,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lco_flow, dim3((unsigned)count), dim3(kLcoThreads), 0, s, X, h, n, out);
  return hipGetLastError();
}

hipError_t launch_lco_local_error(const double* states, const double* h, long long n, long long steps, double delta,
                                  double* err, hipStream_t s) {
  if (steps <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lco_local_error, dim3((unsigned)steps), dim3(kLcoThreads), 0, s, states, h, n, delta, err);
  return hipGetLastError();
}

}  // namespace bs32
