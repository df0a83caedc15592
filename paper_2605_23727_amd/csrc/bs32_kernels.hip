// bs32_kernels.hip -- gfx950 kernels of the BS3(2) hot path.
//
// One attempt of the embedded pair (Sec. 2.2, eq. (Stage-ODE23)) is four launches:
//   S2       : P = A V(Y2) ; K2 = F(Y2) + coupling(P) ; Y3 = X + h a32 K2 ; V(Y3)      N^2
//   S3       : P = A V(Y3) ; K3 ; X^{n+1} = X + h (b1 K1 + b2 K2 + b3 K3) ; V(X^{n+1})    N^2
//   S4       : P = A V(X^{n+1}) ; K4 (FSAL: the next K1) ; error h sum (b_l - bt_l) K_l ;
//              per-block weighted max (eq. (ERROR-O23))                                  N^2
//   finalize : one workgroup: grid max, accept/reject, controller, failure checks,
//              then Y2 = X + h a21 K1 and V(Y2) of the next attempt                     O(N)
// The state is component-major (SoA) on the device, the coupling matrix A is
// row-major with a padded leading dimension, and every stage combination is FP64
// (Sec. 2.3 cast rules).  No workgroup ever waits for another: split-K runs across
// the waves of one workgroup and is reduced through LDS in a fixed order, so
// every sum has a fixed order and a solve is bitwise reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "bs32_internal.hpp"
#include "bs32_mlp.hpp"

// The file compiles as several translation units (BS32_PART = 0 .. 8), each
// instantiating a disjoint family of kernels, so that the build runs them in
// parallel; without BS32_PART it is a single unit holding everything.
#ifndef BS32_PART
#define BS32_PART -1
#endif
#define BS32_IN(p) (BS32_PART < 0 || BS32_PART == (p))

namespace bs32 {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// streaming load of the coupling matrix; NT: non-temporal hint (read once, keep
// the vector operand resident in the caches instead)
template <bool NT, typename T>
__device__ __forceinline__ T ldA(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

#if BS32_IN(0)
int dim_of(int kind) {
  return kind == 1 ? 2 : kind == 2 ? 2 : kind == 3 ? 1 : kind == 4 ? 3 : kind == 5 ? 4 : 0;
}
int vcols_of(int kind, int pairwise) { return (kind == 3 && !pairwise) ? 2 : 1; }
#endif

// constants of the clock / cell-cycle model, paper eq. (CC) (Sec. 2.1); k1 is per cell
constexpr double kCcK0 = 2.0, kCcK2 = 0.144832, kCcK3 = 2.0, kCcA = 2.0, kCcB = 0.7, kCcC = 0.8,
                 kCcEps = 0.228249;
#if BS32_IN(0)
size_t fmt_bytes(int fmt) {
  return fmt == F_F64 ? 8 : (fmt == F_F32 || fmt == F_BF16X2) ? 4 : (fmt == F_BF16 || fmt == F_F16) ? 2 : 1;
}
#endif

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double nanmax(double a, double b) {
  if (a != a || b != b) return __builtin_nan("");
  return a > b ? a : b;
}
__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
// a double moved between lanes by a DPP control (both halves), VALU only
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// maximum over the wave (NaN wins; exact, so the order does not matter): rotations by
// 8, 4, 2, 1 lanes within each row of 16 (DPP row_ror), then across the four rows.
// Every lane of the wave must be active.
__device__ __forceinline__ double wave_nanmax(double v) {
  v = nanmax(v, dpp_f64<0x128>(v));
  v = nanmax(v, dpp_f64<0x124>(v));
  v = nanmax(v, dpp_f64<0x122>(v));
  v = nanmax(v, dpp_f64<0x121>(v));
  v = nanmax(v, __shfl_xor(v, 16, 64));
  return nanmax(v, __shfl_xor(v, 32, 64));
}

// XCD-aware block order: workgroups are dealt to the 8 XCDs round-robin; give each
// XCD a contiguous range of row blocks.
__device__ __forceinline__ int block_row(const Args& a) {
  const int bid = blockIdx.x;
  return (a.nrb % 8 == 0) ? (bid % 8) * (a.nrb / 8) + bid / 8 : bid;
}

// ---------------------------------------------------------------------------
// Storage formats: round to nearest, ties to even, straight from the FP64 bits
// (no intermediate FP32 rounding).  e4m3 is the OCP e4m3fn format with
// saturation to +-448 (the encoding gfx950's FP8 matrix instructions read).
// p: significand bits incl. the implicit one; emin: exponent of the smallest normal.
// ---------------------------------------------------------------------------
struct FmtDesc {
  int p, emin, bias, ebits;
  bool e4m3;
};
__host__ __device__ constexpr FmtDesc fmt_desc(int fmt) {
  return fmt == F_BF16 ? FmtDesc{8, -126, 127, 8, false}
         : fmt == F_F16 ? FmtDesc{11, -14, 15, 5, false}
                        : FmtDesc{4, -6, 7, 4, true};
}

__device__ inline uint32_t encode_rne(double x, FmtDesc f) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const int nb = 1 + f.ebits + (f.p - 1);
  const uint32_t sign = (uint32_t)(u >> 63) << (nb - 1);
  const unsigned long long a = u & 0x7fffffffffffffffULL;
  const uint32_t emask = (1u << f.ebits) - 1u;
  if (a > 0x7ff0000000000000ULL) return f.e4m3 ? (sign | 0x7fu) : (sign | (emask << (f.p - 1)) | (1u << (f.p - 2)));
  if (a == 0x7ff0000000000000ULL) return f.e4m3 ? (sign | 0x7eu) : (sign | (emask << (f.p - 1)));
  const int e = (int)(a >> 52);
  if (e == 0) return sign;  // FP64 subnormals lie far below every target's smallest subnormal
  const int E = e - 1023;
  const unsigned long long mant = (a & 0xfffffffffffffULL) | (1ULL << 52);
  int q = (E > f.emin ? E : f.emin) - (f.p - 1);  // exponent of one target quantum
  const int sh = 52 + q - E;
  if (sh >= 54) return sign;  // below half the smallest subnormal
  unsigned long long r = mant >> sh;
  const unsigned long long rem = mant & ((1ULL << sh) - 1ULL);
  const unsigned long long half = 1ULL << (sh - 1);
  if (rem > half || (rem == half && (r & 1ULL))) ++r;
  if (r == 0) return sign;
  if (r >> f.p) {
    r >>= 1;
    ++q;
  }
  uint32_t bexp, frac;
  if (r < (1ULL << (f.p - 1))) {
    bexp = 0;
    frac = (uint32_t)r;
  } else {
    bexp = (uint32_t)(q + (f.p - 1) + f.bias);
    frac = (uint32_t)(r - (1ULL << (f.p - 1)));
  }
  if (f.e4m3) {
    if (bexp > 15u || (bexp == 15u && frac == 7u)) return sign | 0x7eu;
  } else if (bexp >= emask) {
    return sign | (emask << (f.p - 1));
  }
  return sign | (bexp << (f.p - 1)) | frac;
}

__device__ inline double decode_bits(uint32_t b, FmtDesc f) {
  const int nb = 1 + f.ebits + (f.p - 1);
  const bool s = (b >> (nb - 1)) & 1u;
  const uint32_t emask = (1u << f.ebits) - 1u;
  const uint32_t be = (b >> (f.p - 1)) & emask;
  const uint32_t fr = b & ((1u << (f.p - 1)) - 1u);
  double v;
  if (f.e4m3 && be == emask && fr == 7u) v = __builtin_nan("");
  else if (!f.e4m3 && be == emask) v = fr ? __builtin_nan("") : __builtin_inf();
  else if (be == 0) v = ldexp((double)fr, f.emin - (f.p - 1));
  else v = ldexp((double)(fr + (1u << (f.p - 1))), (int)be - f.bias - (f.p - 1));
  return s ? -v : v;
}

// one pointer of a two-pointer pair in the argument block: a select, never an
// index computed at run time (which would copy the whole by-value block to scratch)
template <typename P>
__device__ __forceinline__ P pick2(P const (&p)[2], int q) {
  return q ? p[1] : p[0];
}

// ---------------------------------------------------------------------------
// vector operand of one agent and its split into reduced-format terms
// ---------------------------------------------------------------------------
// the vector operand of a coupled component y: (sin y, cos y) for the Kuramoto
// matrix-vector form, y itself otherwise (linear couplings, pairwise forms)
__device__ __forceinline__ void vec_of(const Args& a, double y, double* v) {
  if (a.kind == 3 && !a.pairwise) {
    sincos(y, &v[0], &v[1]);
  } else {
    v[0] = v[1] = y;
  }
}

// split terms of a storage format: count and exponent shift between terms
template <int VF>
struct VSplit {
  static constexpr int T = VF == F_E4M3 ? 3 : 2;
  static constexpr int S = VF == F_F32 ? 24 : VF == F_BF16 ? 8 : VF == F_F16 ? 11 : 4;
};

// FP64 -> FP32 rounded to odd: truncate toward zero, then set the last bit when the
// value was inexact.  Rounding that result to a format of at most 22 significant
// bits (to nearest, ties to even) gives the same value as rounding the FP64 value
// straight to that format, so the hardware conversions from FP32 serve as an
// exact FP64 rounding.
__device__ __forceinline__ float f32_round_odd(double x) {
  const float f = (float)x;
  const double b = (double)f;
  if (b == x) return f;
  unsigned u = __float_as_uint(f);
  if (fabs(b) > fabs(x)) --u;  // the nearest value lay away from zero: step back toward it
  return __uint_as_float(u | 1u);
}

// one split term: Q(x) in storage format VF (round to nearest even from FP64; e4m3
// saturates at +-448 like encode_rne); returns the term's value, *bits its encoding
template <int VF>
__device__ __forceinline__ double split_q(double x, uint32_t* bits) {
  if constexpr (VF == F_BF16) {
    const unsigned u = __float_as_uint(f32_round_odd(x));
    const unsigned r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;  // finite inputs: no carry into NaN
    *bits = r;
    return (double)__uint_as_float(r << 16);
  } else if constexpr (VF == F_F16) {
    const _Float16 h = (_Float16)f32_round_odd(x);
    *bits = (uint32_t)__builtin_bit_cast(unsigned short, h);
    return (double)(float)h;
  } else {
    if (x != x) {  // NaN keeps its encoding (the saturating clamp below would turn it into a number)
      *bits = 0x7fu;
      return x;
    }
    const float f = fminf(fmaxf(f32_round_odd(x), -448.0f), 448.0f);
    const uint32_t b = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(f, f, 0, false) & 0xffu;
    *bits = b;
    return (double)__builtin_amdgcn_cvt_f32_fp8((int)b, 0);
  }
}

// Vq layout: [c * T + t][ld]; term t holds Q(r_t 2^(t S)), r_0 = v,
// r_{t+1} = r_t - 2^(-t S) Q(r_t 2^(t S)).  (Scaling by a power of two is exact,
// so the products below equal ldexp.)  Writes column c of agent i.
template <int VF>
__device__ __forceinline__ void write_vq_t(const Args& a, void* Vq, long long i, int c, double v) {
  if constexpr (VF == F_F64) {
    return;
  } else {
    if (Vq == nullptr) return;
    constexpr int T = VSplit<VF>::T, S = VSplit<VF>::S;
    double r = v;
    if (fabs(r) > a.vmax && isfinite(r)) *a.rflag = 1u;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const long long idx = (long long)(c * T + t) * a.ld + i;
      const double x = r * __builtin_ldexp(1.0, t * S);
      double qv;
      if constexpr (VF == F_F32) {
        const float f = (a.vsingle && t > 0) ? 0.0f : (float)x;  // pair terms in single: one term
        ((float*)Vq)[idx] = f;
        qv = (double)f;
      } else {
        uint32_t b;
        qv = split_q<VF>(x, &b);
        if constexpr (VF == F_E4M3) ((uint8_t*)Vq)[idx] = (uint8_t)b;
        else ((uint16_t*)Vq)[idx] = (uint16_t)b;
      }
      r = r - qv * __builtin_ldexp(1.0, -t * S);
    }
  }
}

// columns [c0, c1) of agent i's operand into buffer buf (FP64 copy and split terms)
// (the row epilogues give the two Kuramoto columns to two lanes of one wave: both
// take the one sincos, which runs once for the wave, and split one column each)
template <int VF>
__device__ __forceinline__ void write_operand_t(const Args& a, int buf, long long i, double y, int c0, int c1) {
  double v[2];
  vec_of(a, y, v);
  for (int c = c0; c < c1; ++c) {
    const double vc = c ? v[1] : v[0];
    pick2(a.V64, buf)[i * a.m + c] = vc;
    write_vq_t<VF>(a, pick2(a.Vq, buf), i, c, vc);
  }
}

// every column, with the format known only at run time (prep and finalize serve every format)
__device__ __forceinline__ void write_operand(const Args& a, int buf, long long i, double y) {
  switch (a.vfmt) {
    case F_F32: write_operand_t<F_F32>(a, buf, i, y, 0, a.m); break;
    case F_BF16: write_operand_t<F_BF16>(a, buf, i, y, 0, a.m); break;
    case F_F16: write_operand_t<F_F16>(a, buf, i, y, 0, a.m); break;
    case F_E4M3: write_operand_t<F_E4M3>(a, buf, i, y, 0, a.m); break;
    default: write_operand_t<F_F64>(a, buf, i, y, 0, a.m); break;
  }
}

// F_i(Y_i) + coupling of agent i from the contraction P_i (Sec. 2.1 benchmarks with
// weights A_ij/N).  vself: the agent's own vector operand (sin, cos of theta_i);
// p: its parameter (omega or b); rs: its row sum of the stored weights.
// LEAN: the matrix-vector systems only (ensembles serve no pairwise coupling), so
// that the code of a kernel's per-item tail stays small
template <bool LEAN = false>
__device__ __forceinline__ void rhs_agent(const Args& a, const double* y, const double* P, const double* vself,
                                          double p, double rs, double* k) {
  switch (a.kind) {
    case 1:  // coupled oscillators: x' = v, v' = -w^2 x + (1/N) sum_j A_ij (x_j - x_i)
      k[0] = y[1];
      k[1] = -p * p * y[0] + a.invN * (P[0] - y[0] * rs);
      break;
    case 2:  // paper eq. (LCO): x' = v + (1/N) sum_j A_ij (x_j - x_i), v' = -x
      k[0] = y[1] + a.invN * (P[0] - y[0] * rs);
      k[1] = -y[0];
      break;
    case 3:  // paper eq. (Kuramoto): sum_j A_ij sin(th_j - th_i) = cos th_i (A sin th)_i - sin th_i (A cos th)_i
      if (!LEAN && a.pairwise) k[0] = p + a.gain * a.invN * P[0];  // P = sum_j A_ij sin(th_j - th_i) pair by pair
      else k[0] = p + a.gain * a.invN * (vself[1] * P[0] - vself[0] * P[1]);
      break;
    case 5: {  // paper eq. (CC): P = sum_j A_ij arctan(X_j1 - X_i1), the pair prefactor depends on X_i2
      if constexpr (!LEAN) {
        const double th = p / (kCcK0 - p);
        const double q = kCcK0 * th / (th + y[1] * y[1] * y[1] * y[1]);
        k[0] = q * (kCcA * y[0] * y[0] + 1.0) - p * y[0] + (q * kCcA) * a.gain * a.invN * P[0];
        k[1] = kCcK2 * (y[0] - y[1]);
        k[2] = y[2] * (1.0 - y[2] * y[2] / 3.0) - y[3] + a.stim * (1.0 - kCcK3 * kCcK3 / (kCcK3 * kCcK3 + y[0] * y[0]));
        k[3] = kCcEps * (y[2] + kCcB - kCcC * y[3]);
      }
      break;
    }
    default: {  // Goodwin clock: x' = 1/(1+z^10) - b x + (kappa/N) sum_j C_ij (x_j - x_i)
      const double z2 = y[2] * y[2], z4 = z2 * z2, z8 = z4 * z4;
      k[0] = 1.0 / (1.0 + z8 * z2) - p * y[0] + a.gain * a.invN * (P[0] - y[0] * rs);
      k[1] = y[0] - p * y[1];
      k[2] = y[1] - p * y[2];
      break;
    }
  }
}

// The same right-hand sides with the agent term and the coupling combination in
// FP32 (the recipes' "F in single"): inputs rounded to FP32, FP32 arithmetic.
__device__ __forceinline__ void rhs_agent_f32(const Args& a, const double* y, const double* P, const double* vself,
                                              double pd, double rsd, double* k) {
  const float p = (float)pd, rs = (float)rsd;
  const float invN = (float)a.invN, g = (float)a.gain;
  const float y0 = (float)y[0];
  switch (a.kind) {
    case 1: {
      const float inter = invN * ((float)P[0] - y0 * rs);
      k[0] = (double)(float)y[1];
      k[1] = (double)((-p * p * y0) + inter);
      break;
    }
    case 2: {
      const float inter = invN * ((float)P[0] - y0 * rs);
      k[0] = (double)((float)y[1] + inter);
      k[1] = (double)(-y0);
      break;
    }
    case 3: {
      const float inter = a.pairwise ? g * invN * (float)P[0]
                                     : g * invN * ((float)vself[1] * (float)P[0] - (float)vself[0] * (float)P[1]);
      k[0] = (double)(p + inter);
      break;
    }
    case 5: {
      const float y1 = (float)y[1], y2 = (float)y[2], y3 = (float)y[3];
      const float th = p / ((float)kCcK0 - p);
      const float q = (float)kCcK0 * th / (th + y1 * y1 * y1 * y1);
      const float k3s = (float)kCcK3 * (float)kCcK3;
      const float inter = (q * (float)kCcA) * g * invN * (float)P[0];
      k[0] = (double)((q * ((float)kCcA * y0 * y0 + 1.0f) - p * y0) + inter);
      k[1] = (double)((float)kCcK2 * (y0 - y1));
      k[2] = (double)(y2 * (1.0f - y2 * y2 / 3.0f) - y3 + (float)a.stim * (1.0f - k3s / (k3s + y0 * y0)));
      k[3] = (double)((float)kCcEps * (y2 + (float)kCcB - (float)kCcC * y3));
      break;
    }
    default: {
      const float y1 = (float)y[1], y2 = (float)y[2];
      const float z2 = y2 * y2, z4 = z2 * z2, z8 = z4 * z4;
      const float inter = g * invN * ((float)P[0] - y0 * rs);
      k[0] = (double)((1.0f / (1.0f + z8 * z2) - p * y0) + inter);
      k[1] = (double)(y0 - p * y1);
      k[2] = (double)(y1 - p * y2);
      break;
    }
  }
}

// (LEAN: no recipes either; ensembles run the storage-format modes only)
template <bool LEAN = false>
__device__ __forceinline__ void rhs_eval(const Args& a, const double* y, const double* P, const double* vself,
                                         double p, double rs, double* k) {
  if (!LEAN && a.fsingle) rhs_agent_f32(a, y, P, vself, p, rs, k);
  else rhs_agent<LEAN>(a, y, P, vself, p, rs, k);
}

// Single keeps its solution and stage inputs in FP32
__device__ __forceinline__ double sstore(const Args& a, double v) { return a.sstate ? (double)(float)v : v; }

// ---------------------------------------------------------------------------
// stage epilogue of one row.  Its inputs are loaded by load_row before the
// contraction loop, so that their latency hides behind the stream of A; the
// epilogue returns the row's contributions to the block maxima.
// ---------------------------------------------------------------------------
struct RowIn {
  double x[4], xn[4], k1[4], k2[4], k3[4];  // X^n, X^{n+1}, K1, K2, K3 (those the stage reads)
  double p, rs, vs[2];                      // parameter, row sum, own vector operand
};

__device__ __forceinline__ void load_row(const Args& a, const Ctl* ctl, long long i, RowIn& r) {
  const long long np = a.np;
  const int st = a.stage;
  if (st >= ST_D2) return;  // the Dormand-Prince epilogue loads its own inputs
  const double* X = pick2(a.X, ctl->xi);
  const double* K1 = pick2(a.Kf, ctl->ki);
  const double* Vin = pick2(a.V64, vin_of(st));
  r.p = a.param[i];
  r.rs = a.rsum ? a.rsum[i] : 0.0;  // pairwise systems with uniform weights keep no row sums
  r.vs[0] = Vin[i * a.m];
  r.vs[1] = a.m > 1 ? Vin[i * a.m + 1] : 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    r.x[c] = r.xn[c] = r.k1[c] = r.k2[c] = r.k3[c] = 0.0;
    if (c >= a.d) continue;
    r.x[c] = X[c * np + i];
    if (st != ST_INIT && st != ST_RHS) r.k1[c] = K1[c * np + i];
    if (st == ST_S3 || st == ST_S4) r.k2[c] = a.K2[c * np + i];
    if (st == ST_S4) {
      r.k3[c] = a.K3[c * np + i];
      r.xn[c] = pick2(a.X, 1 - ctl->xi)[c * np + i];
    }
  }
}

// col: the operand column this thread writes (Kuramoto: 0 = sin, 1 = cos, on two
// threads per row so that the two transcendentals and their splits run side by side);
// the thread of column 0 also stores the row's stages and its maxima.  col = -1:
// one thread does all of it.
template <int VF, bool LEAN = false>
__device__ __forceinline__ void epilogue(const Args& a, const Ctl* ctl, long long i, const double* P, const RowIn& r, double* r0,
                         double* r1, int col) {
  const int d = a.d;
  const long long np = a.np;
  double y[4] = {0.0, 0.0, 0.0, 0.0}, k[4] = {0.0, 0.0, 0.0, 0.0};
  const double ha = ctl->ha;
  *r0 = 0.0;
  *r1 = 0.0;
  if (col > 0 && a.stage != ST_S2 && a.stage != ST_S3) return;  // no operand to write
  const bool lead = col <= 0;
  const int c0 = col < 0 ? 0 : col, c1 = col < 0 ? a.m : col + 1;
  switch (a.stage) {
    case ST_INIT:
    case ST_RHS: {
#pragma unroll
      for (int c = 0; c < 4; ++c) y[c] = r.x[c];
      rhs_eval<LEAN>(a, y, P, r.vs, r.p, r.rs, k);
      double* K = pick2(a.Kf, ctl->ki);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c >= d) break;
        K[c * np + i] = k[c];
        const double sc = ctl->atol + ctl->rtol * fabs(y[c]);
        *r0 = nanmax(*r0, fabs(y[c]) / sc);
        *r1 = nanmax(*r1, fabs(k[c]) / sc);
      }
      break;
    }
    case ST_H0: {
#pragma unroll
      for (int c = 0; c < 4; ++c) y[c] = r.x[c] + ctl->h0probe * r.k1[c];
      rhs_eval<LEAN>(a, y, P, r.vs, r.p, r.rs, k);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c >= d) break;
        const double sc = ctl->atol + ctl->rtol * fabs(r.x[c]);
        *r0 = nanmax(*r0, fabs(k[c] - r.k1[c]) / sc);
      }
      break;
    }
    case ST_S2: {
#pragma unroll
      for (int c = 0; c < 4; ++c) y[c] = sstore(a, r.x[c] + ha * (kA21 * r.k1[c]));
      rhs_eval<LEAN>(a, y, P, r.vs, r.p, r.rs, k);
      if (lead) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (c < d) a.K2[c * np + i] = k[c];
      }
      write_operand_t<VF>(a, 1, i, sstore(a, r.x[0] + ha * (kA32 * k[0])), c0, c1);  // stage-3 input
      break;
    }
    case ST_S3: {
      double* Xn = pick2(a.X, 1 - ctl->xi);
#pragma unroll
      for (int c = 0; c < 4; ++c) y[c] = sstore(a, r.x[c] + ha * (kA32 * r.k2[c]));
      rhs_eval<LEAN>(a, y, P, r.vs, r.p, r.rs, k);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c >= d) break;
        const double xn = sstore(a, r.x[c] + ha * (kB1 * r.k1[c] + kB2 * r.k2[c] + kB3 * k[c]));
        if (lead) {
          a.K3[c * np + i] = k[c];
          Xn[c * np + i] = xn;
        }
        y[c] = xn;
      }
      write_operand_t<VF>(a, 0, i, y[0], c0, c1);  // the FSAL stage is evaluated at X^{n+1}
      break;
    }
    case ST_S4: {
      double* K4 = pick2(a.Kf, 1 - ctl->ki);
#pragma unroll
      for (int c = 0; c < 4; ++c) y[c] = r.xn[c];
      rhs_eval<LEAN>(a, y, P, r.vs, r.p, r.rs, k);
      const double floor_w = ctl->atol / ctl->rtol;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c >= d) break;
        K4[c * np + i] = k[c];
        // difference of the two solutions formed from the stages (Sec. 2.2)
        const double e = ha * ((kB1 - kBt1) * r.k1[c] + (kB2 - kBt2) * r.k2[c] + (kB3 - kBt3) * r.k3[c] +
                               (0.0 - kBt4) * k[c]);
        const double xa = fabs(r.x[c]);
        const double W = fmax(fmax(xa, fabs(y[c])), floor_w);
        *r0 = nanmax(*r0, fabs(e) / W);
        *r1 = nanmax(*r1, fabs(r.k1[c]) / fmax(xa, floor_w));
      }
      break;
    }
  }
}

// coefficients of the seven-stage pair in use (a.pair: 2 Fehlberg 4(5), else Dormand-Prince 5(4))
__device__ __forceinline__ double pair_a(const Args& a, int s, int l) { return a.pair == 2 ? kFeA[s][l] : kDpA[s][l]; }
__device__ __forceinline__ double pair_e(const Args& a, int l) {
  return a.pair == 2 ? kFeB[l] - kFeBt[l] : kDpB[l] - kDpBt[l];
}

// Stage s = 2..7 of a seven-stage attempt (Dormand-Prince 5(4), or Fehlberg 4(5)
// with its fourth-order solution in row 6) of one row: K_s from the contraction of the
// stage input, then the next stage's input X + h sum_l a_{s+1,l} K_l (stage 6 writes
// it as X^{n+1} too), or at stage 7 (FSAL, evaluated at X^{n+1}) the difference of
// the two solutions h sum_l (b_l - bt_l) K_l and its weights.  The sums run over l in
// increasing order, FP64.
template <int VF, int S>
__device__ __forceinline__ void epilogue_dp_s(const Args& a, const Ctl* ctl, long long i, const double* P,
                                              double* r0, double* r1, int col) {
  // every index below is a compile-time constant, so the stages live in registers
  const int d = a.d;
  const long long np = a.np;
  const double ha = ctl->ha;
  const double* X = pick2(a.X, ctl->xi);
  double* Xn = pick2(a.X, 1 - ctl->xi);
  auto kbuf = [&](int l) -> double* {  // K_{l+1}
    return l == 0 ? pick2(a.Kf, ctl->ki) : l == 1 ? a.K2 : l == 2 ? a.K3 : l == 6 ? pick2(a.Kf, 1 - ctl->ki) : l == 3 ? a.Kd[0] : l == 4 ? a.Kd[1] : a.Kd[2];
  };
  const double* Vin = pick2(a.V64, vin_of(ST_D2 + S - 2));
  double vs[2];
  vs[0] = Vin[i * a.m];
  vs[1] = a.m > 1 ? Vin[i * a.m + 1] : 0.0;
  const double p = a.param[i];
  const double rs = a.rsum ? a.rsum[i] : 0.0;
  double x[4] = {0, 0, 0, 0}, y[4] = {0, 0, 0, 0}, k[4] = {0, 0, 0, 0}, K[7][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= d) break;
    x[c] = X[c * np + i];
#pragma unroll
    for (int l = 0; l < S - 1; ++l) K[l][c] = kbuf(l)[c * np + i];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= d) break;
    if constexpr (S == 7) {
      y[c] = Xn[c * np + i];
    } else {
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < S - 1; ++l) acc += pair_a(a, S - 1, l) * K[l][c];
      y[c] = x[c] + ha * acc;
    }
  }
  rhs_eval(a, y, P, vs, p, rs, k);
  double* Ks = kbuf(S - 1);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= d) break;
    if (col <= 0) Ks[c * np + i] = k[c];
    K[S - 1][c] = k[c];
  }
  *r0 = 0.0;
  *r1 = 0.0;
  if constexpr (S < 7) {
    double yn[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c >= d) break;
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < S; ++l) acc += pair_a(a, S, l) * K[l][c];
      yn[c] = x[c] + ha * acc;
      if constexpr (S == 6) {
        if (col <= 0) Xn[c * np + i] = yn[c];
      }
    }
    write_operand_t<VF>(a, vin_of(ST_D2 + S - 1), i, yn[0], col < 0 ? 0 : col, col < 0 ? a.m : col + 1);
  } else {
    if (col > 0) return;
    const double floor_w = ctl->atol / ctl->rtol;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c >= d) break;
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < 7; ++l) acc += pair_e(a, l) * K[l][c];
      const double W = fmax(fmax(fabs(x[c]), fabs(y[c])), floor_w);
      *r0 = nanmax(*r0, fabs(ha * acc) / W);
      *r1 = nanmax(*r1, fabs(K[0][c]) / fmax(fabs(x[c]), floor_w));
    }
  }
}

template <int VF>
__device__ __forceinline__ void epilogue_dp(const Args& a, const Ctl* ctl, long long i, const double* P, double* r0,
                                            double* r1, int col) {
  switch (a.stage) {
    case ST_D2: epilogue_dp_s<VF, 2>(a, ctl, i, P, r0, r1, col); break;
    case ST_D3: epilogue_dp_s<VF, 3>(a, ctl, i, P, r0, r1, col); break;
    case ST_D4: epilogue_dp_s<VF, 4>(a, ctl, i, P, r0, r1, col); break;
    case ST_D5: epilogue_dp_s<VF, 5>(a, ctl, i, P, r0, r1, col); break;
    case ST_D6: epilogue_dp_s<VF, 6>(a, ctl, i, P, r0, r1, col); break;
    default: epilogue_dp_s<VF, 7>(a, ctl, i, P, r0, r1, col); break;
  }
}

// Lanes per row of the row epilogues: the 16-bit and e4m3 formats split each operand
// column into terms by rounding, so the two Kuramoto columns get a lane each; the
// FP32 and FP64 operands take one lane per row.
template <int VF>
__device__ __forceinline__ int tail_lanes(const Args& a) {
  return (VF == F_BF16 || VF == F_F16 || VF == F_E4M3) ? a.m : 1;
}

// The row this thread finishes.  Tail threads start at thread tbase (the epilogue
// wave of a single-system kernel, or thread 0); with nl lanes per row, tail threads
// RB c .. RB c + RB - 1 take the block's rows for operand column c (every tile has
// at least 2 RB tail threads).
__device__ __forceinline__ long long tail_row(const Args& a, int rb, int RB, int tbase, int nl) {
  const int tt = (int)threadIdx.x - tbase;
  return (tt >= 0 && tt < RB * nl) ? (long long)rb * RB + tt % RB : -1;
}

// common tail of every contraction kernel: row epilogues and the block maxima (DP: the
// kernel also serves Dormand-Prince attempts; the grouped ensemble kernels do not, and
// leave that code out)
// (tbase > 0: every tail thread is in the last wave, the epilogue wave)
template <int M, int VF, bool DP = true>
__device__ __forceinline__ void contract_tail(const Args& a, int rb, double (*sP)[M], int RB, const RowIn& rin,
                                              int tbase = 0) {
  __shared__ double sRed0[16], sRed1[16];
  const Ctl* ctl = a.ctl;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nl = tail_lanes<VF>(a);
  const long long i = tail_row(a, rb, RB, tbase, nl);
  const int tt = tid - tbase, col = nl > 1 ? tt / RB : -1;
  double r0 = 0.0, r1 = 0.0;
  if (i >= 0 && i < a.n) {
    if constexpr (DP) {
      if (a.stage >= ST_D2) epilogue_dp<VF>(a, ctl, i, sP[tt % RB], &r0, &r1, col);
      else epilogue<VF>(a, ctl, i, sP[tt % RB], rin, &r0, &r1, col);
    } else {  // the grouped ensemble kernels
      epilogue<VF, true>(a, ctl, i, sP[tt % RB], rin, &r0, &r1, col);
    }
  }
  if (a.stage == ST_S2 || a.stage == ST_S3 || a.stage == ST_RHS || (a.stage >= ST_D2 && a.stage < ST_D7)) return;
  if (tbase > 0) {  // one wave holds every row: its maximum is the block's
    if (tid < tbase) return;
    r0 = wave_nanmax(r0);
    r1 = wave_nanmax(r1);
    if (tt == 0) {
      a.ep0[rb] = r0;
      a.ep1[rb] = r1;
    }
    return;
  }
  r0 = wave_nanmax(r0);
  r1 = wave_nanmax(r1);
  const int lane = tid & 63, wave = tid >> 6, nw = (nthr + 63) >> 6;
  if (lane == 0) {
    sRed0[wave] = r0;
    sRed1[wave] = r1;
  }
  __syncthreads();
  if (tid == 0) {
    double m0 = sRed0[0], m1 = sRed1[0];
    for (int w = 1; w < nw; ++w) {
      m0 = nanmax(m0, sRed0[w]);
      m1 = nanmax(m1, sRed1[w]);
    }
    a.ep0[rb] = m0;
    a.ep1[rb] = m1;
  }
}

// loads the tail row's inputs (issued before the contraction loop)
template <int VF>
__device__ __forceinline__ void prefetch_row(const Args& a, int rb, int RB, RowIn& rin, int tbase = 0) {
  const long long i = tail_row(a, rb, RB, tbase, tail_lanes<VF>(a));
  if (i >= 0 && i < a.n) load_row(a, a.ctl, i, rin);
}

// ---------------------------------------------------------------------------
// FP64 contraction on the vector ALUs.  Wave (wr, wk) owns R rows and the k-slice
// [wk KW, (wk+1) KW); lanes stride the row with 16-byte loads (2 doubles) and keep
// U chunks of 128 columns in flight.  The WK slice sums are added in slice order.
// EW (single systems): one more wave, the epilogue wave, loads the rows' epilogue
// inputs while the others stream A and then finishes the rows.  Loads of one wave
// complete in order, so a streaming wave that requested those inputs itself would
// hold up its own stream behind their address dependence on the control state.
// ---------------------------------------------------------------------------
template <int M, int R, int WR, int WK, int U, bool NT, bool DP = true, bool EW = false>
__device__ __forceinline__ void contract_f64(const Args& a, int rb) {
  constexpr int RB = R * WR;
  constexpr int TB = EW ? WR * WK * 64 : 0;  // first tail thread
  __shared__ double sPart[WK][RB][M];
  __shared__ double sP[RB][M];
  if (a.ctl->status != kRunning) return;
  RowIn rin;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (EW && w == WR * WK) {
    prefetch_row<F_F64>(a, rb, RB, rin, TB);
  } else {
    if constexpr (!EW && DP) prefetch_row<F_F64>(a, rb, RB, rin);
    const int wr = w % WR, wk = w / WR;
    const long long row0 = (long long)rb * RB + wr * R;
    const double* __restrict__ Ab = (const double*)a.A + row0 * a.ld;
    const double* __restrict__ V = pick2(a.V64, vin_of(a.stage));
    const long long jb = (long long)wk * a.KW;
    const long long je = min(jb + (long long)a.KW, a.kn);
    double acc[R][M];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < M; ++c) acc[r][c] = 0.0;
    long long j0 = jb;
    for (; j0 + 128 * U <= je; j0 += 128 * U) {
      f64x2 av[U][R];
      f64x2 vv[U][M];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long j = j0 + 128 * u + 2 * lane;
#pragma unroll
        for (int r = 0; r < R; ++r) av[u][r] = ldA<NT>((const f64x2*)(Ab + r * a.ld + j));
#pragma unroll
        for (int c = 0; c < M; ++c) vv[u][c] = *(const f64x2*)(V + j * M + 2 * c);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (M == 1) {
            acc[r][0] = fma(av[u][r].x, vv[u][0].x, acc[r][0]);
            acc[r][0] = fma(av[u][r].y, vv[u][0].y, acc[r][0]);
          } else {
            // vv[u][0] = (V[j][0], V[j][1]), vv[u][1] = (V[j+1][0], V[j+1][1])
            acc[r][0] = fma(av[u][r].x, vv[u][0].x, acc[r][0]);
            acc[r][M - 1] = fma(av[u][r].x, vv[u][0].y, acc[r][M - 1]);
            acc[r][0] = fma(av[u][r].y, vv[u][M - 1].x, acc[r][0]);
            acc[r][M - 1] = fma(av[u][r].y, vv[u][M - 1].y, acc[r][M - 1]);
          }
        }
    }
    for (; j0 < je; j0 += 128) {
      const long long j = j0 + 2 * lane;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const f64x2 x = ldA<NT>((const f64x2*)(Ab + r * a.ld + j));
        const f64x2 v0 = *(const f64x2*)(V + j * M);
        if (M == 1) {
          acc[r][0] = fma(x.x, v0.x, acc[r][0]);
          acc[r][0] = fma(x.y, v0.y, acc[r][0]);
        } else {
          const f64x2 v1 = *(const f64x2*)(V + j * M + 2);
          acc[r][0] = fma(x.x, v0.x, acc[r][0]);
          acc[r][M - 1] = fma(x.x, v0.y, acc[r][M - 1]);
          acc[r][0] = fma(x.y, v1.x, acc[r][0]);
          acc[r][M - 1] = fma(x.y, v1.y, acc[r][M - 1]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const double s = wave_sum(acc[r][c]);
        if (lane == 0) sPart[wk][wr * R + r][c] = s;
      }
  }
  __syncthreads();
  if constexpr (!DP) prefetch_row<F_F64>(a, rb, RB, rin);  // grouped kernels: after the stream
  for (int e = threadIdx.x; e < RB * M; e += blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < WK; ++q) s += sPart[q][e / M][e % M];
    sP[e / M][e % M] = s;
  }
  __syncthreads();
  contract_tail<M, F_F64, DP>(a, rb, sP, RB, rin, TB);
}

// ---------------------------------------------------------------------------
// FP32 contraction on the vector ALUs: A stored FP32, vector operand split into
// T FP32 terms; each lane forms 4-element FP32 dot products per term and adds
// them to FP64 accumulators (FP32 within a chunk, FP64 across chunks).
// ---------------------------------------------------------------------------
template <int M, int T, int R, int WR, int WK, int U, bool NT, bool DP = true, bool EW = false>
__device__ __forceinline__ void contract_f32(const Args& a, int rb) {
  constexpr int RB = R * WR;
  constexpr int NC = M * T;
  constexpr int TB = EW ? WR * WK * 64 : 0;  // first tail thread (EW: the epilogue wave, see contract_f64)
  __shared__ double sPart[WK][RB][NC];
  __shared__ double sP[RB][M];
  if (a.ctl->status != kRunning) return;
  RowIn rin;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (EW && w == WR * WK) {
    prefetch_row<F_F32>(a, rb, RB, rin, TB);
  } else {
    if constexpr (!EW && DP) prefetch_row<F_F32>(a, rb, RB, rin);
    const int wr = w % WR, wk = w / WR;
    const long long row0 = (long long)rb * RB + wr * R;
    const float* __restrict__ Ab = (const float*)a.A + row0 * a.ld;
    const float* __restrict__ Vq = (const float*)pick2(a.Vq, vin_of(a.stage));
    const long long jb = (long long)wk * a.KW;
    const long long je = min(jb + (long long)a.KW, a.kn);
    double acc[R][NC];
    float accf[R][NC];  // the recipes' single sum
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        acc[r][c] = 0.0;
        accf[r][c] = 0.0f;
      }
    long long j0 = jb;
    for (; j0 < je; j0 += 256 * U) {
      const int uu = (int)min((long long)U, (je - j0) / 256);
      f32x4 av[U][R];
      f32x4 vv[U][NC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (u < uu) {
          const long long j = j0 + 256 * u + 4 * lane;
#pragma unroll
          for (int r = 0; r < R; ++r) av[u][r] = ldA<NT>((const f32x4*)(Ab + r * a.ld + j));
#pragma unroll
          for (int c = 0; c < NC; ++c) vv[u][c] = *(const f32x4*)(Vq + c * a.ld + j);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          float s = 0.0f;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (u < uu) {
              s = fmaf(av[u][r].x, vv[u][c].x, s);
              s = fmaf(av[u][r].y, vv[u][c].y, s);
              s = fmaf(av[u][r].z, vv[u][c].z, s);
              s = fmaf(av[u][r].w, vv[u][c].w, s);
            }
          }
          if (a.sum32) accf[r][c] += s;
          else acc[r][c] += (double)s;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double s = a.sum32 ? (double)wave_sum_f32(accf[r][c]) : wave_sum(acc[r][c]);
        if (lane == 0) sPart[wk][wr * R + r][c] = s;
      }
  }
  __syncthreads();
  if constexpr (!DP) prefetch_row<F_F32>(a, rb, RB, rin);  // grouped kernels: after the stream
  for (int e = threadIdx.x; e < RB * M; e += blockDim.x) {
    const int row = e / M, cc = e % M;
    double p = 0.0;
    if (a.sum32) {  // single sum: one FP32 term (vsingle), wave slices added in FP32
      float s = 0.0f;
      for (int q = 0; q < WK; ++q) s += (float)sPart[q][row][cc * T];
      p = (double)s;
    } else {
      for (int t = 0; t < T; ++t) {
        double s = 0.0;
        for (int q = 0; q < WK; ++q) s += sPart[q][row][cc * T + t];
        p += ldexp(s, -t * a.vshift);
      }
    }
    sP[row][cc] = a.scale * p;
  }
  __syncthreads();
  contract_tail<M, F_F32, DP>(a, rb, sP, RB, rin, TB);
}

// ---------------------------------------------------------------------------
// Matrix-core contraction for BF16 / FP16 / FP8-e4m3 storage.
// One 16x16 MFMA tile: A operand = 16 rows of the coupling matrix, B operand =
// the split vector terms as columns (c * T + t < 16; the rest zero).  Lane l
// holds row l%16 and the k-group l/16 (8 elements; 16 for FP8 feeding two MFMAs
// with the same k-permutation on both operands).  FP32 accumulation inside the
// matrix core for KC k-groups, then FP64 accumulation; waves split k and their
// sums are added in slice order.
// Staging: the operand layout above reads 64 bytes of each of 16 rows per load
// instruction, half a cache line per row, which streams HBM markedly slower than
// whole lines.  A batch of U 64-byte steps is therefore loaded as 16/U rows x U*64
// contiguous bytes per instruction, written to the wave's own slab of LDS and read
// back in the operand layout: the same elements meet the same products in the same
// order, only the path from HBM changes.  The slab is private to the wave, and LDS
// operations of one wave complete in order, so no barrier is needed.  The grouped
// ensemble kernels of eight-wave tiles with 8-step batches or two row tiles keep
// the direct path: their per-item loop leaves no registers for the staging.
// ---------------------------------------------------------------------------
template <int FMT>
__device__ __forceinline__ f32x4 mma(u32x4 av, u32x4 bv, f32x4 c) {
  if constexpr (FMT == F_BF16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv), c,
                                                   0, 0, 0);
  } else if constexpr (FMT == F_F16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, av), __builtin_bit_cast(f16x8, bv), c, 0,
                                                  0, 0);
  } else if constexpr (FMT == F_F32) {
    // four 16x16x4 steps; lane group g holds columns 4g..4g+3 of the 16-column
    // block, step e uses column 4g+e on both operands (same k-permutation).
    // (Cast the whole vector: a bit_cast of a single vector element compiles to
    // element 0 with this toolchain.)
    const f32x4 fa = __builtin_bit_cast(f32x4, av), fb = __builtin_bit_cast(f32x4, bv);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[0], fb[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[1], fb[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[2], fb[2], c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x4f32(fa[3], fb[3], c, 0, 0, 0);
  } else {
    const long a0 = (long)(((unsigned long long)av.y << 32) | av.x);
    const long a1 = (long)(((unsigned long long)av.w << 32) | av.z);
    const long b0 = (long)(((unsigned long long)bv.y << 32) | bv.x);
    const long b1 = (long)(((unsigned long long)bv.w << 32) | bv.z);
    c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, c, 0, 0, 0);
  }
}

template <int FMT, int M, int T, int RT, int WR, int WK, int U, bool NT, bool DP = true, bool EW = false>
__device__ __forceinline__ void contract_mfma(const Args& a, int rb) {
  constexpr int NC = M * T;
  static_assert(NC <= 16, "vector terms exceed the MFMA tile width");
  constexpr int RB = 16 * RT * WR;
  static_assert(!EW || 2 * RB <= 64, "the epilogue wave holds every row of the block");
  static_assert(EW || WR * WK * 64 >= 2 * RB, "the tail needs two threads per row (one per operand column)");
  constexpr int TB = EW ? WR * WK * 64 : 0;  // first tail thread (EW: the epilogue wave, see contract_f64)
  constexpr int ES = (FMT == F_E4M3) ? 1 : (FMT == F_F32) ? 4 : 2;  // bytes per element
  constexpr int KC = 8;                        // k-groups kept in FP32 before an FP64 flush
  static_assert(U == 2 || U == 4 || U == 8, "staged batches of 2, 4 or 8 steps");
  constexpr int RPI = 16 / U;                  // rows per staged load instruction
  constexpr int LPR = 64 / RPI;                // lanes per row: U*64 contiguous bytes
  constexpr int SROW = U * 64 + 16;            // slab row stride (padded against bank conflicts)
  constexpr int NQ = RT * U;                   // load instructions per batch
  constexpr bool STAGE = DP || !(WR * WK >= 8 && (U == 8 || RT == 2));
  __shared__ double sPart[WK][RB][NC];
  __shared__ double sP[RB][M];
  __shared__ __attribute__((aligned(16))) unsigned char sA[STAGE ? WR * WK : 1][STAGE ? RT * 16 * SROW : 16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  RowIn rin;
  if (EW && w == WR * WK) {
    if (a.ctl->status != kRunning) return;
    prefetch_row<FMT>(a, rb, RB, rin, TB);
  } else {
    const int wr = w % WR, wk = w / WR;
    const int r16 = lane & 15, g = lane >> 4;
    const long long row_base = (long long)rb * RB + wr * 16 * RT;
    const long long kb = (long long)wk * a.KW;
    const long long ke = min(kb + (long long)a.KW, a.kn);
    const char* Ab = (const char*)a.A;
    const bool bcol = r16 < NC;
    const char* bp = (const char*)pick2(a.Vq, vin_of(a.stage)) + ((long long)(bcol ? r16 : 0) * a.ld + kb) * ES + g * 16;
    // staged path: instruction q reads rows q*RPI + srow of the wave's 16*RT, bytes scol..scol+15
    unsigned char* const slab = sA[STAGE ? w : 0];
    const int srow = lane / LPR, scol = (lane % LPR) * 16;
    const char* const sp = Ab + ((row_base + srow) * a.ld + kb) * ES + scol;
    const long long qstride = (long long)RPI * a.ld * ES;
    f32x4 c[RT];
    double dacc[RT][4];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      c[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      for (int i = 0; i < 4; ++i) dacc[t][i] = 0.0;
    }
    const u32x4 zero = {0u, 0u, 0u, 0u};
    int kc = 0;
    long long off = 0;  // byte offset from the slice start
    const long long span = (ke > kb) ? (ke - kb) * ES : 0;
    // Software pipeline over batches of U 64-byte steps: the loads of the next batch
    // are in flight while the matrix cores consume the current one (two register
    // buffers, ping-pong).  Same products, same order as a plain loop.
    constexpr long long BATCH = 64LL * U;
    const long long full = span / BATCH * BATCH;
    u32x4 a0[NQ], b0[U], a1[NQ], b1[U];
    auto load = [&](u32x4 (&xa)[NQ], u32x4 (&xb)[U], long long o) {
      if constexpr (STAGE) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) xa[q] = ldA<NT>((const u32x4*)(sp + q * qstride + o));
      } else {  // operand layout straight from HBM: element u*RT + t is step u of row tile t
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int t = 0; t < RT; ++t)
            xa[u * RT + t] =
                ldA<NT>((const u32x4*)(Ab + ((row_base + 16 * t + r16) * a.ld + kb) * ES + g * 16 + o + 64 * u));
      }
#pragma unroll
      for (int u = 0; u < U; ++u) xb[u] = bcol ? *(const u32x4*)(bp + o + 64 * u) : zero;
    };
    auto step = [&](const u32x4 (&xa)[NQ], const u32x4 (&xb)[U]) {
      if constexpr (STAGE) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) *(u32x4*)(slab + (q * RPI + srow) * SROW + scol) = xa[q];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            const u32x4 av = *(const u32x4*)(slab + (16 * t + r16) * SROW + 64 * u + 16 * g);
            c[t] = mma<FMT>(av, xb[u], c[t]);
          }
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int t = 0; t < RT; ++t) c[t] = mma<FMT>(xa[u * RT + t], xb[u], c[t]);
      }
      kc += U;
      if (kc >= KC && !a.sum32) {  // FP64 flush (the recipes' single sum keeps FP32 throughout)
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          for (int i = 0; i < 4; ++i) dacc[t][i] += (double)c[t][i];
          c[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        kc = 0;
      }
    };
    // The first batch is in flight while the control state arrives; a finished solve
    // streams nothing more (the host enqueues attempts ahead of its checks, and those
    // of a finished solve must cost no more than their launch).
    if (full > 0) load(a0, b0, 0);
    if (a.ctl->status != kRunning) return;
    if constexpr (!EW && DP) prefetch_row<FMT>(a, rb, RB, rin);
    while (off < full) {
      if (off + BATCH < full) load(a1, b1, off + BATCH);
      step(a0, b0);
      off += BATCH;
      if (off >= full) break;
      if (off + BATCH < full) load(a0, b0, off + BATCH);
      step(a1, b1);
      off += BATCH;
    }
    // steps left over after the last whole batch: operand layout straight from HBM
    for (; off < span; off += 64) {
      u32x4 av[RT];
#pragma unroll
      for (int t = 0; t < RT; ++t)
        av[t] = ldA<NT>((const u32x4*)(Ab + ((row_base + 16 * t + r16) * a.ld + kb) * ES + g * 16 + off));
      const u32x4 bv = bcol ? *(const u32x4*)(bp + off) : zero;
#pragma unroll
      for (int t = 0; t < RT; ++t) c[t] = mma<FMT>(av[t], bv, c[t]);
    }
#pragma unroll
    for (int t = 0; t < RT; ++t)
      for (int i = 0; i < 4; ++i) dacc[t][i] += (double)c[t][i];
    // C layout: lane l holds rows 4 (l/16) + i of column l%16
    if (bcol) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
        for (int i = 0; i < 4; ++i) sPart[wk][wr * 16 * RT + 16 * t + 4 * g + i][r16] = dacc[t][i];
    }
  }
  __syncthreads();
  if constexpr (!DP) prefetch_row<FMT>(a, rb, RB, rin);  // grouped kernels: after the stream
  for (int e = threadIdx.x; e < RB * M; e += blockDim.x) {
    const int row = e / M, cc = e % M;
    double p = 0.0;
    if (a.sum32) {  // single sum: one FP32 term (vsingle), wave slices added in FP32
      float s = 0.0f;
      for (int q = 0; q < WK; ++q) s += (float)sPart[q][row][cc * T];
      p = (double)s;
    } else {
      for (int t = 0; t < T; ++t) {
        double s = 0.0;
        for (int q = 0; q < WK; ++q) s += sPart[q][row][cc * T + t];
        p += ldexp(s, -t * a.vshift);
      }
    }
    sP[row][cc] = a.scale * p;
  }
  __syncthreads();
  contract_tail<M, FMT, DP>(a, rb, sP, RB, rin, TB);
}

// ---------------------------------------------------------------------------
// Pairwise coupling, the paper's own form of its benchmarks (Sec. 2.1, eq. (1)):
// P_i = sum_j w_ij g(x_j - x_i) with one transcendental per pair, g = sin
// (Kuramoto) or arctan (clock / cell cycle).  Each wave owns R rows and sweeps
// every column with its 64 lanes; x_j is read once per lane step and shared by
// the R rows.  G32: the pair term in FP32 (the recipes' "G in single": FP32
// difference, FP32 function, FP32 weight); otherwise FP64.  DENSE: the weights
// come from the stored matrix; uniform weights read nothing.  The sum is FP64,
// or FP32 throughout with sum32.
// ---------------------------------------------------------------------------
template <bool ATAN, bool G32>
__device__ __forceinline__ auto pair_g(double xj, double xi) {
  if constexpr (G32) {
    const float d = (float)xj - (float)xi;
    return ATAN ? atanf(d) : sinf(d);
  } else {
    const double d = xj - xi;
    return ATAN ? atan(d) : sin(d);
  }
}

template <bool ATAN, bool G32, bool DENSE, int R, int WV, int UJ>
__device__ __forceinline__ void contract_pair(const Args& a, int rb) {
  constexpr int RB = R * WV;
  __shared__ double sP[RB][1];
  if (a.ctl->status != kRunning) return;
  RowIn rin;
  prefetch_row<F_F64>(a, rb, RB, rin);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long long row0 = (long long)rb * RB + (long long)w * R;
  const double* __restrict__ V = pick2(a.V64, vin_of(a.stage));
  double xi[R], accd[R];
  float accf[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    xi[r] = (row0 + r < a.n) ? V[row0 + r] : 0.0;
    accd[r] = 0.0;
    accf[r] = 0.0f;
  }
  for (long long j0 = 0; j0 < a.n; j0 += 64 * UJ) {
#pragma unroll
    for (int u = 0; u < UJ; ++u) {
      const long long j = j0 + 64 * u + lane;
      if (j < a.n) {
        const double xj = V[j];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          auto g = pair_g<ATAN, G32>(xj, xi[r]);
          if constexpr (DENSE) {
            using WT = decltype(g);
            g = ((const WT*)a.A)[(row0 + r) * a.ld + j] * g;
          }
          if constexpr (G32) {
            if (a.sum32) accf[r] += g;
            else accd[r] += (double)g;
          } else {
            accd[r] += g;
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double s = a.sum32 ? (double)wave_sum_f32(accf[r]) : wave_sum(accd[r]);
    if (lane == 0) sP[w * R + r][0] = a.scale * s;  // the stored matrix's power-of-two scale
  }
  __syncthreads();
  contract_tail<1, F_F64>(a, rb, sP, RB, rin);
}

// ---------------------------------------------------------------------------
// prep: vector operand of an evaluation from the current state (used for the
// first evaluation of a solve, for bs32_rhs and for kernel timing).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void prep_block(const Args& a, int blk) {
  const Ctl* ctl = a.ctl;
  if (ctl->status != kRunning) return;
  const long long i = (long long)blk * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const double* X = pick2(a.X, ctl->xi);
  const double* K1 = pick2(a.Kf, ctl->ki);
  double y = X[i];
  if (a.stage == ST_H0) y = X[i] + ctl->h0probe * K1[i];
  else if (a.stage == ST_S2) y = sstore(a, X[i] + ctl->ha * (kA21 * K1[i]));
  write_operand(a, 0, i, y);
}
#if BS32_IN(0)
__global__ void k_prep(Args a) { prep_block(a, blockIdx.x); }
#endif

// ---------------------------------------------------------------------------
// kernels of one system (block index = row block) and of an ensemble (each
// workgroup walks the live work items of a grouped launch)
// ---------------------------------------------------------------------------
__device__ __forceinline__ const Args& group_args(const Group& g, const Item& w) {
  return g.inst[((size_t)w.inst * kStages + g.stage) * 2 + g.par];
}
#define BS32_GROUP_LOOP(BODY)                                       \
  const unsigned cnt_ = *g.count;                                   \
  for (unsigned it_ = blockIdx.x; it_ < cnt_; it_ += gridDim.x) {   \
    const Item w_ = g.items[it_];                                   \
    BODY(group_args(g, w_), (int)w_.blk);                           \
    __syncthreads();                                                \
  }
// Contraction lists: workgroups are dispatched to the 8 XCDs in turn (block b to XCD
// b % 8), so the workgroups of XCD x walk their own contiguous range of the list, which
// the host balances by streamed bytes.  An instance's operand then stays in the L2 of
// one XCD (two where a range boundary splits it).  Grids are whole multiples of 8.
#define BS32_GROUP_LOOP_X(BODY)                                                     \
  const unsigned x_ = blockIdx.x & 7u, per_ = gridDim.x >> 3;                       \
  const unsigned end_ = g.xs[x_ + 1];                                               \
  for (unsigned it_ = g.xs[x_] + (blockIdx.x >> 3); it_ < end_; it_ += per_) {      \
    const Item w_ = g.items[it_];                                                   \
    BODY(group_args(g, w_), (int)w_.blk);                                           \
    __syncthreads();                                                                \
  }

// EW: a single-system kernel with one more wave than the tile's streaming waves,
// the epilogue wave (see contract_f64); the autotuner tries both forms
template <int M, int R, int WR, int WK, int U, bool NT, bool EW>
__global__ __launch_bounds__(WR* WK * 64 + (EW ? 64 : 0)) void k_contract_f64(Args a) {
  contract_f64<M, R, WR, WK, U, NT, true, EW>(a, block_row(a));
}
template <int M, int R, int WR, int WK, int U, bool NT>
__global__ __launch_bounds__(WR* WK * 64) void k_group_f64(Group g) {
  BS32_GROUP_LOOP_X((contract_f64<M, R, WR, WK, U, NT, false>))
}
template <int M, int T, int R, int WR, int WK, int U, bool NT, bool EW>
__global__ __launch_bounds__(WR* WK * 64 + (EW ? 64 : 0)) void k_contract_f32(Args a) {
  contract_f32<M, T, R, WR, WK, U, NT, true, EW>(a, block_row(a));
}
template <int M, int T, int R, int WR, int WK, int U, bool NT>
__global__ __launch_bounds__(WR* WK * 64) void k_group_f32(Group g) {
  BS32_GROUP_LOOP_X((contract_f32<M, T, R, WR, WK, U, NT, false>))
}
template <int FMT, int M, int T, int RT, int WR, int WK, int U, bool NT, bool EW>
__global__ __launch_bounds__(WR* WK * 64 + (EW ? 64 : 0)) void k_contract_mfma(Args a) {
  contract_mfma<FMT, M, T, RT, WR, WK, U, NT, true, EW>(a, block_row(a));
}
// Two workgroups per CU for tiles of at most four waves: with the row epilogue's loads
// after the stream (DP = false) every such tile fits in 256 registers per lane without
// spilling.  Tiles of eight waves ask for one.
template <int RT, int WR, int WK, int U>
constexpr int group_mfma_blocks() {
  return WR * WK <= 4 ? 2 : 1;
}
template <int FMT, int M, int T, int RT, int WR, int WK, int U, bool NT>
__global__ __launch_bounds__(WR* WK * 64, (group_mfma_blocks<RT, WR, WK, U>())) void k_group_mfma(Group g) {
  BS32_GROUP_LOOP_X((contract_mfma<FMT, M, T, RT, WR, WK, U, NT, false>))
}
template <bool ATAN, bool G32, bool DENSE, int R, int WV, int UJ>
__global__ __launch_bounds__(WV * 64) void k_contract_pair(Args a) {
  contract_pair<ATAN, G32, DENSE, R, WV, UJ>(a, block_row(a));
}
#if BS32_IN(0)
__global__ __launch_bounds__(256) void k_group_prep(Group g) { BS32_GROUP_LOOP(prep_block) }
#endif

// ---------------------------------------------------------------------------
// Shared-coupling ensembles: B instances with one coupling matrix A, each with
// its own parameters, gain, state, step size and status.  The contraction of a
// stage for all of them is one matrix product P = A [V_1 ... V_B] of N rows and
// B C columns (C = m T operand columns per instance) on the matrix cores, and
// each instance's row epilogue follows in the same launch.
//
// Workgroup tile: BM = 64 RT rows (four waves of 16 RT rows) by BN = 16 CT
// columns (IB = BN / C instances).  A fragments go from memory straight into
// the registers of the wave that owns those rows (A is read once per column
// block); the operand tile of each 256-byte k-chunk is staged in LDS, double
// buffered, and shared by the four waves.  BF16 / FP16 / FP32 storage: FP32
// accumulation in the matrix core within a chunk, FP64 across chunks; FP64
// storage: FP64 matrix cores throughout.  Workgroups are ordered so that the
// eight XCDs each take a contiguous range of row blocks (the column blocks of a
// row block share its A rows in that XCD's L2).
// FROMP: the product itself came from the library (16-bit storage, FP32
// accumulation over the whole k and FP32 output, one product per plane of A); the
// kernel reads its P tile from there and runs the same row epilogues.
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));

// operand format of a storage format (the BF16 pair multiplies BF16 operand terms)
template <int FMT>
constexpr int sh_opfmt() {
  return FMT == F_BF16X2 ? F_BF16 : FMT;
}

template <int FMT>
struct ShAcc {
  using T = f32x4;
};
template <>
struct ShAcc<F_F64> {
  using T = f64x4;
};

template <int FMT>
__device__ __forceinline__ typename ShAcc<FMT>::T sh_mma(u32x4 av, u32x4 bv, typename ShAcc<FMT>::T c) {
  if constexpr (FMT == F_F64) {
    // two 16x16x4 steps; lane group g holds k = 2g, 2g+1 of the 8-wide step on both operands
    const f64x2 fa = __builtin_bit_cast(f64x2, av), fb = __builtin_bit_cast(f64x2, bv);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[0], fb[0], c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f64_16x16x4f64(fa[1], fb[1], c, 0, 0, 0);
  } else {
    return mma<sh_opfmt<FMT>()>(av, bv, c);
  }
}

constexpr int kShChunk = 256;          // bytes of k per operand column and chunk
constexpr int kShPitch = kShChunk + 16;  // LDS pitch of one operand column (spreads the banks)

// 16-bit storage accumulates in FP32 across the whole k range (its products carry
// 8- or 11-bit weights, far coarser than an FP32 sum of N terms) and keeps the P tile
// in FP32; FP32 storage adds each chunk's FP32 partial sums in FP64
template <int FMT>
constexpr bool sh_f32acc() {
  return FMT == F_BF16 || FMT == F_F16;
}

template <int FMT, int RT, int CT, bool FROMP>
constexpr int sh_lds_bytes() {
  constexpr int BM = 64 * RT, BN = 16 * CT;
  constexpr int tiles = FROMP ? 0 : 2 * BN * kShPitch, part = BM * (BN + 1) * (sh_f32acc<FMT>() ? 4 : 8);
  return tiles > part ? tiles : part;
}

#if BS32_IN(0)
int shared_cols(int fmt, int m) {
  if (fmt == F_F64) return m;
  if (fmt == F_F32 || fmt == F_BF16 || fmt == F_F16 || fmt == F_BF16X2) return 2 * m;  // two split terms
  return 0;  // e4m3's three terms do not tile the product's columns
}
#endif

// Row epilogues of a shared-coupling product tile: the P tile sP [BM][BN + 1] of row
// block rb and column block cb is in LDS.  The workgroup makes BM IB / 256 passes over
// the (row, instance) pairs, BM consecutive threads per instance (so a wave serves one
// instance and its arguments come through scalar loads); the row inputs of the next
// pass are requested before the current pass's epilogues, and the block maxima are
// gathered per pass and written once at the end.
template <int FMT, int M, int BM, int BN, typename PT>
__device__ __forceinline__ void shared_rows(const Shared& sh, int rb, int cb, const PT* sP) {
  constexpr int T = FMT == F_F64 ? 1 : 2;
  constexpr int C = M * T, IB = BN / C, PP = BN + 1;
  constexpr int NPASS = BM * IB / 256;  // passes over the tile's (row, instance) pairs
  constexpr int WPI = BM / 64;          // waves per instance in one pass
  static_assert(NPASS * 256 == BM * IB && BM % 64 == 0, "whole waves per instance and pass");
  __shared__ double sMax[2][NPASS][4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int stage = sh.stage;
  const bool reduce = !(stage == ST_S2 || stage == ST_S3 || stage == ST_RHS);
  struct Pair {
    const Args* a;
    long long i;
    int row, ib;
    bool live;
  };
  auto pair_of = [&](int p) {
    Pair q;
    const int e = 256 * p + tid;
    q.ib = __builtin_amdgcn_readfirstlane(e / BM);
    q.row = e % BM;
    q.i = (long long)rb * BM + q.row;
    q.a = nullptr;
    q.live = false;
    const int b = cb * IB + q.ib;
    if (b < sh.B) {
      q.a = &sh.inst[((size_t)b * kStages + stage) * 2 + sh.par];
      q.live = q.a->ctl->status == kRunning && q.i < q.a->n;
    }
    return q;
  };
  Pair nq = pair_of(0);
  RowIn nrin;
  if (nq.live) load_row(*nq.a, nq.a->ctl, nq.i, nrin);
#pragma unroll 1
  for (int p = 0; p < NPASS; ++p) {
    const Pair q = nq;
    const RowIn rin = nrin;
    if (p + 1 < NPASS) {
      nq = pair_of(p + 1);
      if (nq.live) load_row(*nq.a, nq.a->ctl, nq.i, nrin);
    }
    double r0 = 0.0, r1 = 0.0;
    if (q.live) {
      double P[2] = {0.0, 0.0};
#pragma unroll
      for (int mm = 0; mm < M; ++mm) {
        double pv = 0.0;
#pragma unroll
        for (int tt = 0; tt < T; ++tt) pv += ldexp((double)sP[q.row * PP + q.ib * C + mm * T + tt], -tt * sh.vshift);
        P[mm] = sh.scale * pv;
      }
      epilogue<sh_opfmt<FMT>(), true>(*q.a, q.a->ctl, q.i, P, rin, &r0, &r1, -1);
    }
    if (reduce) {
      r0 = wave_nanmax(r0);
      r1 = wave_nanmax(r1);
      if (lane == 0) {
        sMax[0][p][w] = r0;
        sMax[1][p][w] = r1;
      }
    }
  }
  if (!reduce) return;
  __syncthreads();
  // one thread per (pass, instance): the first wave of the instance's group
  if (tid < NPASS * 4 && (tid % 4) % WPI == 0) {
    const int p = tid / 4, w0 = tid % 4;
    const int bq = cb * IB + (256 * p + 64 * w0) / BM;
    double m0 = sMax[0][p][w0], m1 = sMax[1][p][w0];
    for (int q = 1; q < WPI; ++q) {
      m0 = nanmax(m0, sMax[0][p][w0 + q]);
      m1 = nanmax(m1, sMax[1][p][w0 + q]);
    }
    if (bq < sh.B) {
      const Args& a = sh.inst[((size_t)bq * kStages + stage) * 2 + sh.par];
      if (a.ctl->status == kRunning) {
        a.ep0[rb] = m0;
        a.ep1[rb] = m1;
      }
    }
  }
}

template <int FMT, int M, int RT, int CT, bool FROMP = false>
__global__ __launch_bounds__(256) void k_shared_contract(Shared sh) {
  constexpr int ES = FMT == F_F64 ? 8 : FMT == F_F32 ? 4 : 2;  // bytes per element of A (per plane) and operand
  constexpr int T = FMT == F_F64 ? 1 : 2;
  constexpr int C = M * T;
  constexpr int PL = FMT == F_BF16X2 ? 2 : 1;  // planes of A: the BF16 pair adds its remainder plane
  constexpr int BM = 64 * RT, BN = 16 * CT, IB = BN / C;
  constexpr int NSTEP = kShChunk / 64;  // 64-byte lane-group steps per chunk
  constexpr int UNITS = BN * kShChunk / 16 / 256;  // 16-byte operand loads per thread and chunk
  static_assert(BN % C == 0, "whole instances per column block");
  using Acc = typename ShAcc<FMT>::T;
  __shared__ __align__(16) char smem[sh_lds_bytes<FMT, RT, CT, FROMP>()];

  // XCD-aware tile order: blockIdx.x % 8 selects the XCD
  const int total = sh.nrb * sh.ncb;
  const int per = (total + 7) / 8;
  const int lin = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (lin >= total) return;
  const int rb = lin / sh.ncb, cb = lin % sh.ncb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int stage = sh.stage;

  // nothing to do when every instance of the column block has finished
  {
    int live = 0;
    if (tid < IB) {
      const int b = cb * IB + tid;
      if (b < sh.B) live = sh.inst[((size_t)b * kStages + stage) * 2 + sh.par].ctl->status == kRunning;
    }
    if (!__syncthreads_or(live)) return;
  }

  constexpr bool F32ACC = sh_f32acc<FMT>();
  // P tile [BM][BN] (FP32 for 16-bit storage, else FP64)
  using PT = typename std::conditional<F32ACC, float, double>::type;
  PT* sP = (PT*)smem;
  constexpr int PP = BN + 1;
  if constexpr (FROMP) {
    // the library's P of this tile: rows rb*BM.., columns cb*BN.. (the BF16 pair adds its
    // remainder plane's product in FP64)
    const float* P0 = sh.Pg[0] + ((long long)rb * BM) * sh.ldp + (long long)cb * BN;
    const float* P1 = (PL == 2) ? sh.Pg[1] + ((long long)rb * BM) * sh.ldp + (long long)cb * BN : nullptr;
    for (int e = tid; e < BM * BN; e += 256) {
      const int row = e / BN, col = e % BN;
      const long long o = (long long)row * sh.ldp + col;
      if constexpr (PL == 2) sP[row * PP + col] = (PT)((double)P0[o] + (double)P1[o]);
      else sP[row * PP + col] = (PT)P0[o];
    }
  } else {
    const long long ld = sh.ld;
    const long long row_base = (long long)rb * BM + w * 16 * RT;
    const char* ap[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) ap[t] = (const char*)sh.A + ((row_base + 16 * t + r16) * ld) * ES + g * 16;
    const char* Bg = (const char*)sh.Bop[vin_of(stage)];
    const long long nchunk = ld * ES / kShChunk;

    // operand unit q of this thread in a chunk: global source and LDS destination(s)
    auto load_units = [&](u32x4 (&v)[UNITS], long long ch) {
#pragma unroll
      for (int q = 0; q < UNITS; ++q) {
        const int u = tid + 256 * q;
        if constexpr (FMT == F_F64 && M == 2) {
          // [b][ld][2] doubles: 16 bytes = both columns of one k
          const int ib = u / 32, part = u % 32;
          const long long b = (long long)cb * IB + ib;
          v[q] = *(const u32x4*)(Bg + ((b * ld + ch * (kShChunk / 8) + part) * 2) * 8);
        } else {
          const int col = u / 16, part = u % 16;
          v[q] = *(const u32x4*)(Bg + ((long long)(cb * BN + col) * ld) * ES + ch * kShChunk + part * 16);
        }
      }
    };
    auto store_units = [&](const u32x4 (&v)[UNITS], int buf) {
      char* base = smem + buf * BN * kShPitch;
#pragma unroll
      for (int q = 0; q < UNITS; ++q) {
        const int u = tid + 256 * q;
        if constexpr (FMT == F_F64 && M == 2) {
          const int ib = u / 32, part = u % 32;
          const f64x2 x = __builtin_bit_cast(f64x2, v[q]);
          *(double*)(base + (2 * ib) * kShPitch + part * 8) = x[0];
          *(double*)(base + (2 * ib + 1) * kShPitch + part * 8) = x[1];
        } else {
          const int col = u / 16, part = u % 16;
          *(u32x4*)(base + col * kShPitch + part * 16) = v[q];
        }
      }
    };
    const long long plane_bytes = sh.np * ld * ES;
    auto load_a = [&](u32x4 (&av)[NSTEP][RT * PL], long long ch) {
#pragma unroll
      for (int s = 0; s < NSTEP; ++s)
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int q = 0; q < PL; ++q) av[s][t * PL + q] = *(const u32x4*)(ap[t] + q * plane_bytes + ch * kShChunk + s * 64);
    };

    constexpr bool FLUSH = !F32ACC && FMT != F_F64;
    Acc c[RT][CT];
    double dacc[FLUSH ? RT : 1][FLUSH ? CT : 1][4];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int u = 0; u < CT; ++u) c[t][u] = Acc{0, 0, 0, 0};
    if constexpr (FLUSH) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int u = 0; u < CT; ++u)
          for (int i = 0; i < 4; ++i) dacc[t][u][i] = 0.0;
    }

    u32x4 bu[UNITS];
    u32x4 a0[NSTEP][RT * PL], a1[NSTEP][RT * PL];
    load_units(bu, 0);
    load_a(a0, 0);
    store_units(bu, 0);
    __syncthreads();
    auto compute = [&](const u32x4 (&av)[NSTEP][RT * PL], int buf) {
      const char* base = smem + buf * BN * kShPitch;
#pragma unroll
      for (int s = 0; s < NSTEP; ++s) {
#pragma unroll
        for (int u = 0; u < CT; ++u) {
          const u32x4 bv = *(const u32x4*)(base + (16 * u + r16) * kShPitch + s * 64 + g * 16);
#pragma unroll
          for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int q = 0; q < PL; ++q) c[t][u] = sh_mma<FMT>(av[s][t * PL + q], bv, c[t][u]);  // (hi + lo) b
        }
      }
      if constexpr (FLUSH) {  // FP64 across chunks
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int u = 0; u < CT; ++u) {
            for (int i = 0; i < 4; ++i) dacc[t][u][i] += (double)c[t][u][i];
            c[t][u] = Acc{0, 0, 0, 0};
          }
      }
    };
    for (long long ch = 0; ch < nchunk; ch += 2) {
      // chunk ch from buffer 0 / registers a0 while chunk ch+1 is fetched, then the reverse
      const bool more1 = ch + 1 < nchunk;
      if (more1) {
        load_units(bu, ch + 1);
        load_a(a1, ch + 1);
      }
      compute(a0, 0);
      if (!more1) break;
      store_units(bu, 1);
      __syncthreads();
      const bool more2 = ch + 2 < nchunk;
      if (more2) {
        load_units(bu, ch + 2);
        load_a(a0, ch + 2);
      }
      compute(a1, 1);
      if (!more2) break;
      store_units(bu, 0);
      __syncthreads();
    }
    __syncthreads();  // every wave is done with the operand tiles: the LDS now takes P

    // lane (r16, g) holds column r16 of each 16x16 tile: rows 4g + i for the FP32-output
    // instructions, rows g + 4i for the FP64 one (measured)
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int u = 0; u < CT; ++u)
        for (int i = 0; i < 4; ++i) {
          const int rr = (FMT == F_F64) ? g + 4 * i : 4 * g + i;
          const int row = w * 16 * RT + 16 * t + rr, col = 16 * u + r16;
          if constexpr (FLUSH) sP[row * PP + col] = dacc[t][u][i];
          else sP[row * PP + col] = (PT)c[t][u][i];
        }
  }
  __syncthreads();

  shared_rows<FMT, M, BM, BN>(sh, rb, cb, sP);
}

// Shared-coupling product for 16-bit storage as an LDS-tiled matrix product: tiles of
// BM = 64 RT rows by BN = 16 CT columns, four waves in a 2 x 2 grid (each BM/2 x BN/2,
// (BM/32) x (BN/32) matrix-core tiles of 16 x 16), 64 elements of k per stage.  Both
// operands go from memory through registers into LDS (two LDS buffers), and the loads
// of stage s + 2 are issued before the products of stage s, so two stages of latency
// are covered.  Every A and operand fragment read from LDS feeds BN/32 or BM/32 matrix-
// core products.  FP32 accumulation over the whole k (both planes of the BF16 pair go
// into one accumulator); the P tile then takes the LDS and the row epilogues follow.
constexpr int kGemmBK = 128;               // bytes of k per stage (64 16-bit elements; a multiple of 64)
constexpr int kGemmPitch = kGemmBK + 16;   // LDS pitch of one row or operand column

template <int FMT, int RT, int CT>
constexpr int gemm_lds_bytes() {
  constexpr int PL = FMT == F_BF16X2 ? 2 : 1, BM = 64 * RT, BN = 16 * CT;
  constexpr int tiles = 2 * (PL * BM + BN) * kGemmPitch, part = BM * (BN + 1) * 4;
  return tiles > part ? tiles : part;
}

template <int FMT, int M, int RT, int CT>
__global__ __launch_bounds__(256) void k_shared_gemm(Shared sh) {
  static_assert(FMT == F_BF16 || FMT == F_F16 || FMT == F_BF16X2, "16-bit storage");
  constexpr int ES = 2, T = 2, C = M * T;
  constexpr int PL = FMT == F_BF16X2 ? 2 : 1;
  constexpr int BM = 64 * RT, BN = 16 * CT, IB = BN / C, PP = BN + 1;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int SP = kGemmPitch, ABYTES = PL * BM * SP, STB = ABYTES + BN * SP;
  constexpr int LA = PL * BM * kGemmBK / 16 / 256, LB = BN * kGemmBK / 16 / 256;  // 16-byte loads per thread
  static_assert(BN % C == 0 && LA * 4096 == PL * BM * kGemmBK && LB * 4096 == BN * kGemmBK, "tile shape");
  static_assert(kGemmBK % 64 == 0, "whole matrix-core steps of 32 elements per stage");
  __shared__ __align__(16) char smem[gemm_lds_bytes<FMT, RT, CT>()];

  // XCD-aware tile order, as in k_shared_contract
  const int total = sh.nrb * sh.ncb;
  const int per = (total + 7) / 8;
  const int lin = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (lin >= total) return;
  const int rb = lin / sh.ncb, cb = lin % sh.ncb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int wm = w >> 1, wn = w & 1;
  const int stage = sh.stage;
  {
    int live = 0;
    if (tid < IB) {
      const int b = cb * IB + tid;
      if (b < sh.B) live = sh.inst[((size_t)b * kStages + stage) * 2 + sh.par].ctl->status == kRunning;
    }
    if (!__syncthreads_or(live)) return;
  }

  const long long ld = sh.ld;
  const long long plane = sh.np * ld * ES;
  const char* const Ab = (const char*)sh.A + (long long)rb * BM * ld * ES;
  const char* const Bb = (const char*)sh.Bop[vin_of(stage)] + (long long)cb * BN * ld * ES;
  // load unit u = tid + 256 q: row u / SEG of the stacked rows (A: PL planes of BM rows;
  // operand: BN columns), 16-byte segment u % SEG of the stage's kGemmBK bytes
  constexpr int SEG = kGemmBK / 16;
  auto gload = [&](u32x4 (&ra)[LA], u32x4 (&rv)[LB], long long st) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int u = tid + 256 * q, r = u / SEG, seg = u % SEG;
      const int pl = r / BM, row = r % BM;
      ra[q] = *(const u32x4*)(Ab + pl * plane + (long long)row * ld * ES + st * kGemmBK + seg * 16);
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int u = tid + 256 * q, col = u / SEG, seg = u % SEG;
      rv[q] = *(const u32x4*)(Bb + (long long)col * ld * ES + st * kGemmBK + seg * 16);
    }
  };
  auto sstore = [&](const u32x4 (&ra)[LA], const u32x4 (&rv)[LB], int buf) {
    char* base = smem + buf * STB;
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int u = tid + 256 * q;
      *(u32x4*)(base + (u / SEG) * SP + (u % SEG) * 16) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int u = tid + 256 * q;
      *(u32x4*)(base + ABYTES + (u / SEG) * SP + (u % SEG) * 16) = rv[q];
    }
  };
  f32x4 c[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) c[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto compute = [&](int buf) {
    const char* base = smem + buf * STB;
#pragma unroll
    for (int ks = 0; ks < kGemmBK / 64; ++ks) {  // 32 elements of k per matrix-core step
      u32x4 af[PL][TM];
#pragma unroll
      for (int pl = 0; pl < PL; ++pl)
#pragma unroll
        for (int i = 0; i < TM; ++i)
          af[pl][i] = *(const u32x4*)(base + (pl * BM + wm * WM + 16 * i + r16) * SP + ks * 64 + g * 16);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const u32x4 bf = *(const u32x4*)(base + ABYTES + (wn * WN + 16 * j + r16) * SP + ks * 64 + g * 16);
#pragma unroll
        for (int pl = 0; pl < PL; ++pl)
#pragma unroll
          for (int i = 0; i < TM; ++i) c[i][j] = mma<sh_opfmt<FMT>()>(af[pl][i], bf, c[i][j]);
      }
    }
  };
  const long long nst = ld * ES / kGemmBK;
  u32x4 ra0[LA], rv0[LB], ra1[LA], rv1[LB];
  gload(ra0, rv0, 0);
  if (nst > 1) gload(ra1, rv1, 1);
  sstore(ra0, rv0, 0);
  __syncthreads();
  for (long long st = 0; st < nst; st += 2) {
    // stage st is in LDS buffer 0 and stage st + 1 in flight to ra1 / rv1
    if (st + 2 < nst) gload(ra0, rv0, st + 2);
    compute(0);
    if (st + 1 >= nst) break;
    sstore(ra1, rv1, 1);
    __syncthreads();
    if (st + 3 < nst) gload(ra1, rv1, st + 3);
    compute(1);
    if (st + 2 >= nst) break;
    sstore(ra0, rv0, 0);
    __syncthreads();
  }
  __syncthreads();  // every wave is done with the tiles: the LDS now takes P

  float* sP = (float*)smem;
  // C layout: lane (r16, g) holds column r16 of each 16 x 16 tile, rows 4 g + i
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) sP[(wm * WM + 16 * i + 4 * g + e) * PP + wn * WN + 16 * j + r16] = c[i][j][e];
  __syncthreads();
  shared_rows<FMT, M, BM, BN>(sh, rb, cb, sP);
}

// elementary controller (reading of the unspecified step-size correction; the
// estimate is O(h^3), so the exponent is 1/3)
__device__ __forceinline__ double control(const Ctl* c, double h, double E, bool accepted) {
  const double fac = (E > 0.0) ? c->safety * cbrt(c->rtol / E) : c->facmax;
  if (accepted) {
    const double hi = c->last_rejected ? 1.0 : c->facmax;
    return h * fmin(hi, fmax(c->facmin, fac));
  }
  double lo = fmax(c->facmin, fac);
  if (c->last_rejected) lo = fmin(lo, 0.5);
  return h * lo;
}

// grid maxima of the evaluation that just finished -> new control state
// returns true when the learned proposer should choose the next step (features in feat)
__device__ __forceinline__ bool finalize(const Args& a, Ctl* c, double m0, double m1, bool writer, float* feat) {
  switch (a.stage) {
    case ST_INIT: {
      c->n_fev += 1;
      c->d0 = m0;
      c->d1 = m1;
      if (c->h0user > 0.0) {
        c->h = c->h0user;
        c->ha = fmin(c->h, c->t1 - c->t);
      } else {  // Hairer-Norsett-Wanner starting step, first half (reading)
        const double h0 = (m0 < 1e-5 || m1 < 1e-5) ? 1e-6 : 0.01 * m0 / m1;
        c->h0probe = fmin(h0, c->h_max);
      }
      break;
    }
    case ST_H0: {
      c->n_fev += 1;
      const double h0 = c->h0probe;
      const double d2 = m0 / h0;
      const double dm = fmax(c->d1, d2);
      // exponent 1/(p+1) of the order p of the propagated solution: 3 (BS3(2)), 5 (DP5(4)), 4 (RKF4(5))
      const double ex = c->method == 1 ? 1.0 / 6.0 : c->method == 2 ? 0.2 : 0.25;
      const double h1 = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, ex);
      c->h = fmin(fmin(100.0 * h0, h1), c->h_max);
      c->ha = fmin(c->h, c->t1 - c->t);
      break;
    }
    case ST_S4: {
      const double E = m0;
      const double ha = c->ha;
      c->n_fev += 3;
      c->err = E;
      bool accepted;
      if (c->fixed_step) {
        accepted = true;
      } else {
        if (!isfinite(E)) {
          c->status = 6;  // BS32_NONFINITE
          c->n_reject += 1;
          if (c->trace_on) {
            if (writer) a.trace[c->trace_n % c->trace_cap] = TraceRec{c->t, ha, E, m1, 0, c->prop_cur};
            c->trace_n += 1;
          }
          return false;
        }
        accepted = E < c->rtol;  // accept iff the estimate is smaller than Rel (Sec. 2.2)
      }
      if (c->trace_on) {
        if (writer) a.trace[c->trace_n % c->trace_cap] = TraceRec{c->t, ha, E, m1, accepted ? 1 : 0, c->prop_cur};
        c->trace_n += 1;
      }
      double hn;
      if (accepted) {
        c->n_accept += 1;
        c->t = (c->t + ha >= c->t1 - c->snap) ? c->t1 : c->t + ha;
        c->xi = 1 - c->xi;  // keep the third-order solution
        c->ki = 1 - c->ki;  // FSAL: K4 becomes the next K1
        hn = c->fixed_step ? c->h : control(c, ha, E, true);
        c->last_rejected = 0;
        if (ha < c->h_min_seen) c->h_min_seen = ha;
      } else {
        c->n_reject += 1;
        hn = control(c, ha, E, false);
        c->last_rejected = 1;
      }
      c->h_last = ha;
      c->h = hn;  // the standard proposal; finalize_step may replace it
      for (int q = 3; q > 0; --q) {
        c->hist_h[q] = c->hist_h[q - 1];
        c->hist_e[q] = c->hist_e[q - 1];
      }
      c->hist_h[0] = ha;
      c->hist_e[0] = E;
      c->nhist += 1;
      // the learned proposer only after 4 attempts and an accepted step, never at the end
      const bool want = c->use_mlp && a.mlp != nullptr && accepted && c->nhist >= 4 && !c->fixed_step &&
                        c->t < c->t1;
      if (want && feat) {
        for (int q = 0; q < 4; ++q) {
          feat[q] = (float)log(c->hist_h[q]);
          feat[4 + q] = (float)log(fmax(c->hist_e[q], 1e-30 * c->rtol) / c->rtol);
        }
        feat[8] = (float)log(fmax(m1, 1e-300));
      }
      return want;
    }
    case ST_D7: {  // a seven-stage attempt (DP5(4) or RKF4(5)): estimate O(h^5), exponent 1/5
      const double E = m0;
      const double ha = c->ha;
      c->n_fev += 6;
      c->err = E;
      bool accepted = true;
      if (!c->fixed_step) {
        if (!isfinite(E)) {
          c->status = 6;  // BS32_NONFINITE
          c->n_reject += 1;
          if (c->trace_on) {
            if (writer) a.trace[c->trace_n % c->trace_cap] = TraceRec{c->t, ha, E, m1, 0, 0};
            c->trace_n += 1;
          }
          return false;
        }
        accepted = E < c->rtol;
      }
      if (c->trace_on) {
        if (writer) a.trace[c->trace_n % c->trace_cap] = TraceRec{c->t, ha, E, m1, accepted ? 1 : 0, 0};
        c->trace_n += 1;
      }
      const double fac = (E > 0.0) ? c->safety * pow(c->rtol / E, 0.2) : c->facmax;
      if (accepted) {
        c->n_accept += 1;
        c->t = (c->t + ha >= c->t1 - c->snap) ? c->t1 : c->t + ha;
        c->xi = 1 - c->xi;
        c->ki = 1 - c->ki;
        c->h = c->fixed_step ? c->h : ha * fmin(c->last_rejected ? 1.0 : c->facmax, fmax(c->facmin, fac));
        c->last_rejected = 0;
        if (ha < c->h_min_seen) c->h_min_seen = ha;
      } else {
        c->n_reject += 1;
        c->h = ha * fmax(c->facmin, fac);
        c->last_rejected = 1;
      }
      c->h_last = ha;
      return false;
    }
    default: break;
  }
  return false;
}

// second half of the step-size update, after the optional learned proposal:
// choose h, clip to h_max, failure conditions of Sec. 2.2, next attempt's step
__device__ __forceinline__ void finalize_step(Ctl* c, bool want, float delta) {
  double hn = c->h;
  int prop = 0;
  if (want && isfinite(delta)) {
    const double d = (double)delta;
    const double d_std = log(c->h / c->h_last);  // the classical rule's step ratio
    if (d >= fmax(kMlpDeltaMin, d_std - kMlpTrust) && d <= fmin(kMlpDeltaMax, d_std + kMlpTrust)) {
      hn = c->h_last * exp(d);
      prop = 1;
      c->n_mlp += 1;
    }
  }
  c->prop_cur = prop;
  c->h = fmin(hn, c->h_max);
  if (c->t >= c->t1) {
    c->status = 0;
    return;
  }
  // failure conditions of Sec. 2.2 (strict thresholds: reading)
  if (c->n_accept + c->n_reject > c->i_max) { c->status = 1; return; }
  if ((double)c->n_reject > 0.85 * (double)c->i_max) { c->status = 2; return; }
  if (!c->fixed_step && c->h <= c->h_min) { c->status = 3; return; }
  c->ha = fmin(c->h, c->t1 - c->t);
}

// Every workgroup reduces the block maxima of the last evaluation and derives the
// same new control state from the same inputs (fixed-order reduction, so the
// copies agree bit for bit); workgroup 0 alone stores it into the other control
// buffer.  Then each workgroup prepares its slice of the next vector operand.
__device__ __forceinline__ void finalize_block(const Args& a, int blk) {
  __shared__ double sR0[4], sR1[4];
  __shared__ Ctl sc;
  __shared__ int s_next;
  constexpr int kWords = (int)(sizeof(Ctl) / sizeof(unsigned long long));
  static_assert(sizeof(Ctl) % sizeof(unsigned long long) == 0 && kWords <= 256, "control block layout");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const bool writer = blk == 0;
  const long long i = (long long)blk * blockDim.x + tid;
  // issue every independent load at once: the control block, the block maxima and
  // both candidate buffers of this agent (which one is current depends on the decision)
  if (tid < kWords) ((unsigned long long*)&sc)[tid] = ((const unsigned long long*)a.ctl)[tid];
  const unsigned rflag = (tid == 0) ? *a.rflag : 0u;  // read by thread 0 after the reductions
  double xc[2] = {0.0, 0.0}, kc[2] = {0.0, 0.0};
  if (i < a.n) {
    xc[0] = a.X[0][i];
    xc[1] = a.X[1][i];
    kc[0] = a.Kf[0][i];
    kc[1] = a.Kf[1][i];
  }
  double m0 = 0.0, m1 = 0.0;
  for (int q = tid; q < a.nrb; q += blockDim.x) {
    m0 = nanmax(m0, a.ep0[q]);
    m1 = nanmax(m1, a.ep1[q]);
  }
  __syncthreads();
  const long long na0 = sc.n_accept;  // read before workgroup thread 0 updates the copy
  if (sc.status != kRunning) {
    if (writer && tid < kWords) ((unsigned long long*)a.ctl_out)[tid] = ((const unsigned long long*)&sc)[tid];
    return;
  }
  m0 = wave_nanmax(m0);
  m1 = wave_nanmax(m1);
  if (lane == 0) {
    sR0[wave] = m0;
    sR1[wave] = m1;
  }
  __syncthreads();
  __shared__ float s_feat[kMlpIn], s_h1[kMlpHid], s_h2[kMlpHid], s_red[1];
  __shared__ int s_want;
  if (tid == 0) {
    m0 = sR0[0];
    m1 = sR1[0];
    for (int w = 1; w < nw; ++w) {
      m0 = nanmax(m0, sR0[w]);
      m1 = nanmax(m1, sR1[w]);
    }
    s_want = 0;
    // the decision is a chain of dependent updates of the control state: run it on a
    // copy in registers, not field by field in LDS
    Ctl cl = sc;
    if (rflag) cl.status = kStatusRange;
    else s_want = finalize(a, &cl, m0, m1, writer, s_feat) ? 1 : 0;
    s_next = (a.stage == ST_INIT && !(cl.h0user > 0.0)) ? ST_H0 : ST_S2;
    // without a learned proposal the rest of the step-size update follows at once
    if ((a.stage == ST_S4 || a.stage == ST_D7) && cl.status == kRunning && !s_want) finalize_step(&cl, false, 0.0f);
    sc = cl;
  }
  __syncthreads();
  if ((a.stage == ST_S4 || a.stage == ST_D7) && sc.status == kRunning && s_want) {
    // learned proposal (whole workgroup), then the rest of the step-size update
    const float delta = mlp_forward_wg(a.mlp, s_feat, s_h1, s_h2, s_red);
    if (tid == 0) {
      Ctl cl = sc;
      finalize_step(&cl, true, delta);
      sc = cl;
    }
    __syncthreads();
  }
  if (writer && tid < kWords) ((unsigned long long*)a.ctl_out)[tid] = ((const unsigned long long*)&sc)[tid];
  // solution record: the initial value, then the state after every accepted step
  if (a.rec && i < a.n && (a.stage == ST_INIT || ((a.stage == ST_S4 || a.stage == ST_D7) && sc.n_accept != na0))) {
    const long long slot = (a.stage == ST_INIT) ? 0 : sc.n_accept;
    if (slot < a.rec_cap) {
      const double* Xc = pick2(a.X, sc.xi);
      double* dst = a.rec + (slot * a.n + i) * a.d;
      for (int c = 0; c < a.d; ++c) dst[c] = Xc[c * a.np + i];
    }
  }
  if (sc.status != kRunning) return;
  if (i < a.n) {
    const double x = xc[sc.xi], k1 = kc[sc.ki];
    const double a21 = sc.method == 1 ? kDpA[1][0] : sc.method == 2 ? kFeA[1][0] : kA21;
    const double y = (s_next == ST_H0) ? x + sc.h0probe * k1 : sstore(a, x + sc.ha * (a21 * k1));
    write_operand(a, 0, i, y);
  }
}

// ---------------------------------------------------------------------------
// Persistent ensemble launch (PGroup): every workgroup repeatedly claims the next task
// of a listed instance, waits until the task's phase may start, runs it (a row tile of
// S2, S3 or S4 with the grouped contraction, or a finalize slice) and counts it done.
// Instances advance independently, each through its own control blocks.  Claims go to
// instances of the workgroup's own XCD first (their operand stays in that L2), then to
// any.  A task's inputs were written by other workgroups, possibly on other XCDs: the
// completion count is an agent-scope release by thread 0 after the workgroup barrier
// (the barrier completes every wave's stores; the release writes the XCD's L2 back),
// and the start an agent-scope acquire by thread 0 before the barrier (it invalidates
// the CU's vector cache and the XCD's L2, which every wave of the workgroup reads
// through).  Every wait is bounded; a wait that exceeds its bound sets the abort word,
// and every workgroup then leaves.
// ---------------------------------------------------------------------------
// bound of one wait (for a phase to open, or for any open task): 10 s of the
// constant-rate clock (100 MHz); the longest legitimate wait is one phase of one
// instance, milliseconds for the sizes here
constexpr unsigned long long kPersWaitTicks = 1000000000ULL;

__device__ __forceinline__ unsigned pers_phase_start(unsigned k, const PSched& sc) {
  const unsigned a = k / sc.Q, r = k - a * sc.Q;
  const unsigned off = r < sc.TC ? 0u : r < 2 * sc.TC ? sc.TC : r < 3 * sc.TC ? 2 * sc.TC : 3 * sc.TC;
  return a * sc.Q + off;
}
// first ticket after the phase that starts at ticket s
__device__ __forceinline__ unsigned pers_phase_end(unsigned s, const PSched& sc) {
  const unsigned r = s % sc.Q;
  return s + (r < 3 * sc.TC ? sc.TC : sc.Q - 3 * sc.TC);
}

// the finalize slices as a call: compiled apart, its registers do not add to the
// contraction loop's (which would spill otherwise); only the few values live across
// the call are saved around it
__device__ __attribute__((noinline)) void pers_finalize(const Args& a, int blk) { finalize_block(a, blk); }

template <class CONTRACT>
__device__ __forceinline__ void pers_loop(const PGroup& p, CONTRACT contract) {
  __shared__ int s_li;
  __shared__ unsigned s_k;
  const int tid = threadIdx.x;
  const unsigned n = *p.count;
  const unsigned xcd = blockIdx.x & 7u;
  const unsigned lo = min(p.xs[xcd], n), hi = min(p.xs[xcd + 1], n);
  unsigned cursor = blockIdx.x >> 3;
  unsigned long long idle_since = 0;  // thread 0: start of the current wait for an open task
  // thread 0: a run of tasks of one instance and phase whose completions are not yet
  // counted.  The release that counts them writes the XCD's L2 back and costs about as
  // much as a task's other overheads together, so a run takes the instance's next ticket
  // directly while its phase has one left and counts the run with one release; the
  // release follows at once when the phase has no ticket left, and always comes before
  // any wait, so a workgroup never waits while holding completions others may wait for.
  int pend_li = -1;
  unsigned pend_need = 0, pend_n = 0;
  while (true) {
    if (tid == 0) {
      int li_sel = -1;
      unsigned k_sel = 0;
      bool all_claimed = true;
      if (pend_n) {  // continue the run
        const PSched sc = p.sched[pend_li];
        const unsigned total = sc.Q * (unsigned)p.attempts;
        const unsigned end = min(pers_phase_end(pend_need, sc), total);
        if (__hip_atomic_load(&p.tick[pend_li], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < end) {
          const unsigned k = __hip_atomic_fetch_add(&p.tick[pend_li], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (k < total) {  // a later phase's ticket if others took the last ones: released below, then waited for
            li_sel = pend_li;
            k_sel = k;
            all_claimed = false;
          }
        }
        if (li_sel < 0) {  // the phase has no ticket left: count the run now
          __hip_atomic_fetch_add(&p.comp[pend_li], pend_n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          pend_n = 0;
        }
      }
      for (int pass = 0; pass < 2 && li_sel < 0; ++pass) {
        const unsigned base = pass == 0 ? lo : 0u, len = pass == 0 ? hi - lo : n;
        for (unsigned q = 0; q < len; ++q) {
          const unsigned li = base + (cursor + q) % len;
          const PSched sc = p.sched[li];
          const unsigned total = sc.Q * (unsigned)p.attempts;
          const unsigned t = __hip_atomic_load(&p.tick[li], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (t >= total) continue;
          all_claimed = false;
          if (__hip_atomic_load(&p.comp[li], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < pers_phase_start(t, sc))
            continue;  // its next phase is not open yet
          const unsigned k = __hip_atomic_fetch_add(&p.tick[li], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (k >= total) continue;
          li_sel = (int)li;
          k_sel = k;
          cursor = (cursor + q) % (len ? len : 1u);
          break;
        }
      }
      if (__hip_atomic_load(p.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) li_sel = -2;
      else if (li_sel < 0 && all_claimed) li_sel = -2;
      const unsigned need = li_sel >= 0 ? pers_phase_start(k_sel, p.sched[li_sel]) : 0u;
      const bool same = li_sel >= 0 && li_sel == pend_li && need == pend_need;
      if (!same && pend_n) {
        __hip_atomic_fetch_add(&p.comp[pend_li], pend_n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        pend_n = 0;
      }
      if (li_sel >= 0 && !same) {  // wait until the task's phase has opened (the run's next
        // task needs neither: its phase is open and its inputs already acquired)
        pend_li = li_sel;
        pend_need = need;
        const unsigned long long w0 = wall_clock64();
        while (__hip_atomic_load(&p.comp[li_sel], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (wall_clock64() - w0 > kPersWaitTicks ||
              __hip_atomic_load(p.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(p.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            li_sel = -2;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      s_li = li_sel;
      s_k = k_sel;
    }
    __syncthreads();
    const int li = s_li;
    const unsigned k = s_k;
    __syncthreads();  // every thread has read the choice before thread 0 makes the next
    if (li == -2) return;
    if (li == -1) {  // nothing open now: other instances' phases are still running
      if (tid == 0) {
        const unsigned long long now = wall_clock64();
        if (idle_since == 0) idle_since = now;
        else if (now - idle_since > kPersWaitTicks)
          __hip_atomic_store(p.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_sleep(32);
      }
      continue;
    }
    if (tid == 0) idle_since = 0;
    const PSched sc = p.sched[li];
    const unsigned a = k / sc.Q, r = k - a * sc.Q;
    const int par = (p.par0 + (int)a) & 1;
    if (r < 3 * sc.TC) {
      const int st = r < sc.TC ? ST_S2 : r < 2 * sc.TC ? ST_S3 : ST_S4;
      const Args& args = p.inst[((size_t)sc.b * kStages + st) * 2 + par];
      const unsigned j0 = (r % sc.TC) * sc.G, j1 = min(j0 + sc.G, sc.T);
      for (unsigned j = j0; j < j1; ++j) {
        contract(args, (int)j);
        __syncthreads();
      }
    } else {
      const Args& args = p.inst[((size_t)sc.b * kStages + ST_S4) * 2 + par];
      const unsigned j0 = (r - 3 * sc.TC) * sc.GF, j1 = min(j0 + sc.GF, sc.F);
      for (unsigned j = j0; j < j1; ++j) {
        pers_finalize(args, (int)j);
        __syncthreads();
      }
    }
    __syncthreads();  // every wave's stores of the task are done before thread 0 counts it
    if (tid == 0) pend_n += 1;
  }
}

// the persistent kernels of the grouped tile families (four waves: the finalize slices
// take 256 threads)
template <int M, int R, int WR, int WK, int U, bool NT>
__global__ __launch_bounds__(256) void k_pers_f64(PGroup p) {
  static_assert(WR * WK == 4, "four waves");
  pers_loop(p, [](const Args& a, int rb) { contract_f64<M, R, WR, WK, U, NT, false>(a, rb); });
}
template <int M, int T, int R, int WR, int WK, int U, bool NT>
__global__ __launch_bounds__(256) void k_pers_f32(PGroup p) {
  static_assert(WR * WK == 4, "four waves");
  pers_loop(p, [](const Args& a, int rb) { contract_f32<M, T, R, WR, WK, U, NT, false>(a, rb); });
}
template <int FMT, int M, int T, int RT, int WR, int WK, int U, bool NT>
__global__ __launch_bounds__(256, 2) void k_pers_mfma(PGroup p) {
  static_assert(WR * WK == 4, "four waves");
  pers_loop(p, [](const Args& a, int rb) { contract_mfma<FMT, M, T, RT, WR, WK, U, NT, false>(a, rb); });
}
#if BS32_IN(0)
__global__ void k_zero_u32(unsigned* p, unsigned n) {
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}
#endif

#if BS32_IN(0)
__global__ __launch_bounds__(256) void k_finalize(Args a) { finalize_block(a, blockIdx.x); }
__global__ __launch_bounds__(256) void k_group_finalize(Group g) { BS32_GROUP_LOOP(finalize_block) }

__global__ void k_set_status(Ctl* c, int code) {
  if (threadIdx.x == 0 && c->status == kRunning) c->status = code;
}

// ---------------------------------------------------------------------------
// layout conversions and packing of the coupling matrix
// ---------------------------------------------------------------------------
__global__ void k_to_soa(const double* __restrict__ src, double* __restrict__ dst, long long n, int d, long long np) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < d; ++c) dst[c * np + i] = src[i * d + c];
}
__global__ void k_from_soa(const double* __restrict__ src, double* __restrict__ dst, long long n, int d,
                           long long np) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < d; ++c) dst[i * d + c] = src[c * np + i];
}
// dst (rows x ld) <- src (n x n row-major), zero padding; uniform: all ones
__global__ void k_pack_f64(const double* __restrict__ src, double* __restrict__ dst, long long n, long long ld,
                           long long rows, int uniform) {
  const long long total = rows * ld;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / ld, j = e - r * ld;
    double v = 0.0;
    if (r < n && j < n) v = uniform ? 1.0 : src[r * n + j];
    dst[e] = v;
  }
}
// max |A| over the packed matrix; out (zero-initialized) receives the bits of the
// non-negative maximum, whose integer order equals the floating-point order
__global__ void k_absmax(const double* __restrict__ A, long long count, unsigned long long* out) {
  double m = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x)
    m = nanmax(m, fabs(A[e]));
  __shared__ double red[4];
  m = wave_nanmax(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
  }
}
__global__ void k_pack_fmt(const double* __restrict__ A, void* __restrict__ dst, int fmt, double inv_scale,
                           long long count) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x) {
    const double x = A[e] * inv_scale;  // power-of-two scale: exact
    if (fmt == F_BF16X2) {  // hi plane, then the remainder's plane
      const uint32_t hi = encode_rne(x, fmt_desc(F_BF16));
      ((uint16_t*)dst)[e] = (uint16_t)hi;
      ((uint16_t*)dst)[count + e] = (uint16_t)encode_rne(x - decode_bits(hi, fmt_desc(F_BF16)), fmt_desc(F_BF16));
    } else if (fmt == F_F32) ((float*)dst)[e] = (float)x;
    else if (fmt == F_E4M3) ((uint8_t*)dst)[e] = (uint8_t)encode_rne(x, fmt_desc(fmt));
    else ((uint16_t*)dst)[e] = (uint16_t)encode_rne(x, fmt_desc(fmt));
  }
}
__device__ __forceinline__ double stored_value(const void* A, int fmt, long long e, long long plane) {
  switch (fmt) {
    case F_BF16X2:
      return decode_bits(((const uint16_t*)A)[e], fmt_desc(F_BF16)) +
             decode_bits(((const uint16_t*)A)[plane + e], fmt_desc(F_BF16));
    case F_F64: return ((const double*)A)[e];
    case F_F32: return (double)((const float*)A)[e];
    case F_E4M3: return decode_bits(((const uint8_t*)A)[e], fmt_desc(fmt));
    default: return decode_bits(((const uint16_t*)A)[e], fmt_desc(fmt));
  }
}
// row sums of the stored matrix in FP64 (fixed order; one workgroup per row)
__global__ void k_rowsum(const void* __restrict__ A, int fmt, double scale, double* __restrict__ rsum, long long n,
                         long long ld, long long plane) {
  __shared__ double red[4];
  const long long r = blockIdx.x;
  double s = 0.0;
  for (long long j = threadIdx.x; j < n; j += blockDim.x) s += scale * stored_value(A, fmt, r * ld + j, plane);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) rsum[r] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static unsigned grid_for(long long count) { return (unsigned)std::min<long long>((count + 255) / 256, 65536); }

// values rounded to FP32 in place (the Single recipe's initial state)
__global__ void k_round_f32(double* __restrict__ x, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (double)(float)x[i];
}
hipError_t launch_round_f32(double* x, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_round_f32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, n);
  return hipGetLastError();
}

hipError_t launch_to_soa(const double* src, double* dst, long long n, int d, long long np, hipStream_t s) {
  k_to_soa<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, dst, n, d, np);
  return hipGetLastError();
}
hipError_t launch_from_soa(const double* src, double* dst, long long n, int d, long long np, hipStream_t s) {
  k_from_soa<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(src, dst, n, d, np);
  return hipGetLastError();
}
hipError_t launch_pack_f64(const double* src, double* dst, long long n, long long ld, long long rows, int uniform,
                           hipStream_t s) {
  k_pack_f64<<<grid_for(rows * ld), 256, 0, s>>>(src, dst, n, ld, rows, uniform);
  return hipGetLastError();
}
hipError_t launch_absmax(const double* A64, long long count, double* out, hipStream_t s) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(double), s);
  if (e != hipSuccess) return e;
  k_absmax<<<std::min(grid_for(count), 2048u), 256, 0, s>>>(A64, count, (unsigned long long*)out);
  return hipGetLastError();
}
hipError_t launch_pack_fmt(const double* A64, void* dst, int fmt, double inv_scale, long long count, hipStream_t s) {
  k_pack_fmt<<<grid_for(count), 256, 0, s>>>(A64, dst, fmt, inv_scale, count);
  return hipGetLastError();
}
hipError_t launch_rowsum(const void* A, int fmt, double scale, double* rsum, long long n, long long ld,
                         hipStream_t s) {
  const long long plane = (n + 255) / 256 * 256 * ld;  // np x ld values per plane (BF16 pairs)
  k_rowsum<<<(unsigned)n, 256, 0, s>>>(A, fmt, scale, rsum, n, ld, plane);
  return hipGetLastError();
}
hipError_t launch_prep(const Args& a, hipStream_t s) {
  k_prep<<<(unsigned)((a.n + 255) / 256), 256, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_finalize(const Args& a, hipStream_t s) {
  k_finalize<<<(unsigned)((a.n + 255) / 256), 256, 0, s>>>(a);
  return hipGetLastError();
}
hipError_t launch_set_status(Ctl* c, int code, hipStream_t s) {
  k_set_status<<<1, 64, 0, s>>>(c, code);
  return hipGetLastError();
}

int tile_rows(int fmt, const Tile& t) {
  return t.MM == 3 ? 64 * t.R : t.MM == 1 ? 16 * t.R * t.WR : t.R * t.WR;
}
// columns one wave step covers: 64 lanes x 16 bytes (VALU), 4 lane groups x 16 bytes (matrix cores)
int tile_kalign(int fmt, const Tile& t) {
  if (t.MM == 1) return 64 / (int)fmt_bytes(fmt);
  if (t.MM == 2) return 64;
  if (t.MM == 3) return 256;
  return fmt == F_F64 ? 128 : 256;
}

#endif  // BS32_IN(0)

// ---- instantiated tiles ------------------------------------------------------
// (R, WR, WK, U, NT): the candidate set the autotuner times, per kernel family
#define BS32_F64_TILES(X)                                                                                   \
  X(1, 4, 1, 4, 0) X(2, 1, 4, 2, 0) X(2, 2, 2, 2, 0) X(4, 1, 4, 2, 0) X(1, 1, 8, 2, 0) X(1, 1, 4, 8, 0)     \
  X(2, 1, 4, 4, 0) X(1, 1, 8, 4, 0) X(2, 1, 4, 2, 1) X(4, 1, 4, 2, 1) X(1, 1, 4, 8, 1) X(2, 1, 8, 4, 0)     \
  X(2, 2, 2, 2, 1) X(4, 2, 2, 2, 1)
#define BS32_F32_TILES(X)                                                                                   \
  X(1, 4, 1, 2, 0) X(1, 1, 4, 2, 0) X(2, 1, 4, 2, 0) X(1, 1, 8, 2, 0) X(1, 1, 4, 4, 0) X(2, 1, 4, 4, 0)     \
  X(1, 1, 8, 4, 0) X(2, 1, 4, 2, 1) X(1, 1, 8, 4, 1)
#define BS32_MMA_TILES(X)                                                                    \
  X(1, 1, 8, 2, 0) X(1, 1, 8, 4, 0) X(1, 1, 8, 8, 0) X(2, 1, 8, 4, 0) X(1, 1, 4, 8, 0) X(2, 1, 4, 4, 0) \
  X(1, 1, 8, 4, 1) X(2, 1, 8, 4, 1) X(1, 1, 4, 4, 0) X(1, 1, 4, 8, 1) X(1, 1, 8, 8, 1) X(2, 1, 4, 4, 1) \
  X(1, 1, 4, 4, 1) X(2, 2, 2, 4, 0) X(2, 2, 2, 4, 1) X(2, 4, 1, 4, 0) X(2, 4, 1, 4, 1) X(1, 4, 1, 4, 0)  \
  X(1, 4, 1, 4, 1) X(2, 8, 1, 4, 1) X(2, 4, 1, 2, 1)

// the matrix-core tiles that also run with an epilogue wave: one 16-row tile per wave and
// batches of at most four steps (the others would spill with the extra wave's share of
// the register file), and at most 32 rows per block (two lanes per row in one wave)
#define BS32_MMA_EW_OK(R_, WR_, U_) ((R_) == 1 && (U_) <= 4 && (WR_) <= 2)

// pairwise kernels: (R rows per wave, WV waves, UJ column chunks per step)
#define BS32_PAIR_TILES(X) X(2, 4, 1) X(4, 4, 1) X(8, 4, 1) X(4, 4, 2)

// shared-coupling products: (RT 16-row tiles per wave, CT 16-column tiles), four waves;
// RT = 4 only for 16-bit storage (its FP32 P tile fits the LDS)
#define BS32_SHARED_TILES(X) X(2, 4) X(1, 8) X(1, 4) X(2, 2) X(4, 4) X(4, 2)
// LDS-tiled products of 16-bit storage (k_shared_gemm): (RT, CT), tiles of 64 RT x 16 CT
#define BS32_GEMM_TILES(X) X(2, 8) X(2, 4) X(1, 8)

#if BS32_IN(0)
#define BS32_TILE_VALU(R_, WR_, WK_, U_, NT_) Tile{R_, WR_, WK_, U_, NT_, 0},
#define BS32_TILE_MMA(R_, WR_, WK_, U_, NT_) Tile{R_, WR_, WK_, U_, NT_, 1},
#define BS32_TILE_VALU_EW(R_, WR_, WK_, U_, NT_) Tile{R_, WR_, WK_, U_, NT_, 0, 1},
#define BS32_TILE_MMA_EW(R_, WR_, WK_, U_, NT_) BS32_TILE_MMA_EW_##R_##_##U_(R_, WR_, WK_, U_, NT_)
#define BS32_TILE_MMA_EW_1_2(R_, WR_, WK_, U_, NT_) BS32_TILE_MMA_EW_W##WR_(R_, WR_, WK_, U_, NT_)
#define BS32_TILE_MMA_EW_1_4(R_, WR_, WK_, U_, NT_) BS32_TILE_MMA_EW_W##WR_(R_, WR_, WK_, U_, NT_)
#define BS32_TILE_MMA_EW_W1(R_, WR_, WK_, U_, NT_) Tile{R_, WR_, WK_, U_, NT_, 1, 1},
#define BS32_TILE_MMA_EW_W2(R_, WR_, WK_, U_, NT_) Tile{R_, WR_, WK_, U_, NT_, 1, 1},
#define BS32_TILE_MMA_EW_W4(R_, WR_, WK_, U_, NT_)
#define BS32_TILE_MMA_EW_1_8(R_, WR_, WK_, U_, NT_)
#define BS32_TILE_MMA_EW_2_2(R_, WR_, WK_, U_, NT_)
#define BS32_TILE_MMA_EW_2_4(R_, WR_, WK_, U_, NT_)
#define BS32_TILE_MMA_EW_2_8(R_, WR_, WK_, U_, NT_)
// every tile, then (single systems only) the same tiles with an epilogue wave
static const Tile kF64Tiles[] = {BS32_F64_TILES(BS32_TILE_VALU) BS32_F64_TILES(BS32_TILE_VALU_EW)};
static const Tile kF32Tiles[] = {BS32_F32_TILES(BS32_TILE_VALU) BS32_MMA_TILES(BS32_TILE_MMA)
                                     BS32_F32_TILES(BS32_TILE_VALU_EW) BS32_MMA_TILES(BS32_TILE_MMA_EW)};
static const Tile kMmaTiles[] = {BS32_MMA_TILES(BS32_TILE_MMA) BS32_MMA_TILES(BS32_TILE_MMA_EW)};
#define BS32_TILE_PAIR(R_, WV_, UJ_) Tile{R_, WV_, 1, UJ_, 0, 2},
static const Tile kPairTiles[] = {BS32_PAIR_TILES(BS32_TILE_PAIR)};
#undef BS32_TILE_PAIR
#define BS32_TILE_SHARED(RT_, CT_) Tile{RT_, 4, 1, CT_, 0, 3},
#define BS32_TILE_GEMM(RT_, CT_) Tile{RT_, 4, 2, CT_, 0, 3},
static const Tile kSharedTiles[] = {BS32_SHARED_TILES(BS32_TILE_SHARED) Tile{1, 4, 1, 8, 1, 3}, Tile{1, 4, 1, 4, 1, 3},
                                     Tile{1, 4, 1, 2, 1, 3}, BS32_GEMM_TILES(BS32_TILE_GEMM)};
#undef BS32_TILE_SHARED
#undef BS32_TILE_GEMM
#undef BS32_TILE_VALU
#undef BS32_TILE_MMA
#undef BS32_TILE_VALU_EW
#undef BS32_TILE_MMA_EW
#undef BS32_TILE_MMA_EW_1_2
#undef BS32_TILE_MMA_EW_1_4
#undef BS32_TILE_MMA_EW_W1
#undef BS32_TILE_MMA_EW_W2
#undef BS32_TILE_MMA_EW_W4
#undef BS32_TILE_MMA_EW_1_8
#undef BS32_TILE_MMA_EW_2_2
#undef BS32_TILE_MMA_EW_2_4
#undef BS32_TILE_MMA_EW_2_8

const Tile* pair_tile_candidates(int* count) {
  *count = (int)(sizeof(kPairTiles) / sizeof(Tile));
  return kPairTiles;
}

const Tile* tile_candidates(int fmt, int* count) {
  if (fmt == F_F64) {
    *count = (int)(sizeof(kF64Tiles) / sizeof(Tile));
    return kF64Tiles;
  }
  if (fmt == F_F32) {
    *count = (int)(sizeof(kF32Tiles) / sizeof(Tile));
    return kF32Tiles;
  }
  *count = (int)(sizeof(kMmaTiles) / sizeof(Tile));
  return kMmaTiles;
}

const Tile* shared_tile_candidates(int* count) {
  *count = (int)(sizeof(kSharedTiles) / sizeof(Tile));
  return kSharedTiles;
}
#endif  // BS32_IN(0)

// one contraction launch: a single system (a) or an ensemble (g, ggrid workgroups)
struct Launch {
  const Args* a;
  const Group* g;
  unsigned ggrid;
  hipStream_t s;
  bool dry;
  const PGroup* p = nullptr;  // persistent ensemble launch (grid ggrid)
};
// the launchers of each kernel family (each defined in its own part)
template <int M>
hipError_t launch_f64(const Launch& L, const Tile& t);
template <int M>
hipError_t launch_f32(const Launch& L, const Tile& t);
template <int FMT, int M, int T>
hipError_t launch_mma(const Launch& L, const Tile& t);
hipError_t launch_pair(const Launch& L, int fmt, const Tile& t);
// sh == nullptr: only whether the instance exists
hipError_t dispatch_shared(const Shared* sh, int m, int fmt, const Tile& t, hipStream_t s);

#if BS32_IN(8)

template <int FMT, int M>
static hipError_t launch_shared_t(const Shared* sh, const Tile& t, hipStream_t s) {
  const int total = sh ? sh->nrb * sh->ncb : 0;
  const unsigned grid = 8u * (unsigned)((total + 7) / 8);
  if (t.NT) {  // library product + epilogue: 16-bit storage, 64 x 16 CT epilogue tiles
    if constexpr (FMT == F_BF16 || FMT == F_F16 || FMT == F_BF16X2) {
      if (t.R == 1 && (t.U == 8 || t.U == 4 || t.U == 2)) {
        if (!sh) return hipSuccess;
        if (sh->Pg[0] == nullptr || (FMT == F_BF16X2 && sh->Pg[1] == nullptr)) return hipErrorInvalidValue;
        if (total > 0) {
          if (t.U == 8) k_shared_contract<FMT, M, 1, 8, true><<<grid, 256, 0, s>>>(*sh);
          else if (t.U == 4) k_shared_contract<FMT, M, 1, 4, true><<<grid, 256, 0, s>>>(*sh);
          else k_shared_contract<FMT, M, 1, 2, true><<<grid, 256, 0, s>>>(*sh);
        }
        return hipGetLastError();
      }
    }
    return hipErrorInvalidValue;
  }
  if (t.WK == 2) {  // LDS-tiled product: 16-bit storage
    if constexpr (FMT == F_BF16 || FMT == F_F16 || FMT == F_BF16X2) {
#define G(RT_, CT_)                                                                 \
  if (t.R == RT_ && t.U == CT_) {                                                   \
    if constexpr (gemm_lds_bytes<FMT, RT_, CT_>() > 160 * 1024) {                   \
      return hipErrorInvalidValue;                                                  \
    } else {                                                                        \
      if (!sh) return hipSuccess;                                                   \
      if (total > 0) k_shared_gemm<FMT, M, RT_, CT_><<<grid, 256, 0, s>>>(*sh);    \
      return hipGetLastError();                                                     \
    }                                                                               \
  }
      BS32_GEMM_TILES(G)
#undef G
    }
    return hipErrorInvalidValue;
  }
#define X(RT_, CT_)                                                                       \
  if (t.R == RT_ && t.U == CT_) {                                                         \
    if constexpr (RT_ == 4 && !sh_f32acc<FMT>()) {                                        \
      return hipErrorInvalidValue;                                                        \
    } else {                                                                              \
      if (!sh) return hipSuccess;                                                         \
      if (total > 0) k_shared_contract<FMT, M, RT_, CT_><<<grid, 256, 0, s>>>(*sh);      \
      return hipGetLastError();                                                           \
    }                                                                                     \
  }
  BS32_SHARED_TILES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t dispatch_shared(const Shared* sh, int m, int fmt, const Tile& t, hipStream_t s) {
  if (t.MM != 3 || t.WR != 4) return hipErrorInvalidValue;
  switch (fmt) {
    case F_F64: return m == 2 ? launch_shared_t<F_F64, 2>(sh, t, s) : launch_shared_t<F_F64, 1>(sh, t, s);
    case F_F32: return m == 2 ? launch_shared_t<F_F32, 2>(sh, t, s) : launch_shared_t<F_F32, 1>(sh, t, s);
    case F_BF16: return m == 2 ? launch_shared_t<F_BF16, 2>(sh, t, s) : launch_shared_t<F_BF16, 1>(sh, t, s);
    case F_F16: return m == 2 ? launch_shared_t<F_F16, 2>(sh, t, s) : launch_shared_t<F_F16, 1>(sh, t, s);
    case F_BF16X2:
      return m == 2 ? launch_shared_t<F_BF16X2, 2>(sh, t, s) : launch_shared_t<F_BF16X2, 1>(sh, t, s);
    default: return hipErrorInvalidValue;
  }
}

#endif  // BS32_IN(8)

#if BS32_IN(0)
hipError_t launch_shared_contract(const Shared& sh, int m, int fmt, const Tile& t, hipStream_t s) {
  return dispatch_shared(&sh, m, fmt, t, s);
}
#endif
// THREADS: the tile's streaming waves; a single-system kernel with an epilogue wave
// (tile EW) has one more, and the grouped kernels have none
#define BS32_LAUNCH(SINGLE_EW, SINGLE, GROUP, PERS, THREADS) \
  BS32_LAUNCH_IF(true, SINGLE_EW, SINGLE, GROUP, PERS, THREADS)
#define BS32_LAUNCH_IF(EWOK, SINGLE_EW, SINGLE, GROUP, PERS, THREADS)                            \
  if (L.p) {                                                                                     \
    if (t.EW) return hipErrorInvalidValue;                                                       \
    if constexpr ((THREADS) == 256) {                                                            \
      if (!L.dry) PERS<<<L.ggrid, 256, 0, L.s>>>(*L.p);                                           \
      return L.dry ? hipSuccess : hipGetLastError();                                             \
    } else {                                                                                     \
      return hipErrorInvalidValue;                                                               \
    }                                                                                            \
  }                                                                                              \
  if (L.g && t.EW) return hipErrorInvalidValue;                                                  \
  if constexpr (!(EWOK)) {                                                                       \
    if (t.EW) return hipErrorInvalidValue;                                                       \
    if (!L.dry) {                                                                                \
      if (L.g) GROUP<<<L.ggrid, THREADS, 0, L.s>>>(*L.g);                                        \
      else SINGLE<<<(unsigned)L.a->nrb, THREADS, 0, L.s>>>(*L.a);                                \
    }                                                                                            \
  } else {                                                                                       \
    if (!L.dry) {                                                                                \
      if (L.g) GROUP<<<L.ggrid, THREADS, 0, L.s>>>(*L.g);                                        \
      else if (t.EW) SINGLE_EW<<<(unsigned)L.a->nrb, THREADS + 64, 0, L.s>>>(*L.a);              \
      else SINGLE<<<(unsigned)L.a->nrb, THREADS, 0, L.s>>>(*L.a);                                \
    }                                                                                            \
  }                                                                                              \
  return L.dry ? hipSuccess : hipGetLastError();

#if BS32_IN(1)
template <int M>
hipError_t launch_f64(const Launch& L, const Tile& t) {
#define X(R_, WR_, WK_, U_, NT_)                                                                 \
  if (t.R == R_ && t.WR == WR_ && t.WK == WK_ && t.U == U_ && t.NT == NT_) {                     \
    BS32_LAUNCH((k_contract_f64<M, R_, WR_, WK_, U_, NT_, true>), (k_contract_f64<M, R_, WR_, WK_, U_, NT_, false>), \
                (k_group_f64<M, R_, WR_, WK_, U_, NT_>), (k_pers_f64<M, R_, WR_, WK_, U_, NT_>), WR_ * WK_ * 64) \
  }
  BS32_F64_TILES(X)
#undef X
  return hipErrorInvalidValue;
}
template hipError_t launch_f64<1>(const Launch&, const Tile&);
template hipError_t launch_f64<2>(const Launch&, const Tile&);
#endif
#if BS32_IN(2)
template <int M>
hipError_t launch_f32(const Launch& L, const Tile& t) {
#define X(R_, WR_, WK_, U_, NT_)                                                                       \
  if (t.R == R_ && t.WR == WR_ && t.WK == WK_ && t.U == U_ && t.NT == NT_) {                           \
    BS32_LAUNCH((k_contract_f32<M, 2, R_, WR_, WK_, U_, NT_, true>),                                   \
                (k_contract_f32<M, 2, R_, WR_, WK_, U_, NT_, false>),                                  \
                (k_group_f32<M, 2, R_, WR_, WK_, U_, NT_>), (k_pers_f32<M, 2, R_, WR_, WK_, U_, NT_>),  \
                WR_ * WK_ * 64)                                                                        \
  }
  BS32_F32_TILES(X)
#undef X
  return hipErrorInvalidValue;
}
template hipError_t launch_f32<1>(const Launch&, const Tile&);
template hipError_t launch_f32<2>(const Launch&, const Tile&);
#endif
#if BS32_IN(3) || BS32_IN(4) || BS32_IN(5) || BS32_IN(6)
template <int FMT, int M, int T>
hipError_t launch_mma(const Launch& L, const Tile& t) {
#define X(R_, WR_, WK_, U_, NT_)                                                            \
  if (t.R == R_ && t.WR == WR_ && t.WK == WK_ && t.U == U_ && t.NT == NT_) {                \
    BS32_LAUNCH_IF(BS32_MMA_EW_OK(R_, WR_, U_), (k_contract_mfma<FMT, M, T, R_, WR_, WK_, U_, NT_, true>), \
                   (k_contract_mfma<FMT, M, T, R_, WR_, WK_, U_, NT_, false>),                 \
                   (k_group_mfma<FMT, M, T, R_, WR_, WK_, U_, NT_>),                           \
                   (k_pers_mfma<FMT, M, T, R_, WR_, WK_, U_, NT_>), WR_ * WK_ * 64)            \
  }
  BS32_MMA_TILES(X)
#undef X
  return hipErrorInvalidValue;
}
#endif
#if BS32_IN(3)
template hipError_t launch_mma<F_F32, 1, 2>(const Launch&, const Tile&);
template hipError_t launch_mma<F_F32, 2, 2>(const Launch&, const Tile&);
#endif
#if BS32_IN(4)
template hipError_t launch_mma<F_BF16, 1, 2>(const Launch&, const Tile&);
template hipError_t launch_mma<F_BF16, 2, 2>(const Launch&, const Tile&);
#endif
#if BS32_IN(5)
template hipError_t launch_mma<F_F16, 1, 2>(const Launch&, const Tile&);
template hipError_t launch_mma<F_F16, 2, 2>(const Launch&, const Tile&);
#endif
#if BS32_IN(6)
template hipError_t launch_mma<F_E4M3, 1, 3>(const Launch&, const Tile&);
template hipError_t launch_mma<F_E4M3, 2, 3>(const Launch&, const Tile&);
#endif
#if BS32_IN(7)
template <bool ATAN, bool G32, bool DENSE>
static hipError_t launch_pair_t(const Launch& L, const Tile& t) {
#define X(R_, WV_, UJ_)                                                                                  \
  if (t.R == R_ && t.WR == WV_ && t.U == UJ_) {                                                          \
    if (L.dry) return hipSuccess;                                                                        \
    if (L.g) return hipErrorInvalidValue; /* pairwise couplings are not grouped */                      \
    k_contract_pair<ATAN, G32, DENSE, R_, WV_, UJ_><<<(unsigned)L.a->nrb, WV_ * 64, 0, L.s>>>(*L.a);    \
    return hipGetLastError();                                                                            \
  }
  BS32_PAIR_TILES(X)
#undef X
  return hipErrorInvalidValue;
}
// fmt F_F32 selects the FP32 pair term (the recipes), F_F64 the FP64 one
hipError_t launch_pair(const Launch& L, int fmt, const Tile& t) {
  if (L.dry) return launch_pair_t<false, false, false>(L, t);
  if (L.g) return hipErrorInvalidValue;
  const bool atn = L.a->kind == 5, g32 = fmt == F_F32, dense = L.a->A != nullptr;
  if (atn) {
    if (g32) return dense ? launch_pair_t<true, true, true>(L, t) : launch_pair_t<true, true, false>(L, t);
    return dense ? launch_pair_t<true, false, true>(L, t) : launch_pair_t<true, false, false>(L, t);
  }
  if (g32) return dense ? launch_pair_t<false, true, true>(L, t) : launch_pair_t<false, true, false>(L, t);
  return dense ? launch_pair_t<false, false, true>(L, t) : launch_pair_t<false, false, false>(L, t);
}
#endif  // BS32_IN(7)
#undef BS32_LAUNCH

#if BS32_IN(0)
static hipError_t dispatch(const Launch& L, int m, int fmt, const Tile& t);
bool tile_supported(int fmt, int m, const Tile& t);

static hipError_t dispatch(const Launch& L, int m, int fmt, const Tile& t) {
  if (t.MM == 3) return L.dry ? dispatch_shared(nullptr, m, fmt, t, nullptr) : hipErrorInvalidValue;
  if (t.MM == 2) return (fmt == F_F64 || fmt == F_F32) ? launch_pair(L, fmt, t) : hipErrorInvalidValue;
  switch (fmt) {
    case F_F64: return m == 2 ? launch_f64<2>(L, t) : launch_f64<1>(L, t);
    case F_F32:
      if (t.MM) return m == 2 ? launch_mma<F_F32, 2, 2>(L, t) : launch_mma<F_F32, 1, 2>(L, t);
      return m == 2 ? launch_f32<2>(L, t) : launch_f32<1>(L, t);
    case F_BF16: return m == 2 ? launch_mma<F_BF16, 2, 2>(L, t) : launch_mma<F_BF16, 1, 2>(L, t);
    case F_F16: return m == 2 ? launch_mma<F_F16, 2, 2>(L, t) : launch_mma<F_F16, 1, 2>(L, t);
    case F_E4M3: return m == 2 ? launch_mma<F_E4M3, 2, 3>(L, t) : launch_mma<F_E4M3, 1, 3>(L, t);
    default: return hipErrorInvalidValue;
  }
}

int kernel_name(int fmt, int m, const Tile& t, char* buf, size_t cap) {
  if (!tile_supported(fmt, m, t)) return -1;
  const char* nt = t.NT ? "true" : "false";
  if (t.MM == 3 && t.NT)
    return snprintf(buf, cap, "hipBLASLt product + k_shared_contract<%d, %d, %d, %d, true>", fmt, m, t.R, t.U);
  if (t.MM == 3 && t.WK == 2) return snprintf(buf, cap, "k_shared_gemm<%d, %d, %d, %d>", fmt, m, t.R, t.U);
  if (t.MM == 3) return snprintf(buf, cap, "k_shared_contract<%d, %d, %d, %d>", fmt, m, t.R, t.U);
  if (t.MM == 2)  // the system kind and weights also select the instance: name the family and tile
    return snprintf(buf, cap, "k_contract_pair<*, %s, *, %d, %d, %d>", fmt == F_F32 ? "true" : "false", t.R, t.WR,
                    t.U);
  const char* ew = t.EW ? "true" : "false";
  if (fmt == F_F64)
    return snprintf(buf, cap, "k_contract_f64<%d, %d, %d, %d, %d, %s, %s>", m, t.R, t.WR, t.WK, t.U, nt, ew);
  if (fmt == F_F32 && !t.MM)
    return snprintf(buf, cap, "k_contract_f32<%d, 2, %d, %d, %d, %d, %s, %s>", m, t.R, t.WR, t.WK, t.U, nt, ew);
  const int T = fmt == F_E4M3 ? 3 : 2;
  return snprintf(buf, cap, "k_contract_mfma<%d, %d, %d, %d, %d, %d, %d, %s, %s>", fmt, m, T, t.R, t.WR, t.WK, t.U, nt,
                  ew);
}

bool tile_supported(int fmt, int m, const Tile& t) {
  return dispatch(Launch{nullptr, nullptr, 0, nullptr, true}, m, fmt, t) == hipSuccess;
}

hipError_t launch_contract(const Args& a, int fmt, const Tile& t, hipStream_t s) {
  return dispatch(Launch{&a, nullptr, 0, s, false}, a.m, fmt, t);
}
hipError_t launch_group_contract(const Group& g, int m, int fmt, const Tile& t, unsigned grid, hipStream_t s) {
  return dispatch(Launch{nullptr, &g, grid, s, false}, m, fmt, t);
}
hipError_t launch_persistent(const PGroup& p, int m, int fmt, const Tile& t, unsigned grid, unsigned ncounters,
                             hipStream_t s) {
  if (!tile_persistent_ok(fmt, m, t) || grid == 0) return hipErrorInvalidValue;
  // the counters: tick [ncounters] followed by comp [ncounters]
  if (p.comp != p.tick + ncounters) return hipErrorInvalidValue;
  const unsigned nz = 2 * ncounters;
  if (nz) k_zero_u32<<<(nz + 255) / 256, 256, 0, s>>>(p.tick, nz);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  Launch L{nullptr, nullptr, grid, s, false};
  L.p = &p;
  return dispatch(L, m, fmt, t);
}
bool tile_persistent_ok(int fmt, int m, const Tile& t) {
  if (t.MM > 1 || t.EW || t.WR * t.WK != 4) return false;
  PGroup p{};
  Launch L{nullptr, nullptr, 0, nullptr, true};
  L.p = &p;
  return dispatch(L, m, fmt, t) == hipSuccess;
}
hipError_t launch_group_prep(const Group& g, unsigned grid, hipStream_t s) {
  k_group_prep<<<grid, 256, 0, s>>>(g);
  return hipGetLastError();
}
hipError_t launch_group_finalize(const Group& g, unsigned grid, hipStream_t s) {
  k_group_finalize<<<grid, 256, 0, s>>>(g);
  return hipGetLastError();
}
#endif  // BS32_IN(0)

}  // namespace bs32
