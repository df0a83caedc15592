/*
 * bs32_oracle.c -- plain, slow CPU reference of the mixed-precision adaptive
 * Bogacki-Shampine 3(2) solver ("the oracle").
 *
 * TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares nothing with
 * the HIP library.
 *
 * What follows the paper (Al-Sayed Ali, Bernard, Marzorati, Rouzaud-Cornabas,
 * "Mixed-Precision in adaptive Runge-Kutta method for large ODE systems"):
 *   - general pairwise model, Sec. 2.1 eq. (1)-(2): orc_rhs (pairwise sums,
 *     never the matrix-vector rewrite);
 *   - Benchmark 1 (eq. LCO) and Benchmark 2 (eq. Kuramoto): ORC_LCO_PAPER and
 *     ORC_KURAMOTO, with the uniform weights M_ij = 1/N generalised to A_ij/N;
 *   - the BS3(2) pair, Sec. 2.2 eq. (Stage-ODE23) and Table Butcher-O23, with
 *     FSAL (the fourth stage is the next first stage);
 *   - the weighted max error, Sec. 2.2 eq. (ERROR-O23), formed from the stages;
 *   - the accept rule and failure conditions, Sec. 2.2 ("Failure conditions");
 *   - the recipes Single/Mixed1/Mixed2, Sec. 2.3 and Table MP-Distrib.
 * What the paper leaves open is filled with stated readings (the step-size
 * update, the starting step, h_max, the last-step clip, the counter thresholds):
 * each is marked "reading" at the place it is used.
 *
 * Parity pins (tests/test_oracle_*.py): tableau order conditions; the exact
 * one-step and error-estimate polynomials on y' = lambda y; observed orders 3
 * and 2; closed forms of LCO_PAPER (mode decomposition) and OSC2 (symmetric
 * eigendecomposition); uncoupled Kuramoto; the Kuramoto order-parameter
 * identity for uniform weights; the two-oscillator Adler equation; the Goodwin
 * fixed point; quantizer bit patterns; DP5(4) against an independent library
 * integrator; the BF16-pair storage (hi + rounded remainder, the conclusion's
 * extension to other formats) by exact pairs, its 2^-17 bound and its reduction
 * to BF16 on BF16 weights.  The paper recipes: the recipe table against the
 * paper's Table MP-Distrib (a transcribed fixture), the stage each table row
 * serves (one fixed-step attempt composed from single evaluations), and every
 * single-precision branch of orc_rhs_recipe (pair term, its weight, the
 * accumulation, the agent term, the gains and the eq. (CC) prefactor) by values
 * derived by hand on inputs whose every rounding is known in closed form.
 */
#include "bs32_oracle.h"
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Bogacki-Shampine 3(2), Table Butcher-O23                                  */
/* ------------------------------------------------------------------------ */
static const double BS_C[4] = {0.0, 1.0 / 2.0, 3.0 / 4.0, 1.0};
static const double BS_A[4][4] = {
    {0.0, 0.0, 0.0, 0.0},
    {1.0 / 2.0, 0.0, 0.0, 0.0},
    {0.0, 3.0 / 4.0, 0.0, 0.0},
    {2.0 / 9.0, 1.0 / 3.0, 4.0 / 9.0, 0.0},
};
static const double BS_B[4] = {2.0 / 9.0, 1.0 / 3.0, 4.0 / 9.0, 0.0};
static const double BS_BT[4] = {7.0 / 24.0, 1.0 / 4.0, 1.0 / 3.0, 1.0 / 8.0};

void orc_bs32_tableau(double c[4], double a[16], double b[4], double bt[4]) {
  for (int i = 0; i < 4; ++i) {
    c[i] = BS_C[i];
    b[i] = BS_B[i];
    bt[i] = BS_BT[i];
    for (int j = 0; j < 4; ++j) a[4 * i + j] = BS_A[i][j];
  }
}

/* Dormand-Prince 5(4) (Dormand & Prince 1980), the pair behind the paper's
   reference solver; used here only for reference solutions. */
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double DP_A[7][7] = {
    {0, 0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0},
};
static const double DP_B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
static const double DP_BT[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                                -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};

void orc_dp54_tableau(double c[7], double a[49], double b[7], double bt[7]) {
  for (int i = 0; i < 7; ++i) {
    c[i] = DP_C[i];
    b[i] = DP_B[i];
    bt[i] = DP_BT[i];
    for (int j = 0; j < 7; ++j) a[7 * i + j] = DP_A[i][j];
  }
}

/* Fehlberg 4(5) (the embedded Fehlberg pair the paper's conclusion names): six
   stages, the fourth-order solution is propagated and the fifth-order one only
   measures its error.  Published coefficients. */
static const double FE_C[6] = {0.0, 1.0 / 4.0, 3.0 / 8.0, 12.0 / 13.0, 1.0, 1.0 / 2.0};
static const double FE_A[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 4.0, 0, 0, 0, 0, 0},
    {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0, 0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0, 0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0, 0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0, 0},
};
static const double FE_B[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0, 0.0};
static const double FE_BH[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0};

void orc_rkf45_tableau(double c[6], double a[36], double b[6], double bh[6]) {
  for (int i = 0; i < 6; ++i) {
    c[i] = FE_C[i];
    b[i] = FE_B[i];
    bh[i] = FE_BH[i];
    for (int j = 0; j < 6; ++j) a[6 * i + j] = FE_A[i][j];
  }
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int orc_dim(int kind) {
  switch (kind) {
    case ORC_OSC2: return 2;
    case ORC_LCO_PAPER: return 2;
    case ORC_KURAMOTO: return 1;
    case ORC_GOODWIN3: return 3;
    case ORC_CLOCK4: return 4;
    default: return 0;
  }
}

static double weight(const orc_system* s, int64_t i, int64_t j) {
  return s->A ? s->A[i * s->n + j] : 1.0;
}
static double agent_param(const orc_system* s, int64_t i) { return s->param ? s->param[i] : 1.0; }

/* eq. (CC) constants (Sec. 2.1): k0, k2, k3, a, b, c, h = 4, epsilon; k1 per agent
   (the parameter array), theta^h = k1 / (k0 - k1) per agent (reading). */
#define CC_K0 2.0
#define CC_K2 0.144832
#define CC_K3 2.0
#define CC_A 2.0
#define CC_B 0.7
#define CC_C 0.8
#define CC_EPS 0.228249

/* agent term of eq. (CC) and the prefactor of its pair term, FP64 */
static void cc_agent(const double* x, double k1, double I0, double* F, double* pre) {
  const double th = k1 / (CC_K0 - k1);
  const double x2h = x[1] * x[1] * x[1] * x[1]; /* X_{i,2}^h, h = 4 */
  const double q = CC_K0 * th / (th + x2h);
  F[0] = q * (CC_A * x[0] * x[0] + 1.0) - k1 * x[0];
  F[1] = CC_K2 * (x[0] - x[1]);
  F[2] = x[2] * (1.0 - x[2] * x[2] / 3.0) - x[3] + I0 * (1.0 - CC_K3 * CC_K3 / (CC_K3 * CC_K3 + x[0] * x[0]));
  F[3] = CC_EPS * (x[2] + CC_B - CC_C * x[3]);
  *pre = q * CC_A; /* G_ij,1 = pre * K * arctan(X_j1 - X_i1) */
}

/* ------------------------------------------------------------------------ */
/* FP64 right-hand side: agent term F_i plus sum_j M_ij * G_ij (eq. (1)).     */
/* ------------------------------------------------------------------------ */
int orc_rhs(const orc_system* s, double t, const double* X, double* F) {
  (void)t; /* every system here is autonomous */
  const int64_t n = s->n;
  const int d = orc_dim(s->kind);
  if (d == 0 || n <= 0) return ORC_EINVAL;
  const double invN = 1.0 / (double)n;
#pragma omp parallel for schedule(static) if (n >= 64)
  for (int64_t i = 0; i < n; ++i) {
    const double* Xi = X + i * d;
    double* Fi = F + i * d;
    double sum = 0.0; /* sum_j A_ij * G_ij over the coupled component */
    switch (s->kind) {
      case ORC_OSC2: {
        /* G_ij = (0, x_j - x_i): the coupling enters the velocity equation */
        for (int64_t j = 0; j < n; ++j) sum += weight(s, i, j) * (X[j * 2] - Xi[0]);
        double w = agent_param(s, i);
        Fi[0] = Xi[1];
        Fi[1] = -w * w * Xi[0] + invN * sum;
        break;
      }
      case ORC_LCO_PAPER: {
        /* eq. (LCO): F_i = (X_i2, -X_i1), G_ij = (X_j1 - X_i1, 0), M_ij = (1/N, 0) */
        for (int64_t j = 0; j < n; ++j) sum += weight(s, i, j) * (X[j * 2] - Xi[0]);
        Fi[0] = Xi[1] + invN * sum;
        Fi[1] = -Xi[0];
        break;
      }
      case ORC_KURAMOTO: {
        /* eq. (Kuramoto): F_i = omega_i, G_ij = K sin(X_j - X_i), M_ij = 1/N */
        for (int64_t j = 0; j < n; ++j) sum += weight(s, i, j) * sin(X[j] - Xi[0]);
        Fi[0] = agent_param(s, i) + s->gain * invN * sum;
        break;
      }
      case ORC_GOODWIN3: {
        /* x' = 1/(1+z^10) - b x + (kappa/N) sum_j C_ij (x_j - x_i); y' = x - b y; z' = y - b z */
        for (int64_t j = 0; j < n; ++j) sum += weight(s, i, j) * (X[j * 3] - Xi[0]);
        double b = agent_param(s, i);
        Fi[0] = 1.0 / (1.0 + pow(Xi[2], 10.0)) - b * Xi[0] + s->gain * invN * sum;
        Fi[1] = Xi[0] - b * Xi[1];
        Fi[2] = Xi[1] - b * Xi[2];
        break;
      }
      case ORC_CLOCK4: {
        /* eq. (CC): G_ij = (k0 th a / (th + X_i2^h) K arctan(X_j1 - X_i1), 0, 0, 0), M_ij = (1/N, 0, 0, 0) */
        double pre;
        cc_agent(Xi, agent_param(s, i), s->stimulus, Fi, &pre);
        for (int64_t j = 0; j < n; ++j) sum += weight(s, i, j) * (pre * s->gain * atan(X[j * 4] - Xi[0]));
        Fi[0] += invN * sum;
        break;
      }
    }
  }
  return ORC_OK;
}

int orc_rhs_rows(const orc_system* s, const int64_t* rows, int64_t nrows, const double* Arows, double t,
                 const double* X, double* F_rows) {
  const int64_t n = s->n;
  const int d = orc_dim(s->kind);
  if (d == 0 || n <= 0) return ORC_EINVAL;
  for (int64_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= n) return ORC_EINVAL;
  /* a one-row system per listed agent: same pairwise sums as orc_rhs */
#pragma omp parallel for schedule(static) if (nrows >= 8)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    const double* Xi = X + i * d;
    double* Fi = F_rows + r * d;
    const double* Ai = Arows ? Arows + r * n : NULL;
    const double invN = 1.0 / (double)n;
    double sum = 0.0;
    double pre = 0.0;
    if (s->kind == ORC_CLOCK4) cc_agent(Xi, agent_param(s, i), s->stimulus, Fi, &pre);
    for (int64_t j = 0; j < n; ++j) {
      double w = Ai ? Ai[j] : 1.0;
      if (s->kind == ORC_KURAMOTO) sum += w * sin(X[j] - Xi[0]);
      else if (s->kind == ORC_CLOCK4) sum += w * (pre * s->gain * atan(X[j * 4] - Xi[0]));
      else sum += w * (X[j * d] - Xi[0]);
    }
    double p = agent_param(s, i);
    switch (s->kind) {
      case ORC_CLOCK4: Fi[0] += invN * sum; break;
      case ORC_OSC2: Fi[0] = Xi[1]; Fi[1] = -p * p * Xi[0] + invN * sum; break;
      case ORC_LCO_PAPER: Fi[0] = Xi[1] + invN * sum; Fi[1] = -Xi[0]; break;
      case ORC_KURAMOTO: Fi[0] = p + s->gain * invN * sum; break;
      case ORC_GOODWIN3:
        Fi[0] = 1.0 / (1.0 + pow(Xi[2], 10.0)) - p * Xi[0] + s->gain * invN * sum;
        Fi[1] = Xi[0] - p * Xi[1];
        Fi[2] = Xi[1] - p * Xi[2];
        break;
    }
  }
  (void)t;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Number formats: round-to-nearest-even straight from FP64.                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  int p;        /* significand bits including the implicit one */
  int emin;     /* exponent of the smallest normal */
  int ebits;    /* exponent field width */
  int bias;
  double maxf;  /* largest finite */
  int satur;    /* 1: values beyond maxf become maxf (OCP "satfinite") */
} fmt_desc;

static fmt_desc fmt_of(int fmt) {
  fmt_desc f;
  switch (fmt) {
    case ORC_FMT_F32: f.p = 24; f.emin = -126; f.ebits = 8; f.bias = 127; f.maxf = FLT_MAX; f.satur = 0; break;
    case ORC_FMT_BF16: f.p = 8; f.emin = -126; f.ebits = 8; f.bias = 127; f.maxf = ldexp(255.0, 120); f.satur = 0; break;
    case ORC_FMT_F16: f.p = 11; f.emin = -14; f.ebits = 5; f.bias = 15; f.maxf = 65504.0; f.satur = 0; break;
    case ORC_FMT_E4M3: f.p = 4; f.emin = -6; f.ebits = 4; f.bias = 7; f.maxf = 448.0; f.satur = 1; break;
    default: f.p = 53; f.emin = -1022; f.ebits = 11; f.bias = 1023; f.maxf = DBL_MAX; f.satur = 0; break;
  }
  return f;
}

double orc_round_fmt(double x, int fmt) {
  if (fmt == ORC_FMT_F64) return x;
  if (fmt == ORC_FMT_BF16X2) { /* the stored pair's value: hi + round(x - hi), exact in FP64 */
    const double hi = orc_round_fmt(x, ORC_FMT_BF16);
    if (!isfinite(hi)) return hi;
    return hi + orc_round_fmt(x - hi, ORC_FMT_BF16);
  }
  fmt_desc f = fmt_of(fmt);
  if (isnan(x) || x == 0.0) return x;
  double a = fabs(x);
  if (isinf(a)) return f.satur ? copysign(f.maxf, x) : x;
  int e;
  frexp(a, &e);          /* a = m * 2^e with m in [0.5, 1): leading bit has exponent e-1 */
  int lead = e - 1;
  if (lead < f.emin) lead = f.emin;    /* subnormal range: fixed quantum */
  int q = lead - (f.p - 1);            /* exponent of one unit in the last place */
  double r = nearbyint(ldexp(a, -q));  /* default rounding mode: to nearest, ties to even */
  double y = ldexp(r, q);
  if (y > f.maxf) y = f.satur ? f.maxf : INFINITY;
  return copysign(y, x);
}

uint32_t orc_encode_fmt(double x, int fmt) {
  fmt_desc f = fmt_of(fmt);
  int nbits = f.ebits + f.p; /* sign + exponent + (p-1) fraction bits */
  uint32_t sign = signbit(x) ? (1u << (nbits - 1)) : 0u;
  double y = orc_round_fmt(x, fmt);
  uint32_t emask = (1u << f.ebits) - 1u;
  if (isnan(y)) {
    if (fmt == ORC_FMT_E4M3) return sign | 0x7fu; /* e4m3fn has only S.1111.111 as NaN */
    return sign | (emask << (f.p - 1)) | (1u << (f.p - 2));
  }
  double a = fabs(y);
  if (isinf(a)) return sign | (emask << (f.p - 1));
  if (a == 0.0) return sign;
  int e;
  frexp(a, &e);
  int lead = e - 1;
  if (lead < f.emin) { /* subnormal: exponent field 0, fraction = a / 2^(emin-(p-1)) */
    uint32_t frac = (uint32_t)ldexp(a, -(f.emin - (f.p - 1)));
    return sign | frac;
  }
  uint32_t bexp = (uint32_t)(lead + f.bias);
  uint32_t frac = (uint32_t)(ldexp(a, -(lead - (f.p - 1))) - ldexp(1.0, f.p - 1));
  return sign | (bexp << (f.p - 1)) | frac;
}

double orc_decode_fmt(uint32_t bits, int fmt) {
  fmt_desc f = fmt_of(fmt);
  int nbits = f.ebits + f.p;
  int s = (bits >> (nbits - 1)) & 1u;
  uint32_t emask = (1u << f.ebits) - 1u;
  uint32_t be = (bits >> (f.p - 1)) & emask;
  uint32_t fr = bits & ((1u << (f.p - 1)) - 1u);
  double v;
  if (fmt == ORC_FMT_E4M3 && be == emask && fr == 7u) v = NAN;
  else if (fmt != ORC_FMT_E4M3 && be == emask) v = fr ? NAN : INFINITY;
  else if (be == 0) v = ldexp((double)fr, f.emin - (f.p - 1));
  else v = ldexp((double)(fr + (1u << (f.p - 1))), (int)be - f.bias - (f.p - 1));
  return s ? -v : v;
}

/* reading: per-tensor scale s = 2^ceil(log2(max|A| / m)), m = 448 for e4m3 and
   1 otherwise, so that A/s is exact and only the format rounding remains. */
double orc_matrix_scale(const double* A, int64_t count, int fmt) {
  if (fmt == ORC_FMT_F64) return 1.0;
  double mx = 0.0;
  for (int64_t k = 0; k < count; ++k) mx = fmax(mx, fabs(A[k]));
  if (mx == 0.0) return 1.0;
  double fm = (fmt == ORC_FMT_E4M3) ? 448.0 : 1.0;
  return ldexp(1.0, (int)ceil(log2(mx / fm)));
}

void orc_split(double v, int fmt, int terms, int shift, double* out) {
  double r = v;
  for (int k = 0; k < terms; ++k) {
    double q = orc_round_fmt(ldexp(r, k * shift), fmt);
    out[k] = ldexp(q, -k * shift);
    r = r - out[k];
  }
}

/* mode defaults for the split of the vector operand (reading of the
   "compensated" reduced-precision contraction) */
static void split_defaults(int fmt, int* sfmt, int* terms, int* shift) {
  switch (fmt) {
    case ORC_FMT_F32: *sfmt = ORC_FMT_F32; *terms = 2; *shift = 24; break;
    case ORC_FMT_BF16:
    case ORC_FMT_BF16X2: *sfmt = ORC_FMT_BF16; *terms = 2; *shift = 8; break;
    case ORC_FMT_F16: *sfmt = ORC_FMT_F16; *terms = 2; *shift = 11; break;
    case ORC_FMT_E4M3: *sfmt = ORC_FMT_E4M3; *terms = 3; *shift = 4; break;
    default: *sfmt = ORC_FMT_F64; *terms = 1; *shift = 0; break;
  }
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision contraction mode.                                       */
/* The coupling is written as a weighted sum over the coupled component:     */
/*   diffusive systems:  sum_j Ahat_ij (x_j - x_i) = sum_j Ahat_ij xt_j - x_i sum_j Ahat_ij */
/*   Kuramoto:  sum_j Ahat_ij sin(th_j - th_i)                               */
/*            = cos th_i sum_j Ahat_ij st_j - sin th_i sum_j Ahat_ij ct_j     */
/* with xt, st, ct the split reconstructions of x, sin th, cos th.           */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_system* s;
  double* Ahat;  /* dequantized weights, n*n */
  double* rsum;  /* row sums of Ahat */
  int sfmt, terms, shift;
} lowp_ctx;

static int lowp_init(lowp_ctx* c, const orc_system* s, int fmt, int sfmt, int terms, int shift) {
  const int64_t n = s->n;
  c->Ahat = NULL;
  c->rsum = NULL;
  if (s->kind == ORC_CLOCK4) return ORC_EINVAL; /* the arctan pair term has no matrix-vector form */
  c->s = s;
  int dfm, dt, dsh;
  split_defaults(fmt, &dfm, &dt, &dsh);
  c->sfmt = sfmt >= 0 ? sfmt : dfm;
  c->terms = terms > 0 ? terms : dt;
  c->shift = shift > 0 ? shift : dsh;
  c->Ahat = (double*)malloc(sizeof(double) * (size_t)(n * n));
  c->rsum = (double*)malloc(sizeof(double) * (size_t)n);
  if (!c->Ahat || !c->rsum) return ORC_EINVAL;
  if (s->A) {
    double sc = orc_matrix_scale(s->A, n * n, fmt);
    for (int64_t k = 0; k < n * n; ++k) c->Ahat[k] = sc * orc_round_fmt(s->A[k] / sc, fmt);
  } else {
    for (int64_t k = 0; k < n * n; ++k) c->Ahat[k] = 1.0;
  }
  for (int64_t i = 0; i < n; ++i) {
    double r = 0.0;
    for (int64_t j = 0; j < n; ++j) r += c->Ahat[i * n + j];
    c->rsum[i] = r;
  }
  return ORC_OK;
}
static void lowp_free(lowp_ctx* c) {
  free(c->Ahat);
  free(c->rsum);
}

static double split_sum(double v, const lowp_ctx* c) {
  double parts[8];
  orc_split(v, c->sfmt, c->terms, c->shift, parts);
  double r = 0.0;
  for (int k = 0; k < c->terms; ++k) r += parts[k];
  return r;
}

/* split reconstructions of the vector operand: vt[2j] = x_j (or sin th_j),
   vt[2j+1] = cos th_j (Kuramoto) */
static void lowp_operand(const lowp_ctx* c, const double* X, double* vt) {
  const orc_system* s = c->s;
  const int d = orc_dim(s->kind);
  for (int64_t j = 0; j < s->n; ++j) {
    if (s->kind == ORC_KURAMOTO) {
      vt[2 * j] = split_sum(sin(X[j]), c);
      vt[2 * j + 1] = split_sum(cos(X[j]), c);
    } else {
      vt[2 * j] = split_sum(X[j * d], c);
      vt[2 * j + 1] = 0.0;
    }
  }
}

/* agent i from its row of stored weights Ai, their sum rs and the operand vt */
static void lowp_row(const orc_system* s, int64_t i, const double* Ai, double rs, const double* vt, const double* X,
                     double* Fi) {
  const int d = orc_dim(s->kind);
  const double invN = 1.0 / (double)s->n;
  const double* Xi = X + i * d;
  double p0 = 0.0, p1 = 0.0;
  for (int64_t j = 0; j < s->n; ++j) {
    p0 += Ai[j] * vt[2 * j];
    p1 += Ai[j] * vt[2 * j + 1];
  }
  switch (s->kind) {
    case ORC_OSC2: {
      double w = agent_param(s, i);
      Fi[0] = Xi[1];
      Fi[1] = -w * w * Xi[0] + invN * (p0 - Xi[0] * rs);
      break;
    }
    case ORC_LCO_PAPER:
      Fi[0] = Xi[1] + invN * (p0 - Xi[0] * rs);
      Fi[1] = -Xi[0];
      break;
    case ORC_KURAMOTO:
      Fi[0] = agent_param(s, i) + s->gain * invN * (cos(Xi[0]) * p0 - sin(Xi[0]) * p1);
      break;
    case ORC_GOODWIN3: {
      double b = agent_param(s, i);
      Fi[0] = 1.0 / (1.0 + pow(Xi[2], 10.0)) - b * Xi[0] + s->gain * invN * (p0 - Xi[0] * rs);
      Fi[1] = Xi[0] - b * Xi[1];
      Fi[2] = Xi[1] - b * Xi[2];
      break;
    }
  }
}

static int lowp_rhs(const lowp_ctx* c, const double* X, double* F) {
  const orc_system* s = c->s;
  const int64_t n = s->n;
  const int d = orc_dim(s->kind);
  double* vt = (double*)malloc(sizeof(double) * (size_t)(2 * n));
  if (!vt) return ORC_EINVAL;
  lowp_operand(c, X, vt);
#pragma omp parallel for schedule(static) if (n >= 64)
  for (int64_t i = 0; i < n; ++i) lowp_row(s, i, c->Ahat + i * n, c->rsum[i], vt, X, F + i * d);
  free(vt);
  return ORC_OK;
}

int orc_rhs_lowp(const orc_system* s, int fmt, int sfmt, int terms, int shift, double t, const double* X,
                 double* F) {
  (void)t;
  if (orc_dim(s->kind) == 0 || s->n <= 0) return ORC_EINVAL;
  lowp_ctx c;
  int rc = lowp_init(&c, s, fmt, sfmt, terms, shift);
  if (rc == ORC_OK) rc = lowp_rhs(&c, X, F);
  lowp_free(&c);
  return rc;
}

/* The same definition for a subset of rows: the stored weights of the listed rows
   are formed from their FP64 values with the per-tensor scale of the whole matrix
   (passed in: it depends only on max|A|), everything else as in orc_rhs_lowp. */
int orc_rhs_lowp_rows(const orc_system* s, int fmt, double scale, const int64_t* rows, int64_t nrows,
                      const double* Arows, double t, const double* X, double* F_rows) {
  (void)t;
  const int64_t n = s->n;
  const int d = orc_dim(s->kind);
  if (d == 0 || n <= 0 || s->kind == ORC_CLOCK4 || !(scale > 0.0)) return ORC_EINVAL;
  for (int64_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= n) return ORC_EINVAL;
  lowp_ctx c;
  c.s = s;
  c.Ahat = NULL;
  c.rsum = NULL;
  int dfm, dt, dsh;
  split_defaults(fmt, &dfm, &dt, &dsh);
  c.sfmt = dfm;
  c.terms = dt;
  c.shift = dsh;
  double* vt = (double*)malloc(sizeof(double) * (size_t)(2 * n));
  double* Ahat = (double*)malloc(sizeof(double) * (size_t)(nrows * n));
  if (!vt || !Ahat) {
    free(vt);
    free(Ahat);
    return ORC_EINVAL;
  }
  for (int64_t k = 0; k < nrows * n; ++k)
    Ahat[k] = Arows ? scale * orc_round_fmt(Arows[k] / scale, fmt) : 1.0;
  lowp_operand(&c, X, vt);
#pragma omp parallel for schedule(static) if (nrows >= 8)
  for (int64_t r = 0; r < nrows; ++r) {
    double rs = 0.0;
    for (int64_t j = 0; j < n; ++j) rs += Ahat[r * n + j];
    lowp_row(s, rows[r], Ahat + r * n, rs, vt, X, F_rows + r * d);
  }
  free(vt);
  free(Ahat);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Paper recipes (Sec. 2.3, Table MP-Distrib): one stage evaluated with the  */
/* agent term in precision pF, the pair terms G_ij (and their weights) in pG  */
/* and their accumulation in pS; single-precision pair terms are cast to      */
/* double before a double accumulation.                                       */
/* ------------------------------------------------------------------------ */
int orc_rhs_recipe(const orc_system* s, int pF, int pS, int pG, double t, const double* X, double* F) {
  (void)t;
  if (!(pF | pS | pG)) return orc_rhs(s, t, X, F);
  const int64_t n = s->n;
  const int d = orc_dim(s->kind);
  if (d == 0 || n <= 0) return ORC_EINVAL;
#pragma omp parallel for schedule(static) if (n >= 64)
  for (int64_t i = 0; i < n; ++i) {
    const double* Xi = X + i * d;
    double* Fi = F + i * d;
    /* interaction sum: sum_j M_ij G_ij with M_ij = A_ij / N */
    double sumd = 0.0;
    float sumf = 0.0f;
    const float invNf = 1.0f / (float)n;
    const double invN = 1.0 / (double)n;
    /* eq. (CC): the pair term's prefactor k0 th a / (th + X_i2^h) in the G precision */
    double pre_d = 0.0;
    float pre_f = 0.0f;
    if (s->kind == ORC_CLOCK4) {
      double Ftmp[4];
      cc_agent(Xi, agent_param(s, i), s->stimulus, Ftmp, &pre_d);
      const float k1f = (float)agent_param(s, i), x2f = (float)Xi[1];
      const float thf = k1f / ((float)CC_K0 - k1f);
      pre_f = (float)CC_K0 * thf / (thf + x2f * x2f * x2f * x2f) * (float)CC_A;
    }
    for (int64_t j = 0; j < n; ++j) {
      double term;
      if (pG) {
        float g;
        if (s->kind == ORC_KURAMOTO) g = (float)s->gain * sinf((float)X[j] - (float)Xi[0]);
        else if (s->kind == ORC_CLOCK4) g = pre_f * (float)s->gain * atanf((float)X[j * d] - (float)Xi[0]);
        else g = (float)X[j * d] - (float)Xi[0];
        float m = (float)weight(s, i, j) * invNf;
        term = (double)(m * g);
      } else {
        double g;
        if (s->kind == ORC_KURAMOTO) g = s->gain * sin(X[j] - Xi[0]);
        else if (s->kind == ORC_CLOCK4) g = pre_d * s->gain * atan(X[j * d] - Xi[0]);
        else g = X[j * d] - Xi[0];
        term = (weight(s, i, j) * invN) * g;
      }
      if (pS) sumf = sumf + (float)term;
      else sumd += term;
    }
    double inter = pS ? (double)sumf : sumd;
    if (s->kind == ORC_GOODWIN3) inter = pG ? (double)((float)s->gain * (float)inter) : s->gain * inter;
    if (pF) {
      float xf[4] = {(float)Xi[0], d > 1 ? (float)Xi[1] : 0.f, d > 2 ? (float)Xi[2] : 0.f, d > 3 ? (float)Xi[3] : 0.f};
      float intf = (float)inter;
      float pf = (float)agent_param(s, i);
      switch (s->kind) {
        case ORC_CLOCK4: {
          const float thf = pf / ((float)CC_K0 - pf);
          const float q = (float)CC_K0 * thf / (thf + xf[1] * xf[1] * xf[1] * xf[1]);
          const float k3s = (float)CC_K3 * (float)CC_K3;
          Fi[0] = (q * ((float)CC_A * xf[0] * xf[0] + 1.0f) - pf * xf[0]) + intf;
          Fi[1] = (float)CC_K2 * (xf[0] - xf[1]);
          Fi[2] = xf[2] * (1.0f - xf[2] * xf[2] / 3.0f) - xf[3] + (float)s->stimulus * (1.0f - k3s / (k3s + xf[0] * xf[0]));
          Fi[3] = (float)CC_EPS * (xf[2] + (float)CC_B - (float)CC_C * xf[3]);
          break;
        }
        case ORC_OSC2: Fi[0] = xf[1]; Fi[1] = (-pf * pf * xf[0]) + intf; break;
        case ORC_LCO_PAPER: Fi[0] = xf[1] + intf; Fi[1] = -xf[0]; break;
        case ORC_KURAMOTO: Fi[0] = pf + intf; break;
        case ORC_GOODWIN3:
          Fi[0] = (1.0f / (1.0f + powf(xf[2], 10.0f)) - pf * xf[0]) + intf;
          Fi[1] = xf[0] - pf * xf[1];
          Fi[2] = xf[1] - pf * xf[2];
          break;
      }
    } else {
      double p = agent_param(s, i);
      switch (s->kind) {
        case ORC_CLOCK4: {
          double pre;
          cc_agent(Xi, p, s->stimulus, Fi, &pre);
          Fi[0] += inter;
          break;
        }
        case ORC_OSC2: Fi[0] = Xi[1]; Fi[1] = -p * p * Xi[0] + inter; break;
        case ORC_LCO_PAPER: Fi[0] = Xi[1] + inter; Fi[1] = -Xi[0]; break;
        case ORC_KURAMOTO: Fi[0] = p + inter; break;
        case ORC_GOODWIN3:
          Fi[0] = 1.0 / (1.0 + pow(Xi[2], 10.0)) - p * Xi[0] + inter;
          Fi[1] = Xi[0] - p * Xi[1];
          Fi[2] = Xi[1] - p * Xi[2];
          break;
      }
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Stage evaluator used by the integrator: picks the RHS of the mode.        */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_system* s;
  int mode;
  lowp_ctx lp;
  int has_lp;
} evaluator;

/* recipe table (Table MP-Distrib): rows k2, k3, k4; columns F, Sigma, G; 1 = single */
static const int RECIPE[3][3][3] = {
    /* Single */ {{1, 1, 1}, {1, 1, 1}, {1, 1, 1}},
    /* Mixed1 */ {{1, 1, 1}, {1, 1, 1}, {0, 0, 1}},
    /* Mixed2 */ {{0, 0, 1}, {0, 0, 1}, {0, 0, 1}},
};

void orc_recipe_table(int out[27]) {
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k)
      for (int q = 0; q < 3; ++q) out[9 * r + 3 * k + q] = RECIPE[r][k][q];
}

/* stage: 2, 3, 4 (the first stage is always the FSAL copy of stage 4, and the
   very first one uses the stage-4 recipe: reading) */
static int eval_stage(evaluator* e, int stage, double t, const double* Y, double* K) {
  switch (e->mode) {
    case ORC_PREC_FP64: return orc_rhs(e->s, t, Y, K);
    case ORC_PREC_RHS_FP32:
    case ORC_PREC_RHS_BF16:
    case ORC_PREC_RHS_FP16:
    case ORC_PREC_RHS_FP8:
    case ORC_PREC_RHS_BF16X2: return lowp_rhs(&e->lp, Y, K);
    default: {
      const int r = e->mode - ORC_PREC_PAPER_SINGLE;
      const int* p = RECIPE[r][stage - 2];
      return orc_rhs_recipe(e->s, p[0], p[1], p[2], t, Y, K);
    }
  }
}

static int mode_fmt(int mode) {
  switch (mode) {
    case ORC_PREC_RHS_FP32: return ORC_FMT_F32;
    case ORC_PREC_RHS_BF16: return ORC_FMT_BF16;
    case ORC_PREC_RHS_FP16: return ORC_FMT_F16;
    case ORC_PREC_RHS_FP8: return ORC_FMT_E4M3;
    case ORC_PREC_RHS_BF16X2: return ORC_FMT_BF16X2;
    default: return ORC_FMT_F64;
  }
}

/* the paper's weighted max norm, eq. (ERROR-O23):
   E = max_k |err_k| / max(|X^n_k|, |X^{n+1}_k|, Ab/Rel) */
static double weighted_max(const double* err, const double* X, const double* Xn, int64_t m, double rtol,
                           double atol) {
  double E = 0.0;
  const double floor_w = atol / rtol;
  for (int64_t k = 0; k < m; ++k) {
    double W = fmax(fmax(fabs(X[k]), fabs(Xn[k])), floor_w);
    double v = fabs(err[k]) / W;
    if (isnan(v)) return v; /* a NaN anywhere makes the estimate NaN */
    if (v > E) E = v;
  }
  return E;
}

/* Single keeps its solution in single precision (Sec. 2.3): round a stored vector */
static void store_single(double* v, int64_t m) {
  for (int64_t k = 0; k < m; ++k) v[k] = (double)(float)v[k];
}

int orc_bs32_attempt(const orc_system* s, double t, double h, const double* X, const double* K1, double rtol,
                     double atol, double* Xn, double* K4, double* err) {
  const int64_t m = (int64_t)orc_dim(s->kind) * s->n;
  double* K2 = (double*)malloc(sizeof(double) * (size_t)m);
  double* K3 = (double*)malloc(sizeof(double) * (size_t)m);
  double* Y = (double*)malloc(sizeof(double) * (size_t)m);
  double* ev = (double*)malloc(sizeof(double) * (size_t)m);
  if (!K2 || !K3 || !Y || !ev) return ORC_EINVAL;
  for (int64_t k = 0; k < m; ++k) Y[k] = X[k] + h * (BS_A[1][0] * K1[k]);
  orc_rhs(s, t + BS_C[1] * h, Y, K2);
  for (int64_t k = 0; k < m; ++k) Y[k] = X[k] + h * (BS_A[2][0] * K1[k] + BS_A[2][1] * K2[k]);
  orc_rhs(s, t + BS_C[2] * h, Y, K3);
  for (int64_t k = 0; k < m; ++k) Xn[k] = X[k] + h * (BS_B[0] * K1[k] + BS_B[1] * K2[k] + BS_B[2] * K3[k]);
  orc_rhs(s, t + h, Xn, K4);
  for (int64_t k = 0; k < m; ++k)
    ev[k] = h * ((BS_B[0] - BS_BT[0]) * K1[k] + (BS_B[1] - BS_BT[1]) * K2[k] + (BS_B[2] - BS_BT[2]) * K3[k] +
                 (BS_B[3] - BS_BT[3]) * K4[k]);
  *err = weighted_max(ev, X, Xn, m, rtol, atol);
  free(K2);
  free(K3);
  free(Y);
  free(ev);
  return ORC_OK;
}

/* reading of the unspecified step-size correction: elementary controller for an
   error estimate of order q+1 = 3 (the embedded solution is second order). */
static double control(double h, double E, double rtol, int accepted, int last_rejected, double safety,
                      double facmin, double facmax) {
  double fac = (E > 0.0) ? safety * cbrt(rtol / E) : facmax;
  if (accepted) {
    double hi = last_rejected ? 1.0 : facmax;
    return h * fmin(hi, fmax(facmin, fac));
  }
  double lo = fmax(facmin, fac);
  if (last_rejected) lo = fmin(lo, 0.5);
  return h * lo;
}

/* reading of the unspecified starting step: Hairer-Norsett-Wanner (Sec. II.4)
   with the paper's max norm and weights atol + rtol |y0|, order p. */
static double start_step(evaluator* e, int p, double t0, const double* y0, const double* f0, int64_t m,
                         double rtol, double atol, double h_max, int64_t* nfev) {
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  for (int64_t k = 0; k < m; ++k) {
    double sc = atol + rtol * fabs(y0[k]);
    d0 = fmax(d0, fabs(y0[k]) / sc);
    d1 = fmax(d1, fabs(f0[k]) / sc);
  }
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
  h0 = fmin(h0, h_max);
  double* y1 = (double*)malloc(sizeof(double) * (size_t)m);
  double* f1 = (double*)malloc(sizeof(double) * (size_t)m);
  for (int64_t k = 0; k < m; ++k) y1[k] = y0[k] + h0 * f0[k];
  eval_stage(e, 4, t0 + h0, y1, f1);
  *nfev += 1;
  for (int64_t k = 0; k < m; ++k) {
    double sc = atol + rtol * fabs(y0[k]);
    d2 = fmax(d2, fabs(f1[k] - f0[k]) / sc);
  }
  d2 /= h0;
  free(y1);
  free(f1);
  double dm = fmax(d1, d2);
  double h1 = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 1.0 / (double)(p + 1));
  return fmin(fmin(100.0 * h0, h1), h_max);
}

/* learned proposer network, plain FP64 (parameter order as in the header) */
double orc_mlp_forward(const double* w, const double* f) {
  const int I = ORC_MLP_IN, H = ORC_MLP_HID;
  const double* W1 = w;
  const double* b1 = W1 + H * I;
  const double* W2 = b1 + H;
  const double* b2 = W2 + H * H;
  const double* w3 = b2 + H;
  const double b3 = w3[H];
  const double* mu = w3 + H + 1;
  const double* inv_sd = mu + I;
  double x[ORC_MLP_IN], h1[ORC_MLP_HID], h2[ORC_MLP_HID];
  for (int k = 0; k < I; ++k) x[k] = (f[k] - mu[k]) * inv_sd[k];
  for (int j = 0; j < H; ++j) {
    double z = b1[j];
    for (int k = 0; k < I; ++k) z += W1[j * I + k] * x[k];
    h1[j] = tanh(z);
  }
  for (int j = 0; j < H; ++j) {
    double z = b2[j];
    for (int k = 0; k < H; ++k) z += W2[j * H + k] * h1[k];
    h2[j] = tanh(z);
  }
  double y = b3;
  for (int j = 0; j < H; ++j) y += w3[j] * h2[j];
  return y;
}

static void fill_defaults(const orc_options* o, double t0, double t1, double* h_max, int64_t* i_max,
                          double* safety, double* facmin, double* facmax) {
  *h_max = (o->h_max > 0.0) ? o->h_max : 0.1 * fabs(t1 - t0);
  *i_max = (o->i_max > 0) ? o->i_max : 100000;
  *safety = (o->safety > 0.0) ? o->safety : 0.9;
  *facmin = (o->facmin > 0.0) ? o->facmin : 0.2;
  *facmax = (o->facmax > 0.0) ? o->facmax : 5.0;
}

int orc_bs32_solve(const orc_system* s, const orc_options* o, int mode, const double* y0, double t0, double t1,
                   double* y_out, orc_stats* st, orc_trace_rec* trace, int64_t trace_cap, int64_t* trace_len) {
  const int d = orc_dim(s->kind);
  if (d == 0 || s->n <= 0 || !(o->rtol > 0.0) || !(o->atol >= 0.0) || !(t1 >= t0) || mode < 0 || mode > 8)
    return ORC_EINVAL;
  if (o->fixed_step && !(o->h0 > 0.0)) return ORC_EINVAL;
  const int64_t m = (int64_t)d * s->n;
  memset(st, 0, sizeof(*st));
  if (trace_len) *trace_len = 0;
  if (t1 == t0) {
    memmove(y_out, y0, sizeof(double) * (size_t)m);
    st->t_reached = t0;
    st->status = ORC_OK;
    return ORC_OK;
  }
  double h_max, safety, facmin, facmax;
  int64_t i_max;
  fill_defaults(o, t0, t1, &h_max, &i_max, &safety, &facmin, &facmax);
  const int single = (mode == ORC_PREC_PAPER_SINGLE);
  /* Sec. 2.2: h must stay above h_min = 100 eps_m of the format holding the step (reading) */
  const double h_min = 100.0 * (single ? (double)FLT_EPSILON : DBL_EPSILON);

  evaluator ev;
  ev.s = s;
  ev.mode = mode;
  ev.has_lp = 0;
  if ((mode >= ORC_PREC_RHS_FP32 && mode <= ORC_PREC_RHS_FP8) || mode == ORC_PREC_RHS_BF16X2) {
    if (lowp_init(&ev.lp, s, mode_fmt(mode), o->split_fmt, o->split_terms, o->split_shift) != ORC_OK)
      return ORC_EINVAL;
    ev.has_lp = 1;
  }

  double* X = (double*)malloc(sizeof(double) * (size_t)m);
  double* Xn = (double*)malloc(sizeof(double) * (size_t)m);
  double* Y = (double*)malloc(sizeof(double) * (size_t)m);
  double* K1 = (double*)malloc(sizeof(double) * (size_t)m);
  double* K2 = (double*)malloc(sizeof(double) * (size_t)m);
  double* K3 = (double*)malloc(sizeof(double) * (size_t)m);
  double* K4 = (double*)malloc(sizeof(double) * (size_t)m);
  double* E = (double*)malloc(sizeof(double) * (size_t)m);
  memcpy(X, y0, sizeof(double) * (size_t)m);
  if (single) store_single(X, m);

  double t = t0;
  eval_stage(&ev, 4, t, X, K1);
  st->n_fev = 1;
  double h;
  if (o->h0 > 0.0) h = o->h0;
  else h = start_step(&ev, 3, t0, X, K1, m, o->rtol, o->atol, h_max, &st->n_fev);
  st->h_min_seen = INFINITY;
  int last_rejected = 0;
  int status = ORC_OK;
  const double snap = 4.0 * DBL_EPSILON * fabs(t1);
  double hist_h[4] = {0}, hist_e[4] = {0}; /* learned proposer history, most recent first */
  int64_t nhist = 0;
  int proposer = 0; /* 1: the current h came from the learned proposer */

  while (t < t1) {
    const double ha = fmin(h, t1 - t); /* reading: clip the last step onto t1 */
    /* stage 2 and 3 inputs and the third-order solution: always in FP64 (Sec. 2.3) */
    for (int64_t k = 0; k < m; ++k) Y[k] = X[k] + ha * (BS_A[1][0] * K1[k]);
    if (single) store_single(Y, m);
    eval_stage(&ev, 2, t + BS_C[1] * ha, Y, K2);
    for (int64_t k = 0; k < m; ++k) Y[k] = X[k] + ha * (BS_A[2][0] * K1[k] + BS_A[2][1] * K2[k]);
    if (single) store_single(Y, m);
    eval_stage(&ev, 3, t + BS_C[2] * ha, Y, K3);
    for (int64_t k = 0; k < m; ++k)
      Xn[k] = X[k] + ha * (BS_B[0] * K1[k] + BS_B[1] * K2[k] + BS_B[2] * K3[k]);
    if (single) store_single(Xn, m);
    eval_stage(&ev, 4, t + ha, Xn, K4);
    st->n_fev += 3;
    /* the difference of the two solutions, formed from the stages (Sec. 2.2) */
    for (int64_t k = 0; k < m; ++k)
      E[k] = ha * ((BS_B[0] - BS_BT[0]) * K1[k] + (BS_B[1] - BS_BT[1]) * K2[k] + (BS_B[2] - BS_BT[2]) * K3[k] +
                   (BS_B[3] - BS_BT[3]) * K4[k]);
    double err = weighted_max(E, X, Xn, m, o->rtol, o->atol);
    st->err_last = err;
    double fnorm = 0.0; /* weighted size of f(t_n, X^n), a proposer feature */
    for (int64_t k = 0; k < m; ++k) {
      const double v = fabs(K1[k]) / fmax(fabs(X[k]), o->atol / o->rtol);
      if (isnan(v) || isnan(fnorm)) fnorm = NAN;
      else if (v > fnorm) fnorm = v;
    }
    int accepted;
    if (o->fixed_step) accepted = 1;
    else {
      if (!isfinite(err)) {
        status = ORC_NONFINITE;
        if (trace && trace_len && *trace_len < trace_cap) {
          orc_trace_rec r = {t, ha, err, fnorm, 0, proposer};
          trace[(*trace_len)++] = r;
        }
        st->n_reject++;
        break;
      }
      accepted = err < o->rtol; /* Sec. 2.2: accept iff the estimate is smaller than Rel */
    }
    if (trace && trace_len && *trace_len < trace_cap) {
      orc_trace_rec r = {t, ha, err, fnorm, accepted, proposer};
      trace[(*trace_len)++] = r;
    }
    double hn;
    if (accepted) {
      st->n_accept++;
      t = (t + ha >= t1 - snap) ? t1 : t + ha;
      double* tmp = X; X = Xn; Xn = tmp;     /* the third-order solution is kept */
      tmp = K1; K1 = K4; K4 = tmp;           /* FSAL */
      hn = o->fixed_step ? h : control(ha, err, o->rtol, 1, last_rejected, safety, facmin, facmax);
      last_rejected = 0;
      if (ha < st->h_min_seen) st->h_min_seen = ha;
    } else {
      st->n_reject++;
      hn = control(ha, err, o->rtol, 0, last_rejected, safety, facmin, facmax);
      last_rejected = 1;
    }
    st->h_last = ha;
    for (int q = 3; q > 0; --q) {
      hist_h[q] = hist_h[q - 1];
      hist_e[q] = hist_e[q - 1];
    }
    hist_h[0] = ha;
    hist_e[0] = err;
    nhist++;
    proposer = 0;
    /* the learned proposal replaces the controller's after an accepted attempt
       with four attempts recorded, when its standardized features lie inside
       [-4, 4] and its step ratio is finite, inside [0.2, 5] and within a factor
       of 2 of the classical rule's */
    if (o->mlp_w && accepted && nhist >= 4 && !o->fixed_step && t < t1) {
      double f[ORC_MLP_IN];
      for (int q = 0; q < 4; ++q) {
        f[q] = log(hist_h[q]);
        f[4 + q] = log(fmax(hist_e[q], 1e-30 * o->rtol) / o->rtol);
      }
      f[8] = log(fmax(fnorm, 1e-300));
      const double* mu = o->mlp_w + (ORC_MLP_PARAMS - 2 * ORC_MLP_IN);
      const double* inv_sd = mu + ORC_MLP_IN;
      int inside = 1;
      for (int k = 0; k < ORC_MLP_IN; ++k)
        if (!(fabs((f[k] - mu[k]) * inv_sd[k]) <= 4.0)) inside = 0;
      const double delta = orc_mlp_forward(o->mlp_w, f);
      const double d_std = log(hn / ha);
      if (inside && isfinite(delta) && delta >= fmax(log(0.2), d_std - log(2.0)) &&
          delta <= fmin(log(5.0), d_std + log(2.0))) {
        hn = ha * exp(delta);
        proposer = 1;
      }
    }
    hn = fmin(hn, h_max);
    h = hn;
    if (t >= t1) break;
    /* failure conditions of Sec. 2.2 (counter thresholds strict, reading) */
    if (st->n_accept + st->n_reject > i_max) { status = ORC_MAX_STEPS; break; }
    if ((double)st->n_reject > 0.85 * (double)i_max) { status = ORC_MAX_REJECTS; break; }
    if (!o->fixed_step && h <= h_min) { status = ORC_H_TOO_SMALL; break; }
  }
  st->h_next = h;
  st->t_reached = t;
  st->status = status;
  memcpy(y_out, X, sizeof(double) * (size_t)m);
  free(X); free(Xn); free(Y); free(K1); free(K2); free(K3); free(K4); free(E);
  if (ev.has_lp) lowp_free(&ev.lp);
  return status;
}

/* ------------------------------------------------------------------------ */
/* DP5(4) reference integrator (FSAL, weighted max norm, order-5 controller) */
/* ------------------------------------------------------------------------ */
/* Adaptive Fehlberg 4(5) with the paper's acceptance rule and weighted max norm
   (Sec. 2.2): stages K_l = f(X + h sum_q a_lq K_q), the fourth-order solution
   X_new = X + h sum_l b_l K_l, the error h sum_l (b_l - bh_l) K_l against the fifth
   order, accept iff E < Rel; then t += h, X = X_new and K_1 = f(X_new) (the pair has
   no shared last stage).  Step factor safety (Rel / E)^(1/5) clipped to
   [facmin, facmax] (growth capped at 1 right after a rejection); the starting step
   with the order 4. */
int orc_rkf45_solve(const orc_system* s, const orc_options* o, const double* y0, double t0, double t1,
                    double* y_out, orc_stats* st) {
  const int d = orc_dim(s->kind);
  if (d == 0 || s->n <= 0 || !(o->rtol > 0.0) || !(t1 >= t0)) return ORC_EINVAL;
  const int64_t m = (int64_t)d * s->n;
  memset(st, 0, sizeof(*st));
  if (t1 == t0) {
    memmove(y_out, y0, sizeof(double) * (size_t)m);
    st->t_reached = t0;
    return ORC_OK;
  }
  double h_max, safety, facmin, facmax;
  int64_t i_max;
  fill_defaults(o, t0, t1, &h_max, &i_max, &safety, &facmin, &facmax);
  evaluator ev = {s, ORC_PREC_FP64, {0}, 0};
  double* K[6];
  for (int l = 0; l < 6; ++l) K[l] = (double*)malloc(sizeof(double) * (size_t)m);
  double* X = (double*)malloc(sizeof(double) * (size_t)m);
  double* Xn = (double*)malloc(sizeof(double) * (size_t)m);
  double* Y = (double*)malloc(sizeof(double) * (size_t)m);
  memcpy(X, y0, sizeof(double) * (size_t)m);
  double t = t0;
  orc_rhs(s, t, X, K[0]);
  st->n_fev = 1;
  double h = (o->h0 > 0.0) ? o->h0 : start_step(&ev, 4, t0, X, K[0], m, o->rtol, o->atol, h_max, &st->n_fev);
  int last_rejected = 0, status = ORC_OK;
  const double snap = 4.0 * DBL_EPSILON * fabs(t1);
  while (t < t1) {
    const double ha = fmin(h, t1 - t);
    for (int l = 1; l < 6; ++l) {
      for (int64_t k = 0; k < m; ++k) {
        double acc = 0.0;
        for (int q = 0; q < l; ++q) acc += FE_A[l][q] * K[q][k];
        Y[k] = X[k] + ha * acc;
      }
      orc_rhs(s, t + FE_C[l] * ha, Y, K[l]);
    }
    st->n_fev += 5;
    double E = 0.0;
    const double fw = o->atol / o->rtol;
    for (int64_t k = 0; k < m; ++k) {
      double acc = 0.0, err = 0.0;
      for (int q = 0; q < 6; ++q) {
        acc += FE_B[q] * K[q][k];
        err += (FE_B[q] - FE_BH[q]) * K[q][k];
      }
      Xn[k] = X[k] + ha * acc;
      double W = fmax(fmax(fabs(X[k]), fabs(Xn[k])), fw);
      double v = fabs(ha * err) / W;
      if (isnan(v) || isnan(E)) E = NAN;
      else if (v > E) E = v;
    }
    if (!isfinite(E)) { status = ORC_NONFINITE; break; }
    double fac = (E > 0.0) ? safety * pow(o->rtol / E, 0.2) : facmax;
    if (E < o->rtol) {
      st->n_accept++;
      t = (t + ha >= t1 - snap) ? t1 : t + ha;
      double* tmp = X; X = Xn; Xn = tmp;
      orc_rhs(s, t, X, K[0]);
      st->n_fev += 1;
      h = ha * fmin(last_rejected ? 1.0 : facmax, fmax(facmin, fac));
      last_rejected = 0;
    } else {
      st->n_reject++;
      h = ha * fmax(facmin, fac);
      last_rejected = 1;
    }
    h = fmin(h, h_max);
    st->err_last = E;
    if (t >= t1) break;
    if (st->n_accept + st->n_reject > i_max) { status = ORC_MAX_STEPS; break; }
    if (h <= 100.0 * DBL_EPSILON) { status = ORC_H_TOO_SMALL; break; }
  }
  st->t_reached = t;
  st->status = status;
  memcpy(y_out, X, sizeof(double) * (size_t)m);
  for (int l = 0; l < 6; ++l) free(K[l]);
  free(X); free(Xn); free(Y);
  return status;
}

int orc_dp54_solve(const orc_system* s, const orc_options* o, const double* y0, double t0, double t1,
                   double* y_out, orc_stats* st) {
  const int d = orc_dim(s->kind);
  if (d == 0 || s->n <= 0 || !(o->rtol > 0.0) || !(t1 >= t0)) return ORC_EINVAL;
  const int64_t m = (int64_t)d * s->n;
  memset(st, 0, sizeof(*st));
  if (t1 == t0) {
    memmove(y_out, y0, sizeof(double) * (size_t)m);
    st->t_reached = t0;
    return ORC_OK;
  }
  double h_max, safety, facmin, facmax;
  int64_t i_max;
  fill_defaults(o, t0, t1, &h_max, &i_max, &safety, &facmin, &facmax);
  evaluator ev = {s, ORC_PREC_FP64, {0}, 0};
  double* K[7];
  for (int l = 0; l < 7; ++l) K[l] = (double*)malloc(sizeof(double) * (size_t)m);
  double* X = (double*)malloc(sizeof(double) * (size_t)m);
  double* Xn = (double*)malloc(sizeof(double) * (size_t)m);
  double* Y = (double*)malloc(sizeof(double) * (size_t)m);
  memcpy(X, y0, sizeof(double) * (size_t)m);
  double t = t0;
  orc_rhs(s, t, X, K[0]);
  st->n_fev = 1;
  double h = (o->h0 > 0.0) ? o->h0 : start_step(&ev, 5, t0, X, K[0], m, o->rtol, o->atol, h_max, &st->n_fev);
  int last_rejected = 0, status = ORC_OK;
  const double snap = 4.0 * DBL_EPSILON * fabs(t1);
  while (t < t1) {
    const double ha = fmin(h, t1 - t);
    for (int l = 1; l < 7; ++l) {
      double* dst = (l == 6) ? Xn : Y;
      for (int64_t k = 0; k < m; ++k) {
        double acc = 0.0;
        for (int q = 0; q < l; ++q) acc += DP_A[l][q] * K[q][k];
        dst[k] = X[k] + ha * acc;
      }
      orc_rhs(s, t + DP_C[l] * ha, dst, K[l]);
    }
    st->n_fev += 6;
    double E = 0.0;
    const double fw = o->atol / o->rtol;
    for (int64_t k = 0; k < m; ++k) {
      double acc = 0.0;
      for (int q = 0; q < 7; ++q) acc += (DP_B[q] - DP_BT[q]) * K[q][k];
      double W = fmax(fmax(fabs(X[k]), fabs(Xn[k])), fw);
      double v = fabs(ha * acc) / W;
      if (isnan(v) || isnan(E)) E = NAN;
      else if (v > E) E = v;
    }
    if (!isfinite(E)) { status = ORC_NONFINITE; break; }
    double fac = (E > 0.0) ? safety * pow(o->rtol / E, 0.2) : facmax;
    if (E < o->rtol) {
      st->n_accept++;
      t = (t + ha >= t1 - snap) ? t1 : t + ha;
      double* tmp = X; X = Xn; Xn = tmp;
      tmp = K[0]; K[0] = K[6]; K[6] = tmp;
      h = ha * fmin(last_rejected ? 1.0 : facmax, fmax(facmin, fac));
      last_rejected = 0;
    } else {
      st->n_reject++;
      h = ha * fmax(facmin, fac);
      last_rejected = 1;
    }
    h = fmin(h, h_max);
    st->err_last = E;
    if (t >= t1) break;
    if (st->n_accept + st->n_reject > i_max) { status = ORC_MAX_STEPS; break; }
    if (h <= 100.0 * DBL_EPSILON) { status = ORC_H_TOO_SMALL; break; }
  }
  st->t_reached = t;
  st->status = status;
  memcpy(y_out, X, sizeof(double) * (size_t)m);
  for (int l = 0; l < 7; ++l) free(K[l]);
  free(X); free(Xn); free(Y);
  return status;
}
