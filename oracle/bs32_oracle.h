/*
 * bs32_oracle.h -- plain CPU reference ("oracle") of the mixed-precision
 * Bogacki-Shampine 3(2) solver for pairwise-coupled ODE systems.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link,
 * load or call this library: only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark do.  It shares no code, header, table or
 * helper with the HIP library; the two meet only through the seeded input
 * arrays handed to both.
 *
 * Everything is FP64 unless a precision mode says otherwise.  The state is
 * agent-major, X = (X_1, ..., X_N), X_i in R^d, exactly as the paper's
 * general model (Sec. 2.1, eq. (1)-(2)) lays it out.
 *
 * Parity status of each function is listed in the file header of
 * bs32_oracle.c.
 */
#ifndef BS32_ORACLE_H
#define BS32_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* system kinds (same numbering as the public library, written out again here) */
#define ORC_OSC2 1      /* x'' = -w^2 x + (1/N) sum_j A_ij (x_j - x_i)            d = 2 */
#define ORC_LCO_PAPER 2 /* paper Benchmark 1: x' = v + (1/N)sum A_ij(x_j-x_i), v'=-x  d = 2 */
#define ORC_KURAMOTO 3  /* paper Benchmark 2 with weights A_ij/N                    d = 1 */
#define ORC_GOODWIN3 4  /* 3-variable Goodwin clock with diffusive x-coupling       d = 3 */
#define ORC_CLOCK4 5    /* paper Benchmark 3, eq. (CC): clock/cell cycle, arctan coupling  d = 4 */

/* storage formats of the coupling matrix / split vector terms */
#define ORC_FMT_F64 0
#define ORC_FMT_F32 1
#define ORC_FMT_BF16 2
#define ORC_FMT_F16 3
#define ORC_FMT_E4M3 4 /* OCP e4m3fn, saturating */
#define ORC_FMT_BF16X2 5 /* a pair of BF16 values hi + lo, lo = the remainder x - hi rounded to BF16 */

/* precision modes */
#define ORC_PREC_FP64 0
#define ORC_PREC_RHS_FP32 1
#define ORC_PREC_RHS_BF16 2
#define ORC_PREC_RHS_FP16 3
#define ORC_PREC_RHS_FP8 4
#define ORC_PREC_PAPER_SINGLE 5
#define ORC_PREC_PAPER_MIXED1 6
#define ORC_PREC_PAPER_MIXED2 7
#define ORC_PREC_RHS_BF16X2 8 /* coupling as BF16 pairs, operand in two BF16 terms */

/* termination codes (paper Sec. 2.2, "Failure conditions") */
#define ORC_OK 0
#define ORC_MAX_STEPS 1
#define ORC_MAX_REJECTS 2
#define ORC_H_TOO_SMALL 3
#define ORC_NONFINITE 6
#define ORC_EINVAL -1

typedef struct {
  int32_t kind;
  int64_t n;           /* number of agents N */
  const double* A;     /* n*n row-major weights; NULL = all ones (the paper's uniform M_ij = 1/N) */
  const double* param; /* per agent: omega_i (OSC2, KURAMOTO) or b_i (GOODWIN3); NULL = all ones */
  double gain;         /* K (KURAMOTO, CLOCK4), kappa (GOODWIN3); ignored by OSC2 and LCO_PAPER */
  double stimulus;     /* I_0 (CLOCK4); ignored by the others */
} orc_system;

typedef struct {
  double rtol, atol;
  double h_max;        /* <= 0: 0.1*|t1-t0| */
  double h0;           /* > 0: fixed initial step, no starting-step evaluation */
  int64_t i_max;       /* <= 0: 100000 */
  int32_t fixed_step;  /* 1: take h0 every step, accept all, no control (order tests only) */
  double safety, facmin, facmax; /* <= 0: 0.9, 0.2, 5.0 */
  /* split of the vector operand in the reduced-precision RHS modes */
  int32_t split_terms;     /* <= 0: mode default */
  int32_t split_fmt;       /* -1: mode default */
  int32_t split_shift;     /* <= 0: mode default */
  /* learned step-size proposer: ORC_MLP_PARAMS weights, NULL = standard controller only */
  const double* mlp_w;
} orc_options;

typedef struct {
  int64_t n_accept, n_reject, n_fev;
  double t_reached, h_last, h_next, err_last, h_min_seen;
  int32_t status;
} orc_stats;

/* one record per step attempt */
typedef struct {
  double t, h, err;
  double fnorm;        /* max_k |K1_k| / max(|X^n_k|, atol/rtol) at the start of the attempt */
  int32_t accepted;
  int32_t proposer;    /* 1: the learned proposer chose h */
} orc_trace_rec;

int orc_dim(int kind);

/* OpenMP threads of the row loops (n <= 0 leaves the setting); the count in use. */
void orc_set_threads(int n);
int orc_get_threads(void);

/* ---- right-hand sides -------------------------------------------------- */
/* FP64 pairwise definition: F(t,X) + [M*G](t,X), sums over j in increasing order. */
int orc_rhs(const orc_system* sys, double t, const double* X, double* F);

/* FP64 pairwise definition for a subset of rows only: rows[r] is the agent index,
   Arows holds those agents' rows of the weights (nrows*n, NULL = all ones), F_rows
   receives d values per listed row.  For checks of sampled outputs at full size. */
int orc_rhs_rows(const orc_system* sys, const int64_t* rows, int64_t nrows, const double* Arows, double t,
                 const double* X, double* F_rows);

/* Reduced-precision contraction mode (fmt = ORC_FMT_*): the coupling weights are
   replaced by their stored values A_hat = s*Q(A/s) and the vector operand by its
   split reconstruction; the contraction itself is evaluated exactly in FP64. */
int orc_rhs_lowp(const orc_system* sys, int fmt, int split_fmt, int split_terms, int split_shift,
                 double t, const double* X, double* F);

/* The reduced-precision definition for a subset of rows (checks of sampled outputs
   at full size): Arows holds the listed agents' FP64 rows (nrows*n, NULL = all
   ones), scale the per-tensor scale of the whole matrix (orc_matrix_scale; it
   depends only on max|A|), the split of the vector operand the format's default. */
int orc_rhs_lowp_rows(const orc_system* sys, int fmt, double scale, const int64_t* rows, int64_t nrows,
                      const double* Arows, double t, const double* X, double* F_rows);

/* Paper recipe evaluation of one stage (Sec. 2.3, Table MP-Distrib): pF, pS, pG in
   {0 = double, 1 = single} for the agent term, the accumulation and the pair term. */
int orc_rhs_recipe(const orc_system* sys, int pF, int pS, int pG, double t, const double* X, double* F);

/* The recipe table the integrator uses (Table MP-Distrib): out[9 r + 3 k + q] for
   solver r (0 Single, 1 Mixed1, 2 Mixed2), stage row k (0 k2, 1 k3, 2 k4) and
   column q (0 F, 1 Sigma, 2 G); 1 = single, 0 = double. */
void orc_recipe_table(int out[27]);

/* ---- number formats ---------------------------------------------------- */
/* Round-to-nearest-even of an FP64 value straight to the format (no double rounding);
   returns the rounded value as a double. */
double orc_round_fmt(double x, int fmt);
/* Same rounding, returned as the format's bit pattern (low bits of the result). */
uint32_t orc_encode_fmt(double x, int fmt);
double orc_decode_fmt(uint32_t bits, int fmt);
/* Per-tensor power-of-two scale of a coupling matrix stored in fmt. */
double orc_matrix_scale(const double* A, int64_t count, int fmt);
/* Split v into terms: out[k] = 2^(-k*shift) * Q(r_k * 2^(k*shift)), r_0 = v, r_{k+1} = r_k - out[k]. */
void orc_split(double v, int fmt, int terms, int shift, double* out);

/* ---- the integrators ---------------------------------------------------- */
/* Adaptive BS3(2) with FSAL (Sec. 2.2), y0/y_out agent-major, may alias. */
int orc_bs32_solve(const orc_system* sys, const orc_options* opt, int prec_mode,
                   const double* y0, double t0, double t1, double* y_out, orc_stats* st,
                   orc_trace_rec* trace, int64_t trace_cap, int64_t* trace_len);

/* Adaptive Dormand-Prince 5(4) in FP64, used only to build reference solutions. */
int orc_dp54_solve(const orc_system* sys, const orc_options* opt,
                   const double* y0, double t0, double t1, double* y_out, orc_stats* st);

/* Fehlberg 4(5): the embedded Fehlberg pair (published coefficients), fourth-order
   solution propagated, the same norm, acceptance rule and step factor exponent 1/5 as
   orc_dp54_solve; K_1 is evaluated afresh after every accepted step (no shared last
   stage), so n_fev = 1 + (starting step) + 5 attempts + accepted steps. */
void orc_rkf45_tableau(double c[6], double a[36], double b[6], double bh[6]);
int orc_rkf45_solve(const orc_system* sys, const orc_options* opt,
                    const double* y0, double t0, double t1, double* y_out, orc_stats* st);

/* ---- learned step-size proposer ----------------------------------------
   An extension: Sec. 2.2 only says that the error estimate drives the step-size
   correction.  9 -> 64 -> 64 -> 1 network with tanh hidden layers on standardized
   features x_k = (f_k - mu_k) inv_sd_k; parameter vector W1[64][9], b1[64],
   W2[64][64], b2[64], w3[64], b3, mu[9], inv_sd[9].  Features after an
   accepted attempt n: log h_n..h_{n-3}, log(max(E, 1e-30 Rel)/Rel) of the same
   attempts, log max(fnorm_n, 1e-300); output log(h_{n+1}/h_n), used when finite
   and inside [log 0.2, log 5] once four attempts are recorded. */
#define ORC_MLP_IN 9
#define ORC_MLP_HID 64
#define ORC_MLP_PARAMS 4883
/* FP64 evaluation of the network on one feature vector. */
double orc_mlp_forward(const double* w, const double* features);

/* Butcher tables as the oracle holds them (for the tableau tests). */
void orc_bs32_tableau(double c[4], double a[16], double b[4], double bt[4]);
void orc_dp54_tableau(double c[7], double a[49], double b[7], double bt[7]);

/* One BS3(2) attempt from (t, X, K1) with step h: Xn, K4 and the weighted max error. */
int orc_bs32_attempt(const orc_system* sys, double t, double h, const double* X, const double* K1,
                     double rtol, double atol, double* Xn, double* K4, double* err);

#ifdef __cplusplus
}
#endif
#endif
