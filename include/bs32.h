/*
 * bs32.h -- C ABI of the MI355X (gfx950) mixed-precision Bogacki-Shampine 3(2)
 * solver for large, fully pairwise-coupled ODE systems.
 *
 * The problem is the paper's general model (Sec. 2.1, eq. (1)-(2)):
 *     dX_i/dt = F_i(t, X_i) + sum_j M_ij (.) G_ij(t, X_i, X_j),   i = 1..N,
 * with X in R^{dN} stored agent-major, X_i = (X_{(i-1)d+1}, ..., X_{id}), and the
 * weights M_ij = A_ij / N given by a dense N x N matrix A (uniform weights
 * M_ij = 1/N when A is NULL).  The integrator is the BS3(2) embedded pair with
 * FSAL (Sec. 2.2, Table Butcher-O23), the weighted max error estimate of
 * eq. (ERROR-O23), the accept rule "error smaller than Rel", and the failure
 * conditions of Sec. 2.2.  The reduced-precision modes put the N^2 coupling
 * contraction in FP32, BF16, FP16 or FP8 while every stage combination, the
 * error estimate, time and step size stay FP64 (the cast rules of Sec. 2.3).
 *
 * Conventions
 *  - Ownership: the caller owns every buffer it passes; the library copies what
 *    it needs during the call and keeps no caller pointer afterwards.
 *  - Pointers may be host or device (HIP) memory; the library tells them apart
 *    with hipPointerGetAttributes.  Device pointers must be on the context's device.
 *  - Every call returns a bs32_status.  Negative codes are argument or device
 *    errors: the context is left as it was and bs32_last_error() explains.
 *    Positive codes are solver terminations (Sec. 2.2): y_out then holds the last
 *    accepted state and bs32_stats() reports the time reached.
 *  - Calls on one context are synchronous with respect to the host and must not
 *    overlap; use one context per host thread.  Contexts are independent.
 */
#ifndef BS32_H
#define BS32_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bs32_ctx bs32_ctx; /* opaque; owns every device buffer it uses */

typedef enum {
  BS32_OK = 0,
  BS32_MAX_STEPS = 1,     /* failed + accepted steps > I_max (Sec. 2.2) */
  BS32_MAX_REJECTS = 2,   /* failed steps > 0.85 I_max (Sec. 2.2) */
  BS32_H_TOO_SMALL = 3,   /* step size fell to h_min = 100 eps_m (Sec. 2.2) */
  BS32_TIMEOUT = 4,       /* wall time over the limit (Sec. 2.2) */
  BS32_TOO_SLOW = 5,      /* wall time over the slow limit with < 10% of [t0,t1] done (Sec. 2.2) */
  BS32_NONFINITE = 6,     /* the error estimate is NaN or infinite */
  BS32_RANGE = 7,         /* a vector operand left the range of the reduced storage format */
  BS32_EINVAL = -1,       /* invalid argument */
  BS32_ENOMEM = -2,       /* device allocation failed */
  BS32_EDEVICE = -3,      /* HIP runtime error */
  BS32_ESTATE = -4,       /* call out of order (e.g. solve before set_system) */
  BS32_EUNSUPPORTED = -5  /* valid but not supported combination */
} bs32_status;

/* System kinds.  d = components per agent; the coupled component is the first. */
typedef enum {
  BS32_SYS_OSC2 = 1,      /* x' = v, v' = -w_i^2 x + (1/N) sum_j A_ij (x_j - x_i)          d = 2 */
  BS32_SYS_LCO_PAPER = 2, /* paper Benchmark 1, eq. (LCO): x' = v + (1/N) sum_j A_ij (x_j - x_i),
                             v' = -x                                                       d = 2 */
  BS32_SYS_KURAMOTO = 3,  /* paper Benchmark 2, eq. (Kuramoto):
                             th' = w_i + (K/N) sum_j A_ij sin(th_j - th_i)                 d = 1 */
  BS32_SYS_GOODWIN3 = 4,  /* x' = 1/(1+z^10) - b_i x + (kappa/N) sum_j A_ij (x_j - x_i),
                             y' = x - b_i y, z' = y - b_i z                                d = 3 */
  BS32_SYS_CLOCK4 = 5     /* paper Benchmark 3, eq. (CC), clock / cell cycle:
                             X1' = q (a X1^2 + 1) - k1_i X1 + (K/N) sum_j A_ij q a arctan(X_j1 - X_i1),
                             q = k0 th / (th + X2^4), th = k1_i / (k0 - k1_i),
                             X2' = k2 (X1 - X2), X3' = X3 (1 - X3^2/3) - X4 + I0 (1 - k3^2/(k3^2 + X1^2)),
                             X4' = eps (X3 + b - c X4); k0 = 2, k2 = 0.144832, k3 = 2, a = 2,
                             b = 0.7, c = 0.8, eps = 0.228249                               d = 4 */
} bs32_system_kind;

/* Precision of the coupling contraction (Sec. 2.3).  In modes 0-4 the stage
   combinations, the error estimate and its norm, t, h and the controller are
   FP64.  Modes 1-4 store A as Q(A / s), Q = round to nearest even from FP64,
   s = 2^ceil(log2(max|A| / m)) with m = 448 for e4m3 and 1 otherwise, and split
   the vector operand v into T terms of the storage format, term t = Q(r_t 2^(t S)),
   r_0 = v, r_(t+1) = r_t - 2^(-t S) term_t (the later terms compensate the first);
   products are summed in FP32 within groups of at most 128 (FP32), 256 (BF16,
   FP16) or 512 (e4m3) products and in FP64 across groups; the diffusive terms use
   FP64 row sums of the stored matrix.  A vector term outside the format's range
   stops the solve with BS32_RANGE. */
typedef enum {
  BS32_PREC_FP64 = 0,         /* the paper's "Double" */
  BS32_PREC_RHS_FP32 = 1,     /* FP32 storage, T = 2, S = 24 (vector ALU or 16x16x4 f32 matrix cores) */
  BS32_PREC_RHS_BF16 = 2,     /* BF16 storage, T = 2, S = 8 (16x16x32 bf16 matrix cores) */
  BS32_PREC_RHS_FP16 = 3,     /* IEEE binary16 storage, T = 2, S = 11 (16x16x32 f16 matrix cores) */
  BS32_PREC_RHS_FP8_E4M3 = 4, /* OCP e4m3fn storage, T = 3, S = 4 (16x16x32 fp8 matrix cores) */
  /* The paper's recipes (Table MP-Distrib, rows k2, k3, k4; the first K1, the
     starting-step probe and bs32_rhs use the k4 row).  Pair terms G in single
     everywhere: A stored FP32 and the vector operand one FP32 term.  "F in S":
     the agent term and the coupling combination in FP32; "Sigma in S": the
     interaction sum accumulated in FP32 throughout (else FP32 groups, FP64 across
     them).  Not available for ensembles. */
  BS32_PREC_PAPER_SINGLE = 5, /* k2, k3, k4 all single; solution and stage inputs stored FP32;
                                 h_min = 100 eps of FP32 */
  BS32_PREC_PAPER_MIXED1 = 6, /* k2, k3 all single; k4: F and Sigma double, G single */
  BS32_PREC_PAPER_MIXED2 = 7, /* k2, k3, k4: F and Sigma double, G single */
  /* each weight stored as a BF16 pair hi + lo (lo = the remainder A/s - hi rounded to
     BF16: about 16 significant bits), the operand split into two BF16 terms, the
     contraction (hi + lo) V accumulated in FP32 on the matrix cores within 128-element
     chunks and in FP64 across them; the conclusion's extension of the approach to
     other number formats.  Shared-coupling ensembles only (EUNSUPPORTED elsewhere);
     bs32_get_packed_coupling returns the hi plane followed by the lo plane. */
  BS32_PREC_RHS_BF16X2 = 8
} bs32_precision_mode;

typedef struct {
  int32_t kind;               /* bs32_system_kind */
  int32_t coupling_on_device; /* ignored (pointers are classified by the runtime); kept for ABI stability */
  int64_t n;                  /* number of agents N >= 1 */
  const double* coupling;     /* N*N row-major FP64 A_ij, or NULL for uniform weights (all ones) */
  const double* agent_param;  /* N values: w_i (OSC2, KURAMOTO), b_i (GOODWIN3), k1_i (CLOCK4); NULL = ones */
  double gain;                /* K (KURAMOTO, CLOCK4), kappa (GOODWIN3); ignored by OSC2 and LCO_PAPER */
  double stimulus;            /* I0 (CLOCK4); ignored by the others */
  int32_t pairwise;           /* KURAMOTO: 1 = evaluate K sin(th_j - th_i) pair by pair (N^2 sines, the
                                 paper's own form) instead of the matrix-vector identity; CLOCK4 is
                                 always pairwise (its arctan pair term has no such identity).  Pairwise
                                 systems run in modes 0 and 5-7 only, and not in ensembles; with
                                 coupling == NULL they store no matrix at all. */
  int32_t reserved;           /* 0 */
} bs32_system_desc;

typedef struct {
  int64_t n_accept, n_reject, n_fev; /* accepted / rejected attempts; RHS evaluations */
  double pair_interactions;          /* n_fev * N^2 */
  double t_reached, h_last, h_min_seen, err_last;
  double solve_ms;                   /* host wall time of the last solve */
  double kernel_ms;                  /* device time between the first and last kernel of the solve */
  int32_t status;                    /* bs32_status of the last solve */
  int32_t mode;                      /* precision mode of the last solve */
  int64_t n_learned;                 /* steps whose size the learned proposer chose */
  int32_t tile;                      /* contraction tile used (index as in options.tile) */
  int32_t reserved;
} bs32_stats_t;

typedef struct {
  int64_t i_max;         /* attempt limit (default 100000, Sec. 2.2) */
  double time_limit_s;   /* wall-time limit (default 5400 s, Sec. 2.2); <= 0 disables */
  double slow_limit_s;   /* "slow solver" time (default 2700 s, Sec. 2.2); <= 0 disables.
                            Both are checked by the host between chunks of attempts (2..64):
                            the chunk in flight when a limit is noticed still runs, so up to
                            64 more attempts count; the solve then returns BS32_TIMEOUT /
                            BS32_TOO_SLOW with y_out the last accepted state and the time and
                            counts reached in bs32_stats (per instance for a batch) */
  double h_max;          /* <= 0: 0.1 |t1 - t0| */
  double h0;             /* > 0: initial step (skips the starting-step evaluation) */
  double safety, facmin, facmax; /* controller constants (defaults 0.9, 0.2, 5) */
  int32_t fixed_step;    /* 1: every step h0, all accepted (order studies) */
  int32_t use_graph;     /* 1 (default): replay attempts from captured HIP graphs */
  int32_t trace;         /* 1: record one bs32_trace_rec per attempt (ring of trace_cap) */
  int32_t trace_cap;     /* ring capacity (default 65536) */
  int32_t controller;    /* 0 standard, 1 learned proposer (needs bs32_set_controller) */
  int32_t tile;          /* contraction tile configuration; -1 = autotuned default */
  int32_t method;        /* bs32_method: the embedded pair (default BS32_METHOD_BS32) */
  int32_t ensemble_launch; /* batches of independent systems (bs32_set_ensemble, not shared
                            couplings): 0 (default) one grouped launch per stage of an attempt;
                            1 one persistent launch per chunk of attempts, in which every
                            instance advances through its own stages from a device task
                            queue (contraction tiles of four waves only) */
} bs32_options;

/* Embedded Runge-Kutta pair of bs32_solve.  The paper's method is the
   Bogacki-Shampine 3(2) pair with FSAL (Sec. 2.2); its reference solver uses the
   Dormand-Prince 5(4) pair (Sec. 2.4, ode45) and its conclusion names other
   embedded pairs as generalisations.  BS32_METHOD_DP54 runs the same contraction
   kernels and storage formats (precision modes 0-4, pairwise couplings included)
   with seven FSAL stages per attempt, the same weighted max norm and acceptance
   rule (E < Rel) and the step factor safety * (Rel / E)^(1/5), clipped to
   [facmin, facmax] (growth capped at 1 right after a rejection); the starting
   step uses the exponent 1/6.  BS32_METHOD_RKF45 runs the embedded Fehlberg pair
   the conclusion also names (Fehlberg 4(5), published coefficients) on the same
   kernels: six stages, the fourth-order solution propagated and the fifth-order one
   measuring its error, the same norm, acceptance rule and step factor
   (exponent 1/5), starting step exponent 1/5; each attempt also evaluates f at
   its new solution, which becomes the next first stage (six evaluations per
   attempt, like DP5(4)).  Neither seven-stage pair serves the paper's recipes
   (modes 5-7), the learned proposer or ensembles (EUNSUPPORTED). */
typedef enum { BS32_METHOD_BS32 = 0, BS32_METHOD_DP54 = 1, BS32_METHOD_RKF45 = 2 } bs32_method;

/* One record per step attempt of the last solve (when options.trace = 1). */
typedef struct {
  double t, h, err, fnorm; /* time, attempted step, weighted error, weighted max norm of K1 */
  int32_t accepted, proposer; /* proposer: 1 if the learned proposer chose h */
} bs32_trace_rec;

/* The recipe row the library evaluates (Table MP-Distrib) for precision_mode 5-7
   and stage_row 0, 1, 2 (the paper's k2, k3, k4; the k4 row also serves the first
   K1, the starting-step probe and bs32_rhs): flags[0] = F, flags[1] = Sigma,
   flags[2] = G, each 1 for single and 0 for double.  Host only (no device or
   context needed); EINVAL for other modes or rows. */
bs32_status bs32_recipe_row(int precision_mode, int stage_row, int32_t flags[3]);

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to run on, or
   NULL for a library-owned stream (default priority). */
bs32_status bs32_create(bs32_ctx** out, int device, void* hip_stream);

/* Default options (the values quoted above). */
bs32_status bs32_default_options(bs32_options* out);
bs32_status bs32_set_options(bs32_ctx* ctx, const bs32_options* opt);

/* Copy and pack the system: A into padded row-major storage (FP64 first, other
   formats on first use by a solve), per-agent parameters, gain.  Replaces any
   previous system. */
bs32_status bs32_set_system(bs32_ctx* ctx, const bs32_system_desc* desc);

/* Integrate from (t0, y0) to t1.  y0 and y_out: d*N FP64 agent-major (may be the
   same buffer).  rtol > 0, atol >= 0, t1 >= t0 (t1 == t0 copies y0).
   precision_mode: bs32_precision_mode. */
bs32_status bs32_solve(bs32_ctx* ctx, const double* y0, double t0, double t1, double rtol, double atol,
                       int precision_mode, double* y_out);

/* Statistics of the last solve. */
bs32_status bs32_stats(const bs32_ctx* ctx, bs32_stats_t* out);

/* Evaluate the right-hand side once in a precision mode: f = F(X) + [M*G](X)
   (agent-major, d*N values).  For kernel tests and roofline timing: `repeat` > 1
   evaluates it that many times back to back and returns the last. */
bs32_status bs32_rhs(bs32_ctx* ctx, const double* y, int precision_mode, int repeat, double* f_out);

/* Time the N^2 contraction kernel of one stage evaluation (the hot kernel of
   eq. (Stage-ODE23)) in a precision mode, at the launch configuration bs32_solve
   uses: `repeat` back-to-back launches between two HIP events on the context's
   stream; *avg_ms receives the mean duration of one launch.  With an ensemble
   set, times the grouped launch over every instance.  Overwrites the context's
   stage buffers (call between solves). */
bs32_status bs32_time_contraction(bs32_ctx* ctx, int precision_mode, int repeat, double* avg_ms);

/* Name of the contraction kernel instance that precision_mode (0-4) runs with
   candidate tile `tile` (the index options.tile and bs32_stats_t.tile use) on the
   context's system or ensemble, as profilers list it without namespace and
   parameter list, e.g. "k_contract_f64<2, 2, 1, 4, 2, false>"; NUL-terminated
   into buf (cap bytes).  For matching profiler output to a solve. */
bs32_status bs32_kernel_name(bs32_ctx* ctx, int precision_mode, int tile, char* buf, size_t cap);

/* Copy the coupling matrix as stored for a precision mode (packing it first if
   needed): N rows of N elements of the storage format (8, 4, 2, 2, 1 bytes for
   FP64, FP32, BF16, FP16, e4m3), row-major without padding, into the host buffer
   dst of `bytes` bytes; *scale receives the per-tensor power-of-two scale s
   (A ~= s * stored).  For inspection and tests of the quantizer. */
bs32_status bs32_get_packed_coupling(bs32_ctx* ctx, int precision_mode, void* dst, size_t bytes, double* scale);

/* ---- ensembles -------------------------------------------------------------
   Many independent instances of the general model (each its own N, A, parameters,
   initial value and interval) solved together: each stage of an attempt is one
   grouped launch over the row blocks of every running instance, each instance
   keeps its own step size, counters and status (Sec. 2.2 applies per instance). */

/* Copy and pack `count` systems, all of the same kind (descs as for
   bs32_set_system).  Replaces any previous system or ensemble. */
bs32_status bs32_set_ensemble(bs32_ctx* ctx, int32_t count, const bs32_system_desc* descs);

/* Solve instance b from (t0[b], y0_b) to t1[b] for every b, with shared rtol, atol
   and precision mode.  y0_concat, y_out_concat: the instances' agent-major vectors
   concatenated in instance order (sum_b d N_b FP64 values; host or device; may be
   the same buffer).  t0, t1: host arrays of `count` values (t1[b] >= t0[b]).
   status_out: host array of `count` bs32_status values (may be NULL).  Returns
   BS32_OK when every instance reached its t1, otherwise the status of the first
   instance that did not. */
bs32_status bs32_solve_batch(bs32_ctx* ctx, const double* y0_concat, const double* t0, const double* t1,
                             double rtol, double atol, int precision_mode, double* y_out_concat,
                             int32_t* status_out);

/* Statistics of instance `instance` of the last batch solve (bs32_stats gives the
   totals: counts summed, time of the whole batch). */
bs32_status bs32_batch_stats(const bs32_ctx* ctx, int32_t instance, bs32_stats_t* out);

/* Ensemble of `count` instances that share one coupling matrix (parameter sweeps
   on one network): desc gives the kind (a matrix-vector system: not
   BS32_SYS_CLOCK4, pairwise = 0), N and the coupling A (host or device, NULL =
   all ones); params holds count x N agent parameters, instance-major (host or
   device; NULL = desc->agent_param for every instance, or ones); gains holds
   count gains (host; NULL = desc->gain).  Each instance keeps its own state,
   step size, counters and status; bs32_solve_batch and bs32_batch_stats work as
   for bs32_set_ensemble, and precision modes 0-3 (FP64, FP32, BF16, FP16
   storage of A) and 8 (the BF16 pair) are available.  The contraction of a stage
   for all instances is one matrix product A [V_1 ... V_B] on the matrix cores
   (B x m x T operand columns), followed by each instance's row epilogue in the
   same launch; this is the general model (Sec. 2.1, eq. (1)) evaluated for many
   parameter sets at once.  With 16-bit storage (modes 2, 3, 8) one more tile
   candidate computes the product as a plain library GEMM (hipBLASLt, FP32
   accumulation and output, one product per plane of the BF16 pair) and then
   launches the row epilogues on it; the autotuner takes it when it is faster,
   and that path is enqueued eagerly (no graph capture) and allocates its P
   buffer and workspace on first use.  Replaces any system or ensemble; count in
   [1, 65536]. */
bs32_status bs32_set_shared_ensemble(bs32_ctx* ctx, const bs32_system_desc* desc, int32_t count,
                                     const double* params, const double* gains);

/* Trace records of the last solve, oldest first; *n_records receives the count copied. */
bs32_status bs32_get_trace(bs32_ctx* ctx, bs32_trace_rec* buf, size_t cap, size_t* n_records);

/* ---- accuracy diagnostics -----------------------------------------------------
   The paper studies the solvers' accuracy through the real local error of each
   step of the coupled linear oscillators (Sec. 2.4, eq. (LCO-Local-Error)): the
   numerical solution after a step against the analytic solution started from the
   solution before it.  These calls provide the trajectory and that analytic flow. */

/* Record the solution of later bs32_solve calls into `states` (device memory,
   cap * d * N doubles, agent-major like y0): slot 0 receives the initial value
   as the solver holds it (rounded to FP32 in the Single recipe), slot k the
   state after the k-th accepted step; slots beyond cap - 1 are not written.  A
   solve ending after n_accept steps fills min(n_accept + 1, cap) slots (the
   last one equals y_out).  states = NULL or cap = 0 stops recording.  Needs a
   single system (ESTATE otherwise); bs32_set_system and bs32_set_ensemble stop
   recording.  The buffer stays owned by the caller and must outlive the solves. */
bs32_status bs32_set_record(bs32_ctx* ctx, double* states, int64_t cap);

/* Analytic solution of the coupled linear oscillators (paper Benchmark 1,
   eq. (LCO), uniform weights M_ij = 1/N, in FP64): out[k] = exp(h[k] L) X[k] for
   `count` states of 2N agent-major doubles each.  X, h (count values) and out
   are device memory; out must not overlap X.  Runs on the context's stream and
   returns when done; any system set on the context is left alone. */
bs32_status bs32_lco_flow(bs32_ctx* ctx, int64_t n, int64_t count, const double* X, const double* h, double* out);

/* Real local error of eq. (LCO-Local-Error) for `steps` consecutive steps of a
   recorded trajectory: err[k] = max over the 2N components of
   |states[k+1] - X_ex| / max(|X_ex|, delta), with X_ex = exp(h[k] L) states[k]
   and delta > 0 (the paper takes Abs / Rel).  states holds steps + 1 states of
   2N agent-major doubles (as bs32_set_record writes them), h the accepted step
   sizes (bs32_get_trace records with accepted = 1), err receives `steps`
   values; all device memory.  A non-finite state gives NaN. */
bs32_status bs32_lco_local_error(bs32_ctx* ctx, int64_t n, int64_t steps, const double* states, const double* h,
                                 double delta, double* err);

/* ---- learned step-size proposer ---------------------------------------------
   The paper says only that the error estimate drives the step-size correction
   (Sec. 2.2).  This extension lets a small network propose the next step while
   the estimate stays the only judge of acceptance: a step is accepted iff
   E < Rel whatever proposed it.

   Network: 9 -> 64 -> 64 -> 1, tanh hidden layers, BF16-valued weights, FP32
   accumulation, on standardized features x_k = (f_k - mu_k) * inv_sd_k (FP32).
   Parameter vector of BS32_MLP_PARAMS floats, in this order: W1[64][9], b1[64],
   W2[64][64], b2[64], w3[64], b3 (4865 network weights, used rounded to BF16),
   mu[9], inv_sd[9] (used as given).
   Features after an accepted attempt n (most recent first):
     f[0..3] = log h_n, log h_{n-1}, log h_{n-2}, log h_{n-3}   (attempted steps)
     f[4..7] = log(max(E, 1e-30 Rel) / Rel) of the same attempts
     f[8]    = log max(fnorm_n, 1e-300), fnorm_n = max_k |K1_k| / max(|X^n_k|, Ab/Rel),
               the weighted size of f(t_n, X^n) (trace field fnorm)
   Output: delta = log(h_{n+1} / h_n).  The proposal is used only after an
   accepted attempt with four attempts recorded, when every |x_k| <= 4 (the
   features lie where the network was trained) and delta is finite, inside
   [log 0.2, log 5] and within log 2 of the standard controller's own
   log(h_{n+1} / h_n); otherwise the standard controller chooses (it always does
   in the attempt after a rejection).  The step is then clipped to h_max and t1. */
#define BS32_MLP_PARAMS 4883

/* Training samples from a trace (bs32_get_trace of a solve with tolerance rtol):
   one per accepted attempt n >= 3 whose next attempt n+1 is not the last record
   and has 0 < E < inf.  features: 9 floats per sample (layout above) or NULL;
   labels: 1 float per sample or NULL, the step that would have put attempt n+1's
   estimate at 0.8 Rel under E ~ h^3:
     label = log(h_{n+1} / h_n) + (1/3) log(0.8 Rel / E_{n+1}).
   Buffers must hold n-4 samples; *n_samples receives the count.  Host only. */
bs32_status bs32_mlp_features(const bs32_trace_rec* trace, size_t n, double rtol, float* features, float* labels,
                              size_t* n_samples);

/* Train the network on the GPU: mu and inv_sd from the mean and deviation of the
   n feature vectors; Glorot-uniform initial weights, zero biases and the epoch
   shuffles drawn from `seed` (splitmix64); minibatch Adam (beta 0.9 / 0.999,
   eps 1e-8, learning rate lr) on FP32 master weights, every forward pass with
   their BF16-rounded copies; loss (1/B) sum w (y - label)^2 with w = 4 when the
   prediction overshoots the label (a rejection costs three RHS) and 1 otherwise.
   weights_out: BS32_MLP_PARAMS values, the FP32 master weights and the
   standardization (host).  loss_per_epoch: `epochs` values (host, may be NULL),
   the loss over all n samples after each epoch.  Host buffers; n >= 2; the last
   partial minibatch of an epoch is dropped. */
bs32_status bs32_mlp_train(bs32_ctx* ctx, const float* features, const float* labels, size_t n, int epochs,
                           int batch, float lr, uint64_t seed, float* weights_out, float* loss_per_epoch);

/* Gradient of that loss over n samples (features as the solver forms them; the
   weights' own standardization is applied) at the BF16-rounded network weights,
   by the training kernels.  grad_out: BS32_MLP_PARAMS doubles (zero for mu and
   inv_sd, which are not trained); loss_out: the loss (may be NULL).  Host
   buffers.  For tests of the training kernels. */
bs32_status bs32_mlp_grad(bs32_ctx* ctx, const float* weights, const float* features, const float* labels, size_t n,
                          double* grad_out, double* loss_out);

/* Allocation-free variant of bs32_mlp_grad, for callers that cannot allocate device
   memory (code under HIP graph capture, tight serving loops, harnesses that forbid
   allocation).  Same kernels and the same result, bit for bit, as bs32_mlp_grad on
   the same inputs; no call allocates or frees memory.  Every buffer is device memory
   on the context's device, owned by the caller: weights (BS32_MLP_PARAMS floats, the
   layout above), features (9 n raw floats), labels (n floats), grad_out
   (BS32_MLP_PARAMS doubles; zero for mu and inv_sd) and loss_out (one double, may be
   NULL).  1 <= n <= BS32_MLP_NOALLOC_MAX, else BS32_EINVAL.  Intermediate results
   live in a fixed device array of the library (about 5.3 MiB per GPU, held until the
   process ends), shared by every call on that GPU: calls that overlap on one GPU
   (several contexts or streams) race and must be serialized by the caller.  The
   work is enqueued on the context's stream and the call returns without waiting;
   the outputs are valid once that stream has completed it. */
#define BS32_MLP_NOALLOC_MAX 16384
bs32_status bs32_mlp_grad_noalloc(bs32_ctx* ctx, const float* weights, const float* features, const float* labels,
                                  size_t n, double* grad_out, double* loss_out);

/* Select the step-size controller of later solves: kind 0 = standard (weights
   ignored), kind 1 = learned proposer with `count` = BS32_MLP_PARAMS finite FP32
   values (host); the network weights are stored rounded to BF16.  Sets
   options.controller. */
bs32_status bs32_set_controller(bs32_ctx* ctx, int kind, const float* weights, size_t count);

/* Message of the last negative status on this context (never NULL). */
const char* bs32_last_error(const bs32_ctx* ctx);

void bs32_destroy(bs32_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* BS32_H */
