// bs32_internal.hpp -- shared declarations of the gfx950 BS3(2) library
// (host orchestration in bs32_capi.cpp, kernels in bs32_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bs32 {

// ---- BS3(2) tableau (Sec. 2.2, Table Butcher-O23) --------------------------
constexpr double kA21 = 1.0 / 2.0;
constexpr double kA32 = 3.0 / 4.0;
constexpr double kB1 = 2.0 / 9.0, kB2 = 1.0 / 3.0, kB3 = 4.0 / 9.0;
constexpr double kBt1 = 7.0 / 24.0, kBt2 = 1.0 / 4.0, kBt3 = 1.0 / 3.0, kBt4 = 1.0 / 8.0;

// ---- Dormand-Prince 5(4) with FSAL: the pair of the paper's reference solver
// (Sec. 2.4, ode45) and a method its conclusion names the approach for; the
// published coefficients.  Row s of kDpA builds the input of stage s + 1; the
// last row equals the fifth-order weights, so stage 7 is evaluated at X^{n+1}.
constexpr double kDpA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0},
};
constexpr double kDpB[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
constexpr double kDpBt[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0, -92097.0 / 339200.0,
                             187.0 / 2100.0, 1.0 / 40.0};

// ---- Fehlberg 4(5), the embedded Fehlberg pair of the conclusion, laid out like the
// Dormand-Prince arrays above: rows 1..5 build the inputs of stages 2..6, row 6 holds
// the propagated fourth-order weights (the seventh evaluation, at X^{n+1}, becomes the
// next step's first stage), and the error weights b - bt leave the seventh stage out.
// Published coefficients.
constexpr double kFeA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 4.0, 0, 0, 0, 0, 0},
    {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0, 0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0, 0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0, 0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0, 0},
    {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0, 0.0},
};
constexpr double kFeB[7] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0, 0.0, 0.0};
constexpr double kFeBt[7] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0, 0.0};

// internal solver status (public codes are bs32_status values >= 0)
constexpr int kRunning = 100;
constexpr int kStatusRange = 7;  // BS32_RANGE

// stages of one contraction launch
// (ST_D2 .. ST_D7: the six contractions of a Dormand-Prince 5(4) attempt)
enum Stage : int {
  ST_INIT = 0, ST_H0 = 1, ST_S2 = 2, ST_S3 = 3, ST_S4 = 4, ST_RHS = 5,
  ST_D2 = 6, ST_D3 = 7, ST_D4 = 8, ST_D5 = 9, ST_D6 = 10, ST_D7 = 11
};

// storage formats of the coupling matrix
// (F_BF16X2: each weight as a BF16 pair hi + lo, lo = the remainder rounded to BF16,
// stored as two planes of np x ld values; the shared-coupling product only)
enum Fmt : int { F_F64 = 0, F_F32 = 1, F_BF16 = 2, F_F16 = 3, F_E4M3 = 4, F_BF16X2 = 5 };

// Device-resident control block of one solve: the step-size state lives on the
// GPU so that attempts run back to back without host round trips.  Two buffers
// alternate: each finalize launch reads one and workgroup 0 writes the other, so
// no launch ever reads a block that the same launch writes.
struct Ctl {
  double t, h, ha;        // time, proposed step, step of the current attempt (clipped to t1)
  double t0, t1, rtol, atol;
  double h_max, h_min, snap;
  double safety, facmin, facmax;
  double err, h_last, h_min_seen;
  double h0probe;         // starting-step probe size (Hairer-Norsett-Wanner)
  double h0user;          // > 0: user initial step
  double d0, d1;          // starting-step norms of y0 and f0
  long long n_accept, n_reject, n_fev, i_max;
  int status;             // kRunning or a final bs32_status
  int xi;                 // current solution buffer (X^n = X[xi], X^{n+1} -> X[1-xi])
  int ki;                 // current first-stage buffer (K1 = Kf[ki], K4 -> Kf[1-ki])
  int last_rejected;
  int fixed_step;
  int trace_on;
  int trace_cap;
  int use_mlp;            // 1: the learned proposer chooses h when its conditions hold
  long long trace_n;      // attempts recorded so far (ring index = trace_n % cap)
  double hist_h[4];       // attempted steps, most recent first (learned proposer features)
  double hist_e[4];       // their error estimates
  long long nhist;        // attempts recorded in the history
  long long n_mlp;        // steps chosen by the learned proposer
  int prop_cur;           // 1 if the current step size came from the learned proposer
  int method;             // 0: Bogacki-Shampine 3(2), 1: Dormand-Prince 5(4), 2: Fehlberg 4(5)
};

struct TraceRec {
  double t, h, err, fnorm;
  int accepted, proposer;
};

// operand buffer a contraction reads: stage 3 of BS3(2) and the odd Dormand-Prince
// stages read buffer 1, the rest buffer 0 (each stage writes the next one's input
// into the other buffer)
__host__ __device__ inline int vin_of(int stage) {
  if (stage >= ST_D2) return (stage - ST_D2) & 1;
  return stage == ST_S3 ? 1 : 0;
}

// Arguments of the contraction / prep / finalize kernels (passed by value).
struct Args {
  const void* A;          // packed coupling, rows_pad x ld, storage format
  const double* rsum;     // row sums of the stored (dequantized) A, length np
  const double* param;    // per-agent parameter (omega or b), length np
  double* X[2];           // SoA state ping-pong, d x np each
  double* Kf[2];          // first/last stage ping-pong (FSAL)
  double* K2;
  double* K3;
  double* Kd[3];          // K4, K5, K6 of a Dormand-Prince attempt
  double* V64[2];         // FP64 vector operand ping-pong, [ld][m]
  void* Vq[2];            // split vector operand terms for reduced formats, [m*T][ld]
  double* ep0;            // per-row-block partial maxima
  double* ep1;
  Ctl* ctl;               // control state read by this launch
  Ctl* ctl_out;           // finalize: where the next control state goes (the other buffer)
  unsigned* rflag;        // sticky flag: a vector term left the storage format's range
  const float* mlp;       // learned proposer weights (BF16 values as FP32), or null
  TraceRec* trace;
  double gain, invN, scale; // coupling gain, 1/N, per-tensor scale of A (power of two)
  double vmax;            // largest magnitude the vector terms may hold (format range check)
  long long n, np, ld;    // agents, padded rows, leading dimension (elements)
  long long kn;           // columns the contraction streams: n rounded up to the tile's k step (<= ld)
  int kind, d, m;         // system kind, components per agent, vector columns
  int stage;
  int nrb;                // row blocks (workgroups of the contraction)
  int RB;                 // rows per block
  int KW;                 // columns per wave k-slice
  int vfmt;               // format of the vector terms (F_F64 = no terms)
  int vterms;             // split terms of the vector operand
  int vshift;             // exponent shift between consecutive terms
  // the paper's recipes (Sec. 2.3, Table MP-Distrib), per stage
  int vsingle;            // pair terms in single: the vector operand is one FP32 term
  int fsingle;            // agent term F and the coupling combination in FP32
  int sum32;              // the interaction sum accumulated in FP32 throughout
  int sstate;             // solution and stage inputs stored in FP32 (Single)
  int pairwise;           // coupling evaluated pair by pair (g(x_j - x_i)); operand = the coupled component
  double stim;            // I_0 of the clock / cell-cycle model
  double* rec;            // solution record (initial value, then one state per accepted step), or null
  long long rec_cap;      // states the record holds (d * n agent-major doubles each)
  int pair;               // seven-stage attempts (ST_D2 .. ST_D7): 1 Dormand-Prince 5(4), 2 Fehlberg 4(5)
};

// Ensembles: one work item = (instance, row block) for a contraction, or
// (instance, 256-agent slice) for prep / finalize.
struct Item {
  unsigned inst, blk;
};
constexpr int kStages = 6;  // Args copies per instance and control parity: one per Stage
struct Group {
  const Args* inst;       // [(instance * kStages + stage) * 2 + parity]
  const Item* items;      // live work items
  const unsigned* count;  // number of live items
  const unsigned* xs;     // contraction lists: item ranges of the 8 XCDs, xs[x] .. xs[x + 1]
  int stage, par;
};

// Persistent ensemble launch: one kernel runs `attempts` attempts of every listed
// instance.  An instance's work is a sequence of tasks, per attempt TC tasks of each
// of the stages S2, S3, S4 (a task: G consecutive row tiles of the T) and then FC
// finalize tasks (GF consecutive slices of 256 agents of the F), Q = 3 TC + FC tasks;
// workgroups claim the next task of an instance from its counter `tick` and may start
// it once `comp` (tasks completed) has reached the first task of its phase.
struct PSched {
  unsigned b;       // instance
  unsigned T, G;    // row tiles of a stage; row tiles per task
  unsigned F, GF;   // finalize slices; slices per task
  unsigned TC, FC;  // tasks per stage, finalize tasks
  unsigned Q;       // tasks per attempt, 3 TC + FC
};
struct PGroup {
  const Args* inst;       // [(instance * kStages + stage) * 2 + parity]
  const PSched* sched;    // listed instances
  const unsigned* count;  // number of listed instances
  const unsigned* xs;     // listed-instance ranges of the 8 XCDs, xs[x] .. xs[x + 1]
  unsigned* tick;         // [listed] tasks claimed (zeroed before each launch)
  unsigned* comp;         // [listed] tasks completed (zeroed before each launch)
  unsigned* abort;        // set when a wait exceeded its bound: every workgroup leaves
  int attempts;           // attempts of this launch
  int par0;               // control parity of the first attempt
};

// Shared-coupling ensembles: B instances with one coupling matrix; the stage
// contraction of all of them is one matrix product A [V_1 ... V_B].
struct Shared {
  const void* A;          // the shared coupling, np x ld in the storage format
  const Args* inst;       // per-instance arguments [(instance * kStages + stage) * 2 + parity]
  const void* Bop[2];     // operand pools by buffer: split terms [Bpad][m T][ld] (FP64: [Bpad][ld][m])
  long long ld, np;
  int stage, par;
  int B;                  // instances (the pools hold whole column tiles of zero-padded instances beyond)
  int nrb, ncb;           // row and column blocks of the product
  double scale;           // power-of-two scale of the stored coupling
  int vshift;             // exponent shift between the operand's split terms
  const float* Pg[2];     // library product tile source (tile NT = 1): P of A (and of the BF16
                          // pair's remainder plane), [np][ldp] FP32; null for the fused kernels
  long long ldp;          // row stride of Pg (operand columns of all pooled instances)
};

// Contraction tile: WR row groups x WK k-slices of waves per workgroup; each wave
// owns R rows (VALU kernels) or R tiles of 16 rows (matrix-core kernels) and
// keeps U loads per row in flight.  Pairwise kernels: WR waves of R rows, U
// column chunks of 64 per step.
struct Tile {
  int R, WR, WK, U, NT;  // NT: non-temporal loads of A (shared products: 1 = library product + epilogue)
  int MM;                // 0: vector-ALU kernel, 1: matrix-core kernel (16-row tiles), 2: pairwise kernel,
                         // 3: shared-coupling product (R: 16-row tiles per wave of 4, U: 16-column tiles)
  int EW = 0;            // single systems: one more wave that loads the rows' epilogue inputs and finishes them
};
const Tile* tile_candidates(int fmt, int* count);
const Tile* pair_tile_candidates(int* count);
const Tile* shared_tile_candidates(int* count);
// columns of the shared product one instance occupies in a storage format (0: not supported)
int shared_cols(int fmt, int m);

// host launchers (bs32_kernels.hip)
int dim_of(int kind);
int vcols_of(int kind, int pairwise);
size_t fmt_bytes(int fmt);
int tile_rows(int fmt, const Tile& t);
int tile_kalign(int fmt, const Tile& t);
bool tile_supported(int fmt, int m, const Tile& t);
// name of the contraction kernel instance (as profilers list it); < 0 if unsupported
int kernel_name(int fmt, int m, const Tile& t, char* buf, size_t cap);
hipError_t launch_prep(const Args& a, hipStream_t s);
hipError_t launch_finalize(const Args& a, hipStream_t s);
hipError_t launch_set_status(Ctl* c, int code, hipStream_t s);
hipError_t launch_contract(const Args& a, int fmt, const Tile& t, hipStream_t s);
hipError_t launch_group_contract(const Group& g, int m, int fmt, const Tile& t, unsigned grid, hipStream_t s);
hipError_t launch_group_prep(const Group& g, unsigned grid, hipStream_t s);
// persistent ensemble launch (tiles of four waves; see PGroup); zeroes the counters first
hipError_t launch_persistent(const PGroup& p, int m, int fmt, const Tile& t, unsigned grid, unsigned ncounters,
                             hipStream_t s);
bool tile_persistent_ok(int fmt, int m, const Tile& t);
hipError_t launch_group_finalize(const Group& g, unsigned grid, hipStream_t s);
hipError_t launch_shared_contract(const Shared& sh, int m, int fmt, const Tile& t, hipStream_t s);

// plain library product for 16-bit shared products (bs32_blas.cpp)
struct BlasProduct;
BlasProduct* blas_create(char* err, size_t cap);
void blas_destroy(BlasProduct* b);
int blas_product(BlasProduct* b, int fmt, const void* A, const void* B, long long rows, long long m, long long ld,
                 float* P, hipStream_t stream, char* err, size_t cap);

// learned proposer training (bs32_mlp.hip)
hipError_t launch_mlp_grad(const float* W, const float* X, const float* Y, const int* idx, int nb, float inv_n,
                           float over_w, float* part, double* loss_part, hipStream_t s);
hipError_t launch_mlp_reduce(const float* part, int nparts, double* out, hipStream_t s);
hipError_t launch_mlp_adam(float* master, float* m1, float* m2, float* wq, const float* part, int nparts, float lr,
                           float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t s);
hipError_t launch_bf16_copy(const float* src, float* dst, int n_round, int n, hipStream_t s);
// allocation-free gradient: samples at most kNaMaxSamples; noalloc_bind (once per device,
// with that device current) looks up the device's copy of the scratch array
constexpr int kNaMaxSamples = 16384;  // BS32_MLP_NOALLOC_MAX
hipError_t noalloc_bind(int device);
hipError_t launch_mlp_grad_noalloc(int device, const float* W, const float* F, const float* Y, int n, double* grad,
                                   double* loss, hipStream_t s);
hipError_t launch_round_f32(double* x, long long n, hipStream_t s);
// analytic solution of the coupled linear oscillators and the real local error (bs32_lco.hip)
hipError_t launch_lco_flow(const double* X, const double* h, long long n, long long count, double* out,
                           hipStream_t s);
hipError_t launch_lco_local_error(const double* states, const double* h, long long n, long long steps, double delta,
                                  double* err, hipStream_t s);
hipError_t launch_to_soa(const double* src, double* dst, long long n, int d, long long np, hipStream_t s);
hipError_t launch_from_soa(const double* src, double* dst, long long n, int d, long long np, hipStream_t s);
hipError_t launch_pack_f64(const double* src, double* dst, long long n, long long ld, long long rows, int uniform,
                           hipStream_t s);
hipError_t launch_absmax(const double* A64, long long count, double* out, hipStream_t s);
hipError_t launch_pack_fmt(const double* A64, void* dst, int fmt, double inv_scale, long long count, hipStream_t s);
hipError_t launch_rowsum(const void* A, int fmt, double scale, double* rsum, long long n, long long ld,
                         hipStream_t s);

}  // namespace bs32
