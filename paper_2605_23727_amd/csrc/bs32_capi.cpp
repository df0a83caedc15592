// bs32_capi.cpp -- C ABI and host orchestration of the gfx950 BS3(2) solver.
//
// A solve runs from device-resident state: the control block (t, h, counters,
// status, FSAL and solution buffer indices) lives in device memory and only the
// single-workgroup finalize kernel updates it.  The host enqueues attempts in
// chunks (replayed from captured HIP graphs), reads the control block back once
// per chunk, and enforces the wall-clock failure conditions of Sec. 2.2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/bs32.h"
#include "bs32_internal.hpp"
#include "bs32_mlp.hpp"

using namespace bs32;

namespace {

constexpr int kNumFmt = 6;

// per-format vector-operand split (reading of the reduced-precision contraction)
struct VecSplit {
  int vfmt, terms, shift;
  double vmax;
};
VecSplit vec_split(int fmt) {
  switch (fmt) {
    case F_F32: return {F_F32, 2, 24, 3.0e38};
    case F_BF16:
    case F_BF16X2: return {F_BF16, 2, 8, 3.0e38};
    case F_F16: return {F_F16, 2, 11, 65504.0};
    case F_E4M3: return {F_E4M3, 3, 4, 448.0};
    default: return {F_F64, 1, 0, INFINITY};
  }
}
double fmt_max(int fmt) { return fmt == F_E4M3 ? 448.0 : 1.0; }

int mode_fmt(int mode) {
  switch (mode) {
    case BS32_PREC_RHS_FP32: return F_F32;
    case BS32_PREC_RHS_BF16: return F_BF16;
    case BS32_PREC_RHS_FP16: return F_F16;
    case BS32_PREC_RHS_FP8_E4M3: return F_E4M3;
    case BS32_PREC_RHS_BF16X2: return F_BF16X2;
    case BS32_PREC_PAPER_SINGLE:
    case BS32_PREC_PAPER_MIXED1:
    case BS32_PREC_PAPER_MIXED2: return F_F32;  // the recipes' single-precision pair terms
    default: return F_F64;
  }
}

// candidate tiles per format for the autotuner (the instantiated set of bs32_kernels.hip)
std::vector<Tile> candidates(int fmt) {
  int cnt = 0;
  const Tile* t = tile_candidates(fmt, &cnt);
  return std::vector<Tile>(t, t + cnt);
}

struct Geom {
  Tile t;
  int RB, nrb, KW;
  long long kn;
};

}  // namespace

struct bs32_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  bs32_options opt{};
  std::string arch;

  // system
  bool has_sys = false;
  int cur_mode = 0;  // precision mode of the current solve / evaluation
  int pairwise = 0;  // coupling evaluated pair by pair (clock / cell cycle; Kuramoto on request)
  double stim = 0.0; // I_0 of the clock / cell-cycle model
  bool uniform = false;  // pairwise system with uniform weights: no stored matrix
  int kind = 0, d = 0, m = 0;
  long long n = 0, np = 0, ld = 0;
  double gain = 1.0;
  double* param = nullptr;
  void* Aq[kNumFmt] = {};       // packed coupling per storage format (FP64 always present)
  double* rsum[kNumFmt] = {};   // row sums of the stored matrix per format
  double scale[kNumFmt] = {1, 1, 1, 1, 1, 1};
  bool tuned[kNumFmt] = {};
  Tile best[kNumFmt] = {};

  // state buffers
  bool have_state = false;
  double* X[2] = {nullptr, nullptr};
  double* Kf[2] = {nullptr, nullptr};
  double* K2 = nullptr;
  double* K3 = nullptr;
  double* Kd[3] = {nullptr, nullptr, nullptr};  // K4..K6 of the Dormand-Prince 5(4) pair
  double* V64[2] = {nullptr, nullptr};
  void* Vq[2] = {nullptr, nullptr};
  int vq_fmt = -1;  // storage format the split-operand buffers were last cleared for
  double* ep0 = nullptr;
  double* ep1 = nullptr;
  double* stage_buf = nullptr;  // d*n staging for host <-> device copies
  double* scratch = nullptr;    // small device scratch (max reductions)
  Ctl* ctlbuf[2] = {nullptr, nullptr};  // alternating device control blocks
  int par = 0;                          // index of the block holding the current state
  Ctl* ctl_d() const { return ctlbuf[par]; }
  Ctl* ctl_h[2] = {nullptr, nullptr};  // pinned host mirrors
  TraceRec* trace_d = nullptr;
  int trace_alloc = 0;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_chunk[2] = {nullptr, nullptr};

  // captured attempt chunks, keyed by the number of attempts; dropped when the launch set changes
  std::map<int, hipGraphExec_t> graphs;
  std::string graph_key;

  bs32_stats_t st{};

  // solution record (bs32_set_record): written by solves only
  double* rec = nullptr;
  long long rec_cap = 0;
  bool in_solve = false;

  struct EnsembleState* ens = nullptr;  // set by bs32_set_ensemble (bs32_ensemble.inc)
  bool shared_ens = false;              // the ensemble shares one coupling (bs32_set_shared_ensemble)
  float* mlp_w = nullptr;               // learned proposer weights (BF16 values), bs32_set_controller
};
void ens_free(bs32_ctx* c);

namespace {

bs32_status fail(bs32_ctx* c, bs32_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHK(ctx, call)                                                                              \
  do {                                                                                                 \
    hipError_t e_ = (call);                                                                            \
    if (e_ != hipSuccess) {                                                                            \
      return fail(ctx, e_ == hipErrorOutOfMemory ? BS32_ENOMEM : BS32_EDEVICE, "%s failed: %s", #call, \
                  hipGetErrorString(e_));                                                              \
    }                                                                                                  \
  } while (0)

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

long long roundup(long long x, long long m) { return (x + m - 1) / m * m; }

void ignore(hipError_t) {}

// the context's candidate tiles: pairwise systems have their own kernels
std::vector<Tile> candidates_for(const bs32_ctx* c, int fmt) {
  if (c->shared_ens) {
    int cnt = 0;
    const Tile* t = shared_tile_candidates(&cnt);
    return std::vector<Tile>(t, t + cnt);
  }
  if (c->pairwise) {
    int cnt = 0;
    const Tile* t = pair_tile_candidates(&cnt);
    return std::vector<Tile>(t, t + cnt);
  }
  return candidates(fmt);
}


void free_graphs(bs32_ctx* c) {
  for (auto& kv : c->graphs) ignore(hipGraphExecDestroy(kv.second));
  c->graphs.clear();
  c->graph_key.clear();
}

template <typename T>
void dfree(T*& p) {
  if (p) ignore(hipFree((void*)p));
  p = nullptr;
}

void free_state(bs32_ctx* c) {
  free_graphs(c);
  for (int q = 0; q < 2; ++q) {
    dfree(c->X[q]);
    dfree(c->Kf[q]);
    dfree(c->V64[q]);
    dfree(c->Vq[q]);
  }
  dfree(c->K2);
  dfree(c->K3);
  for (int q = 0; q < 3; ++q) dfree(c->Kd[q]);
  dfree(c->ep0);
  dfree(c->ep1);
  dfree(c->stage_buf);
  dfree(c->scratch);
  c->have_state = false;
}

void free_system(bs32_ctx* c) {
  free_state(c);
  for (int f = 0; f < kNumFmt; ++f) {
    dfree(c->Aq[f]);
    dfree(c->rsum[f]);
    c->scale[f] = 1.0;
    c->tuned[f] = false;
  }
  dfree(c->param);
  c->has_sys = false;
  c->rec = nullptr;  // the record's layout belongs to the system it was set for
  c->rec_cap = 0;
}

bs32_status ensure_state(bs32_ctx* c) {
  if (c->have_state) return BS32_OK;
  const long long np = c->np;
  const size_t sv = sizeof(double) * (size_t)(c->d * np);
  auto alloc0 = [&](void** p, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) e = hipMemset(*p, 0, bytes);
    return e;
  };
  for (int q = 0; q < 2; ++q) {
    HIPCHK(c, alloc0((void**)&c->X[q], sv));
    HIPCHK(c, alloc0((void**)&c->Kf[q], sv));
    HIPCHK(c, alloc0((void**)&c->V64[q], sizeof(double) * (size_t)(2 * c->ld)));
    HIPCHK(c, alloc0((void**)&c->Vq[q], sizeof(float) * 6 * (size_t)c->ld));
    c->vq_fmt = -1;
  }
  HIPCHK(c, alloc0((void**)&c->K2, sv));
  HIPCHK(c, alloc0((void**)&c->K3, sv));
  for (int q = 0; q < 3; ++q) HIPCHK(c, alloc0((void**)&c->Kd[q], sv));
  HIPCHK(c, alloc0((void**)&c->ep0, sizeof(double) * (size_t)np));
  HIPCHK(c, alloc0((void**)&c->ep1, sizeof(double) * (size_t)np));
  HIPCHK(c, alloc0((void**)&c->stage_buf, sv));
  HIPCHK(c, alloc0((void**)&c->scratch, 64));
  c->have_state = true;
  return BS32_OK;
}

Geom geometry(const bs32_ctx* c, int fmt, const Tile& t) {
  Geom g;
  g.t = t;
  g.RB = tile_rows(fmt, t);
  // row blocks that hold a row below n, and columns up to n rounded to the tile's k
  // step: the zero padding of the stored matrix beyond them is never streamed
  g.nrb = (int)((c->n + g.RB - 1) / g.RB);
  g.kn = std::min<long long>(c->ld, roundup(c->n, tile_kalign(fmt, t)));
  g.KW = (int)roundup((g.kn + t.WK - 1) / t.WK, tile_kalign(fmt, t));
  return g;
}

// The paper's recipes (Sec. 2.3, Table MP-Distrib): rows k2, k3, k4 of Single,
// Mixed1 and Mixed2; columns F, Sigma, G with 1 = single.
constexpr int kRecipe[3][3][3] = {
    {{1, 1, 1}, {1, 1, 1}, {1, 1, 1}},  // Single
    {{1, 1, 1}, {1, 1, 1}, {0, 0, 1}},  // Mixed1
    {{0, 0, 1}, {0, 0, 1}, {0, 0, 1}},  // Mixed2
};

// Table row a stage evaluates: S2 and S3 take rows k2 and k3; S4 takes k4, which
// also serves the first K1, the starting-step probe and single evaluations.
int recipe_row(int stage) { return stage == ST_S2 ? 0 : stage == ST_S3 ? 1 : 2; }

// The recipes on this path: the pair terms G are single in every recipe (A
// stored FP32, the vector operand one FP32 term); "F in S" evaluates the agent
// term and the coupling combination in FP32 and "Sigma in S" accumulates the
// interaction sum in FP32; Single also keeps the solution and stage inputs in FP32.
void set_recipe(Args& a, int mode, int stage) {
  if (mode < BS32_PREC_PAPER_SINGLE || mode > BS32_PREC_PAPER_MIXED2) return;
  const int* p = kRecipe[mode - BS32_PREC_PAPER_SINGLE][recipe_row(stage)];
  a.fsingle = p[0];
  a.sum32 = p[1];
  a.vsingle = p[2];
  a.sstate = mode == BS32_PREC_PAPER_SINGLE ? 1 : 0;
}

Args make_args(bs32_ctx* c, int fmt, const Geom& g, int stage) {
  Args a{};
  a.A = c->Aq[fmt];
  a.rsum = c->rsum[fmt];
  a.param = c->param;
  for (int q = 0; q < 2; ++q) {
    a.X[q] = c->X[q];
    a.Kf[q] = c->Kf[q];
    a.V64[q] = c->V64[q];
    a.Vq[q] = (fmt == F_F64) ? nullptr : c->Vq[q];
  }
  a.K2 = c->K2;
  a.K3 = c->K3;
  for (int q = 0; q < 3; ++q) a.Kd[q] = c->Kd[q];
  a.ep0 = c->ep0;
  a.ep1 = c->ep1;
  a.ctl = c->ctlbuf[c->par];
  a.ctl_out = c->ctlbuf[1 - c->par];
  a.rflag = (unsigned*)((char*)c->scratch + 32);
  a.mlp = c->mlp_w;
  a.trace = c->trace_d;
  a.gain = c->gain;
  a.invN = 1.0 / (double)c->n;
  a.scale = c->scale[fmt];
  const VecSplit vs = vec_split(fmt);
  a.vmax = vs.vmax;
  a.vfmt = vs.vfmt;
  a.vterms = vs.terms;
  a.vshift = vs.shift;
  set_recipe(a, c->cur_mode, stage);
  a.pairwise = c->pairwise;
  a.stim = c->stim;
  if (c->in_solve && c->rec) {
    a.rec = c->rec;
    a.rec_cap = c->rec_cap;
  }
  if (c->pairwise) {  // the pair kernels read the FP64 operand; no split terms
    a.vfmt = F_F64;
    a.vterms = 1;
    a.Vq[0] = a.Vq[1] = nullptr;
  }
  a.n = c->n;
  a.np = c->np;
  a.ld = c->ld;
  a.kind = c->kind;
  a.d = c->d;
  a.m = c->m;
  a.stage = stage;
  a.nrb = g.nrb;
  a.RB = g.RB;
  a.KW = g.KW;
  a.kn = g.kn;
  a.pair = c->opt.method;
  return a;
}

// store the matrix in a reduced format: A_stored = Q(A / s), s = 2^ceil(log2(max|A| / m))
bs32_status ensure_packed(bs32_ctx* c, int fmt) {
  if (c->Aq[fmt] || c->uniform) return BS32_OK;
  const long long count = c->np * c->ld;
  double* Aq = nullptr;
  (void)Aq;
  void* dst = nullptr;
  HIPCHK(c, hipMalloc(&dst, fmt_bytes(fmt) * (size_t)count));
  HIPCHK(c, launch_absmax((const double*)c->Aq[F_F64], count, c->scratch, c->stream));
  double mx = 0.0;
  HIPCHK(c, hipMemcpyAsync(&mx, c->scratch, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double s = 1.0;
  if (mx > 0.0 && std::isfinite(mx)) s = std::ldexp(1.0, (int)std::ceil(std::log2(mx / fmt_max(fmt))));
  HIPCHK(c, launch_pack_fmt((const double*)c->Aq[F_F64], dst, fmt, 1.0 / s, count, c->stream));
  double* rs = nullptr;
  HIPCHK(c, hipMalloc((void**)&rs, sizeof(double) * (size_t)c->np));
  HIPCHK(c, hipMemsetAsync(rs, 0, sizeof(double) * (size_t)c->np, c->stream));
  HIPCHK(c, launch_rowsum(dst, fmt, s, rs, c->n, c->ld, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->Aq[fmt] = dst;
  c->rsum[fmt] = rs;
  c->scale[fmt] = s;
  return BS32_OK;
}

// upload an agent-major vector (host or device) into SoA buffer dst
bs32_status upload_state(bs32_ctx* c, const double* y, double* dst) {
  const size_t bytes = sizeof(double) * (size_t)(c->d * c->n);
  HIPCHK(c, hipMemcpyAsync(c->stage_buf, y, bytes,
                           is_device_ptr(y) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_to_soa(c->stage_buf, dst, c->n, c->d, c->np, c->stream));
  return BS32_OK;
}

bs32_status download_state(bs32_ctx* c, const double* src, double* y) {
  const size_t bytes = sizeof(double) * (size_t)(c->d * c->n);
  HIPCHK(c, launch_from_soa(src, c->stage_buf, c->n, c->d, c->np, c->stream));
  HIPCHK(c, hipMemcpyAsync(y, c->stage_buf, bytes,
                           is_device_ptr(y) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return BS32_OK;
}

bs32_status set_ctl_scratch(bs32_ctx* c) {
  Ctl* h = c->ctl_h[0];
  std::memset(h, 0, sizeof(Ctl));
  h->status = kRunning;
  h->rtol = 1.0;
  h->atol = 1.0;
  h->trace_cap = 1;
  HIPCHK(c, hipMemcpyAsync(c->ctl_d(), h, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemsetAsync((char*)c->scratch + 32, 0, sizeof(unsigned), c->stream));
  return BS32_OK;
}

// Autotuner: time every candidate tile of the format on this system (S2 contraction,
// event-timed) and keep the fastest.  All candidates produce bit-identical sums.
bs32_status autotune(bs32_ctx* c, int fmt) {
  if (c->tuned[fmt]) return BS32_OK;
  bs32_status s = set_ctl_scratch(c);
  if (s != BS32_OK) return s;
  float best_ms = 1e30f;
  Tile best{};
  bool found = false;
  for (const Tile& t : candidates_for(c, fmt)) {
    if (!tile_supported(fmt, c->m, t)) continue;
    Geom g = geometry(c, fmt, t);
    Args a = make_args(c, fmt, g, ST_S2);
    HIPCHK(c, launch_prep(a, c->stream));
    HIPCHK(c, launch_contract(a, fmt, t, c->stream));
    HIPCHK(c, hipEventRecord(c->ev_start, c->stream));
    // 20 launches: the candidates of a small system differ by a few percent, below the
    // spread of a handful of launches
    for (int r = 0; r < 20; ++r) HIPCHK(c, launch_contract(a, fmt, t, c->stream));
    HIPCHK(c, hipEventRecord(c->ev_stop, c->stream));
    HIPCHK(c, hipEventSynchronize(c->ev_stop));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev_start, c->ev_stop));
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
      found = true;
    }
  }
  if (!found) return fail(c, BS32_EUNSUPPORTED, "no contraction tile for format %d", fmt);
  c->best[fmt] = best;
  c->tuned[fmt] = true;
  return BS32_OK;
}

// index of a tile in the context's candidate list (the value options.tile takes)
int tile_index(const bs32_ctx* c, int fmt, const Tile& t) {
  const std::vector<Tile> cand = candidates_for(c, fmt);
  for (size_t q = 0; q < cand.size(); ++q)
    if (std::memcmp(&cand[q], &t, sizeof(Tile)) == 0) return (int)q;
  return -1;
}

// picks the tile: explicit option index into the candidate list, else the autotuned one
bs32_status prepare(bs32_ctx* c, int mode, Geom* g, int* fmt) {
  if (!c->has_sys) return fail(c, BS32_ESTATE, "no system set");
  if (mode < 0 || mode > BS32_PREC_RHS_BF16X2) return fail(c, BS32_EINVAL, "unknown precision mode %d", mode);
  if (mode == BS32_PREC_RHS_BF16X2)
    return fail(c, BS32_EUNSUPPORTED, "BF16-pair storage serves the shared-coupling product (bs32_set_shared_ensemble)");
  if (c->pairwise && mode >= BS32_PREC_RHS_FP32 && mode <= BS32_PREC_RHS_FP8_E4M3)
    return fail(c, BS32_EUNSUPPORTED, "pairwise couplings have no stored-matrix formats (modes 0, 5-7)");
  *fmt = mode_fmt(mode);
  c->cur_mode = mode;
  bs32_status s = ensure_state(c);
  if (s != BS32_OK) return s;
  s = ensure_packed(c, *fmt);
  if (s != BS32_OK) return s;
  Tile t;
  const std::vector<Tile> cand = candidates_for(c, *fmt);
  if (c->opt.tile >= 0) {
    if (c->opt.tile >= (int)cand.size()) return fail(c, BS32_EINVAL, "tile index %d out of range", c->opt.tile);
    t = cand[(size_t)c->opt.tile];
  } else {
    s = autotune(c, *fmt);
    if (s != BS32_OK) return s;
    t = c->best[*fmt];
  }
  *g = geometry(c, *fmt, t);
  // The contraction reads the operand terms over the padded row length, where A is
  // zero; bytes another format left in the padding could decode as Inf or NaN
  // (0 * Inf = NaN), so the buffers start from zero whenever the format changes.
  if (*fmt != F_F64 && c->vq_fmt != *fmt) {
    for (int q = 0; q < 2; ++q) HIPCHK(c, hipMemsetAsync(c->Vq[q], 0, sizeof(float) * 6 * (size_t)c->ld, c->stream));
    c->vq_fmt = *fmt;
  }
  char key[128];
  snprintf(key, sizeof key, "%d/%d/%d/%d/%d/%d/%d/%d/%p/%p/%lld/%d", mode, t.R, t.WR, t.WK, t.U, t.NT, t.MM, t.EW,
           (void*)c->trace_d, (void*)(c->in_solve ? c->rec : nullptr), c->rec_cap, c->opt.method);
  if (c->graph_key != key) {
    free_graphs(c);
    c->graph_key = key;
  }
  return BS32_OK;
}

hipError_t enqueue_attempt(bs32_ctx* c, int fmt, const Geom& g) {
  hipError_t e;
  Args a{};
  if (c->opt.method != BS32_METHOD_BS32) {  // Dormand-Prince 5(4) or Fehlberg 4(5): six contractions
    for (int st = ST_D2; st <= ST_D7; ++st) {
      a = make_args(c, fmt, g, st);
      if ((e = launch_contract(a, fmt, g.t, c->stream)) != hipSuccess) return e;
    }
  } else {
    for (int st : {ST_S2, ST_S3, ST_S4}) {  // each stage with its own recipe row (Table MP-Distrib)
      a = make_args(c, fmt, g, st);
      if ((e = launch_contract(a, fmt, g.t, c->stream)) != hipSuccess) return e;
    }
  }
  e = launch_finalize(a, c->stream);
  c->par ^= 1;  // the finalize wrote the other control block
  return e;
}

bs32_status run_chunk(bs32_ctx* c, int fmt, const Geom& g, int attempts) {
  if (!c->opt.use_graph) {
    for (int q = 0; q < attempts; ++q) HIPCHK(c, enqueue_attempt(c, fmt, g));
    return BS32_OK;
  }
  // an even number of attempts flips the control block an even number of times, so
  // a captured chunk is replayable whenever it starts from the same block
  const int key = attempts * 2 + c->par;
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    hipGraph_t graph;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int q = 0; q < attempts && e == hipSuccess; ++q) e = enqueue_attempt(c, fmt, g);
    const hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
    if (e != hipSuccess) return fail(c, BS32_EDEVICE, "launch during capture failed: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(c, BS32_EDEVICE, "graph capture failed: %s", hipGetErrorString(e2));
    hipGraphExec_t ex;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    ignore(hipGraphDestroy(graph));
    if (e != hipSuccess) return fail(c, BS32_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    it = c->graphs.emplace(key, ex).first;
  } else {
    c->par ^= (attempts & 1);
  }
  HIPCHK(c, hipGraphLaunch(it->second, c->stream));
  return BS32_OK;
}

bs32_status ens_time_contraction(bs32_ctx* c, int mode, int repeat, double* avg_ms);  // bs32_ensemble.inc
int ens_vcols(const bs32_ctx* c);                                                     // bs32_ensemble.inc

}  // namespace

extern "C" {

bs32_status bs32_default_options(bs32_options* o) {
  if (!o) return BS32_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->i_max = 100000;
  o->time_limit_s = 5400.0;
  o->slow_limit_s = 2700.0;
  o->safety = 0.9;
  o->facmin = 0.2;
  o->facmax = 5.0;
  o->use_graph = 1;
  o->trace_cap = 65536;
  o->tile = -1;
  return BS32_OK;
}

bs32_status bs32_recipe_row(int mode, int stage_row, int32_t flags[3]) {
  if (!flags || mode < BS32_PREC_PAPER_SINGLE || mode > BS32_PREC_PAPER_MIXED2 || stage_row < 0 || stage_row > 2)
    return BS32_EINVAL;
  const int stage = stage_row == 0 ? ST_S2 : stage_row == 1 ? ST_S3 : ST_S4;
  Args a{};
  set_recipe(a, mode, stage);
  flags[0] = a.fsingle;
  flags[1] = a.sum32;
  flags[2] = a.vsingle;
  return BS32_OK;
}

bs32_status bs32_create(bs32_ctx** out, int device, void* hip_stream) {
  if (!out) return BS32_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return BS32_EDEVICE;
  if (device < 0 || device >= ndev) return BS32_EINVAL;
  bs32_ctx* c = new bs32_ctx();
  c->device = device;
  bs32_default_options(&c->opt);
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return BS32_EDEVICE;
  }
  hipDeviceProp_t pr;
  if (hipGetDeviceProperties(&pr, device) == hipSuccess) c->arch = pr.gcnArchName;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return BS32_EDEVICE;
    }
    c->own_stream = true;
  }
  const bool ok = hipMalloc((void**)&c->ctlbuf[0], sizeof(Ctl)) == hipSuccess &&
                  hipMalloc((void**)&c->ctlbuf[1], sizeof(Ctl)) == hipSuccess &&
                  hipHostMalloc((void**)&c->ctl_h[0], sizeof(Ctl), hipHostMallocDefault) == hipSuccess &&
                  hipHostMalloc((void**)&c->ctl_h[1], sizeof(Ctl), hipHostMallocDefault) == hipSuccess &&
                  hipEventCreate(&c->ev_start) == hipSuccess && hipEventCreate(&c->ev_stop) == hipSuccess &&
                  hipEventCreateWithFlags(&c->ev_chunk[0], hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->ev_chunk[1], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    bs32_destroy(c);
    return BS32_ENOMEM;
  }
  // the allocation-free gradient's scratch array: this device's copy, looked up once
  if (noalloc_bind(device) != hipSuccess) {
    bs32_destroy(c);
    return BS32_EDEVICE;
  }
  std::memset(c->ctl_h[0], 0, sizeof(Ctl));
  std::memset(c->ctl_h[1], 0, sizeof(Ctl));
  *out = c;
  return BS32_OK;
}

void bs32_destroy(bs32_ctx* c) {
  if (!c) return;
  ignore(hipSetDevice(c->device));
  if (c->stream) ignore(hipStreamSynchronize(c->stream));
  ens_free(c);
  free_system(c);
  dfree(c->ctlbuf[0]);
  dfree(c->ctlbuf[1]);
  dfree(c->trace_d);
  dfree(c->mlp_w);
  for (int q = 0; q < 2; ++q)
    if (c->ctl_h[q]) ignore(hipHostFree(c->ctl_h[q]));
  if (c->ev_start) ignore(hipEventDestroy(c->ev_start));
  if (c->ev_stop) ignore(hipEventDestroy(c->ev_stop));
  for (int q = 0; q < 2; ++q)
    if (c->ev_chunk[q]) ignore(hipEventDestroy(c->ev_chunk[q]));
  if (c->own_stream && c->stream) ignore(hipStreamDestroy(c->stream));
  delete c;
}

const char* bs32_last_error(const bs32_ctx* c) { return c ? c->err.c_str() : "null context"; }

bs32_status bs32_set_options(bs32_ctx* c, const bs32_options* o) {
  if (!c || !o) return fail(c, BS32_EINVAL, "null argument");
  if (o->i_max <= 0) return fail(c, BS32_EINVAL, "i_max must be positive");
  if (!(o->safety > 0 && o->facmin > 0 && o->facmax >= 1.0 && o->facmin <= 1.0))
    return fail(c, BS32_EINVAL, "controller constants out of range");
  if (o->trace && (o->trace_cap <= 0 || o->trace_cap > (1 << 26))) return fail(c, BS32_EINVAL, "bad trace_cap");
  if (o->fixed_step && !(o->h0 > 0)) return fail(c, BS32_EINVAL, "fixed_step needs h0 > 0");
  if (o->controller != 0 && o->controller != 1) return fail(c, BS32_EINVAL, "unknown controller %d", o->controller);
  if (o->controller == 1 && !c->mlp_w) return fail(c, BS32_ESTATE, "learned controller needs bs32_set_controller");
  if (o->method != BS32_METHOD_BS32 && o->method != BS32_METHOD_DP54 && o->method != BS32_METHOD_RKF45)
    return fail(c, BS32_EINVAL, "unknown method %d", o->method);
  if (o->ensemble_launch != 0 && o->ensemble_launch != 1)
    return fail(c, BS32_EINVAL, "ensemble_launch must be 0 or 1");
  c->opt = *o;
  free_graphs(c);
  return BS32_OK;
}

bs32_status bs32_set_system(bs32_ctx* c, const bs32_system_desc* sd) {
  if (!c || !sd) return fail(c, BS32_EINVAL, "null argument");
  const int d = dim_of(sd->kind);
  if (d == 0) return fail(c, BS32_EINVAL, "unknown system kind %d", sd->kind);
  if (sd->n < 1 || sd->n > (1LL << 20)) return fail(c, BS32_EINVAL, "n out of range: %lld", (long long)sd->n);
  if (!std::isfinite(sd->gain)) return fail(c, BS32_EINVAL, "gain must be finite");
  if (!std::isfinite(sd->stimulus)) return fail(c, BS32_EINVAL, "stimulus must be finite");
  if (sd->pairwise != 0 && sd->pairwise != 1) return fail(c, BS32_EINVAL, "pairwise must be 0 or 1");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  ens_free(c);
  free_system(c);
  c->kind = sd->kind;
  c->d = d;
  c->pairwise = (sd->kind == BS32_SYS_CLOCK4 || (sd->kind == BS32_SYS_KURAMOTO && sd->pairwise)) ? 1 : 0;
  c->stim = sd->stimulus;
  c->uniform = c->pairwise && sd->coupling == nullptr;
  c->m = vcols_of(sd->kind, c->pairwise);
  c->n = sd->n;
  c->gain = sd->gain;
  c->np = roundup(c->n, 256);
  c->ld = roundup(c->n, 256);
  bs32_status s = ensure_state(c);
  if (s != BS32_OK) return s;
  double* tmp = nullptr;
  if (!c->uniform) {  // a pairwise system with uniform weights stores no matrix
    const size_t abytes = sizeof(double) * (size_t)c->np * (size_t)c->ld;
    HIPCHK(c, hipMalloc(&c->Aq[F_F64], abytes));
    const double* src = sd->coupling;
    if (src && !is_device_ptr(src)) {
      HIPCHK(c, hipMalloc((void**)&tmp, sizeof(double) * (size_t)(c->n * c->n)));
      HIPCHK(c, hipMemcpyAsync(tmp, src, sizeof(double) * (size_t)(c->n * c->n), hipMemcpyHostToDevice, c->stream));
      src = tmp;
    }
    HIPCHK(c, launch_pack_f64(src, (double*)c->Aq[F_F64], c->n, c->ld, c->np, src == nullptr ? 1 : 0, c->stream));
    HIPCHK(c, hipMalloc((void**)&c->rsum[F_F64], sizeof(double) * (size_t)c->np));
    HIPCHK(c, hipMemsetAsync(c->rsum[F_F64], 0, sizeof(double) * (size_t)c->np, c->stream));
    HIPCHK(c, launch_rowsum(c->Aq[F_F64], F_F64, 1.0, c->rsum[F_F64], c->n, c->ld, c->stream));
  }
  HIPCHK(c, hipMalloc((void**)&c->param, sizeof(double) * (size_t)c->np));
  std::vector<double> ones;
  if (sd->agent_param) {
    HIPCHK(c, hipMemcpyAsync(c->param, sd->agent_param, sizeof(double) * (size_t)c->n,
                             is_device_ptr(sd->agent_param) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             c->stream));
  } else {
    ones.assign((size_t)c->n, 1.0);
    HIPCHK(c, hipMemcpyAsync(c->param, ones.data(), sizeof(double) * (size_t)c->n, hipMemcpyHostToDevice,
                             c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (tmp) ignore(hipFree(tmp));
  c->has_sys = true;
  std::memset(&c->st, 0, sizeof(c->st));
  return BS32_OK;
}

bs32_status bs32_stats(const bs32_ctx* c, bs32_stats_t* out) {
  if (!c || !out) return BS32_EINVAL;
  *out = c->st;
  return BS32_OK;
}

bs32_status bs32_rhs(bs32_ctx* c, const double* y, int mode, int repeat, double* f_out) {
  if (!c || !y || !f_out) return fail(c, BS32_EINVAL, "null argument");
  if (repeat < 1) return fail(c, BS32_EINVAL, "repeat must be >= 1");
  HIPCHK(c, hipSetDevice(c->device));
  Geom g;
  int fmt;
  bs32_status s = prepare(c, mode, &g, &fmt);
  if (s != BS32_OK) return s;
  s = set_ctl_scratch(c);
  if (s != BS32_OK) return s;
  s = upload_state(c, y, c->X[0]);
  if (s != BS32_OK) return s;
  Args a = make_args(c, fmt, g, ST_RHS);
  for (int r = 0; r < repeat; ++r) {
    HIPCHK(c, launch_prep(a, c->stream));
    HIPCHK(c, launch_contract(a, fmt, g.t, c->stream));
  }
  unsigned rflag = 0;
  HIPCHK(c, hipMemcpyAsync(&rflag, (char*)c->scratch + 32, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  s = download_state(c, c->Kf[0], f_out);
  if (s != BS32_OK) return s;
  if (rflag) return fail(c, BS32_RANGE, "vector operand outside the storage format's range");
  return BS32_OK;
}

bs32_status bs32_time_contraction(bs32_ctx* c, int mode, int repeat, double* avg_ms) {
  if (!c || !avg_ms) return fail(c, BS32_EINVAL, "null argument");
  if (repeat < 1) return fail(c, BS32_EINVAL, "repeat must be >= 1");
  HIPCHK(c, hipSetDevice(c->device));
  if (c->ens) return ens_time_contraction(c, mode, repeat, avg_ms);
  Geom g;
  int fmt;
  bs32_status s = prepare(c, mode, &g, &fmt);
  if (s != BS32_OK) return s;
  s = set_ctl_scratch(c);
  if (s != BS32_OK) return s;
  Args a = make_args(c, fmt, g, ST_S2);
  HIPCHK(c, launch_prep(a, c->stream));
  HIPCHK(c, launch_contract(a, fmt, g.t, c->stream));  // warm-up
  HIPCHK(c, hipEventRecord(c->ev_start, c->stream));
  for (int r = 0; r < repeat; ++r) HIPCHK(c, launch_contract(a, fmt, g.t, c->stream));
  HIPCHK(c, hipEventRecord(c->ev_stop, c->stream));
  HIPCHK(c, hipEventSynchronize(c->ev_stop));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev_start, c->ev_stop));
  *avg_ms = (double)ms / repeat;
  return BS32_OK;
}

bs32_status bs32_kernel_name(bs32_ctx* c, int mode, int tile, char* buf, size_t cap) {
  if (!c || !buf || cap == 0) return fail(c, BS32_EINVAL, "null argument");
  if (mode < 0 || mode > BS32_PREC_RHS_BF16X2) return fail(c, BS32_EINVAL, "unknown precision mode %d", mode);
  int m = 0;
  if (c->has_sys) m = c->m;
  else if (c->ens) m = ens_vcols(c);
  else return fail(c, BS32_ESTATE, "no system set");
  if (c->pairwise && mode != BS32_PREC_FP64) mode = BS32_PREC_PAPER_MIXED2;  // every recipe: the FP32 pair term
  const int fmt = mode_fmt(mode);
  const std::vector<Tile> cand = candidates_for(c, fmt);
  if (tile < 0 || tile >= (int)cand.size()) return fail(c, BS32_EINVAL, "tile index %d out of range", tile);
  const int r = kernel_name(fmt, m, cand[(size_t)tile], buf, cap);
  if (r < 0) return fail(c, BS32_EUNSUPPORTED, "tile %d is not instantiated for this system", tile);
  if ((size_t)r >= cap) return fail(c, BS32_EINVAL, "buffer too small");
  return BS32_OK;
}

bs32_status bs32_get_packed_coupling(bs32_ctx* c, int mode, void* dst, size_t bytes, double* scale) {
  if (!c || !dst || !scale) return fail(c, BS32_EINVAL, "null argument");
  if (!c->has_sys) return fail(c, BS32_ESTATE, "no system set");
  if (mode < 0 || (mode > BS32_PREC_RHS_FP8_E4M3 && mode != BS32_PREC_RHS_BF16X2))
    return fail(c, BS32_EINVAL, "mode %d has no packed matrix", mode);
  if (c->uniform) return fail(c, BS32_ESTATE, "a pairwise system with uniform weights stores no matrix");
  HIPCHK(c, hipSetDevice(c->device));
  const int fmt = mode_fmt(mode);
  const size_t es = fmt_bytes(fmt);
  if (bytes < es * (size_t)(c->n * c->n)) return fail(c, BS32_EINVAL, "buffer too small");
  bs32_status s = ensure_state(c);
  if (s != BS32_OK) return s;
  s = ensure_packed(c, fmt);
  if (s != BS32_OK) return s;
  if (fmt == F_BF16X2) {  // the hi plane, then the remainder plane, each N x N BF16
    const size_t plane = 2 * (size_t)c->np * (size_t)c->ld;
    for (int q = 0; q < 2; ++q)
      HIPCHK(c, hipMemcpy2DAsync((char*)dst + q * 2 * (size_t)(c->n * c->n), 2 * (size_t)c->n,
                                 (const char*)c->Aq[fmt] + q * plane, 2 * (size_t)c->ld, 2 * (size_t)c->n, (size_t)c->n,
                                 hipMemcpyDeviceToHost, c->stream));
  } else {
    HIPCHK(c, hipMemcpy2DAsync(dst, es * (size_t)c->n, c->Aq[fmt], es * (size_t)c->ld, es * (size_t)c->n,
                               (size_t)c->n, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *scale = c->scale[fmt];
  return BS32_OK;
}

bs32_status bs32_solve(bs32_ctx* c, const double* y0, double t0, double t1, double rtol, double atol, int mode,
                       double* y_out) {
  if (!c || !y0 || !y_out) return fail(c, BS32_EINVAL, "null argument");
  if (!(rtol > 0.0) || !(atol >= 0.0) || !std::isfinite(rtol) || !std::isfinite(atol))
    return fail(c, BS32_EINVAL, "need rtol > 0 and atol >= 0");
  if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 >= t0)) return fail(c, BS32_EINVAL, "need t1 >= t0");
  HIPCHK(c, hipSetDevice(c->device));
  struct InSolve {  // the record is written by this solve's kernels only
    bs32_ctx* c;
    explicit InSolve(bs32_ctx* x) : c(x) { c->in_solve = true; }
    ~InSolve() { c->in_solve = false; }
  } in_solve(c);
  const bs32_options& o = c->opt;
  if (o.method != BS32_METHOD_BS32) {
    if (mode >= BS32_PREC_PAPER_SINGLE)
      return fail(c, BS32_EUNSUPPORTED, "the paper's recipes are defined for the Bogacki-Shampine stages");
    if (o.controller == 1) return fail(c, BS32_EUNSUPPORTED, "the learned proposer serves the Bogacki-Shampine pair");
  }
  if (o.trace && c->trace_alloc < o.trace_cap) {
    dfree(c->trace_d);
    HIPCHK(c, hipMalloc((void**)&c->trace_d, sizeof(TraceRec) * (size_t)o.trace_cap));
    c->trace_alloc = o.trace_cap;
  }
  Geom g;
  int fmt;
  bs32_status s = prepare(c, mode, &g, &fmt);
  if (s != BS32_OK) return s;
  const auto wall0 = std::chrono::steady_clock::now();
  std::memset(&c->st, 0, sizeof(c->st));
  c->st.mode = mode;
  if (t1 == t0) {
    if (y_out != y0) {
      const size_t bytes = sizeof(double) * (size_t)(c->d * c->n);
      const bool di = is_device_ptr(y0), dout = is_device_ptr(y_out);
      HIPCHK(c, hipMemcpyAsync(y_out, y0, bytes,
                               di ? (dout ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost)
                                  : (dout ? hipMemcpyHostToDevice : hipMemcpyHostToHost),
                               c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->st.t_reached = t0;
    c->st.status = BS32_OK;
    return BS32_OK;
  }
  Ctl* h = c->ctl_h[0];
  std::memset(h, 0, sizeof(Ctl));
  h->t = t0;
  h->t0 = t0;
  h->t1 = t1;
  h->rtol = rtol;
  h->atol = atol;
  h->h_max = o.h_max > 0.0 ? o.h_max : 0.1 * std::fabs(t1 - t0);
  // 100 eps of the format holding h (Sec. 2.2): FP32 in the Single recipe, FP64 otherwise
  h->h_min = 100.0 * (mode == BS32_PREC_PAPER_SINGLE ? 1.1920928955078125e-07 : 2.220446049250313e-16);
  h->snap = 4.0 * 2.220446049250313e-16 * std::fabs(t1);
  h->safety = o.safety;
  h->facmin = o.facmin;
  h->facmax = o.facmax;
  h->h_min_seen = INFINITY;
  h->h0user = o.h0 > 0.0 ? o.h0 : 0.0;
  h->i_max = o.i_max;
  h->status = kRunning;
  h->fixed_step = o.fixed_step;
  h->trace_on = o.trace ? 1 : 0;
  h->trace_cap = o.trace ? o.trace_cap : 1;
  h->use_mlp = (o.controller == 1 && c->mlp_w) ? 1 : 0;
  h->method = o.method;
  c->par = 0;
  HIPCHK(c, hipMemcpyAsync(c->ctl_d(), h, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemsetAsync((char*)c->scratch + 32, 0, sizeof(unsigned), c->stream));
  s = upload_state(c, y0, c->X[0]);
  if (s != BS32_OK) return s;
  if (mode == BS32_PREC_PAPER_SINGLE) HIPCHK(c, launch_round_f32(c->X[0], (long long)c->d * c->np, c->stream));
  HIPCHK(c, hipEventRecord(c->ev_start, c->stream));
  {
    // first stage K1 = f(t0, y0), then the starting-step probe (a2)
    Args a = make_args(c, fmt, g, ST_INIT);
    HIPCHK(c, launch_prep(a, c->stream));
    HIPCHK(c, launch_contract(a, fmt, g.t, c->stream));
    HIPCHK(c, launch_finalize(a, c->stream));
    c->par ^= 1;
    if (!(o.h0 > 0.0)) {
      a = make_args(c, fmt, g, ST_H0);
      HIPCHK(c, launch_contract(a, fmt, g.t, c->stream));
      HIPCHK(c, launch_finalize(a, c->stream));
      c->par ^= 1;
    }
  }
  // attempt chunks; one chunk is always in flight ahead of the one being checked,
  // and its kernels return at once when the solve is over
  int chunk = 2;
  int k = 0;
  s = run_chunk(c, fmt, g, chunk);
  if (s != BS32_OK) return s;
  HIPCHK(c, hipMemcpyAsync(c->ctl_h[0], c->ctl_d(),sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipEventRecord(c->ev_chunk[0], c->stream));
  int final_status = kRunning;
  while (true) {
    s = run_chunk(c, fmt, g, chunk);
    if (s != BS32_OK) return s;
    HIPCHK(c, hipMemcpyAsync(c->ctl_h[(k + 1) & 1], c->ctl_d(),sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipEventRecord(c->ev_chunk[(k + 1) & 1], c->stream));
    HIPCHK(c, hipEventSynchronize(c->ev_chunk[k & 1]));
    const Ctl* cur = c->ctl_h[k & 1];
    if (cur->status != kRunning) break;
    // wall-clock failure conditions of Sec. 2.2
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
    const double frac = (cur->t - t0) / (t1 - t0);
    if (o.time_limit_s > 0 && el > o.time_limit_s) {
      final_status = BS32_TIMEOUT;
      break;
    }
    if (o.slow_limit_s > 0 && el > o.slow_limit_s && frac < 0.1) {
      final_status = BS32_TOO_SLOW;
      break;
    }
    // size the next chunk from the attempts the current step size suggests are left
    const double est = (cur->h > 0) ? (t1 - cur->t) / cur->h : 1e9;
    const int want = (int)std::min(64.0, std::max(2.0, std::ceil(0.5 * est)));
    int p2 = 2;
    while (p2 < want) p2 <<= 1;
    chunk = std::min(64, std::max(2, std::min(p2, chunk * 2)));
    ++k;
  }
  if (final_status != kRunning) HIPCHK(c, launch_set_status(c->ctl_d(),final_status, c->stream));
  HIPCHK(c, hipEventRecord(c->ev_stop, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->ctl_h[0], c->ctl_d(),sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const Ctl fin = *c->ctl_h[0];
  s = download_state(c, c->X[fin.xi], y_out);
  if (s != BS32_OK) return s;
  float kms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&kms, c->ev_start, c->ev_stop));
  c->st.n_accept = fin.n_accept;
  c->st.n_reject = fin.n_reject;
  c->st.n_fev = fin.n_fev;
  c->st.pair_interactions = (double)fin.n_fev * (double)c->n * (double)c->n;
  c->st.t_reached = fin.t;
  c->st.h_last = fin.h_last;
  c->st.h_min_seen = fin.h_min_seen;
  c->st.err_last = fin.err;
  c->st.n_learned = fin.n_mlp;
  c->st.tile = tile_index(c, fmt, g.t);
  c->st.kernel_ms = kms;
  c->st.status = fin.status;
  c->st.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
  return (bs32_status)fin.status;
}

bs32_status bs32_set_record(bs32_ctx* c, double* states, int64_t cap) {
  if (!c) return BS32_EINVAL;
  if (cap < 0) return fail(c, BS32_EINVAL, "record capacity must be >= 0");
  if (!states || cap == 0) {
    c->rec = nullptr;
    c->rec_cap = 0;
    return BS32_OK;
  }
  if (!c->has_sys || c->ens) return fail(c, BS32_ESTATE, "the record needs a single system (bs32_set_system)");
  if (!is_device_ptr(states)) return fail(c, BS32_EINVAL, "the record must be device memory");
  c->rec = states;
  c->rec_cap = cap;
  return BS32_OK;
}

bs32_status bs32_lco_flow(bs32_ctx* c, int64_t n, int64_t count, const double* X, const double* h, double* out) {
  if (!c) return BS32_EINVAL;
  if (n < 1 || n > (1LL << 30)) return fail(c, BS32_EINVAL, "n out of range: %lld", (long long)n);
  if (count < 0 || count > 0x7fffffffLL) return fail(c, BS32_EINVAL, "count out of range");
  if (count == 0) return BS32_OK;
  if (!X || !h || !out) return fail(c, BS32_EINVAL, "null argument");
  if (!is_device_ptr(X) || !is_device_ptr(h) || !is_device_ptr(out))
    return fail(c, BS32_EINVAL, "states, steps and output must be device memory");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, launch_lco_flow(X, h, n, count, out, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return BS32_OK;
}

bs32_status bs32_lco_local_error(bs32_ctx* c, int64_t n, int64_t steps, const double* states, const double* h,
                                 double delta, double* err) {
  if (!c) return BS32_EINVAL;
  if (n < 1 || n > (1LL << 30)) return fail(c, BS32_EINVAL, "n out of range: %lld", (long long)n);
  if (steps < 0 || steps > 0x7fffffffLL) return fail(c, BS32_EINVAL, "steps out of range");
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(c, BS32_EINVAL, "delta must be positive and finite");
  if (steps == 0) return BS32_OK;
  if (!states || !h || !err) return fail(c, BS32_EINVAL, "null argument");
  if (!is_device_ptr(states) || !is_device_ptr(h) || !is_device_ptr(err))
    return fail(c, BS32_EINVAL, "states, steps and output must be device memory");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, launch_lco_local_error(states, h, n, steps, delta, err, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return BS32_OK;
}

bs32_status bs32_get_trace(bs32_ctx* c, bs32_trace_rec* buf, size_t cap, size_t* n_records) {
  if (!c || !n_records || (cap && !buf)) return fail(c, BS32_EINVAL, "null argument");
  *n_records = 0;
  if (!c->trace_d || !c->opt.trace) return BS32_OK;
  const long long total = c->ctl_h[0]->trace_n;
  const long long ring = c->opt.trace_cap;
  const long long have = std::min(total, ring);
  const long long first = total - have;
  std::vector<TraceRec> tmp((size_t)ring);
  HIPCHK(c, hipMemcpy(tmp.data(), c->trace_d, sizeof(TraceRec) * (size_t)ring, hipMemcpyDeviceToHost));
  size_t outn = 0;
  for (long long q = first; q < total && outn < cap; ++q) {
    const TraceRec& r = tmp[(size_t)(q % ring)];
    buf[outn].t = r.t;
    buf[outn].h = r.h;
    buf[outn].err = r.err;
    buf[outn].fnorm = r.fnorm;
    buf[outn].accepted = r.accepted;
    buf[outn].proposer = r.proposer;
    ++outn;
  }
  *n_records = outn;
  return BS32_OK;
}

}  // extern "C"

#include "bs32_ensemble.inc"
#include "bs32_mlp.inc"
