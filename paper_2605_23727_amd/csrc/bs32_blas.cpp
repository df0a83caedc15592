// Plain library product for the shared-coupling ensembles: P = A [V_1 ... V_B]
// with 16-bit A and operand terms and FP32 accumulation and output (hipBLASLt).
// The per-instance row epilogue stays in the library's own kernel, which reads P.
//
// Layouts (row-major as the rest of the library holds them):
//   A   rows x ld, 16-bit, row i contiguous over k;
//   B   m operand columns, column j contiguous over k at B + j*ld;
//   P   rows x m FP32, row stride m:  P[i][j] = sum_k A[i][k] B[j][k].
// In hipBLASLt's column-major terms this is D (m x rows) = B^T (m x ld) . A^T
// (ld x rows): matrix "A" of the call is B read transposed, matrix "B" is A.

#include <hip/hip_runtime.h>
#include <hipblaslt/hipblaslt.h>

#include <cstdio>
#include <map>
#include <tuple>

#include "bs32_internal.hpp"

namespace bs32 {

namespace {

struct Plan {
  hipblasLtMatmulDesc_t desc = nullptr;
  hipblasLtMatrixLayout_t la = nullptr, lb = nullptr, lc = nullptr;
  hipblasLtMatmulAlgo_t algo{};
  size_t ws = 0;
};

}  // namespace

struct BlasProduct {
  hipblasLtHandle_t h = nullptr;
  std::map<std::tuple<int, long long, long long, long long>, Plan> plans;
  void* ws = nullptr;
  size_t ws_bytes = 0;
};

static constexpr size_t kMaxWorkspace = 64u << 20;

BlasProduct* blas_create(char* err, size_t cap) {
  BlasProduct* b = new BlasProduct();
  const hipblasStatus_t s = hipblasLtCreate(&b->h);
  if (s != HIPBLAS_STATUS_SUCCESS) {
    snprintf(err, cap, "hipblasLtCreate failed (status %d)", (int)s);
    delete b;
    return nullptr;
  }
  return b;
}

void blas_destroy(BlasProduct* b) {
  if (!b) return;
  for (auto& kv : b->plans) {
    Plan& p = kv.second;
    if (p.la) hipblasLtMatrixLayoutDestroy(p.la);
    if (p.lb) hipblasLtMatrixLayoutDestroy(p.lb);
    if (p.lc) hipblasLtMatrixLayoutDestroy(p.lc);
    if (p.desc) hipblasLtMatmulDescDestroy(p.desc);
  }
  if (b->ws) (void)hipFree(b->ws);
  if (b->h) hipblasLtDestroy(b->h);
  delete b;
}

// descriptors and the heuristic's first algorithm for one shape, made once
static bool plan_for(BlasProduct* b, int fmt, long long rows, long long m, long long ld, Plan** out, char* err,
                     size_t cap) {
  const auto key = std::make_tuple(fmt, rows, m, ld);
  auto it = b->plans.find(key);
  if (it != b->plans.end()) {
    *out = &it->second;
    return true;
  }
  const hipDataType in = fmt == F_F16 ? HIP_R_16F : HIP_R_16BF;
  Plan p;
  hipblasStatus_t s = hipblasLtMatmulDescCreate(&p.desc, HIPBLAS_COMPUTE_32F, HIP_R_32F);
  const int32_t opT = HIPBLAS_OP_T, opN = HIPBLAS_OP_N;
  if (s == HIPBLAS_STATUS_SUCCESS)
    s = hipblasLtMatmulDescSetAttribute(p.desc, HIPBLASLT_MATMUL_DESC_TRANSA, &opT, sizeof(opT));
  if (s == HIPBLAS_STATUS_SUCCESS)
    s = hipblasLtMatmulDescSetAttribute(p.desc, HIPBLASLT_MATMUL_DESC_TRANSB, &opN, sizeof(opN));
  if (s == HIPBLAS_STATUS_SUCCESS) s = hipblasLtMatrixLayoutCreate(&p.la, in, (uint64_t)ld, (uint64_t)m, ld);
  if (s == HIPBLAS_STATUS_SUCCESS) s = hipblasLtMatrixLayoutCreate(&p.lb, in, (uint64_t)ld, (uint64_t)rows, ld);
  if (s == HIPBLAS_STATUS_SUCCESS) s = hipblasLtMatrixLayoutCreate(&p.lc, HIP_R_32F, (uint64_t)m, (uint64_t)rows, m);
  hipblasLtMatmulPreference_t pref = nullptr;
  if (s == HIPBLAS_STATUS_SUCCESS) s = hipblasLtMatmulPreferenceCreate(&pref);
  const uint64_t wsmax = kMaxWorkspace;
  if (s == HIPBLAS_STATUS_SUCCESS)
    s = hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &wsmax, sizeof(wsmax));
  hipblasLtMatmulHeuristicResult_t res[4];
  int nres = 0;
  if (s == HIPBLAS_STATUS_SUCCESS)
    s = hipblasLtMatmulAlgoGetHeuristic(b->h, p.desc, p.la, p.lb, p.lc, p.lc, pref, 4, res, &nres);
  if (pref) hipblasLtMatmulPreferenceDestroy(pref);
  if (s != HIPBLAS_STATUS_SUCCESS || nres < 1) {
    snprintf(err, cap, "hipBLASLt has no algorithm for a %lld x %lld x %lld product (status %d)", m, rows, ld,
             (int)s);
    if (p.la) hipblasLtMatrixLayoutDestroy(p.la);
    if (p.lb) hipblasLtMatrixLayoutDestroy(p.lb);
    if (p.lc) hipblasLtMatrixLayoutDestroy(p.lc);
    if (p.desc) hipblasLtMatmulDescDestroy(p.desc);
    return false;
  }
  p.algo = res[0].algo;
  p.ws = res[0].workspaceSize;
  *out = &(b->plans[key] = p);
  return true;
}

// P (rows x m, FP32) = A (rows x ld) B^T (B: m columns of ld), fmt F_BF16 or F_F16.
// Returns 0 or a negative hipBLASLt / HIP status with a message in err.  Allocates
// its workspace on first use of a shape (never inside a captured graph: the callers
// run this path eagerly).
int blas_product(BlasProduct* b, int fmt, const void* A, const void* B, long long rows, long long m, long long ld,
                 float* P, hipStream_t stream, char* err, size_t cap) {
  if (fmt != F_BF16 && fmt != F_F16) {
    snprintf(err, cap, "library product serves BF16 and FP16 storage only");
    return -1;
  }
  Plan* p = nullptr;
  if (!plan_for(b, fmt, rows, m, ld, &p, err, cap)) return -2;
  if (p->ws > b->ws_bytes) {
    if (b->ws) (void)hipFree(b->ws);
    b->ws = nullptr;
    b->ws_bytes = 0;
    const hipError_t e = hipMalloc(&b->ws, p->ws);
    if (e != hipSuccess) {
      snprintf(err, cap, "workspace of %zu bytes: %s", p->ws, hipGetErrorString(e));
      return -3;
    }
    b->ws_bytes = p->ws;
  }
  const float one = 1.0f, zero = 0.0f;
  const hipblasStatus_t s = hipblasLtMatmul(b->h, p->desc, &one, B, p->la, A, p->lb, &zero, P, p->lc, P, p->lc,
                                            &p->algo, b->ws, p->ws, stream);
  if (s != HIPBLAS_STATUS_SUCCESS) {
    snprintf(err, cap, "hipblasLtMatmul failed (status %d)", (int)s);
    return -4;
  }
  return 0;
}

}  // namespace bs32
