// The dense Gaussian sketch with a stored C (Section 3.2, eq. (eq:YCX); Section 3.3's
// Gaussian measurement matrix) as a plain library GEMM: once C (bfloat16 or OCP e4m3,
// pixel-major) and the video (split into S pixel slices of Ks: exact bfloat16, or for the
// FP8 form two exact e4m3 parts, 16 hi and lo, of each byte) are in device memory, the
// sketch is S independent products part[s] = C[:, slice s] X[slice s, :] with float32
// accumulation and float32 output, batched in one hipBLASLt call (two for FP8, the second
// adding into the first), then summed over s in float64 (reduce_gauss).  In the library's
// column-major terms, with no transposes:
//   A = Ct[s]  p x Ks,  ld p   (pixel-major C: element (r, j) at j p + r)
//   B = Xs[s]  Ks x m,  ld Ks  (frame-major video slice: element (j, t) at t Ks + j)
//   D = part[s] p x m,  ld p   (frame-major partial sketch: element (r, t) at t p + r)
#include "sketch_gemm.hpp"

#include <hipblaslt/hipblaslt.h>

namespace cdmd {
namespace blas {

constexpr int kMaxCandidates = 8;

struct SketchGemm {
  hipblasLtHandle_t handle = nullptr;
  hipblasLtMatmulDesc_t desc = nullptr;
  hipblasLtMatrixLayout_t la = nullptr, lb = nullptr, ld = nullptr;
  hipblasLtMatmulHeuristicResult_t cand[kMaxCandidates];  // the library's candidates, best guess first
  int ncand = 0, cur = 0;
  void* ws = nullptr;  // sized for the largest candidate
  size_t ws_bytes = 0;
  ~SketchGemm() {
    if (ws) (void)hipFree(ws);
    if (la) (void)hipblasLtMatrixLayoutDestroy(la);
    if (lb) (void)hipblasLtMatrixLayoutDestroy(lb);
    if (ld) (void)hipblasLtMatrixLayoutDestroy(ld);
    if (desc) (void)hipblasLtMatmulDescDestroy(desc);
    if (handle) (void)hipblasLtDestroy(handle);
  }
};

namespace {
bool batched(hipblasLtMatrixLayout_t l, int32_t S, int64_t stride) {
  return hipblasLtMatrixLayoutSetAttribute(l, HIPBLASLT_MATRIX_LAYOUT_BATCH_COUNT, &S, sizeof(S)) ==
             HIPBLAS_STATUS_SUCCESS &&
         hipblasLtMatrixLayoutSetAttribute(l, HIPBLASLT_MATRIX_LAYOUT_STRIDED_BATCH_OFFSET, &stride, sizeof(stride)) ==
             HIPBLAS_STATUS_SUCCESS;
}
}  // namespace

SketchGemm* sketch_gemm_create(int p, int64_t Ks, int64_t m, int S, int fp8, std::string* err) {
  SketchGemm* g = new SketchGemm();
  auto bad = [&](const char* what) -> SketchGemm* {
    if (err) *err = what;
    delete g;
    return nullptr;
  };
  if (hipblasLtCreate(&g->handle) != HIPBLAS_STATUS_SUCCESS) return bad("hipblasLtCreate failed");
  if (hipblasLtMatmulDescCreate(&g->desc, HIPBLAS_COMPUTE_32F, HIP_R_32F) != HIPBLAS_STATUS_SUCCESS)
    return bad("hipblasLtMatmulDescCreate failed");
  const int32_t opN = HIPBLAS_OP_N;
  if (hipblasLtMatmulDescSetAttribute(g->desc, HIPBLASLT_MATMUL_DESC_TRANSA, &opN, sizeof(opN)) !=
          HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatmulDescSetAttribute(g->desc, HIPBLASLT_MATMUL_DESC_TRANSB, &opN, sizeof(opN)) !=
          HIPBLAS_STATUS_SUCCESS)
    return bad("setting the GEMM operations failed");
  const hipDataType in = fp8 ? HIP_R_8F_E4M3 : HIP_R_16BF;  // OCP e4m3fn codes, or bfloat16
  if (hipblasLtMatrixLayoutCreate(&g->la, in, (uint64_t)p, (uint64_t)Ks, p) != HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatrixLayoutCreate(&g->lb, in, (uint64_t)Ks, (uint64_t)m, Ks) != HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatrixLayoutCreate(&g->ld, HIP_R_32F, (uint64_t)p, (uint64_t)m, p) != HIPBLAS_STATUS_SUCCESS)
    return bad("hipblasLtMatrixLayoutCreate failed");
  if (!batched(g->la, S, Ks * (int64_t)p) || !batched(g->lb, S, m * Ks) || !batched(g->ld, S, m * (int64_t)p))
    return bad("setting the batch layout failed");
  hipblasLtMatmulPreference_t pref = nullptr;
  if (hipblasLtMatmulPreferenceCreate(&pref) != HIPBLAS_STATUS_SUCCESS) return bad("no GEMM preference");
  const uint64_t max_ws = (uint64_t)256 << 20;
  (void)hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &max_ws,
                                              sizeof(max_ws));
  hipblasLtMatmulHeuristicResult_t res[kMaxCandidates];
  int got = 0;
  const hipblasStatus_t hs = hipblasLtMatmulAlgoGetHeuristic(g->handle, g->desc, g->la, g->lb, g->ld, g->ld, pref,
                                                             kMaxCandidates, res, &got);
  (void)hipblasLtMatmulPreferenceDestroy(pref);
  if (hs != HIPBLAS_STATUS_SUCCESS) return bad("hipBLASLt has no algorithm for the sketch GEMM");
  for (int i = 0; i < got && i < kMaxCandidates; ++i) {
    if (res[i].state != HIPBLAS_STATUS_SUCCESS) continue;
    g->cand[g->ncand++] = res[i];
    if (res[i].workspaceSize > g->ws_bytes) g->ws_bytes = res[i].workspaceSize;
  }
  if (g->ncand < 1) return bad("hipBLASLt has no algorithm for the sketch GEMM");
  if (g->ws_bytes > 0 && hipMalloc(&g->ws, g->ws_bytes) != hipSuccess) {
    (void)hipGetLastError();
    g->ws = nullptr;
    return bad("no device memory for the GEMM workspace");
  }
  return g;
}

bool sketch_gemm_run(SketchGemm* g, const void* Ct, const void* Xs, float* part, hipStream_t stream,
                     bool accumulate) {
  const float alpha = 1.0f, beta = accumulate ? 1.0f : 0.0f;
  return hipblasLtMatmul(g->handle, g->desc, &alpha, Ct, g->la, Xs, g->lb, &beta, part, g->ld, part, g->ld,
                         &g->cand[g->cur].algo, g->ws, g->ws_bytes, stream) == HIPBLAS_STATUS_SUCCESS;
}

int sketch_gemm_candidates(const SketchGemm* g) { return g->ncand; }
int sketch_gemm_choice(const SketchGemm* g) { return g->cur; }
bool sketch_gemm_select(SketchGemm* g, int i) {
  if (i < 0 || i >= g->ncand) return false;
  g->cur = i;
  return true;
}

void sketch_gemm_free(SketchGemm* g) { delete g; }

}  // namespace blas
}  // namespace cdmd
