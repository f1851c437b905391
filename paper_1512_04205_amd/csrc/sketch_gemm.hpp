// The dense Gaussian sketch with a stored C as batched library GEMMs (sketch_gemm.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace cdmd {
namespace blas {

struct SketchGemm;

// Plan of S products part[s] (p x m, float32) = Ct[s] (p x Ks) Xs[s] (Ks x m), both bfloat16
// (fp8 = 0) or both OCP e4m3 (fp8 = 1), with its workspace.  Null (and *err set) when the
// library offers no algorithm or memory runs out.
SketchGemm* sketch_gemm_create(int p, int64_t Ks, int64_t m, int S, int fp8, std::string* err);
// Enqueues the S products on `stream` with the selected candidate algorithm, written to part
// or, with accumulate, added to it; false if the library refuses the call.
bool sketch_gemm_run(SketchGemm* g, const void* Ct, const void* Xs, float* part, hipStream_t stream,
                     bool accumulate = false);
// The library's candidate algorithms for the shape (up to 8, its first guess first, all
// with the same results up to float32 summation order), and the one in use (default 0).
int sketch_gemm_candidates(const SketchGemm* g);
int sketch_gemm_choice(const SketchGemm* g);
bool sketch_gemm_select(SketchGemm* g, int i);
void sketch_gemm_free(SketchGemm* g);

}  // namespace blas
}  // namespace cdmd
