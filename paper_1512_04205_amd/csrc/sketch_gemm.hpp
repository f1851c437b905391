// The dense Gaussian sketch with a stored C as batched library GEMMs (sketch_gemm.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace cdmd {
namespace blas {

struct SketchGemm;

// Plan of S products part[s] (p x m, float32) = Ct[s] (p x Ks, bfloat16) Xs[s] (Ks x m,
// bfloat16), with its workspace.  Null (and *err set) when the library offers no algorithm
// or memory runs out.
SketchGemm* sketch_gemm_create(int p, int64_t Ks, int64_t m, int S, std::string* err);
// Enqueues the S products on `stream`; false if the library refuses the call.
bool sketch_gemm_run(SketchGemm* g, const void* Ct, const void* Xs, float* part, hipStream_t stream);
void sketch_gemm_free(SketchGemm* g);

}  // namespace blas
}  // namespace cdmd
