// HIP kernels of the cDMD hot path for gfx950 (CDNA4, wave64).
//
//   sketch  Y^ = C D         (Algorithm 1 step 3; sparse / single-pixel C of Section 3.3)
//   Gram    Y^T Y            (route to the truncated SVD of step 4 and to A~ of step 6)
//   lift    Phi = X' G       (step 8, eq. (Eq:cDMDModes), G = V S^-1 W) fused with the
//                            per-block partial sums of Phi^H Phi and Phi^H x_1 that the
//                            amplitude least squares of step 9 / eq. (eq:b) needs
//   bgfg    L = Re(Phi_S diag(beta) V_S) (eq. (equ:DMDTerms)) fused with the
//           threshold |x - L| > tau (eq. (eq:thres)); Phi_S is recomputed from X' per
//           pixel so the modes never travel through HBM.
#include "kernels.hpp"

#include <hip/hip_runtime.h>

namespace cdmd {
namespace k {

template <typename T>
__device__ __forceinline__ float ldx(const T* p) {
  return static_cast<float>(*p);
}

// ============================================================================
// sparse sketch, uint8 video
// One block = one segment of pixel-sorted (pixel, row, sign) triples x FPB frames.
// Integer accumulation in LDS (exact, so atomic order does not matter).
template <int FPB>
__global__ __launch_bounds__(512) void k_sketch_sparse_u8(
    const uint8_t* __restrict__ D, int64_t ld, int64_t m, const int32_t* __restrict__ tri_pix,
    const uint32_t* __restrict__ tri_rs, const int32_t* __restrict__ seg, int p,
    int32_t* __restrict__ Yout) {
  extern __shared__ int32_t acc[];  // [FPB][nrows]
  const int s = blockIdx.x;
  const int begin = seg[5 * s + 0], end = seg[5 * s + 1];
  const int r0 = seg[5 * s + 2], nrows = seg[5 * s + 3], slot = seg[5 * s + 4];
  const int64_t t0 = (int64_t)blockIdx.y * FPB;
  const int nf = (int)((m - t0) < FPB ? (m - t0) : FPB);
  for (int i = threadIdx.x; i < FPB * nrows; i += blockDim.x) acc[i] = 0;
  __syncthreads();
  const uint8_t* Dt = D + t0 * ld;
  const int stride = blockDim.x;
  int e = begin + threadIdx.x;
  for (; e + stride < end; e += 2 * stride) {
    const int pa = tri_pix[e], pb = tri_pix[e + stride];
    const uint32_t ra = tri_rs[e], rb = tri_rs[e + stride];
    int va[FPB], vb[FPB];
#pragma unroll
    for (int f = 0; f < FPB; ++f) {
      va[f] = (f < nf) ? (int)Dt[f * ld + pa] : 0;
      vb[f] = (f < nf) ? (int)Dt[f * ld + pb] : 0;
    }
    const int rowa = (int)(ra & 0x7fffffffu), rowb = (int)(rb & 0x7fffffffu);
#pragma unroll
    for (int f = 0; f < FPB; ++f) {
      if (f < nf) {
        atomicAdd(&acc[f * nrows + rowa], (ra >> 31) ? -va[f] : va[f]);
        atomicAdd(&acc[f * nrows + rowb], (rb >> 31) ? -vb[f] : vb[f]);
      }
    }
  }
  if (e < end) {
    const int pa = tri_pix[e];
    const uint32_t ra = tri_rs[e];
    const int rowa = (int)(ra & 0x7fffffffu);
#pragma unroll
    for (int f = 0; f < FPB; ++f) {
      if (f < nf) {
        const int v = (int)Dt[f * ld + pa];
        atomicAdd(&acc[f * nrows + rowa], (ra >> 31) ? -v : v);
      }
    }
  }
  __syncthreads();
  int32_t* Y = Yout + (int64_t)slot * m * p;
  for (int i = threadIdx.x; i < nf * nrows; i += blockDim.x) {
    const int f = i / nrows, r = i - f * nrows;
    Y[(t0 + f) * p + r0 + r] = acc[i];
  }
}

hipError_t sketch_sparse_u8(const uint8_t* D, int64_t ld, int64_t m, const int32_t* tri_pix,
                            const uint32_t* tri_rs, const int32_t* seg, int nseg, int p,
                            int max_rows, int fpb, int32_t* Yout, int nslot,
                            hipStream_t stream) {
  (void)nslot;
  const dim3 grid(nseg, (unsigned)((m + fpb - 1) / fpb));
  const size_t lds = (size_t)fpb * max_rows * sizeof(int32_t);
  switch (fpb) {
    case 1: hipLaunchKernelGGL(k_sketch_sparse_u8<1>, grid, dim3(512), lds, stream, D, ld, m, tri_pix, tri_rs, seg, p, Yout); break;
    case 2: hipLaunchKernelGGL(k_sketch_sparse_u8<2>, grid, dim3(512), lds, stream, D, ld, m, tri_pix, tri_rs, seg, p, Yout); break;
    case 4: hipLaunchKernelGGL(k_sketch_sparse_u8<4>, grid, dim3(512), lds, stream, D, ld, m, tri_pix, tri_rs, seg, p, Yout); break;
    case 8: hipLaunchKernelGGL(k_sketch_sparse_u8<8>, grid, dim3(512), lds, stream, D, ld, m, tri_pix, tri_rs, seg, p, Yout); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ void k_reduce_slots(const int32_t* __restrict__ Yp, int nslot, int64_t count,
                               int32_t* __restrict__ Y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    int32_t s = 0;
    for (int q = 0; q < nslot; ++q) s += Yp[(int64_t)q * count + i];
    Y[i] = s;
  }
}

hipError_t reduce_slots_i32(const int32_t* Ypart, int nslot, int64_t count, int32_t* Y,
                            hipStream_t stream) {
  int blocks = (int)((count + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_reduce_slots, dim3(blocks), dim3(256), 0, stream, Ypart, nslot, count, Y);
  return hipGetLastError();
}

// ============================================================================
// sparse sketch, float32 video: one thread per (row, frame), row order, float64 sum
__global__ void k_sketch_sparse_f32(const float* __restrict__ D, int64_t ld, int64_t m,
                                    const int32_t* __restrict__ idx,
                                    const int8_t* __restrict__ sign, int p, int nnz,
                                    double* __restrict__ Y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t t = blockIdx.y;
  if (r >= p) return;
  const float* Dt = D + t * ld;
  double s = 0.0;
  for (int j = 0; j < nnz; ++j) {
    const double v = (double)Dt[idx[(int64_t)r * nnz + j]];
    s += sign[(int64_t)r * nnz + j] < 0 ? -v : v;
  }
  Y[t * p + r] = s;
}

hipError_t sketch_sparse_f32(const float* D, int64_t ld, int64_t m, const int32_t* idx,
                             const int8_t* sign, int p, int nnz, double* Y,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_sketch_sparse_f32, dim3((p + 255) / 256, (unsigned)m), dim3(256), 0,
                     stream, D, ld, m, idx, sign, p, nnz, Y);
  return hipGetLastError();
}

// ============================================================================
// Gram of the sketch, float64: 32x32 output tiles, upper triangle of tiles computed
// and mirrored.  Each thread owns a 2x2 sub-tile.
template <typename T>
__global__ __launch_bounds__(256) void k_gram(const T* __restrict__ Y, int p, int64_t m,
                                              double* __restrict__ Gr) {
  if (blockIdx.y < blockIdx.x) return;
  __shared__ double sa[32][33];
  __shared__ double sb[32][33];
  const int64_t a0 = (int64_t)blockIdx.x * 32, b0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double c00 = 0, c01 = 0, c10 = 0, c11 = 0;
  for (int r0 = 0; r0 < p; r0 += 32) {
    for (int q = threadIdx.x; q < 32 * 32; q += 256) {
      const int fr = q >> 5, rr = q & 31;
      const int r = r0 + rr;
      sa[fr][rr] = (a0 + fr < m && r < p) ? (double)Y[(a0 + fr) * p + r] : 0.0;
      sb[fr][rr] = (b0 + fr < m && r < p) ? (double)Y[(b0 + fr) * p + r] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < 32; ++rr) {
      const double x0 = sa[ty][rr], x1 = sa[ty + 16][rr];
      const double y0 = sb[tx][rr], y1 = sb[tx + 16][rr];
      c00 = fma(x0, y0, c00);
      c01 = fma(x0, y1, c01);
      c10 = fma(x1, y0, c10);
      c11 = fma(x1, y1, c11);
    }
    __syncthreads();
  }
  const double cv[2][2] = {{c00, c01}, {c10, c11}};
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      const int64_t a = a0 + ty + 16 * u, b = b0 + tx + 16 * v;
      if (a < m && b < m) {
        Gr[a * m + b] = cv[u][v];
        Gr[b * m + a] = cv[u][v];
      }
    }
}

hipError_t gram_i32(const int32_t* Y, int p, int64_t m, double* Gr, hipStream_t stream) {
  const unsigned t = (unsigned)((m + 31) / 32);
  hipLaunchKernelGGL(k_gram<int32_t>, dim3(t, t), dim3(256), 0, stream, Y, p, m, Gr);
  return hipGetLastError();
}
hipError_t gram_f64(const double* Y, int p, int64_t m, double* Gr, hipStream_t stream) {
  const unsigned t = (unsigned)((m + 31) / 32);
  hipLaunchKernelGGL(k_gram<double>, dim3(t, t), dim3(256), 0, stream, Y, p, m, Gr);
  return hipGetLastError();
}

// ============================================================================
// lift (fp32): one thread per pixel, NC accumulators; G rows are wave-uniform and
// are read through the scalar path.  Persistent blocks walk pixel tiles of LIFT_NT.
constexpr int LIFT_NT = 128;
constexpr int LIFT_UNROLL = 8;

template <int NC>
struct LiftEPT {
  static constexpr int ne = NC * (NC + 1) / 2 + NC + 1;
  static constexpr int value = (ne + LIFT_NT - 1) / LIFT_NT;
};

template <typename Tin, int NC>
__global__ __launch_bounds__(LIFT_NT) void k_lift(
    const Tin* __restrict__ D, int64_t ld, int64_t n, int64_t m, const float* __restrict__ G,
    int nc, const uint32_t* __restrict__ pairs, int npair, double* __restrict__ part,
    float* __restrict__ phi, int kmodes, float xscale) {
  constexpr int EPT = LiftEPT<NC>::value;
  __shared__ float sphi[LIFT_NT][NC + 1];
  __shared__ float sx1[LIFT_NT];
  const int ne = npair + nc + 1;
  double pacc[EPT];
#pragma unroll
  for (int s = 0; s < EPT; ++s) pacc[s] = 0.0;
  const int64_t ntiles = (n + LIFT_NT - 1) / LIFT_NT;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t i = tile * LIFT_NT + threadIdx.x;
    const bool valid = i < n;
    const Tin* Dp = D + (valid ? i : 0);
    float acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.f;
    int64_t t = 1;
    for (; t + LIFT_UNROLL <= m; t += LIFT_UNROLL) {
      float xs[LIFT_UNROLL];
#pragma unroll
      for (int u = 0; u < LIFT_UNROLL; ++u) xs[u] = valid ? ldx(Dp + (t + u) * ld) : 0.f;
#pragma unroll
      for (int u = 0; u < LIFT_UNROLL; ++u) {
        const float* g = G + (t + u - 1) * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = fmaf(xs[u], g[c], acc[c]);
      }
    }
    for (; t < m; ++t) {
      const float x = valid ? ldx(Dp + t * ld) : 0.f;
      const float* g = G + (t - 1) * NC;
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = fmaf(x, g[c], acc[c]);
    }
    const float x1 = valid ? ldx(Dp) * xscale : 0.f;
    if (phi != nullptr && valid) {
      for (int j = 0; j < kmodes; ++j) {
        float2 v;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (c == j) v.x = acc[c];
          if (c == kmodes + j) v.y = acc[c];
        }
        reinterpret_cast<float2*>(phi)[(int64_t)j * n + i] = v;
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) sphi[threadIdx.x][c] = acc[c];
    sx1[threadIdx.x] = x1;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
      const int e = threadIdx.x + s * LIFT_NT;
      if (e < npair) {
        const uint32_t pr = pairs[e];
        const int a = (int)(pr & 0xffffu), b = (int)(pr >> 16);
        double sum = 0.0;
        for (int q = 0; q < LIFT_NT; ++q) sum = fma((double)sphi[q][a], (double)sphi[q][b], sum);
        pacc[s] += sum;
      } else if (e < npair + nc) {
        const int a = e - npair;
        double sum = 0.0;
        for (int q = 0; q < LIFT_NT; ++q) sum = fma((double)sphi[q][a], (double)sx1[q], sum);
        pacc[s] += sum;
      } else if (e < ne) {
        double sum = 0.0;
        for (int q = 0; q < LIFT_NT; ++q) sum = fma((double)sx1[q], (double)sx1[q], sum);
        pacc[s] += sum;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < EPT; ++s) {
    const int e = threadIdx.x + s * LIFT_NT;
    if (e < ne) part[(int64_t)blockIdx.x * ne + e] = pacc[s];
  }
}

int lift_grid(int64_t n) {
  const int64_t tiles = (n + LIFT_NT - 1) / LIFT_NT;
  return (int)(tiles < 2048 ? tiles : 2048);
}

template <typename Tin>
static hipError_t lift_dispatch(const Tin* D, int64_t ld, int64_t n, int64_t m, const float* G,
                                int NC, int nc, const uint32_t* pairs, int npair, double* part,
                                int grid, float* phi, int kmodes, float xscale,
                                hipStream_t s) {
#define LIFT_CASE(NCV)                                                                       \
  case NCV:                                                                                  \
    hipLaunchKernelGGL((k_lift<Tin, NCV>), dim3(grid), dim3(LIFT_NT), 0, s, D, ld, n, m, G,  \
                       nc, pairs, npair, part, phi, kmodes, xscale);                         \
    break;
  switch (NC) {
    LIFT_CASE(8)
    LIFT_CASE(16)
    LIFT_CASE(24)
    LIFT_CASE(32)
    LIFT_CASE(40)
    LIFT_CASE(48)
    LIFT_CASE(56)
    LIFT_CASE(64)
    LIFT_CASE(72)
    LIFT_CASE(80)
    default:
      return hipErrorInvalidValue;
  }
#undef LIFT_CASE
  return hipGetLastError();
}

hipError_t lift_fp32(const void* D, int dtype, int64_t ld, int64_t n, int64_t m, const float* G,
                     int NC, int nc, const uint32_t* pairs, int npair, double* part, int grid,
                     float* phi, int kmodes, float xscale, hipStream_t stream) {
  if (dtype == 0)
    return lift_dispatch((const uint8_t*)D, ld, n, m, G, NC, nc, pairs, npair, part, grid, phi,
                         kmodes, xscale, stream);
  return lift_dispatch((const float*)D, ld, n, m, G, NC, nc, pairs, npair, part, grid, phi,
                       kmodes, xscale, stream);
}

__global__ void k_reduce_partials(const double* __restrict__ part, int grid, int ne,
                                  double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double s = 0.0;
  for (int b = 0; b < grid; ++b) s += part[(int64_t)b * ne + e];
  out[e] = s;
}

hipError_t reduce_partials(const double* part, int grid, int ne, double* out,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_reduce_partials, dim3((ne + 127) / 128), dim3(128), 0, stream, part, grid,
                     ne, out);
  return hipGetLastError();
}

// ============================================================================
// fused background + foreground
constexpr int BGFG_NT = 256;

template <typename Tin, int NS>
__global__ __launch_bounds__(BGFG_NT) void k_bgfg(const Tin* __restrict__ D, int64_t ld,
                                                 int64_t n, int64_t m,
                                                 const float* __restrict__ Gs,
                                                 const float* __restrict__ Vc, float tau,
                                                 float xscale, int mode, void* __restrict__ out,
                                                 int64_t t0, int64_t t1, int64_t ldL) {
  const int64_t i = (int64_t)blockIdx.x * BGFG_NT + threadIdx.x;
  const bool valid = i < n;
  const Tin* Dp = D + (valid ? i : 0);
  float acc[NS];
#pragma unroll
  for (int c = 0; c < NS; ++c) acc[c] = 0.f;
  int64_t t = 1;
  for (; t + 8 <= m; t += 8) {
    float xs[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) xs[u] = valid ? ldx(Dp + (t + u) * ld) : 0.f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float* g = Gs + (t + u - 1) * NS;
#pragma unroll
      for (int c = 0; c < NS; ++c) acc[c] = fmaf(xs[u], g[c], acc[c]);
    }
  }
  for (; t < m; ++t) {
    const float x = valid ? ldx(Dp + t * ld) : 0.f;
    const float* g = Gs + (t - 1) * NS;
#pragma unroll
    for (int c = 0; c < NS; ++c) acc[c] = fmaf(x, g[c], acc[c]);
  }
  const int lane = threadIdx.x & 63;
  const int64_t i0 = i - lane;
  const int64_t words = (n + 31) >> 5;
  for (int64_t tt = t0; tt < t1; ++tt) {
    const float* v = Vc + tt * NS;
    float L = 0.f;
#pragma unroll
    for (int c = 0; c < NS; ++c) L = fmaf(acc[c], v[c], L);
    if (mode == 2) {
      if (valid) reinterpret_cast<float*>(out)[(tt - t0) * ldL + i] = L;
      continue;
    }
    const float x = valid ? ldx(Dp + tt * ld) * xscale : 0.f;
    const bool fg = valid && (fabsf(x - L) > tau);
    if (mode == 1) {
      if (valid) reinterpret_cast<uint8_t*>(out)[tt * n + i] = fg ? 1 : 0;
    } else {
      const uint64_t bal = __ballot(fg);
      if (lane == 0 && i0 < n) {
        uint32_t* w = reinterpret_cast<uint32_t*>(out) + tt * words + (i0 >> 5);
        w[0] = (uint32_t)bal;
        if ((i0 >> 5) + 1 < words) w[1] = (uint32_t)(bal >> 32);
      }
    }
  }
}

template <typename Tin>
static hipError_t bgfg_dispatch(const Tin* D, int64_t ld, int64_t n, int64_t m, const float* Gs,
                                int NS, const float* Vc, float tau, float xscale, int mode,
                                void* out, int64_t t0, int64_t t1, int64_t ldL,
                                hipStream_t s) {
  const dim3 grid((unsigned)((n + BGFG_NT - 1) / BGFG_NT));
#define BGFG_CASE(NSV)                                                                        \
  case NSV:                                                                                   \
    hipLaunchKernelGGL((k_bgfg<Tin, NSV>), grid, dim3(BGFG_NT), 0, s, D, ld, n, m, Gs, Vc,   \
                       tau, xscale, mode, out, t0, t1, ldL);                                  \
    break;
  switch (NS) {
    BGFG_CASE(4)
    BGFG_CASE(8)
    BGFG_CASE(12)
    BGFG_CASE(16)
    BGFG_CASE(20)
    BGFG_CASE(24)
    BGFG_CASE(32)
    BGFG_CASE(40)
    BGFG_CASE(48)
    BGFG_CASE(64)
    BGFG_CASE(80)
    default:
      return hipErrorInvalidValue;
  }
#undef BGFG_CASE
  return hipGetLastError();
}

hipError_t bgfg(const void* D, int dtype, int64_t ld, int64_t n, int64_t m, const float* Gs,
                int NS, const float* Vc, float tau, float xscale, int mode, void* out,
                int64_t t0, int64_t t1, int64_t ldL, hipStream_t stream) {
  if (dtype == 0)
    return bgfg_dispatch((const uint8_t*)D, ld, n, m, Gs, NS, Vc, tau, xscale, mode, out, t0, t1,
                         ldL, stream);
  return bgfg_dispatch((const float*)D, ld, n, m, Gs, NS, Vc, tau, xscale, mode, out, t0, t1, ldL,
                       stream);
}

__global__ __launch_bounds__(256) void k_mask_counts(const uint32_t* __restrict__ mask,
                                                     int64_t words, int64_t* __restrict__ counts) {
  __shared__ long long red[256];
  const uint32_t* w = mask + (int64_t)blockIdx.x * words;
  long long s = 0;
  for (int64_t q = threadIdx.x; q < words; q += 256) s += __popc(w[q]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

hipError_t mask_counts(const uint32_t* mask, int64_t words, int64_t m, int64_t* counts,
                       hipStream_t stream) {
  hipLaunchKernelGGL(k_mask_counts, dim3((unsigned)m), dim3(256), 0, stream, mask, words, counts);
  return hipGetLastError();
}

}  // namespace k
}  // namespace cdmd
