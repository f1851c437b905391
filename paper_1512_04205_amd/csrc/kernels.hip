// HIP kernels of the cDMD hot path for gfx950 (CDNA4, wave64).
//
//   sketch  Y^ = C D         (eq. (eq:YCX); sparse / single-pixel C of Section 3.3)
//   Gram    Y^T Y            (route to the truncated SVD, eq. svd, and to A~, Section 3.2)
//   lift    Phi = X' G       (eq. (Eq:cDMDModes), G = V S^-1 W) fused with the
//                            per-block partial sums of Phi^H Phi and Phi^H x_1 that the
//                            amplitude least squares of eq. (eq:b) needs
//   bgfg    L = Re(Phi_S diag(beta) V_S) (eq. (equ:DMDTerms)) fused with the
//           threshold |x - L| > tau (eq. (eq:thres)); Phi_S is recomputed from X' per
//           pixel so the modes never travel through HBM.
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <atomic>

#include "team_la.hpp"

namespace cdmd {
namespace k {

template <typename T>
__device__ __forceinline__ float ldx(const T* p) {
  return static_cast<float>(*p);
}

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// x rounded to the nearest bf16 (8 significant bits, ties to even), as bits; and back.
__device__ __forceinline__ uint16_t bf16_bits_d(double x) {
  if (x == 0.0) return signbit(x) ? 0x8000 : 0;
  int e;
  const double f = frexp(fabs(x), &e);
  const double q = ldexp(rint(ldexp(f, 8)), e - 8);
  const uint32_t u = __float_as_uint((float)q) >> 16;
  return (uint16_t)(u | (x < 0 ? 0x8000u : 0u));
}
__device__ __forceinline__ double bf16_val_d(uint16_t b) {
  return (double)__uint_as_float((uint32_t)b << 16);
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

// Streaming form for 16-byte aligned frames: block (pixel range, frame group, row block)
// reads its pixel range of SK_F frames in chunks of SK_CH bytes with coalesced 16-byte
// loads (each video byte read once in total) into LDS, then the triples of the chunk
// (pixel-sorted, located by chunk_off) add the staged bytes into per-row LDS sums.
// Integer sums, so the atomic order does not matter.  Output: Ypart[range][t][r].
constexpr int SK_CH = 8192;   // finest chunk: 512 threads x 16 bytes (chunk_off granularity)
constexpr int SK_NT = 512;

// V: 16-byte vectors per thread and frame, chunk = V * SK_CH bytes.
template <int F, int V>
__global__ __launch_bounds__(SK_NT) void k_sketch_stream_u8(
    const uint8_t* __restrict__ D, int64_t ld, int64_t n, int64_t m, const int32_t* __restrict__ tri_pix,
    const uint32_t* __restrict__ tri_rs, const int32_t* __restrict__ chunk_off, int nchunk,
    const int32_t* __restrict__ rblk, int cpr, int p, int max_rows, int32_t* __restrict__ Ypart) {
  constexpr int CH = V * SK_CH;
  extern __shared__ int32_t lds[];
  int32_t* acc = lds;                                                    // [F][nrows]
  uint8_t* stage = reinterpret_cast<uint8_t*>(lds + F * max_rows);       // [F][CH]
  const int pr = blockIdx.x, b = blockIdx.z;
  const int64_t t0 = (int64_t)blockIdx.y * F;
  const int nf = (int)((m - t0) < F ? (m - t0) : F);
  const int r0 = rblk[2 * b], nrows = rblk[2 * b + 1];
  const int c_begin = pr * cpr, c_end = (pr + 1) * cpr < nchunk ? (pr + 1) * cpr : nchunk;
  const int* off = chunk_off + (int64_t)b * (nchunk + 1);
  for (int i = threadIdx.x; i < F * nrows; i += SK_NT) acc[i] = 0;
  const int tid = threadIdx.x;
  // chunk c covers bytes [c CH, (c+1) CH); vector u of thread tid is at 16 (u SK_NT + tid)
  auto load = [&](int c, uint4 (*v)[V]) {
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
      for (int u = 0; u < V; ++u) {
        const int64_t j = (int64_t)c * CH + 16 * (u * SK_NT + tid);
        uint4 x = make_uint4(0u, 0u, 0u, 0u);
        if (f < nf && j < n) {
          const uint8_t* src = D + (t0 + f) * ld + j;
          if (j + 16 <= n) {
            x = *reinterpret_cast<const uint4*>(src);
          } else {
            uint32_t w[4] = {0u, 0u, 0u, 0u};
            for (int e = 0; j + e < n; ++e) w[e >> 2] |= (uint32_t)src[e] << (8 * (e & 3));
            x = make_uint4(w[0], w[1], w[2], w[3]);
          }
        }
        v[f][u] = x;
      }
  };
  const int nck = (nchunk + V - 1) / V;  // chunks of this size
  const int cb = c_begin, ce = c_end < nck ? c_end : nck;
  uint4 cur[F][V];
  if (cb < ce) load(cb, cur);
  for (int c = cb; c < ce; ++c) {
    __syncthreads();  // previous chunk's triples are done with the stage
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
      for (int u = 0; u < V; ++u)
        *reinterpret_cast<uint4*>(stage + f * CH + 16 * (u * SK_NT + tid)) = cur[f][u];
    __syncthreads();
    if (c + 1 < ce) load(c + 1, cur);  // next chunk in flight while this one is summed
    const int fe = (c + 1) * V < nchunk ? (c + 1) * V : nchunk;
    const int e0 = off[c * V], e1 = off[fe];
    const int64_t c0 = (int64_t)c * CH;
    for (int e = e0 + tid; e < e1; e += SK_NT) {
      const int px = (int)(tri_pix[e] - c0);
      const uint32_t rs = tri_rs[e];
      const int row = (int)(rs & 0x7fffffffu);
      const bool neg = (rs >> 31) != 0;
#pragma unroll
      for (int f = 0; f < F; ++f)
        if (f < nf) {
          const int v = (int)stage[f * CH + px];
          atomicAdd(&acc[f * nrows + row], neg ? -v : v);
        }
    }
  }
  __syncthreads();
  int32_t* Y = Ypart + (int64_t)pr * m * p;
  for (int i = threadIdx.x; i < nf * nrows; i += SK_NT) {
    const int f = i / nrows, r = i - f * nrows;
    Y[(t0 + f) * p + r0 + r] = acc[i];
  }
}

bool sketch_stream_fits(int F, int V, int max_rows) {
  return (size_t)F * max_rows * sizeof(int32_t) + (size_t)F * V * SK_CH <= 65536;
}

hipError_t sketch_stream_u8(const uint8_t* D, int64_t ld, int64_t n, int64_t m, const int32_t* tri_pix,
                            const uint32_t* tri_rs, const int32_t* chunk_off, int nchunk, const int32_t* rblk,
                            int nblk, int nrange, int p, int max_rows, int F, int V, int32_t* Ypart,
                            hipStream_t stream) {
  if (!sketch_stream_fits(F, V, max_rows)) return hipErrorInvalidValue;
  const int nck = (nchunk + V - 1) / V;
  const int cpr = (nck + nrange - 1) / nrange;
  const dim3 grid((unsigned)nrange, (unsigned)((m + F - 1) / F), (unsigned)nblk);
  const size_t lds = (size_t)F * max_rows * sizeof(int32_t) + (size_t)F * V * SK_CH;
#define SK_LAUNCH(FF, VV)                                                                                  \
  hipLaunchKernelGGL((k_sketch_stream_u8<FF, VV>), grid, dim3(SK_NT), lds, stream, D, ld, n, m, tri_pix, \
                     tri_rs, chunk_off, nchunk, rblk, cpr, p, max_rows, Ypart)
  if (F == 4 && V == 1) SK_LAUNCH(4, 1);
  else if (F == 2 && V == 1) SK_LAUNCH(2, 1);
  else if (F == 2 && V == 2) SK_LAUNCH(2, 2);
  else if (F == 1 && V == 1) SK_LAUNCH(1, 1);
  else if (F == 1 && V == 2) SK_LAUNCH(1, 2);
  else if (F == 1 && V == 4) SK_LAUNCH(1, 4);
  else return hipErrorInvalidValue;
#undef SK_LAUNCH
  return hipGetLastError();
}

int sketch_stream_chunk() { return SK_CH; }

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
    const int32_t i = idx[(int64_t)r * nnz + j];
    if (i < 0) continue;  // empty slot of a shorter row
    const double v = (double)Dt[i];
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

// Gram of the sketch on FP64 MFMA 16x16x4: a workgroup per 16 x 16 tile of the upper
// triangle (mirrored); its 4 waves take interleaved 64-row chunks of the inner (sketch-row)
// index and their partial tiles are added in wave order.  Within a chunk the inner index
// is permuted so that lane (i, q) reads runs of four consecutive rows, the same
// permutation for both operands (the sum runs over the same terms).  For an integer sketch
// every partial sum is an integer below 2^53, so the result is exact in any order.
template <typename T>
__global__ __launch_bounds__(256) void k_gram_mfma(const T* __restrict__ Y, int p, int64_t m,
                                                   double* __restrict__ Gr) {
  if (blockIdx.y < blockIdx.x) return;
  __shared__ f64x4_t s_part[4][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, kq = l >> 4;
  const int64_t a0 = (int64_t)blockIdx.x * 16, b0 = (int64_t)blockIdx.y * 16;
  const int64_t a = a0 + i, b = b0 + i;
  const T* ya = Y + (a < m ? a : 0) * (int64_t)p;
  const T* yb = Y + (b < m ? b : 0) * (int64_t)p;
  f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = 64 * w; r0 < p; r0 += 256) {  // 16 steps per chunk, all loads issued first
    double av[16], bv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = r0 + 16 * (u >> 2) + 4 * kq + (u & 3);
      av[u] = a < m && r < p ? (double)ya[r] : 0.0;
      bv[u] = b < m && r < p ? (double)yb[r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
  }
  s_part[w][l] = acc;
  __syncthreads();
  if (w == 0) {
    f64x4_t t = s_part[0][l];
#pragma unroll
    for (int q = 1; q < 4; ++q) t += s_part[q][l];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int64_t ra = a0 + 4 * rr + kq, cb = b0 + i;
      if (ra < m && cb < m) {
        Gr[ra * m + cb] = t[rr];
        Gr[cb * m + ra] = t[rr];
      }
    }
  }
}

hipError_t gram_i32(const int32_t* Y, int p, int64_t m, double* Gr, hipStream_t stream) {
  const unsigned t = (unsigned)((m + 15) / 16);
  hipLaunchKernelGGL(k_gram_mfma<int32_t>, dim3(t, t), dim3(256), 0, stream, Y, p, m, Gr);
  return hipGetLastError();
}
hipError_t gram_f64(const double* Y, int p, int64_t m, double* Gr, hipStream_t stream) {
  const unsigned t = (unsigned)((m + 15) / 16);
  hipLaunchKernelGGL(k_gram_mfma<double>, dim3(t, t), dim3(256), 0, stream, Y, p, m, Gr);
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

// ============================================================================
// lift on MFMA (uint8 video): Phi = X' G with X' exact in bf16 and G given as NSPLIT
// bf16 terms (1: bf16 lift; 3: 24-bit G, float32-accurate products), float32
// accumulation.  Block = 4 waves, tile = 256 pixels, wave w owns pixels 64w..64w+63
// as two 32-row MFMA blocks x NB 32-column blocks.  Frames stream through LDS in
// chunks of 32 or 64 ([frame][pixel] bytes); per k-step each lane gathers its 8 frames of
// one pixel.
// The fused reduction P = Phi_ext^T Phi_ext (Phi_ext = [Phi | x_1 in column nc]) is
// computed from the accumulator registers themselves: a lane holds 16 pixel rows of
// one column, and the same register order is used for both operands, so the pixel
// order inside a K block is a consistent permutation.  P uses hi/lo bf16 splits and all
// four products (dropping lo*lo would bias the diagonal by ~2^-18), float32 accumulation
// over the block's pixels; what remains is the zero-mean rounding of the split.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint32_t pack_u8pair_bf16(uint32_t lo8, uint32_t hi8) {
  // integers 0..255 are exact in bf16: the high half of their float32 encoding
  const uint32_t a = __float_as_uint((float)lo8) >> 16;
  const uint32_t b = __float_as_uint((float)hi8) & 0xffff0000u;
  return a | b;
}

__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// split 8 float32 values into hi and lo bf16 vectors
__device__ __forceinline__ void split8(const float* v, bf16x8_t& hi, bf16x8_t& lo) {
  uint32_t h[4], q[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t h0 = bf16_rne_bits(v[2 * i]), h1 = bf16_rne_bits(v[2 * i + 1]);
    const float r0 = v[2 * i] - __uint_as_float(h0 << 16);
    const float r1 = v[2 * i + 1] - __uint_as_float(h1 << 16);
    h[i] = h0 | (h1 << 16);
    q[i] = bf16_rne_bits(r0) | (bf16_rne_bits(r1) << 16);
  }
  hi = __builtin_bit_cast(bf16x8_t, make_uint4(h[0], h[1], h[2], h[3]));
  lo = __builtin_bit_cast(bf16x8_t, make_uint4(q[0], q[1], q[2], q[3]));
}

constexpr int LM_TILE = 256;
constexpr int LM_SA = 264;       // LDS row stride (bytes) of a frame row

// X' G on MFMA for one 256-pixel tile: acc[mb][nb] (wave w, rows 64w + 32mb + ...)
// Frames 1..m-1 stream through `lds` in chunks of 16 KPC frames ([16 KPC][LM_SA] bytes,
// then the B operands of one chunk; KPC = 2 or 4, each thread loads 16 KPC bytes of one
// frame row per chunk).  The caller synchronises before reusing `lds`.
template <int NB, int NSPLIT, int KPC>
__device__ __forceinline__ void xprime_g_tile(const uint8_t* __restrict__ D, int64_t ld, int64_t n,
                                              int64_t m, const uint4* __restrict__ Gp, int nksteps,
                                              int64_t base, uint8_t* lds, f32x16_t (&acc)[2][NB]) {
  static_assert(KPC == 2 || KPC == 4, "16 KPC frames per chunk, 16 KPC bytes per thread");
  constexpr int LM_CH = 16 * KPC;                 // frames per chunk
  constexpr int NV = KPC;                         // 16-byte loads per thread and chunk
  constexpr int TPR = 16 / KPC;                   // threads per 256-byte frame row
  constexpr int BCH = KPC * NB * NSPLIT * 64;     // uint4 B operands per chunk
  uint8_t(*sA)[LM_SA] = reinterpret_cast<uint8_t(*)[LM_SA]>(lds);
  uint4* sB = reinterpret_cast<uint4*>(lds + LM_CH * LM_SA);
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int64_t N = m - 1;
  const int nchunks = (nksteps + KPC - 1) / KPC;
  const int fr = tid / TPR, seg = (tid % TPR) * (16 * NV);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[mb][nb][j] = 0.f;
  uint4 ra[NV];
  uint4 rb[(BCH + 255) / 256];
  auto gload = [&](int c) {
    const int64_t f = 1 + (int64_t)c * LM_CH + fr;
    const int64_t px = base + seg;
    if (f <= N && px + 16 * NV <= n) {
      const uint4* src = reinterpret_cast<const uint4*>(D + f * ld + px);
#pragma unroll
      for (int q = 0; q < NV; ++q) ra[q] = src[q];
    } else {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        uint32_t wds[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          uint32_t v = 0;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int64_t pp = px + 16 * q + 4 * r + b;
            if (f <= N && pp < n) v |= (uint32_t)D[f * ld + pp] << (8 * b);
          }
          wds[r] = v;
        }
        ra[q] = make_uint4(wds[0], wds[1], wds[2], wds[3]);
      }
    }
#pragma unroll
    for (int q = 0; q < (BCH + 255) / 256; ++q) {
      const int e = tid + q * 256;
      if (e < BCH) {
        const int ks = KPC * c + e / (NB * NSPLIT * 64);
        rb[q] = ks < nksteps ? Gp[(int64_t)KPC * c * NB * NSPLIT * 64 + e] : make_uint4(0, 0, 0, 0);
      }
    }
  };
  gload(0);
  for (int c = 0; c < nchunks; ++c) {
    __syncthreads();
    {  // rows are 8-byte aligned (stride 264): 8-byte stores
      uint2* dst = reinterpret_cast<uint2*>(&sA[fr][seg]);
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        dst[2 * q] = make_uint2(ra[q].x, ra[q].y);
        dst[2 * q + 1] = make_uint2(ra[q].z, ra[q].w);
      }
    }
#pragma unroll
    for (int q = 0; q < (BCH + 255) / 256; ++q) {
      const int e = tid + q * 256;
      if (e < BCH) sB[e] = rb[q];
    }
    __syncthreads();
    if (c + 1 < nchunks) gload(c + 1);
#pragma unroll
    for (int ks = 0; ks < KPC; ++ks) {
      bf16x8_t a[2];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const int pxl = 64 * w + 32 * mb + (l & 31);
        const int k0 = 16 * ks + 8 * (l >> 5);
        uint32_t wv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          wv[i] = pack_u8pair_bf16(sA[k0 + 2 * i][pxl], sA[k0 + 2 * i + 1][pxl]);
        a[mb] = __builtin_bit_cast(bf16x8_t, make_uint4(wv[0], wv[1], wv[2], wv[3]));
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int s = 0; s < NSPLIT; ++s) {
          const bf16x8_t b = __builtin_bit_cast(bf16x8_t, sB[((ks * NB + nb) * NSPLIT + s) * 64 + l]);
#pragma unroll
          for (int mb = 0; mb < 2; ++mb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mb], b, acc[mb][nb], 0, 0, 0);
        }
    }
  }
}

template <int NB, int NSPLIT, int KPC>
constexpr int xg_lds_bytes() {
  return 16 * KPC * LM_SA + KPC * NB * NSPLIT * 64 * 16;
}

// The occupancy hints keep the accumulators in the unified register file at the wave
// count that still needs no spills (checked with the compiler's resource report): more
// resident waves keep more of the video in flight.
template <int NB, int NSPLIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NB == 1 ? 3 : NB == 2 ? 2 : 1))) void k_lift_mfma(
    const uint8_t* __restrict__ D, int64_t ld, int64_t n, int64_t m, const uint4* __restrict__ Gp,
    int nksteps, int nc, float xscale, double* __restrict__ part, float* __restrict__ phi,
    int kmodes) {
  constexpr int NP = NB * (NB + 1) / 2;
  constexpr int RED_BYTES = 4 * NP * 16 * 64 * 4;
  constexpr int MAIN_BYTES = xg_lds_bytes<NB, NSPLIT, 4>();
  constexpr int LDS_BYTES = RED_BYTES > MAIN_BYTES ? RED_BYTES : MAIN_BYTES;
  __shared__ __align__(16) uint8_t lds[LDS_BYTES];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int64_t ntiles = (n + LM_TILE - 1) / LM_TILE;
  f32x16_t P[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) P[q][j] = 0.f;

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t base = tile * LM_TILE;
    f32x16_t acc[2][NB];
    xprime_g_tile<NB, NSPLIT, 4>(D, ld, n, m, Gp, nksteps, base, lds, acc);
    // x_1 (scaled) into column nc of Phi_ext
    if ((l & 31) == (nc & 31)) {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int64_t px = base + 64 * w + 32 * mb + (j >> 2) * 8 + (l >> 5) * 4 + (j & 3);
          const float x1 = px < n ? (float)D[px] * xscale : 0.f;
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            if (nb == (nc >> 5)) acc[mb][nb][j] = x1;
        }
    }
    if (phi != nullptr) {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int col = 32 * nb + (l & 31);
          if (col < 2 * kmodes) {
            const int mode = col < kmodes ? col : col - kmodes;
            const int part_im = col < kmodes ? 0 : 1;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
              const int64_t px = base + 64 * w + 32 * mb + (j >> 2) * 8 + (l >> 5) * 4 + (j & 3);
              if (px < n) phi[2 * ((int64_t)mode * n + px) + part_im] = acc[mb][nb][j];
            }
          }
        }
    }
    // P += Phi_ext^T Phi_ext over this wave's 64 pixels
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        bf16x8_t hi[NB], lo[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          float v[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) v[i] = acc[mb][nb][8 * h + i];
          split8(v, hi[nb], lo[nb]);
        }
        int q = 0;
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = a; b < NB; ++b, ++q) {
            P[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi[a], hi[b], P[q], 0, 0, 0);
            P[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hi[a], lo[b], P[q], 0, 0, 0);
            P[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo[a], hi[b], P[q], 0, 0, 0);
            P[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lo[a], lo[b], P[q], 0, 0, 0);
          }
      }
  }
  // reduce the four waves' P in LDS, write the block partial (float64)
  __syncthreads();
  float* red = reinterpret_cast<float*>(lds);
#pragma unroll
  for (int q = 0; q < NP; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) red[((w * NP + q) * 16 + j) * 64 + l] = P[q][j];
  __syncthreads();
  constexpr int NE = NP * 16 * 64;
  for (int e = tid; e < NE; e += 256) {
    double s = 0.0;
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) s += (double)red[ww * NE + e];
    part[(int64_t)blockIdx.x * NE + e] = s;
  }
}

// ============================================================================
// Background reconstruction and foreground threshold in one read of the video
// (eq. (equ:DMDTerms) with its real-part footnote, eq. (eq:thres)).  A workgroup of
// four waves owns 128 pixels (32 per wave) and first copies all their frames into LDS,
// transposed to one row per pixel (frame t at byte t of the row), so HBM delivers each
// video byte once.  Two workgroups fit a CU's LDS, which gives every SIMD two waves: one
// computes while the other waits for its tile.
//
//   phase 1: T^T = G~'^T X on bf16 MFMA 32x32x16, where G~'[t] = [Re | Im] of
//            G_S[t-1] diag(beta_S) xscale (G~'[0] = 0, so the k-steps start at frame 0
//            and every B fragment is one aligned 8-byte LDS read: 8 frames of a pixel)
//            in NSG bf16 terms; float32 accumulation.  Wave w keeps acc[mb] = T^T of
//            its pixel blocks 32 (RC_MB w + mb) (rows: columns c; lane columns: pixels).
//   phase 2: L = V~ T on bf16 MFMA 32x32x16 per 32-frame block.  The B operands are
//            the phase-1 accumulators split into NTV bf16 terms: a lane of the phase-1
//            result holds one pixel and 16 columns, exactly a B fragment once the K order
//            of phase 2 is the fixed permutation sigma(16q + 8h + i) = 16q + 8(i/4) +
//            4h + i%4.  The A operands V~[t][c] (Re lambda_s^t or -Im lambda_s^t, NTV
//            terms, in that K order) come prepared.  Products of split terms whose orders
//            sum below NTV accumulate in float32 (NTV = 3: six products; NTV = 2: three).
//   output:  |x - L| > tau per element, bit-packed by wave ballots (mode 0), as bytes
//            (mode 1), or L itself (mode 2).
//
// Columns: mode s (< 16) sits in lane half h = s & 1 at slot j = 2 (s >> 1) + part
// (part 0 = Re, 1 = Im), i.e. column rc_col(s, part).
constexpr int RC_TP = 128;  // pixels per workgroup
constexpr int RC_MB = 1;    // 32-pixel blocks per wave
constexpr int RC_NT = 64 * RC_TP / (32 * RC_MB);  // four waves
constexpr int RC_PF = 4;    // k-steps of G~' operands loaded ahead
constexpr int RC_LB = 8;    // 4x16-byte blocks a thread loads per batch of the tile load

__host__ __device__ inline int rc_col(int s, int part) {
  const int h = s & 1, j = 2 * (s >> 1) + part;
  return 16 * (j >> 3) + 8 * ((j >> 2) & 1) + 4 * h + (j & 3);
}
// LDS bytes per pixel row for `rows` frames: congruent to 8 modulo 256, so the 32 rows
// a half-wave reads with 8-byte (or 4-byte) loads fall on distinct banks.
__host__ __device__ inline int rc_stride(int rows) { return ((rows + 247) / 256) * 256 + 8; }

size_t recon_lds_bytes(int64_t m) {
  const int64_t rows = 64 * ((m + 63) / 64);
  return (size_t)RC_TP * rc_stride((int)rows);
}

template <int NT>
__device__ __forceinline__ void split_terms(const float* v, bf16x8_t (&o)[NT]) {
  float r[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = v[i];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    uint32_t wv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t b0 = bf16_rne_bits(r[2 * i]), b1 = bf16_rne_bits(r[2 * i + 1]);
      if (t + 1 < NT) {
        r[2 * i] -= __uint_as_float(b0 << 16);
        r[2 * i + 1] -= __uint_as_float(b1 << 16);
      }
      wv[i] = b0 | (b1 << 16);
    }
    o[t] = __builtin_bit_cast(bf16x8_t, make_uint4(wv[0], wv[1], wv[2], wv[3]));
  }
}

// 8 frames of one pixel (bytes, frame order) as bf16 (integers 0..255 are exact)
__device__ __forceinline__ bf16x8_t u8x8_bf16(uint2 v) {
  uint32_t wv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t src = q < 2 ? v.x : v.y;
    const int sh = 16 * (q & 1);
    const float lo = (float)((src >> sh) & 0xffu), hi = (float)((src >> (sh + 8)) & 0xffu);
    wv[q] = __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x07060302u);
  }
  return __builtin_bit_cast(bf16x8_t, make_uint4(wv[0], wv[1], wv[2], wv[3]));
}

// v_writelane_b32 through the compiler's intrinsic (so that it inserts the wait states a
// VALU-written SGPR needs before v_writelane reads it)
extern "C" __device__ int cdmd_amdgcn_writelane(int src, int lane, int old) __asm("llvm.amdgcn.writelane.i32");
// v with lane LANE replaced by the wave-uniform value u
template <int LANE>
__device__ __forceinline__ uint32_t writelane_u32(uint32_t v, uint32_t u) {
  return (uint32_t)cdmd_amdgcn_writelane((int)u, LANE, (int)v);
}
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// keep v in registers as computed (the compiler may not recompute it later)
__device__ __forceinline__ void pin(bf16x8_t& v) {
  uint4 u = __builtin_bit_cast(uint4, v);
  asm volatile("" : "+v"(u.x), "+v"(u.y), "+v"(u.z), "+v"(u.w));
  v = __builtin_bit_cast(bf16x8_t, u);
}

// One workgroup's tile: pixels [base, base + 128) of the reconstruction a.  MODE 0:
// bit-packed mask, 1: byte mask, 2: L.  RAGGED: the tile runs past n (only the last one),
// so its loads and stores check every pixel.
template <int NSG, int NTV, int MODE, bool RAGGED>
__device__ __forceinline__ void recon_tile(const ReconArgs& a, const int64_t base) {
  extern __shared__ __align__(16) uint4 rc_lds[];
  uint8_t* sV = reinterpret_cast<uint8_t*>(rc_lds);
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, h = l >> 5, fl = l & 31;
  const int64_t n = a.n, ld = a.ld;
  const int m = (int)a.m;
  const int KS = a.KS;               // 16-frame k-steps of phase 1, a multiple of 4
  const int S = rc_stride(16 * KS);

  // ---- the tile's frames into LDS, transposed: per block a thread takes 16 pixels
  // (chunk tid % 8) x 4 frames, transposes 4x4 bytes and stores one word per pixel
  {
    const int pc = tid & 7;
    const int64_t px = base + 16 * pc;
    constexpr int QS = RC_NT / 8;    // frame quads per batch row
    const int nquads = 4 * KS;       // a multiple of 16: the bounds below are uniform per wave
    const uint8_t* src = a.D + px;
    uint8_t* dstc = sV + (size_t)(16 * pc) * S;
    for (int q0 = tid >> 3; q0 < nquads; q0 += QS * RC_LB) {
      uint4 r[RC_LB][4];
#pragma unroll
      for (int b = 0; b < RC_LB; ++b) {
        const int fq = q0 + QS * b;
        if (fq >= nquads) break;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int f = min(4 * fq + i, m - 1);  // beyond the video: finite bytes (their G~' rows are 0)
          if (!RAGGED) {
            r[b][i] = *reinterpret_cast<const uint4*>(src + (int64_t)f * ld);
          } else {
            uint32_t wd[4] = {0, 0, 0, 0};
            for (int e = 0; e < 16; ++e)
              if (px + e < n) wd[e >> 2] |= (uint32_t)src[(int64_t)f * ld + e] << (8 * (e & 3));
            r[b][i] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
          }
        }
      }
#pragma unroll
      for (int b = 0; b < RC_LB; ++b) {
        const int fq = q0 + QS * b;
        if (fq >= nquads) break;
#pragma unroll
        for (int d = 0; d < 4; ++d) {  // dword d of the rows: pixels 4d..4d+3 of the chunk
          const uint32_t r0 = (&r[b][0].x)[d], r1 = (&r[b][1].x)[d], r2 = (&r[b][2].x)[d], r3 = (&r[b][3].x)[d];
          const uint32_t t01lo = __builtin_amdgcn_perm(r1, r0, 0x05010400u), t01hi = __builtin_amdgcn_perm(r1, r0, 0x07030602u);
          const uint32_t t23lo = __builtin_amdgcn_perm(r3, r2, 0x05010400u), t23hi = __builtin_amdgcn_perm(r3, r2, 0x07030602u);
          uint8_t* row = dstc + (size_t)(4 * d) * S + 4 * fq;
          *reinterpret_cast<uint32_t*>(row) = __builtin_amdgcn_perm(t23lo, t01lo, 0x05040100u);
          *reinterpret_cast<uint32_t*>(row + S) = __builtin_amdgcn_perm(t23lo, t01lo, 0x07060302u);
          *reinterpret_cast<uint32_t*>(row + 2 * S) = __builtin_amdgcn_perm(t23hi, t01hi, 0x05040100u);
          *reinterpret_cast<uint32_t*>(row + 3 * S) = __builtin_amdgcn_perm(t23hi, t01hi, 0x07060302u);
        }
      }
    }
  }
  __syncthreads();

  // ---- phase 1 (Gp holds KS + RC_PF k-steps, the last RC_PF zero)
  f32x16_t acc[RC_MB];
#pragma unroll
  for (int mb = 0; mb < RC_MB; ++mb)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[mb][j] = 0.f;
  const uint8_t* rowp[RC_MB];
#pragma unroll
  for (int mb = 0; mb < RC_MB; ++mb) rowp[mb] = sV + (32 * (RC_MB * w + mb) + fl) * S + 8 * h;
  {
    const uint4* gp = a.Gp + l;
    uint4 gq[RC_PF][NSG];
#pragma unroll
    for (int p = 0; p < RC_PF; ++p)
#pragma unroll
      for (int t = 0; t < NSG; ++t) gq[p][t] = gp[(p * NSG + t) * 64];
    for (int K0 = 0; K0 < KS; K0 += RC_PF) {
#pragma unroll
      for (int p = 0; p < RC_PF; ++p) {
        const int K = K0 + p;
        bf16x8_t xb[RC_MB];
#pragma unroll
        for (int mb = 0; mb < RC_MB; ++mb) xb[mb] = u8x8_bf16(*reinterpret_cast<const uint2*>(rowp[mb] + 16 * K));
#pragma unroll
        for (int t = NSG - 1; t >= 0; --t) {
          const bf16x8_t ga = __builtin_bit_cast(bf16x8_t, gq[p][t]);
#pragma unroll
          for (int mb = 0; mb < RC_MB; ++mb) acc[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ga, xb[mb], acc[mb], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < NSG; ++t) gq[p][t] = gp[((K + RC_PF) * NSG + t) * 64];
      }
    }
  }

  // ---- phase 2 (Vp holds NFB + 1 frame blocks, the last zero).  The MFMAs of frame
  // block i + 1 are issued before the threshold of block i, so the matrix cores and the
  // vector ALU overlap.
  const int nq = a.ns <= 8 ? 1 : 2;
  bf16x8_t tb[RC_MB][2][NTV];
#pragma unroll
  for (int mb = 0; mb < RC_MB; ++mb)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      float v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = acc[mb][8 * q + i];
      split_terms<NTV>(v, tb[mb][q]);
#pragma unroll
      for (int t = 0; t < NTV; ++t) pin(tb[mb][q][t]);
    }
  const int ts = MODE == 2 ? (int)a.t0 : 0, te = MODE == 2 ? (int)a.t1 : m;
  const int64_t words = (n + 31) >> 5;
  const int fb0 = ts >> 5, fb1 = (te + 31) >> 5;
  const uint4* vp = a.Vp + l;
  const int pxw = 32 * RC_MB * w;               // this wave's first pixel in the tile
  bool pvb[RC_MB];
#pragma unroll
  for (int mb = 0; mb < RC_MB; ++mb) pvb[mb] = !RAGGED || base + pxw + 32 * mb + fl < n;

  // L of frame block fbi for the wave's pixel blocks
  auto products = [&](int fbi, f32x16_t (&C)[RC_MB]) {
    bf16x8_t va[2][NTV];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int t = 0; t < NTV; ++t)
        va[q][t] = __builtin_bit_cast(bf16x8_t, vp[(((int64_t)fbi * 2 + q) * NTV + t) * 64]);
#pragma unroll
    for (int mb = 0; mb < RC_MB; ++mb)
#pragma unroll
      for (int j = 0; j < 16; ++j) C[mb][j] = 0.f;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q >= nq) break;
#pragma unroll
      for (int mb = 0; mb < RC_MB; ++mb) {  // independent accumulation chains
        if constexpr (NTV >= 3) {  // small products first
          C[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va[q][2], tb[mb][q][0], C[mb], 0, 0, 0);
          C[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va[q][0], tb[mb][q][2], C[mb], 0, 0, 0);
          C[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va[q][1], tb[mb][q][1], C[mb], 0, 0, 0);
        }
        if constexpr (NTV >= 2) {
          C[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va[q][1], tb[mb][q][0], C[mb], 0, 0, 0);
          C[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va[q][0], tb[mb][q][1], C[mb], 0, 0, 0);
        }
        C[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va[q][0], tb[mb][q][0], C[mb], 0, 0, 0);
      }
    }
  };
  // the output of frame block fbi; EDGE: the block runs past [ts, te) (checks per frame)
  auto emit = [&](int fbi, const f32x16_t (&C)[RC_MB], auto edge_c) {
    constexpr bool EDGE = decltype(edge_c)::value;
    const int fb = 32 * fbi;
    uint32_t wmine[RC_MB];
#pragma unroll
    for (int mb = 0; mb < RC_MB; ++mb) {
      // C[mb][j]: frame fb + 8(j/4) + 4h + j%4, pixel base + pxw + 32mb + fl
      const int pxl = pxw + 32 * mb + fl;
      const int64_t px = base + pxl;
      const bool pv = pvb[mb];
      wmine[mb] = 0u;
      if constexpr (MODE == 2) {
        float* out = reinterpret_cast<float*>(a.out) + px;
        static_for<0, 16>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          const int f = fb + 8 * (j >> 2) + 4 * h + (j & 3);
          if ((!RAGGED || pv) && (!EDGE || (f >= ts && f < te))) out[(int64_t)(f - ts) * a.ldL] = C[mb][j];
        });
      } else {
        uint32_t xw[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) xw[g] = *reinterpret_cast<const uint32_t*>(sV + pxl * S + fb + 8 * g + 4 * h);
        uint32_t wm = 0u;
        static_for<0, 16>([&](auto jc) {
          constexpr int j = decltype(jc)::value, g = j >> 2, e = j & 3;
          const float x = (float)((xw[g] >> (8 * e)) & 0xffu);
          bool fgd = fabsf(fmaf(x, a.xscale, -C[mb][j])) > a.tau;
          if constexpr (RAGGED || EDGE) {
            const int f = fb + 8 * g + 4 * h + e;
            fgd = fgd && (!RAGGED || pv) && (!EDGE || f < te);
          }
          if constexpr (MODE == 1) {
            const int f = fb + 8 * g + 4 * h + e;
            if ((!RAGGED || pv) && (!EDGE || f < te)) reinterpret_cast<uint8_t*>(a.out)[(int64_t)f * n + px] = fgd ? 1 : 0;
          } else {
            // lanes 0-31 hold frame fb + 8g + e, lanes 32-63 frame fb + 8g + 4 + e: one
            // mask word each; lane r of half 0 collects the word of frame fb + r
            const uint64_t bal = __ballot(fgd);
            wm = writelane_u32<8 * g + e>(wm, (uint32_t)bal);
            wm = writelane_u32<8 * g + 4 + e>(wm, (uint32_t)(bal >> 32));
          }
        });
        wmine[mb] = wm;
      }
    }
    if constexpr (MODE == 0) {
      const int f = fb + fl;
      if (h == 0 && (!EDGE || f < te)) {
        uint32_t* wd = reinterpret_cast<uint32_t*>(a.out) + (int64_t)f * words + ((base + pxw) >> 5);
#pragma unroll
        for (int mb = 0; mb < RC_MB; ++mb)
          if (!RAGGED || base + pxw + 32 * mb < n) wd[mb] = wmine[mb];
      }
    }
  };
  auto emit_any = [&](int fbi, const f32x16_t (&C)[RC_MB]) {
    if (32 * fbi < ts || 32 * fbi + 32 > te) emit(fbi, C, std::true_type{});
    else emit(fbi, C, std::false_type{});
  };
  f32x16_t Ca[RC_MB], Cb[RC_MB];
  products(fb0, Ca);
  int fbi = fb0;
  for (; fbi + 2 <= fb1; fbi += 2) {
    products(fbi + 1, Cb);
    emit_any(fbi, Ca);
    products(fbi + 2, Ca);   // block fb1 is the zero block past the end when fbi + 2 == fb1
    emit_any(fbi + 1, Cb);
  }
  if (fbi < fb1) emit_any(fbi, Ca);
}

// Blocks are dealt to the eight XCDs in turn; XCD x takes the contiguous tiles
// [x per, (x + 1) per), so neighbouring tiles run together on one XCD and their 16-byte
// pieces of each frame's mask line meet in its L2 before they are written back.
__device__ __forceinline__ int64_t recon_xcd_tile(int64_t ntiles) {
  const int64_t per = (ntiles + 7) / 8;
  return (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// Tiles tile0 .. tile0 + ntiles - 1 of one reconstruction.
template <int NSG, int NTV, int MODE, bool RAGGED>
__global__ __launch_bounds__(RC_NT) void k_recon(ReconArgs a, int64_t tile0, int64_t ntiles) {
  const int64_t tile = recon_xcd_tile(ntiles);
  if (tile >= ntiles) return;  // uniform
  recon_tile<NSG, NTV, MODE, RAGGED>(a, (tile0 + tile) * RC_TP);
}

// The tiles of several reconstructions in one launch (the masks of a batch of models):
// entry e of the work list owns the launch's tiles [start_e, start_e + ntiles_e), which are
// tiles tile0_e .. of its reconstruction; starts increase from 0, total = the last start
// plus its tile count, nw <= 64.  The tiles are dealt to the XCDs in chunks of eight (the
// tiles sharing a 128-byte line of each frame's mask stay on one XCD), chunk c to XCD
// c mod 8, so every entry spreads over all XCDs whatever its cost per tile: block b =
// 64 J + 8 r + x (XCD x) takes tile 64 J + 8 x + r.  A workgroup finds its entry with one
// wave-wide comparison (lane e tests start_e <= tile: the set lanes are a prefix).
template <int NSG, int NTV, int MODE, bool RAGGED>
__global__ __launch_bounds__(RC_NT) void k_recon_list(const ReconWork* __restrict__ list, int nw, int64_t total) {
  const int64_t b = blockIdx.x;
  const int64_t tile = (b & ~(int64_t)63) + 8 * (b & 7) + ((b >> 3) & 7);
  if (tile >= total) return;  // uniform
  const int lane = threadIdx.x & 63;
  const bool mine = lane < nw && list[lane].start <= tile;
  const int e = __builtin_amdgcn_readfirstlane(__popcll(__ballot(mine)) - 1);
  const ReconArgs a = list[e].a;
  recon_tile<NSG, NTV, MODE, RAGGED>(a, (list[e].tile0 + tile - list[e].start) * RC_TP);
}

// Operands of k_recon, from G (N x k complex float64, row t at t*k, mode s in column
// col[s]):
//   Gp [KS + RC_PF][NSG][lane][8] bf16: element i of lane l is G~'[16ks + 8(l/32) + i][l%32]
//      with G~'[t] = [Re | Im](G[t-1, col_s] beta_s xscale) in the columns of rc_col (row 0,
//      rows t > N and the RC_PF k-steps past KS are 0), NSG bf16 terms;
//   Vp [NFB + 1][2][NTV][lane][8] bf16 (the last block 0): element i of lane l (h = l/32) is, at frame t =
//      32 fb + l%32 and K slot 16q + 8h + i, i.e. column c = 16q + 8(i/4) + 4h + i%4,
//      Re lambda_s^t (part 0) or -Im lambda_s^t (part 1) of the mode in column c (0 for
//      unused columns), lambda^t by binary powering in float64 (1 for the static model),
//      NTV bf16 terms of its float32 value.
__global__ __launch_bounds__(256) void k_recon_prep(const double* __restrict__ G, ReconPrep rp,
                                                    uint16_t* __restrict__ Gp, uint16_t* __restrict__ Vp) {
  const int ns = rp.ns, N = rp.N, k = rp.k;
  const int64_t ng = (int64_t)(rp.KS + RC_PF) * 64 * 8, nv = (int64_t)(rp.NFB + 1) * 2 * 64 * 8;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ng + nv; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e & 7);
    const int l = (int)((e >> 3) & 63);
    if (e < ng) {
      const int ks = (int)(e >> 9);
      const int t = 16 * ks + 8 * (l >> 5) + i;
      const int c = l & 31;
      const int hh = (c >> 2) & 1, j = 8 * (c >> 4) + 4 * ((c >> 3) & 1) + (c & 3);
      const int s = 2 * (j >> 1) + hh, part = j & 1;
      double g = 0.0;
      if (ks < rp.KS && t >= 1 && t - 1 < N && s < ns) {
        const double* z = G + 2 * ((int64_t)(t - 1) * k + rp.col[s]);
        const double br = rp.beta[2 * s], bi = rp.beta[2 * s + 1];
        g = part == 0 ? (z[0] * br - z[1] * bi) * rp.xscale : (z[0] * bi + z[1] * br) * rp.xscale;
      }
      double rem = g;
      for (int sp = 0; sp < rp.NSG; ++sp) {
        const uint16_t bits = bf16_bits_d(rem);
        rem -= bf16_val_d(bits);
        Gp[(((int64_t)ks * rp.NSG + sp) * 64 + l) * 8 + i] = bits;
      }
    } else {
      const int64_t ev = e - ng;
      const int q = (int)((ev >> 9) & 1);
      const int64_t fbi = ev >> 10;
      const int hh = l >> 5;
      const int64_t t = 32 * fbi + (l & 31);
      const int j = 8 * q + i;                 // slot of half hh (column 16q + 8(i/4) + 4hh + i%4)
      const int s = 2 * (j >> 1) + hh, part = j & 1;
      float v = 0.f;
      if (fbi < rp.NFB && s < ns) {
        double pr = 1.0, pi = 0.0;
        if (!rp.static_bg) {
          double br = rp.lam[2 * s], bi = rp.lam[2 * s + 1];
          for (int64_t ex = t; ex > 0; ex >>= 1) {
            if (ex & 1) {
              const double nr = pr * br - pi * bi, ni = pr * bi + pi * br;
              pr = nr;
              pi = ni;
            }
            const double sr = br * br - bi * bi, si = 2.0 * br * bi;
            br = sr;
            bi = si;
          }
        }
        v = part == 0 ? (float)pr : (float)(-pi);
      }
      float rem = v;
      for (int sp = 0; sp < rp.NTV; ++sp) {
        const uint32_t bits = bf16_rne_bits(rem);
        rem -= __uint_as_float(bits << 16);
        Vp[((((fbi * 2 + q) * rp.NTV + sp) * 64 + l) * 8) + i] = (uint16_t)bits;
      }
    }
  }
}

hipError_t recon_prep(const double* G, const ReconPrep& rp, void* Gp, void* Vp, hipStream_t s) {
  if (rp.ns < 0 || rp.ns > 16 || rp.NSG < 1 || rp.NSG > 3 || rp.NTV < 1 || rp.NTV > 3) return hipErrorInvalidValue;
  const int64_t total = (int64_t)(rp.KS + RC_PF) * 64 * 8 + (int64_t)(rp.NFB + 1) * 2 * 64 * 8;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 1024);
  hipLaunchKernelGGL(k_recon_prep, dim3(grid), dim3(256), 0, s, G, rp, (uint16_t*)Gp, (uint16_t*)Vp);
  return hipGetLastError();
}

int recon_column(int s, int part) { return rc_col(s, part); }

template <int NSG, int NTV, int MODE, bool RAGGED>
static hipError_t launch_recon1(const ReconArgs& a, size_t lds, int64_t tile0, int64_t tiles, hipStream_t s) {
  static std::atomic<bool> attr{false};  // the larger dynamic LDS limit, set once per instantiation
  if (!attr.load(std::memory_order_acquire)) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_recon<NSG, NTV, MODE, RAGGED>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr.store(true, std::memory_order_release);
  }
  const int64_t blocks = 8 * ((tiles + 7) / 8);
  hipLaunchKernelGGL((k_recon<NSG, NTV, MODE, RAGGED>), dim3((unsigned)blocks), dim3(RC_NT), lds, s, a, tile0, tiles);
  return hipGetLastError();
}

template <int NSG, int NTV, int MODE>
static hipError_t launch_recon(const ReconArgs& a, size_t lds, hipStream_t s) {
  const int64_t full = a.n / RC_TP;
  if (full > 0) {
    const hipError_t e = launch_recon1<NSG, NTV, MODE, false>(a, lds, 0, full, s);
    if (e != hipSuccess) return e;
  }
  if (a.n % RC_TP) return launch_recon1<NSG, NTV, MODE, true>(a, lds, full, 1, s);
  return hipSuccess;
}

template <int NSG, int NTV, int MODE, bool RAGGED>
static hipError_t launch_recon_list(const ReconWork* list, int nw, int64_t total, size_t lds, hipStream_t s) {
  static std::atomic<bool> attr{false};
  if (!attr.load(std::memory_order_acquire)) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_recon_list<NSG, NTV, MODE, RAGGED>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr.store(true, std::memory_order_release);
  }
  const int64_t blocks = 64 * ((total + 63) / 64);
  hipLaunchKernelGGL((k_recon_list<NSG, NTV, MODE, RAGGED>), dim3((unsigned)blocks), dim3(RC_NT), lds, s, list, nw,
                     total);
  return hipGetLastError();
}

hipError_t recon_mfma_list(const ReconWork* list, int nw, int64_t total, size_t lds, int nsg, int ntv, int mode,
                           bool ragged, hipStream_t s) {
  if (list == nullptr || nw < 1 || nw > 64 || total < 1 || total > ((int64_t)1 << 31) - 64 || lds > 160 * 1024 ||
      mode < 0 || mode > 2)
    return hipErrorInvalidValue;
#define RL_MODE(G, T, R)                                                   \
  if (mode == 0) return launch_recon_list<G, T, 0, R>(list, nw, total, lds, s); \
  if (mode == 1) return launch_recon_list<G, T, 1, R>(list, nw, total, lds, s); \
  return launch_recon_list<G, T, 2, R>(list, nw, total, lds, s);
#define RL_CASE(G, T)                 \
  if (nsg == G && ntv == T) {         \
    if (ragged) {                     \
      RL_MODE(G, T, true)             \
    }                                 \
    RL_MODE(G, T, false)              \
  }
  RL_CASE(2, 3)
  RL_CASE(1, 2)
#undef RL_CASE
#undef RL_MODE
  return hipErrorInvalidValue;
}

int recon_tile_pixels() { return RC_TP; }
int recon_ksteps(int64_t m) { return (int)(4 * ((m + 63) / 64)); }
int recon_frame_blocks(int64_t m) { return (int)((m + 31) / 32); }

hipError_t recon_mfma(const ReconArgs& a, int nsg, int ntv, hipStream_t s) {
  if (a.ns < 0 || a.ns > 16 || a.n < 1 || a.m < 2 || a.m >= (1 << 30) || a.KS != recon_ksteps(a.m) ||
      a.NFB != recon_frame_blocks(a.m) || a.mode < 0 || a.mode > 2)
    return hipErrorInvalidValue;
  if (a.mode == 2 && (a.t0 < 0 || a.t1 > a.m || a.t0 >= a.t1)) return hipErrorInvalidValue;
  const size_t lds = recon_lds_bytes(a.m);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
#define RC_CASE(G, T)                                                    \
  if (nsg == G && ntv == T) {                                            \
    if (a.mode == 0) return launch_recon<G, T, 0>(a, lds, s);            \
    if (a.mode == 1) return launch_recon<G, T, 1>(a, lds, s);            \
    return launch_recon<G, T, 2>(a, lds, s);                             \
  }
  RC_CASE(2, 3)
  RC_CASE(1, 2)
#undef RC_CASE
  return hipErrorInvalidValue;
}

int lift_mfma_grid(int64_t n) {
  const int64_t tiles = (n + LM_TILE - 1) / LM_TILE;
  return (int)(tiles < 512 ? tiles : 512);
}

hipError_t lift_mfma(const uint8_t* D, int64_t ld, int64_t n, int64_t m, const void* Gp, int nb,
                     int nsplit, int nksteps, int nc, float xscale, double* part, int grid,
                     float* phi, int kmodes, hipStream_t s) {
#define LM_CASE(NBV, NSV)                                                                    \
  if (nb == NBV && nsplit == NSV) {                                                          \
    hipLaunchKernelGGL((k_lift_mfma<NBV, NSV>), dim3(grid), dim3(256), 0, s, D, ld, n, m,    \
                       (const uint4*)Gp, nksteps, nc, xscale, part, phi, kmodes);            \
    return hipGetLastError();                                                                \
  }
  LM_CASE(1, 1)
  LM_CASE(1, 3)
  LM_CASE(2, 1)
  LM_CASE(2, 3)
  LM_CASE(3, 1)
  LM_CASE(3, 3)
#undef LM_CASE
  return hipErrorInvalidValue;
}

// Deterministic column sums of part[grid][ne]: block = 16 entries x 16 row groups; row
// group g sums blocks b = g, g+16, ... in order, then the 16 group sums are added in
// order.
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ part, int grid,
                                                         int ne, double* __restrict__ out) {
  __shared__ double red[16][17];
  const int e = blockIdx.x * 16 + (threadIdx.x & 15), g = threadIdx.x >> 4;
  double s = 0.0;
  if (e < ne)
    for (int b = g; b < grid; b += 16) s += part[(int64_t)b * ne + e];
  red[g][threadIdx.x & 15] = s;
  __syncthreads();
  if (threadIdx.x < 16 && blockIdx.x * 16 + threadIdx.x < ne) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += red[q][threadIdx.x];
    out[blockIdx.x * 16 + threadIdx.x] = t;
  }
}

hipError_t reduce_partials(const double* part, int grid, int ne, double* out,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_reduce_partials, dim3((ne + 15) / 16), dim3(256), 0, stream, part, grid,
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

// 3x3 median of a binary H x W mask (pixel i = y W + x of a frame): the majority of the
// nine neighbours, rows and columns beyond the border replicated from the edge.
__device__ __forceinline__ int median3_count(int64_t y, int64_t x, int64_t H, int64_t W, const uint32_t* words,
                                             const uint8_t* bytes) {
  int cnt = 0;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy) {
    const int64_t yy = y + dy < 0 ? 0 : (y + dy >= H ? H - 1 : y + dy);
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int64_t xx = x + dx < 0 ? 0 : (x + dx >= W ? W - 1 : x + dx);
      const int64_t j = yy * W + xx;
      cnt += words != nullptr ? (int)((words[j >> 5] >> (j & 31)) & 1u) : (bytes[j] != 0 ? 1 : 0);
    }
  }
  return cnt;
}

// bit-packed: a thread per output word (32 pixels) of frame blockIdx.y
__global__ __launch_bounds__(256) void k_mask_median3_bits(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                           int64_t H, int64_t W, int64_t words) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= words) return;
  const int64_t n = H * W, t = blockIdx.y;
  const uint32_t* f = in + t * words;
  uint32_t o = 0;
  for (int b = 0; b < 32; ++b) {
    const int64_t i = w * 32 + b;
    if (i >= n) break;
    if (median3_count(i / W, i % W, H, W, f, nullptr) >= 5) o |= 1u << b;
  }
  out[t * words + w] = o;
}

// bit-packed with W a multiple of 32 (every row starts a word): a thread per output word,
// the nine neighbours as nine shifted words (left and right neighbours by shifting across
// the adjacent words, the edge pixel replicated at the row ends), their majority by a
// bit-sliced adder: the count is s + 2T with s the parity of the nine and T the sum of the
// four carries; count >= 5 iff T >= 3, or T == 2 and s == 1.
__device__ __forceinline__ void csa(uint32_t a, uint32_t b, uint32_t c, uint32_t& s, uint32_t& cy) {
  const uint32_t ab = a ^ b;
  s = ab ^ c;
  cy = (a & b) | (c & ab);
}

__global__ __launch_bounds__(256) void k_mask_median3_rows(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                           int H, int wpr) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;  // word of the frame
  if (w >= H * wpr) return;
  const int y = w / wpr, c = w - y * wpr;
  const int64_t words = (int64_t)H * wpr;
  const uint32_t* f = in + (int64_t)blockIdx.y * words;
  uint32_t rs[3], rc[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int yy = y + d - 1;
    yy = yy < 0 ? 0 : (yy >= H ? H - 1 : yy);
    const uint32_t* row = f + (int64_t)yy * wpr;
    const uint32_t C = row[c];
    const uint32_t L = c > 0 ? row[c - 1] : 0u, R = c + 1 < wpr ? row[c + 1] : 0u;
    const uint32_t left = (C << 1) | (c > 0 ? L >> 31 : (C & 1u));                    // pixel x - 1
    const uint32_t right = (C >> 1) | (c + 1 < wpr ? R << 31 : (C & 0x80000000u));     // pixel x + 1
    csa(left, C, right, rs[d], rc[d]);
  }
  uint32_t s, cc;
  csa(rs[0], rs[1], rs[2], s, cc);           // weight 1: s; weight 2: cc
  uint32_t u, v;
  csa(rc[0], rc[1], rc[2], u, v);            // T = u + cc + 2 v (in units of 2)
  const uint32_t w1 = u ^ cc, ca = u & cc;   // T = w1 + 2 (v + ca)
  const uint32_t one = v ^ ca, two = v & ca; // v + ca == 1, == 2
  out[(int64_t)blockIdx.y * words + w] = two | (one & w1) | (one & ~w1 & s);
}

// uint8 (0/1): a thread per pixel of frame blockIdx.y
__global__ __launch_bounds__(256) void k_mask_median3_u8(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                         int64_t H, int64_t W) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = H * W, t = blockIdx.y;
  if (i >= n) return;
  out[t * n + i] = median3_count(i / W, i % W, H, W, nullptr, in + t * n) >= 5 ? 1 : 0;
}

hipError_t mask_median3(const void* in, void* out, int64_t H, int64_t W, int64_t m, int bitpacked,
                        hipStream_t stream) {
  const int64_t n = H * W;
  if (bitpacked && W % 32 == 0 && n < ((int64_t)1 << 31)) {
    const int wpr = (int)(W / 32);
    const int64_t words = n / 32;
    hipLaunchKernelGGL(k_mask_median3_rows, dim3((unsigned)((words + 255) / 256), (unsigned)m), dim3(256), 0, stream,
                       (const uint32_t*)in, (uint32_t*)out, (int)H, wpr);
  } else if (bitpacked) {
    const int64_t words = (n + 31) / 32;
    hipLaunchKernelGGL(k_mask_median3_bits, dim3((unsigned)((words + 255) / 256), (unsigned)m), dim3(256), 0, stream,
                       (const uint32_t*)in, (uint32_t*)out, H, W, words);
  } else {
    hipLaunchKernelGGL(k_mask_median3_u8, dim3((unsigned)((n + 255) / 256), (unsigned)m), dim3(256), 0, stream,
                       (const uint8_t*)in, (uint8_t*)out, H, W);
  }
  return hipGetLastError();
}


// ============================================================================
// small float64 linear algebra on the device: one 1024-thread workgroup runs
// The truncated SVD, A~ and eig(A~) of Section 3.2 and G = V S^-1 W (team_la.hpp), then writes the B operands
// of the lift (bf16 terms of G * xscale in MFMA order) so the fit needs no host round
// trip between the Gram and the lift.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ double lane_f64(double v, int l) {
  const uint64_t u = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// One wave of a workgroup acting alone: lanes are its threads, and a synchronisation is a
// wave-level memory fence (the wave's LDS and global accesses then complete in order).
struct WaveTeam {
  int tid, nt, lane, wsize, wave, nwaves;
  __device__ void sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __device__ void stamp(int) {}
  __device__ void tick(int) {}
  // Sum over the wave, the same bits on every lane: within each row of 16 lanes a DPP
  // butterfly (lane pairs i^1, i^2, then the 8- and 16-lane mirrors; every pair adds the
  // same two values), then the four row sums are read as scalars and added in fixed order.
  __device__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
  }
  // the sums over lanes 0..31 (lo) and 32..63 (hi), the same bits on every lane
  __device__ void half_sums(double v, double& lo, double& hi) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    lo = lane_f64(v, 0) + lane_f64(v, 16);
    hi = lane_f64(v, 32) + lane_f64(v, 48);
  }
  __device__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
  }
  // maximum value, lowest index among equal values; identical on every lane
  __device__ void wave_argmax(double& v, int& i) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(v, o, 64);
      const int oi = __shfl_xor(i, o, 64);
      if (ov > v || (ov == v && oi < i)) v = ov, i = oi;
    }
  }
  __device__ int wave_first(bool b) {
    const unsigned long long m = __ballot(b);
    return m ? __ffsll((long long)m) - 1 : 64;
  }
  __device__ double sum(double v) { return wave_sum(v); }
  __device__ double maxv(double v) { return wave_max(v); }
  __device__ WaveTeam wave_team() { return *this; }
  // 1/x from the hardware estimate and two Newton steps (x normal and finite)
  __device__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
  }
};

struct DevTeam : WaveTeam {
  double* red;
  double* tslots;     // phase clocks (wall_clock64 ticks): [0] tridiagonal checks, [2..9]
  uint64_t t_last;    // marks, [10..12] Lanczos sub-phases
  uint64_t t_tick;
  __device__ void sync() { __syncthreads(); }
  // 0: start of a convergence check, 1: its end (accumulated in slot 0); 2..: phase marks
  __device__ __forceinline__ void stamp(int i) {
    if (tid != 0 || tslots == nullptr) return;
    const uint64_t t = wall_clock64();
    if (i == 0) t_last = t;
    else if (i == 1) tslots[0] += (double)(t - t_last);
    else tslots[i] = (double)t;
  }
  // accumulate the time since the previous tick into slot i (i < 0: restart)
  __device__ __forceinline__ void tick(int i) {
    if (tid != 0 || tslots == nullptr) return;
    const uint64_t t = wall_clock64();
    if (i >= 0) tslots[i] += (double)(t - t_tick);
    t_tick = t;
  }
  __device__ __forceinline__ double sum(double v) {
    v = wave_sum(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += red[w];
    __syncthreads();
    return s;
  }
  __device__ WaveTeam wave_team() {
    WaveTeam t;
    t.tid = lane;
    t.nt = wsize;
    t.lane = lane;
    t.wsize = wsize;
    t.wave = 0;
    t.nwaves = 1;
    return t;
  }
};

constexpr int SLA_NMAX = 1024;
constexpr int SLA_JMAX = 320;
constexpr int SLA_FAST = tla::kLaFast;  // LDS doubles: tridiagonal eigen-solve work, later scratch


// The small linear algebra of one solve runs as five kernels, each with a grid row
// (blockIdx.y, or blockIdx.x for the one-workgroup kernels) per solve of a batch:
//   k_la_a     one workgroup: non-finite check, Lanczos, Ritz vectors Z of T_J
//   k_la_ritz  a workgroup per kLaRows rows: V = Q_J Z
//   k_la_tv    a workgroup per kLaRows rows: TV = M12 V and the block partials of V^T TV
//   k_la_b     one workgroup: A~ from the partials, its eigenvalues and eigenvectors
//   k_la_g     a workgroup per kLaRows rows: G = V S^-1 W and the lift's bf16 operands
// Every kernel after the first returns at once when the solve's status is not OK.
constexpr int SLA_ROWS_NT = 512;
constexpr int SLA_STAGE = 8192;  // LDS doubles of the row kernels

__device__ __forceinline__ const SLADesc& la_desc(const SLADesc& d1, const SLADesc* ds, int q) {
  return ds != nullptr ? ds[q] : d1;
}

__device__ __forceinline__ void la_team(DevTeam& tm, double* red, double* tslots) {
  tm.tid = threadIdx.x;
  tm.nt = blockDim.x;
  tm.lane = threadIdx.x & 63;
  tm.wsize = 64;
  tm.wave = threadIdx.x >> 6;
  tm.nwaves = blockDim.x >> 6;
  tm.red = red;
  tm.tslots = tslots;
  tm.t_last = 0;
  tm.t_tick = 0;
}

__device__ void la_work(tla::SmallLAWork& ws, const SLADesc& d, double* s_q, double* s_w, double* s_h,
                        double* s_alpha, double* s_beta, double* s_fast, int* s_flag, double* s_qc = nullptr) {
  using namespace tla;
  const SmallLALayout Ls = small_la_layout(d.m - 1, d.k, d.Jmax);
  double* scratch = d.scratch;
  ws.lz = LanczosWork{s_q, s_w, s_h, s_alpha, s_beta, scratch + Ls.T, s_fast, SLA_FAST, s_qc,
                      s_qc != nullptr ? tla::kLaQCache : 0};
  ws.Q = scratch + Ls.Q;
  ws.V = scratch + Ls.V;
  ws.Z = scratch + Ls.Z;
  ws.TV = scratch + Ls.TV;
  ws.P = scratch + Ls.P;
  ws.nu = scratch + Ls.nu;
  ws.At = scratch + Ls.At;
  ws.Hs = scratch + Ls.Hs;
  ws.LU = reinterpret_cast<cpx*>(scratch + Ls.LU);
  ws.bb = reinterpret_cast<cpx*>(scratch + Ls.bb);
  ws.yy = reinterpret_cast<cpx*>(scratch + Ls.yy);
  ws.piv = reinterpret_cast<int*>(scratch + Ls.piv);
  ws.flag = s_flag;
}

// Exchange between the workgroups of one solve (the row groups of the Lanczos vectors).
// The shares travel through global memory as device-scope (agent) atomic stores and loads,
// which are performed at the device's coherence point, so no cache write-back or
// invalidation is needed: each wave waits for its stores to complete, one thread arrives
// at a counter and waits for all groups, then every wave loads the shares.  The wait is
// bounded: past kSpinLimit polls the exchange reports failure and the kernel returns.
constexpr unsigned kSpinLimit = 1u << 21;

__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct GridX {
  int g, G, r0, r1, N, NQ, PS;
  double* xb;       // two buffers of G*PS partials and an NQ-vector (128-byte aligned)
  unsigned* bar;    // arrivals (zeroed before the launch)
  unsigned nx;      // exchanges so far
  int* s_ok;        // LDS: the wait's outcome
  __device__ __forceinline__ bool exchange(DevTeam& tm, const double* part, int n, double* sum, const double* slice,
                                           double* full) {
    tm.sync();
    if (G == 1) {
      if (sum != part)
        for (int i = tm.tid; i < n; i += tm.nt) sum[i] = part[i];
      if (slice != nullptr && full != slice)
        for (int t = r0 + tm.tid; t < r1; t += tm.nt) full[t] = slice[t];
      tm.sync();
      return true;
    }
    // consecutive exchanges use alternate buffers: a buffer is written again only after
    // every group has passed the exchange in between, so after all have read it
    double* base = xb + (int64_t)(nx & 1u) * ((int64_t)G * PS + NQ);
    for (int i = tm.tid; i < n; i += tm.nt) st_dev(&base[(int64_t)g * PS + i], part[i]);
    if (slice != nullptr)
      for (int t = r0 + tm.tid; t < r1; t += tm.nt) st_dev(&base[(int64_t)G * PS + t], slice[t]);
    ++nx;
    tm.tick(11);  // phase clock: the work before the exchange
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have completed
    __syncthreads();
    if (tm.tid == 0) {
      const unsigned target = nx * (unsigned)G;
      __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int ok = 1;
      unsigned spins = 0;
      while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > kSpinLimit) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      s_ok[0] = ok;
    }
    __syncthreads();
    if (s_ok[0] == 0) return false;  // uniform
    tm.tick(8);  // the wait
    for (int i = tm.tid; i < n; i += tm.nt) {
      double v = 0.0;  // in group order; eight loads in flight
      for (int q0 = 0; q0 < G; q0 += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = q0 + u < G ? ld_dev(&base[(int64_t)(q0 + u) * PS + i]) : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (q0 + u < G) v += x[u];
      }
      sum[i] = v;
    }
    if (full != nullptr)
      for (int t = tm.tid; t < N; t += tm.nt) full[t] = ld_dev(&base[(int64_t)G * PS + t]);
    tm.sync();
    tm.tick(9);  // the loads of the shares
    return true;
  }
};

// Clears a solve's status, Krylov size, phase clocks and exchange counter.
__global__ __launch_bounds__(64) void k_la_prep(SLADesc d1, const SLADesc* __restrict__ ds) {
  using namespace tla;
  const SLADesc& d = la_desc(d1, ds, blockIdx.x);
  const int N = d.m - 1;
  const SmallLAOutLayout Lo = small_la_out_layout(N, d.k);
  const SmallLALayout Ls = small_la_layout(N, d.k, d.Jmax);
  const int t = threadIdx.x;
  if (t < 16) d.out[Lo.timing + t] = 0.0;
  if (t == 0) {
    d.out[Lo.status] = 0.0;
    d.out[Lo.J] = 0.0;
    *reinterpret_cast<unsigned*>(d.scratch + Ls.X) = 0u;
  }
}

// Lanczos and the Ritz vectors of T_J: la_groups(N) workgroups of SLA_A_NT threads per solve
// (blockIdx.x), each owning a range of rows of the Lanczos vectors; group 0 runs the
// convergence checks and writes the results.
constexpr int SLA_A_NT = 512;  // Lanczos workgroup size: 256 registers per thread

__global__ __launch_bounds__(SLA_A_NT) void k_la_a(SLADesc d1, const SLADesc* __restrict__ ds) {
  using namespace tla;
  const SLADesc& d = la_desc(d1, ds, blockIdx.y);
  const int m = d.m, k = d.k, N = m - 1;
  const int G = d.groups > 0 ? (d.groups < N ? d.groups : N) : la_groups(N), g = blockIdx.x;
  if (g >= G) return;  // uniform: this solve needs fewer groups than the grid has
  __shared__ double s_q[SLA_NMAX], s_w[SLA_NMAX];
  __shared__ double s_h[SLA_JMAX + 4], s_alpha[SLA_JMAX + 4], s_beta[SLA_JMAX + 4];
  __shared__ double s_red[16];
  __shared__ int s_flag[1], s_ok[1];
  __shared__ double s_fast[SLA_FAST];
  __shared__ double s_qc[tla::kLaQCache];
  __shared__ double s_ts[16];  // group 0's phase clocks, accumulated in LDS and written at the end
  const SmallLAOutLayout Lo = small_la_out_layout(N, k);
  const SmallLALayout Ls = small_la_layout(N, k, d.Jmax);
  double* out = d.out;
  if (threadIdx.x < 16) s_ts[threadIdx.x] = 0.0;
  __syncthreads();
  DevTeam tm;
  la_team(tm, s_red, g == 0 ? s_ts : nullptr);
  tm.tick(-1);
  SmallLAWork ws;
  la_work(ws, d, s_q, s_w, s_h, s_alpha, s_beta, s_fast, s_flag, s_qc);
  GridX xg;
  xg.g = g;
  xg.G = G;
  la_group_rows(N, G, g, &xg.r0, &xg.r1);
  xg.N = N;
  xg.NQ = la_ldq(N);
  xg.PS = la_xps(d.Jmax);
  xg.bar = reinterpret_cast<unsigned*>(d.scratch + Ls.X);
  xg.xb = d.scratch + Ls.X + 16;
  xg.nx = 0;
  xg.s_ok = s_ok;
  int J = 0;
  const int st = small_la_phase_a(tm, xg, d.Gr, m, k, d.rtol, d.Jmax, ws, out + Lo.mu, ws.Z, &J);
  __syncthreads();
  // slots 4..7 belong to the kernels after this one
  if (g == 0 && threadIdx.x < 16 && (threadIdx.x < 4 || threadIdx.x >= 8)) out[Lo.timing + threadIdx.x] = s_ts[threadIdx.x];
  if (tm.tid == 0) {
    if (g == 0) {
      out[Lo.status] = (double)st;
      out[Lo.J] = (double)J;
    } else if (st == kDevice) {
      out[Lo.status] = (double)st;
    }
  }
}

// Dense products of the small LA on FP64 MFMA (v_mfma_f64_16x16x4f64: lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; item r of lane l is D[4r + l/16][l%16]).  A workgroup
// of 4 waves takes kLaRows = 64 rows, a wave 16 rows x up to 64 columns (four 16-column
// tiles), the inner dimension 4 at a time with its loads issued ahead.
constexpr int SLA_MM_NT = 256;

// out[c*ldo + r] = sum_{q < K} A(r, q) B(q, c) for rows r in [r0, r0 + 16) (< R) and
// columns c < C (<= 64), with A(r, q) = pa[q*lda + r] and B(q, c) = pb[q*ldb + c*cstride].
// The same products over the inner indices q in [qb, qe) only (qb a multiple of 16),
// added into acc (the caller zeroes it).
__device__ __forceinline__ void mfma_rows16_acc(const double* __restrict__ pa, int64_t lda,
                                                const double* __restrict__ pb, int64_t ldb, int64_t cstride,
                                                int qb, int qe, int r0, int R, int C, f64x4_t (&acc)[4]) {
  const int l = threadIdx.x & 63, i = l & 15, kq = l >> 4;
  const int CT = (C + 15) >> 4;
  const int r = r0 + i;
  for (int q0 = qb; q0 < qe; q0 += 16) {
    double av[4], bv[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = q0 + 4 * u + kq;
      av[u] = r < R && q < qe ? pa[(int64_t)q * lda + r] : 0.0;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int c = 16 * ct + i;
        bv[u][ct] = ct < CT && q < qe && c < C ? pb[(int64_t)q * ldb + (int64_t)c * cstride] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
        if (ct < CT) acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u][ct], acc[ct], 0, 0, 0);
  }
}

__device__ __forceinline__ void mfma_rows16(const double* __restrict__ pa, int64_t lda, const double* __restrict__ pb,
                                            int64_t ldb, int64_t cstride, int K, int r0, int R, int C,
                                            double* __restrict__ out, int64_t ldo) {
  const int l = threadIdx.x & 63, i = l & 15, kq = l >> 4;
  const int CT = (C + 15) >> 4;
  f64x4_t acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = f64x4_t{0.0, 0.0, 0.0, 0.0};
  mfma_rows16_acc(pa, lda, pb, ldb, cstride, 0, K, r0, R, C, acc);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int ro = r0 + 4 * rr + kq, c = 16 * ct + i;
      if (ct < CT && ro < R && c < C) out[(int64_t)c * ldo + ro] = acc[ct][rr];
    }
}

// V = Q_J Z over the workgroup's kLaRows rows.
__global__ __launch_bounds__(SLA_MM_NT) void k_la_ritz(SLADesc d1, const SLADesc* __restrict__ ds) {
  using namespace tla;
  const SLADesc& d = la_desc(d1, ds, blockIdx.y);
  const int N = d.m - 1, k = d.k;
  const int t0 = blockIdx.x * kLaRows;
  const SmallLAOutLayout Lo = small_la_out_layout(N, k);
  if (t0 >= N || d.out[Lo.status] != 0.0) return;  // uniform over the workgroup
  const SmallLALayout Ls = small_la_layout(N, k, d.Jmax);
  const int J = (int)d.out[Lo.J];
  if (k <= 64) {
    // V(t, c) = sum_i Q(i, t) Z(i, c): A(t, i) = Q[i*ldq + t], B(i, c) = Z[i*k + c]
    mfma_rows16(d.scratch + Ls.Q, la_ldq(N), d.scratch + Ls.Z, k, 1, J, t0 + 16 * (threadIdx.x >> 6), N, k,
                d.scratch + Ls.V, N);
    return;
  }
  __shared__ double s_red[SLA_MM_NT / 64];
  DevTeam tm;
  la_team(tm, s_red, nullptr);
  ritz_rows(tm, d.scratch + Ls.Q, N, J, d.scratch + Ls.Z, k, d.scratch + Ls.V, t0,
            t0 + kLaRows < N ? t0 + kLaRows : N);
}

// TV = M12 V over the workgroup's rows, and the block's partials of V^T TV and |v_i|^2.
// TV = M12 V: 8 waves, the inner index (length N) split in two halves between waves
// 0-3 and 4-7 (each wave 16 rows), the halves added in that order through LDS.
constexpr int SLA_TV_NT = 512;
__global__ __launch_bounds__(SLA_TV_NT) void k_la_tv(SLADesc d1, const SLADesc* __restrict__ ds) {
  using namespace tla;
  const SLADesc& d = la_desc(d1, ds, blockIdx.y);
  const int m = d.m, N = m - 1, k = d.k;
  const int t0 = blockIdx.x * kLaRows;
  const SmallLAOutLayout Lo = small_la_out_layout(N, k);
  if (t0 >= N || d.out[Lo.status] != 0.0) return;
  __shared__ double s_red[SLA_TV_NT / 64];
  __shared__ double s_stage[SLA_STAGE];
  DevTeam tm;
  la_team(tm, s_red, nullptr);
  const SmallLALayout Ls = small_la_layout(N, k, d.Jmax);
  const int t1 = t0 + kLaRows < N ? t0 + kLaRows : N;
  double* V = d.scratch + Ls.V;
  double* TV = d.scratch + Ls.TV;
  if (k <= 64) {
    // TV(a, c) = sum_b M12(a, b) V(b, c) with M12(a, b) = Gram[(b+1)*m + a] (symmetric):
    // A(a, b) = Gr[(b+1)*m + a], B(b, c) = V[c*N + b]
    const int w = threadIdx.x >> 6, rg = w & 3, half = w >> 2, l = threadIdx.x & 63;
    const int Kh = ((N + 31) / 32) * 16;  // first half [0, Kh), a multiple of 16
    const int rw = t0 + 16 * rg;
    f64x4_t acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    mfma_rows16_acc(d.Gr + m, m, V, 1, N, half == 0 ? 0 : Kh, half == 0 ? (Kh < N ? Kh : N) : N, rw, N, k, acc);
    // s_stage as the exchange: [rg][ct][rr][lane], 4 * 4 * 4 * 64 = 4096 doubles
    if (half == 1)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) s_stage[((rg * 4 + ct) * 4 + rr) * 64 + l] = acc[ct][rr];
    __syncthreads();
    if (half == 0) {
      const int i = l & 15, kq = l >> 4, CT = (k + 15) >> 4;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int ro = rw + 4 * rr + kq, c = 16 * ct + i;
          if (ct < CT && ro < N && c < k)
            TV[(int64_t)c * N + ro] = acc[ct][rr] + s_stage[((rg * 4 + ct) * 4 + rr) * 64 + l];
        }
    }
    __syncthreads();
  } else {
    m12v_rows(tm, d.Gr, m, N, k, V, TV, t0, t1, s_stage, SLA_STAGE);
  }
  block_gram(tm, V, TV, N, k, t0, t1, d.scratch + Ls.P + (int64_t)blockIdx.x * ((int64_t)k * k + k), s_stage,
             SLA_STAGE);
}

// A~ from the block partials and its eigenvalues (one workgroup per solve).
__global__ __launch_bounds__(1024) void k_la_b(SLADesc d1, const SLADesc* __restrict__ ds) {
  using namespace tla;
  const SLADesc& d = la_desc(d1, ds, blockIdx.x);
  const int N = d.m - 1, k = d.k;
  const SmallLAOutLayout Lo = small_la_out_layout(N, k);
  double* out = d.out;
  if (out[Lo.status] != 0.0) return;
  __shared__ double s_w[SLA_NMAX];
  __shared__ double s_red[16];
  __shared__ int s_flag[1];
  __shared__ double s_fast[SLA_FAST];
  DevTeam tm;
  la_team(tm, s_red, out + Lo.timing);
  SmallLAWork ws;
  la_work(ws, d, nullptr, s_w, nullptr, nullptr, nullptr, s_fast, s_flag);
  const int nblk = (N + kLaRows - 1) / kLaRows;
  const int st = small_la_phase_b1(tm, N, k, d.sketch_scale, ws, nblk, out + Lo.mu, out + Lo.sigma,
                                   reinterpret_cast<cpx*>(out + Lo.lam));
  if (tm.tid == 0 && st != kOk) out[Lo.status] = (double)st;
}

// One eigenvector of A~ per single-wave workgroup (blockIdx.x = its index), so that the
// inverse iterations run on separate compute units; the second member of a conjugate pair
// is left to k_la_b3.  LU work in LDS (dynamic, 2k^2 + 5k doubles for the largest k of
// the launch, so the workgroup fits beside others) for k <= 64, else in the solve's
// global scratch.

__global__ __launch_bounds__(64) void k_la_v(SLADesc d1, const SLADesc* __restrict__ ds) {
  using namespace tla;
  const SLADesc& d = la_desc(d1, ds, blockIdx.y);
  const int N = d.m - 1, k = d.k, j = blockIdx.x;
  const SmallLAOutLayout Lo = small_la_out_layout(N, k);
  double* out = d.out;
  if (j >= k || out[Lo.status] != 0.0) return;
  const cpx* lam = reinterpret_cast<const cpx*>(out + Lo.lam);
  if (conj_second(lam, j)) return;
  extern __shared__ double s_lu[];
  const SmallLALayout Ls = small_la_layout(N, k, d.Jmax);
  WaveTeam wt;
  wt.tid = wt.lane = threadIdx.x;
  wt.nt = wt.wsize = 64;
  wt.wave = 0;
  wt.nwaves = 1;
  cpx *LU, *b, *y;
  int* piv;
  if (k <= 64) {
    LU = reinterpret_cast<cpx*>(s_lu);
    b = LU + (int64_t)k * k;
    y = b + k;
    piv = reinterpret_cast<int*>(y + k);
  } else {
    LU = reinterpret_cast<cpx*>(d.scratch + Ls.LU) + (int64_t)j * k * k;
    b = reinterpret_cast<cpx*>(d.scratch + Ls.bb) + (int64_t)j * k;
    y = reinterpret_cast<cpx*>(d.scratch + Ls.yy) + (int64_t)j * k;
    piv = reinterpret_cast<int*>(d.scratch + Ls.piv) + (int64_t)j * k;
  }
  const bool ok = eigvec_wave(wt, d.scratch + Ls.At, k, lam[j].re, lam[j].im, LU, b, y, piv,
                              reinterpret_cast<cpx*>(out + Lo.W) + (int64_t)j * k);
  if (!ok && threadIdx.x == 0) out[Lo.status] = (double)kNumeric;
}

// The conjugate partners and the normalisation of W (one workgroup per solve).
__global__ __launch_bounds__(256) void k_la_b3(SLADesc d1, const SLADesc* __restrict__ ds) {
  using namespace tla;
  const SLADesc& d = la_desc(d1, ds, blockIdx.x);
  const int N = d.m - 1, k = d.k;
  const SmallLAOutLayout Lo = small_la_out_layout(N, k);
  double* out = d.out;
  if (out[Lo.status] != 0.0) return;
  __shared__ double s_red[4];
  DevTeam tm;
  la_team(tm, s_red, out + Lo.timing);
  small_la_phase_b3(tm, k, reinterpret_cast<const cpx*>(out + Lo.lam), reinterpret_cast<cpx*>(out + Lo.W));
}

// G = V S^-1 W over the workgroup's rows.
__global__ __launch_bounds__(SLA_ROWS_NT) void k_la_g(SLADesc d1, const SLADesc* __restrict__ ds) {
  using namespace tla;
  const SLADesc& d = la_desc(d1, ds, blockIdx.y);
  const int N = d.m - 1, k = d.k;
  const int t0 = blockIdx.x * kLaRows;
  const SmallLAOutLayout Lo = small_la_out_layout(N, k);
  double* out = d.out;
  if (t0 >= N || out[Lo.status] != 0.0) return;
  __shared__ double s_red[SLA_ROWS_NT / 64];
  DevTeam tm;
  la_team(tm, s_red, blockIdx.x == 0 ? out + Lo.timing : nullptr);
  const SmallLALayout Ls = small_la_layout(N, k, d.Jmax);
  g_rows(tm, d.scratch + Ls.V, N, k, d.scratch + Ls.nu, out + Lo.sigma, reinterpret_cast<const cpx*>(out + Lo.W),
         reinterpret_cast<cpx*>(out + Lo.G), t0, t0 + kLaRows < N ? t0 + kLaRows : N);
  tm.stamp(7);
}

// The lift's B operands of the real basis V S^-1 (the modes are (X' V S^-1) W; the lift
// forms X' V S^-1 and W is applied to its k x k products in float64 on the host), for the
// 16-row groups of the workgroup's 64 rows: [ks][nb][split][lane][8], element i of lane l
// is row 16ks + 8(l/32) + i, column 32nb + l%32 (< k) of V S^-1, times xscale, split into
// NS bf16 terms; other columns zero.  nu and sigma are formed as in phase B (the column
// norms of V from the block partials, sigma = sqrt(mu) * sketch_scale), so this kernel
// needs nothing from the A~ eigen-solve and runs beside it.
__global__ __launch_bounds__(SLA_ROWS_NT) void k_la_gp(SLADesc d1, const SLADesc* __restrict__ ds) {
  using namespace tla;
  const SLADesc& d = la_desc(d1, ds, blockIdx.y);
  const int N = d.m - 1, k = d.k, NB = d.NB, NS = d.NS, KS = d.KS;
  const int t0 = blockIdx.x * kLaRows;
  const SmallLAOutLayout Lo = small_la_out_layout(N, k);
  const double* out = d.out;
  if ((t0 >= N && t0 >= 16 * KS) || out[Lo.status] != 0.0) return;
  __shared__ double s_nu[SLA_NMAX / 2], s_sig[SLA_NMAX / 2];
  const SmallLALayout Ls = small_la_layout(N, k, d.Jmax);
  const double* P = d.scratch + Ls.P;
  const double* V = d.scratch + Ls.V;
  const int nblk = (N + kLaRows - 1) / kLaRows;
  const int64_t ne = (int64_t)k * k + k;
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    double q = 0.0;
    for (int b = 0; b < nblk; ++b) q += P[b * ne + (int64_t)k * k + i];
    s_nu[i] = sqrt(q);
    s_sig[i] = sqrt(out[Lo.mu + i]) * d.sketch_scale;
  }
  __syncthreads();
  const int ks0 = t0 / 16, ks1 = (t0 + kLaRows) / 16 < KS ? (t0 + kLaRows) / 16 : KS;
  const int64_t total = (int64_t)(ks1 - ks0) * NB * 64 * 8;
  uint16_t* __restrict__ Gp = d.Gp;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = (int)(e & 7);
    const int l = (int)((e >> 3) & 63);
    const int64_t r = e >> 9;
    const int nb = (int)(r % NB);
    const int ks = ks0 + (int)(r / NB);
    const int row = 16 * ks + 8 * (l >> 5) + i;
    const int col = 32 * nb + (l & 31);
    double g = 0.0;
    if (row < N && col < k) g = V[(int64_t)col * N + row] / s_nu[col] / s_sig[col] * d.xscale;
    double rem = g;
    for (int sp = 0; sp < NS; ++sp) {
      const uint16_t bits = bf16_bits_d(rem);
      rem -= bf16_val_d(bits);
      Gp[((((int64_t)ks * NB + nb) * NS + sp) * 64 + l) * 8 + i] = bits;
    }
  }
}

// The small LA in three parts: the head (Lanczos, V, M12 V), then side by side the lift's
// operands (followed by the lift) and the tail (the A~ eigen-solve and G).
// Workgroups of k_la_a the current device holds at once (occupancy per CU times CUs).
// The row groups of one solve wait for each other at every exchange, so they must all be
// resident together: a launch whose solves need more groups than this is refused.  With
// several solves, workgroups are dispatched in grid order (x fastest), so the groups of
// one solve are consecutive; every resident group belongs to a solve whose groups have all
// been dispatched or are next in line, so some solve always has all its groups resident,
// finishes and frees its compute units (the waits are bounded in any case: past
// kSpinLimit polls a solve reports a device error instead of hanging).
static int la_a_capacity() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_la_a), SLA_A_NT, 0) !=
      hipSuccess)
    return 0;
  return per_cu * cus;
}

static hipError_t launch_la_head(const SLADesc& d1, const SLADesc* ds, int count, int nmax,
                                 hipStream_t stream, hipEvent_t after_lanczos, int ngroups) {
  const int rb = (nmax + tla::kLaRows - 1) / tla::kLaRows;
  static std::atomic<int> cap{-1};  // one device model per process: the library targets MI355X
  int capacity = cap.load(std::memory_order_relaxed);
  if (capacity < 0) cap.store(capacity = la_a_capacity(), std::memory_order_relaxed);
  if (capacity > 0 && ngroups > capacity) return hipErrorInvalidConfiguration;  // 0: the query failed
  hipLaunchKernelGGL(k_la_prep, dim3(count), dim3(64), 0, stream, d1, ds);
  hipLaunchKernelGGL(k_la_a, dim3(ngroups, count), dim3(SLA_A_NT), 0, stream, d1, ds);
  if (after_lanczos != nullptr) (void)hipEventRecord(after_lanczos, stream);
  hipLaunchKernelGGL(k_la_ritz, dim3(rb, count), dim3(SLA_MM_NT), 0, stream, d1, ds);
  hipLaunchKernelGGL(k_la_tv, dim3(rb, count), dim3(SLA_TV_NT), 0, stream, d1, ds);
  return hipGetLastError();
}

static hipError_t launch_la_gp(const SLADesc& d1, const SLADesc* ds, int count, int gmax, hipStream_t stream) {
  const int gb = (gmax + tla::kLaRows - 1) / tla::kLaRows;
  hipLaunchKernelGGL(k_la_gp, dim3(gb, count), dim3(SLA_ROWS_NT), 0, stream, d1, ds);
  return hipGetLastError();
}

static hipError_t launch_la_tail(const SLADesc& d1, const SLADesc* ds, int count, int nmax, int kmax,
                                 hipStream_t stream) {
  const int rb = (nmax + tla::kLaRows - 1) / tla::kLaRows;
  hipLaunchKernelGGL(k_la_b, dim3(count), dim3(1024), 0, stream, d1, ds);
  const size_t vlds = kmax <= 64 ? sizeof(double) * (2 * (size_t)kmax * kmax + 5 * (size_t)kmax) : 0;
  hipLaunchKernelGGL(k_la_v, dim3(kmax, count), dim3(64), vlds, stream, d1, ds);
  hipLaunchKernelGGL(k_la_b3, dim3(count), dim3(256), 0, stream, d1, ds);
  hipLaunchKernelGGL(k_la_g, dim3(rb, count), dim3(SLA_ROWS_NT), 0, stream, d1, ds);
  return hipGetLastError();
}

bool small_la_fits(int m, int k, int Jmax) {
  return m - 1 <= SLA_NMAX && Jmax <= SLA_JMAX && 2 * k <= SLA_NMAX;
}

static SLADesc la_desc_of(const double* Gr, int m, int k, double rtol, int Jmax, double sketch_scale,
                          double xscale, double* scratch, double* out, void* Gp, int NB, int NS, int KS,
                          int groups) {
  return SLADesc{Gr, scratch, out, (uint16_t*)Gp, rtol, sketch_scale, xscale, m, k, Jmax, NB, NS, KS, groups};
}

hipError_t small_la_head(const double* Gr, int m, int k, double rtol, int Jmax, double sketch_scale,
                         double xscale, double* scratch, double* out, void* Gp, int NB, int NS, int KS,
                         int groups, hipStream_t stream, hipEvent_t after_lanczos) {
  if (!small_la_fits(m, k, Jmax)) return hipErrorInvalidValue;
  const SLADesc d = la_desc_of(Gr, m, k, rtol, Jmax, sketch_scale, xscale, scratch, out, Gp, NB, NS, KS, groups);
  return launch_la_head(d, nullptr, 1, m - 1, stream, after_lanczos, groups > 0 ? std::min(groups, m - 1) : tla::la_groups(m - 1));
}

hipError_t small_la_gp(const double* Gr, int m, int k, double rtol, int Jmax, double sketch_scale,
                       double xscale, double* scratch, double* out, void* Gp, int NB, int NS, int KS,
                       int groups, hipStream_t stream) {
  if (!small_la_fits(m, k, Jmax)) return hipErrorInvalidValue;
  const SLADesc d = la_desc_of(Gr, m, k, rtol, Jmax, sketch_scale, xscale, scratch, out, Gp, NB, NS, KS, groups);
  return launch_la_gp(d, nullptr, 1, std::max(m - 1, 16 * KS), stream);
}

hipError_t small_la_tail(const double* Gr, int m, int k, double rtol, int Jmax, double sketch_scale,
                         double xscale, double* scratch, double* out, void* Gp, int NB, int NS, int KS,
                         int groups, hipStream_t stream) {
  if (!small_la_fits(m, k, Jmax)) return hipErrorInvalidValue;
  const SLADesc d = la_desc_of(Gr, m, k, rtol, Jmax, sketch_scale, xscale, scratch, out, Gp, NB, NS, KS, groups);
  return launch_la_tail(d, nullptr, 1, m - 1, k, stream);
}

// Remark 3 (Section 3.2): the Gram of the compressed modes' real basis from the sketch
// Gram, for rows [t0, t0 + 64) of the normalised basis B = V diag(1 / (nu s)) (the basis
// of G = B W): R = Gr[1:m, 1:m] V over those rows (in the TV scratch, free once the head
// has run), then the block's shares of B^T Gr[1:m, 1:m] B (k x k, row-major) and of B^T g0
// (g0[t] = Gr[(1+t) m], the products with the first frame), and in block 0 Gr[0][0].
// part: [block][k^2 + k + 1].  Needs only the head: nu (the column norms of V) and s =
// sqrt(mu) are formed here as the eigen-solve's first phase forms them, so this kernel
// runs beside the tail.
constexpr int SLA_PY_KMAX = 64;
__global__ __launch_bounds__(SLA_MM_NT) void k_la_py(SLADesc d, double* __restrict__ part) {
  using namespace tla;
  const int m = d.m, N = m - 1, k = d.k;
  const int t0 = blockIdx.x * kLaRows;
  const SmallLAOutLayout Lo = small_la_out_layout(N, k);
  if (t0 >= N || d.out[Lo.status] != 0.0) return;  // uniform over the workgroup
  __shared__ double s_red[SLA_MM_NT / 64];
  __shared__ double s_stage[SLA_STAGE];
  __shared__ double s_ns[2 * SLA_PY_KMAX];
  DevTeam tm;
  la_team(tm, s_red, nullptr);
  const SmallLALayout Ls = small_la_layout(N, k, d.Jmax);
  const int t1 = t0 + kLaRows < N ? t0 + kLaRows : N;
  const double* V = d.scratch + Ls.V;
  double* R = d.scratch + Ls.TV;
  {
    const int nblk = (N + kLaRows - 1) / kLaRows;
    const int64_t pe = (int64_t)k * k + k;
    const double* Pp = d.scratch + Ls.P;
    const double* mu = d.out + Lo.mu;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
      double q = 0.0;
      for (int b = 0; b < nblk; ++b) q += Pp[b * pe + (int64_t)k * k + i];
      s_ns[i] = sqrt(q);
      s_ns[SLA_PY_KMAX + i] = sqrt(mu[i]);
    }
    __syncthreads();
  }
  const double* nu = s_ns;
  const double* sv = s_ns + SLA_PY_KMAX;
  if (k <= 64) {
    // R(a, c) = sum_b Gr[(b+1) m + (a+1)] V(b, c): A(a, b) = (Gr + m + 1)[b m + a]
    mfma_rows16(d.Gr + m + 1, m, V, 1, N, N, t0 + 16 * (threadIdx.x >> 6), N, k, R, N);
    __syncthreads();
  } else {
    m12v_rows(tm, d.Gr + 1, m, N, k, V, R, t0, t1, s_stage, SLA_STAGE);
    __syncthreads();
  }
  const int ne = k * k + k + 1;
  double* out = part + (int64_t)blockIdx.x * ne;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    double acc = 0.0;
    if (e < k * k) {
      const int a = e / k, c = e % k;
      for (int t = t0; t < t1; ++t) acc += V[(int64_t)a * N + t] * R[(int64_t)c * N + t];
      acc /= nu[a] * sv[a] * nu[c] * sv[c];
    } else if (e < k * k + k) {
      const int a = e - k * k;
      for (int t = t0; t < t1; ++t) acc += V[(int64_t)a * N + t] * d.Gr[(int64_t)(1 + t) * m];
      acc /= nu[a] * sv[a];
    } else if (blockIdx.x == 0) {
      acc = d.Gr[0];
    }
    out[e] = acc;
  }
}

hipError_t small_la_py(const double* Gr, int m, int k, double rtol, int Jmax, double sketch_scale,
                       double* scratch, double* out, double* part, hipStream_t stream) {
  if (!small_la_fits(m, k, Jmax) || k > SLA_PY_KMAX) return hipErrorInvalidValue;
  const SLADesc d = la_desc_of(Gr, m, k, rtol, Jmax, sketch_scale, 1.0, scratch, out, nullptr, 1, 1, 1, 0);
  const int nblk = (m - 1 + tla::kLaRows - 1) / tla::kLaRows;
  hipLaunchKernelGGL(k_la_py, dim3(nblk), dim3(SLA_MM_NT), 0, stream, d, part);
  return hipGetLastError();
}

int small_la_py_blocks(int m) { return (m - 1 + tla::kLaRows - 1) / tla::kLaRows; }

hipError_t small_la_batch_head(const SLADesc* d_descs, int count, int nmax, int ngroups, hipStream_t stream) {
  if (count < 1) return hipSuccess;
  const SLADesc none{};
  return launch_la_head(none, d_descs, count, nmax, stream, nullptr, ngroups);
}

hipError_t small_la_batch_gp(const SLADesc* d_descs, int count, int gmax, hipStream_t stream) {
  if (count < 1) return hipSuccess;
  const SLADesc none{};
  return launch_la_gp(none, d_descs, count, gmax, stream);
}

hipError_t small_la_batch_tail(const SLADesc* d_descs, int count, int nmax, int kmax, hipStream_t stream) {
  if (count < 1) return hipSuccess;
  const SLADesc none{};
  return launch_la_tail(none, d_descs, count, nmax, kmax, stream);
}

int64_t small_la_scratch_doubles(int m, int k, int Jmax) {
  return tla::small_la_layout(m - 1, k, Jmax).total;
}
int64_t small_la_out_doubles(int m, int k) { return tla::small_la_out_layout(m - 1, k).total; }

}  // namespace k
}  // namespace cdmd
