// Dense Gaussian sketch Y^ = C X (Section 3.2, eq. (eq:YCX), with a Gaussian measurement matrix,
// Section "Measurement Matrices").  Every entry of C is a pure function of (seed, row,
// pixel), drawn by the workgroup that needs it, or, for the FP8 form, read from a copy of
// C the library stored in device memory once (gauss_fill: the same entries, bit for bit),
// which trades the per-entry draw for p n bytes of HBM reads per sketch.  (A stored BF16 C
// makes the sketch a plain product: gauss_fill_t stores it pixel-major for the library
// GEMM of sketch_gemm.cpp.)
//
// Entry definition: for row r and pixel j, Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
// SC'11) with key (seed mod 2^32, seed >> 32) on the counter (j >> 2, r, 0, 0) gives four
// words w0..w3; u = (w + 1) 2^-32; Box-Muller on (w0, w1) gives the normals of pixels
// 4(j >> 2) + 0, 1 and on (w2, w3) those of + 2, 3.  The sums are scaled by 1/sqrt(p)
// after accumulation.
//
// Forms:
//  * FP32: the normals are computed in float64 and rounded once to float32; products on
//    FP32 MFMA (16x16x4), float32 accumulation inside a workgroup's pixel slice, float64
//    across slices.
//  * BF16: the normals are computed in float32 with the hardware log/sqrt/sin/cos and
//    rounded to bfloat16 (ties to even); uint8 pixels are exact in bfloat16; products on
//    BF16 MFMA (32x32x16) with float32 accumulation, float64 across slices.
//  * FP8: as BF16 with the normals rounded to OCP e4m3 and each pixel byte split into
//    two exact e4m3 operands (16 hi, lo) on FP8 MFMA.
//
// Work split (BF16 / FP8 forms): a workgroup owns a tile of sketch rows (64, or 128 for
// the BF16 form's 512-frame tiles) x a tile of frames (256 or 512) x a slice of
// pixels.  It draws its C tile once per pixel step into LDS (each entry drawn once per
// frame tile) and reads the video bytes straight into MFMA operands.  Blocks are dealt to
// the eight XCDs in turn, so block b runs on XCD b mod 8; its index b / 8 there picks the
// row tile (fastest) and the (slice, frame tile) combination 8 (index / row tiles) +
// b mod 8.  The row tiles of one combination thus start together on one XCD, step
// through the same pixels at about the same pace and share each video tile through that
// XCD's L2, so the video is read from HBM about (row tiles / workgroups per XCD) times
// instead of once per row tile.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"

namespace cdmd {
namespace k {

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

struct Words4 {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t k0, uint32_t k1,
                                                uint32_t c3in = 0u) {
  uint32_t c2 = 0u, c3 = c3in;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  return Words4{c0, c1, c2, c3};
}

// Box-Muller in float64, each normal rounded once to float32
__device__ __forceinline__ void box_muller_f64(uint32_t wa, uint32_t wb, float& z0, float& z1) {
  const double u1 = ((double)wa + 1.0) * 0x1p-32;
  const double u2 = ((double)wb + 1.0) * 0x1p-32;
  const double r = sqrt(-2.0 * log(u1));
  const double ang = (2.0 * 3.141592653589793) * u2;
  z0 = (float)(r * cos(ang));
  z1 = (float)(r * sin(ang));
}

// Box-Muller in float32 with the hardware transcendentals (v_log_f32 is log2,
// v_sin_f32 / v_cos_f32 take the angle in turns)
__device__ __forceinline__ void box_muller_f32(uint32_t wa, uint32_t wb, float& z0, float& z1) {
  const float u1 = ((float)wa + 1.0f) * 0x1p-32f;
  const float u2 = ((float)wb + 1.0f) * 0x1p-32f;
  const float r = __builtin_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
  z0 = r * __builtin_amdgcn_cosf(u2);
  z1 = r * __builtin_amdgcn_sinf(u2);
}

__device__ __forceinline__ uint32_t bf16_bits_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// 8 bytes (pixels 0..7, little-endian) -> 8 exact bfloat16
__device__ __forceinline__ bf16x8_t u8x8_to_bf16(uint32_t lo, uint32_t hi) {
  uint32_t q[4];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const uint32_t v = i ? hi : lo;
    const uint32_t b0 = __float_as_uint((float)(v & 0xffu)) >> 16;
    const uint32_t b1 = __float_as_uint((float)((v >> 8) & 0xffu)) & 0xffff0000u;
    const uint32_t b2 = __float_as_uint((float)((v >> 16) & 0xffu)) >> 16;
    const uint32_t b3 = __float_as_uint((float)(v >> 24)) & 0xffff0000u;
    q[2 * i] = b0 | b1;
    q[2 * i + 1] = b2 | b3;
  }
  return __builtin_bit_cast(bf16x8_t, make_uint4(q[0], q[1], q[2], q[3]));
}

// ------------------------------------------------------------------------ BF16 form
constexpr int GB_ROWS = 64;   // sketch rows per workgroup of the FP8 form (2 MFMA row blocks)
constexpr int GB_KT = 64;     // pixels per step (4 MFMA k-steps)
constexpr int GB_AS = 72;     // LDS row stride of the C tile (bf16 elements)
constexpr int GB_NW = 8;      // waves per workgroup

// NFB: 32-frame blocks per wave (frames per workgroup = 32 NFB GB_NW); RB: 32-row blocks
// (rows per workgroup = 32 RB, shared by the eight waves); RB NFB <= 8 keeps the
// accumulators within 128 registers.  More rows per workgroup let each drawn C entry and
// each converted video fragment feed more products (gauss_plan picks RB).  Video: uint8,
// frames 16-byte aligned (ld % 16 == 0, aligned base).  K order inside a step: lane half h
// of a wave reads pixels [32h, 32h + 32) of its frame with two 16-byte loads; k-step ks
// takes pixels 32h + 8ks + (0..7).  The C tile is stored in pixel order, so the A
// fragment of (row, h, ks) is the 16 bytes at pixel 32h + 8ks.
// (With a stored C the BF16 form is a plain product and goes to the library GEMM instead.)
template <int NFB, int RB>
__global__ __launch_bounds__(64 * GB_NW) void k_sketch_gauss_bf16(const uint8_t* __restrict__ D, int64_t ld,
                                                                 int64_t n, int64_t m, int p, uint64_t seed,
                                                                 int64_t pps, int nft, int nsplit,
                                                                 float* __restrict__ part) {
  constexpr int FRAMES = 32 * NFB * GB_NW;
  constexpr int ROWS = 32 * RB;
  static_assert(RB >= 2 && RB % 2 == 0 && RB * NFB <= 8, "tile shape");
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][ROWS * GB_AS];
  const int combos = nft * nsplit, nrt = (p + ROWS - 1) / ROWS;
  const int xcd = blockIdx.x & 7, loc = blockIdx.x >> 3;
  const int rt = loc % nrt, cidx = (loc / nrt) * 8 + xcd;
  if (cidx >= combos) return;  // padding of the last group of eight combinations
  const int s = cidx / nft, ft = cidx % nft;
  const int r0 = rt * ROWS;
  const int64_t t0 = (int64_t)ft * FRAMES;
  const int64_t jb = (int64_t)s * pps;
  int64_t je = jb + pps;
  if (je > n) je = n;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int h = l >> 5, lc = l & 31;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  // drawing role: rows gr + 64 i (i < RB / 2), pixels 8 gg .. 8 gg + 7 of the step
  const int gr = tid >> 3, gg = tid & 7;

  // Steps inside the slice in a row tile inside [0, p) (all but the last step of the last
  // slice and the last row tile) take the branch-free forms of draw and load_b, chosen by
  // a workgroup-uniform test.
  const bool rows_in = r0 + ROWS <= p;
  auto draw = [&](int buf, int64_t j0) {
    const int64_t j = j0 + 8 * gg;
    const bool inner = rows_in && j0 + GB_KT <= je;
#pragma unroll
    for (int i = 0; i < RB / 2; ++i) {
      const int lr = gr + 64 * i, grow = r0 + lr;
      uint32_t q[4] = {0u, 0u, 0u, 0u};
      if (inner) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          const Words4 wd = philox4x32_10((uint32_t)((j >> 2) + half), (uint32_t)grow, k0, k1);
          float z[4];
          box_muller_f32(wd.w0, wd.w1, z[0], z[1]);
          box_muller_f32(wd.w2, wd.w3, z[2], z[3]);
          q[2 * half] = bf16_bits_rne(z[0]) | (bf16_bits_rne(z[1]) << 16);
          q[2 * half + 1] = bf16_bits_rne(z[2]) | (bf16_bits_rne(z[3]) << 16);
        }
      } else if (grow < p && j < je) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          const Words4 wd = philox4x32_10((uint32_t)((j >> 2) + half), (uint32_t)grow, k0, k1);
          float z[4];
          box_muller_f32(wd.w0, wd.w1, z[0], z[1]);
          box_muller_f32(wd.w2, wd.w3, z[2], z[3]);
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (j + 4 * half + e >= je) z[e] = 0.f;
          q[2 * half] = bf16_bits_rne(z[0]) | (bf16_bits_rne(z[1]) << 16);
          q[2 * half + 1] = bf16_bits_rne(z[2]) | (bf16_bits_rne(z[3]) << 16);
        }
      }
      *reinterpret_cast<uint4*>(&sA[buf][lr * GB_AS + 8 * gg]) = make_uint4(q[0], q[1], q[2], q[3]);
    }
  };

  // this lane's frames: t0 + 32 NFB w + 32 fb + lc (wave w owns 32 NFB frames)
  uint4 bcur[NFB][2], bnext[NFB][2];
  auto load_b = [&](uint4 (*dst)[2], int64_t j0) {
    const int64_t j = j0 + 32 * h;
    if (j0 + GB_KT <= je) {
      // frames past m read frame m - 1 instead: finite bytes whose output columns are
      // never stored (column t of each product depends on frame t alone)
#pragma unroll
      for (int fb = 0; fb < NFB; ++fb) {
        const int64_t t = t0 + 32 * NFB * w + 32 * fb + lc;
        const uint4* src = reinterpret_cast<const uint4*>(D + (t < m ? t : m - 1) * ld + j);
        dst[fb][0] = src[0];
        dst[fb][1] = src[1];
      }
      return;
    }
#pragma unroll
    for (int fb = 0; fb < NFB; ++fb) {
      const int64_t t = t0 + 32 * NFB * w + 32 * fb + lc;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int64_t ju = j + 16 * u;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (t < m && ju < je) {
          const uint8_t* src = D + t * ld + ju;
          if (ju + 16 <= je) {
            v = *reinterpret_cast<const uint4*>(src);
          } else {
            uint32_t wv[4] = {0u, 0u, 0u, 0u};
            for (int e = 0; e < 16 && ju + e < je; ++e) wv[e >> 2] |= (uint32_t)src[e] << (8 * (e & 3));
            v = make_uint4(wv[0], wv[1], wv[2], wv[3]);
          }
        }
        dst[fb][u] = v;
      }
    }
  };

  f32x16_t acc[RB][NFB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int fb = 0; fb < NFB; ++fb)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[rb][fb][e] = 0.f;

  const int64_t nsteps = je > jb ? (je - jb + GB_KT - 1) / GB_KT : 0;
  if (nsteps > 0) {
    draw(0, jb);
    load_b(bcur, jb);
  }
  __syncthreads();
  for (int64_t st = 0; st < nsteps; ++st) {
    const int buf = (int)(st & 1);
    const int64_t jn = jb + (st + 1) * GB_KT;
    const bool more = st + 1 < nsteps;
    auto products = [&]() {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        bf16x8_t a[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
          a[rb] = *reinterpret_cast<const bf16x8_t*>(&sA[buf][(32 * rb + lc) * GB_AS + 32 * h + 8 * ks]);
#pragma unroll
        for (int fb = 0; fb < NFB; ++fb) {
          const uint4 v = bcur[fb][ks >> 1];
          const bf16x8_t b = (ks & 1) ? u8x8_to_bf16(v.z, v.w) : u8x8_to_bf16(v.x, v.y);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            acc[rb][fb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[rb], b, acc[rb][fb], 0, 0, 0);
        }
      }
    };
    // Waves w and w + 4 share a SIMD: the lower four draw the next step's C entries first
    // and multiply after, the upper four the other way round, so on every SIMD one wave's
    // draw (vector ALU) runs beside the other's products (matrix core) instead of both
    // drawing and then both multiplying.  The fences keep the compiler from moving the
    // video loads above the draw (which would lengthen their registers' lifetime).
    if (w < GB_NW / 2) {
      if (more) draw(buf ^ 1, jn);
      __builtin_amdgcn_sched_barrier(0);
      if (more) load_b(bnext, jn);
      products();
    } else {
      if (more) load_b(bnext, jn);
      products();
      __builtin_amdgcn_sched_barrier(0);
      if (more) draw(buf ^ 1, jn);
    }
    __syncthreads();
#pragma unroll
    for (int fb = 0; fb < NFB; ++fb) {
      bcur[fb][0] = bnext[fb][0];
      bcur[fb][1] = bnext[fb][1];
    }
  }
  // accumulators: lane l, register e -> row 32 rb + 8 (e / 4) + 4 h + e % 4, frame lc
  float* out = part + (int64_t)s * m * p;
#pragma unroll
  for (int fb = 0; fb < NFB; ++fb) {
    const int64_t t = t0 + 32 * NFB * w + 32 * fb + lc;
    if (t >= m) continue;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = r0 + 32 * rb + 8 * (e >> 2) + 4 * h + (e & 3);
        if (r < p) out[t * p + r] = acc[rb][fb][e];
      }
  }
}

// ------------------------------------------------------------------------ FP8 form
// OCP e4m3fn (bias 7, 3 mantissa bits, largest finite 448, no infinities): round to
// nearest, ties to even, saturating to +-448; below 2^-6 the subnormal grid of 2^-9.
__device__ __forceinline__ uint32_t e4m3_rne(float x) {
  const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fabsf(x);
  if (!(a < 448.0f)) return sign | 0x7Eu;
  if (a < 0x1p-6f) return sign | (uint32_t)rintf(a * 512.0f);  // 8 gives 0x08 = 2^-6
  uint32_t u = __float_as_uint(a);
  u += 0x7ffffu + ((u >> 20) & 1u);  // round the float mantissa to 3 bits
  const uint32_t e = (u >> 23) - 127u + 7u, mant = (u >> 20) & 7u;
  return sign | (e << 3) | mant;
}

// e4m3 codes of the integers v (lut_lo) and 16 v (lut_hi), v = 0..15, as byte tables
// for v_perm_b32: entries 0..7 in (t0h:t0l), 8..15 in (t1h:t1l).
__device__ __forceinline__ uint32_t nibble_codes(uint32_t nib4, uint32_t t0l, uint32_t t0h, uint32_t t1l,
                                                 uint32_t t1h) {
  const uint32_t idx = nib4 & 0x07070707u;
  const uint32_t r0 = __builtin_amdgcn_perm(t0h, t0l, idx);
  const uint32_t r1 = __builtin_amdgcn_perm(t1h, t1l, idx);
  const uint32_t m = ((nib4 >> 3) & 0x01010101u) * 0xFFu;
  return (r1 & m) | (r0 & ~m);
}

// As the BF16 form with C rounded to e4m3 and each video byte u = 16 hi + lo split into
// two exact e4m3 operands (16 hi and lo), multiplied by two FP8 MFMAs (32x32x16) into the
// same float32 accumulator: only C is quantised.
// STORED: C is read from Cm (e4m3 codes, row r at Cm + r ldc) instead of drawn.
template <int NFB, bool STORED>
__global__ __launch_bounds__(64 * GB_NW) void k_sketch_gauss_fp8(const uint8_t* __restrict__ D, int64_t ld,
                                                                int64_t n, int64_t m, int p, uint64_t seed,
                                                                int64_t pps, int nft, int nsplit,
                                                                const uint8_t* __restrict__ Cm, int64_t ldc,
                                                                float* __restrict__ part) {
  constexpr int FRAMES = 32 * NFB * GB_NW;
  constexpr int AS = 80;  // LDS row stride of the C tile (bytes)
  __shared__ __attribute__((aligned(16))) uint8_t sA[2][GB_ROWS * AS];
  const int combos = nft * nsplit, nrt = (p + GB_ROWS - 1) / GB_ROWS;
  const int xcd = blockIdx.x & 7, loc = blockIdx.x >> 3;
  const int rt = loc % nrt, cidx = (loc / nrt) * 8 + xcd;
  if (cidx >= combos) return;  // padding of the last group of eight combinations
  const int s = cidx / nft, ft = cidx % nft;
  const int r0 = rt * GB_ROWS;
  const int64_t t0 = (int64_t)ft * FRAMES;
  const int64_t jb = (int64_t)s * pps;
  int64_t je = jb + pps;
  if (je > n) je = n;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int h = l >> 5, lc = l & 31;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const int gr = tid >> 3, gg = tid & 7;
  const int grow = r0 + gr;
  // code tables: v -> e4m3(v) and v -> e4m3(16 v)
  const uint32_t L0l = 0x44403800u, L0h = 0x4E4C4A48u, L1l = 0x53525150u, L1h = 0x57565554u;
  const uint32_t H0l = 0x64605800u, H0h = 0x6E6C6A68u, H1l = 0x73727170u, H1h = 0x77767574u;

  auto draw = [&](int buf, int64_t j0) {
    const int64_t j = j0 + 8 * gg;
    uint32_t q[2] = {0u, 0u};
    if (grow < p && j < je) {
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const Words4 wd = philox4x32_10((uint32_t)((j >> 2) + half), (uint32_t)grow, k0, k1);
        float z[4];
        box_muller_f32(wd.w0, wd.w1, z[0], z[1]);
        box_muller_f32(wd.w2, wd.w3, z[2], z[3]);
        uint32_t word = 0u;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t c = j + 4 * half + e >= je ? 0u : e4m3_rne(z[e]);
          word |= c << (8 * e);
        }
        q[half] = word;
      }
    }
    *reinterpret_cast<uint2*>(&sA[buf][gr * AS + 8 * gg]) = make_uint2(q[0], q[1]);
  };
  // the same eight codes from the stored C (pixels of the next slice read as 0)
  auto fetch = [&](int64_t j0) -> uint2 {
    const int64_t j = j0 + 8 * gg;
    uint2 v = make_uint2(0u, 0u);
    if (grow < p && j < je) {
      v = *reinterpret_cast<const uint2*>(Cm + (int64_t)grow * ldc + j);
      if (j + 8 > je) {
        uint32_t q[2] = {v.x, v.y};
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (j + e >= je) q[e >> 2] &= ~(0xffu << (8 * (e & 3)));
        v = make_uint2(q[0], q[1]);
      }
    }
    return v;
  };
  auto put = [&](int buf, uint2 v) { *reinterpret_cast<uint2*>(&sA[buf][gr * AS + 8 * gg]) = v; };

  uint4 bcur[NFB][2], bnext[NFB][2];
  auto load_b = [&](uint4 (*dst)[2], int64_t j0) {
    const int64_t j = j0 + 32 * h;
    if (j0 + GB_KT <= je) {
      // frames past m read frame m - 1 instead: finite bytes whose output columns are
      // never stored (column t of each product depends on frame t alone)
#pragma unroll
      for (int fb = 0; fb < NFB; ++fb) {
        const int64_t t = t0 + 32 * NFB * w + 32 * fb + lc;
        const uint4* src = reinterpret_cast<const uint4*>(D + (t < m ? t : m - 1) * ld + j);
        dst[fb][0] = src[0];
        dst[fb][1] = src[1];
      }
      return;
    }
#pragma unroll
    for (int fb = 0; fb < NFB; ++fb) {
      const int64_t t = t0 + 32 * NFB * w + 32 * fb + lc;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int64_t ju = j + 16 * u;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (t < m && ju < je) {
          const uint8_t* src = D + t * ld + ju;
          if (ju + 16 <= je) {
            v = *reinterpret_cast<const uint4*>(src);
          } else {
            uint32_t wv[4] = {0u, 0u, 0u, 0u};
            for (int e = 0; e < 16 && ju + e < je; ++e) wv[e >> 2] |= (uint32_t)src[e] << (8 * (e & 3));
            v = make_uint4(wv[0], wv[1], wv[2], wv[3]);
          }
        }
        dst[fb][u] = v;
      }
    }
  };

  f32x16_t acc[2][NFB];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int fb = 0; fb < NFB; ++fb)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[rb][fb][e] = 0.f;

  const int64_t nsteps = je > jb ? (je - jb + GB_KT - 1) / GB_KT : 0;
  if (nsteps > 0) {
    if constexpr (STORED) put(0, fetch(jb));
    else draw(0, jb);
    load_b(bcur, jb);
  }
  __syncthreads();
  uint2 cnext = make_uint2(0u, 0u);
  for (int64_t st = 0; st < nsteps; ++st) {
    const int buf = (int)(st & 1);
    const int64_t jn = jb + (st + 1) * GB_KT;
    const bool more = st + 1 < nsteps;
    auto products = [&]() {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      long a[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
        a[rb] = *reinterpret_cast<const long*>(&sA[buf][(32 * rb + lc) * AS + 32 * h + 8 * ks]);
#pragma unroll
      for (int fb = 0; fb < NFB; ++fb) {
        const uint4 v = bcur[fb][ks >> 1];
        const uint32_t w0 = (ks & 1) ? v.z : v.x, w1 = (ks & 1) ? v.w : v.y;
        const uint32_t lo0 = nibble_codes(w0 & 0x0F0F0F0Fu, L0l, L0h, L1l, L1h);
        const uint32_t lo1 = nibble_codes(w1 & 0x0F0F0F0Fu, L0l, L0h, L1l, L1h);
        const uint32_t hi0 = nibble_codes((w0 >> 4) & 0x0F0F0F0Fu, H0l, H0h, H1l, H1h);
        const uint32_t hi1 = nibble_codes((w1 >> 4) & 0x0F0F0F0Fu, H0l, H0h, H1l, H1h);
        const long blo = (long)(((uint64_t)lo1 << 32) | lo0), bhi = (long)(((uint64_t)hi1 << 32) | hi0);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          acc[rb][fb] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a[rb], bhi, acc[rb][fb], 0, 0, 0);
          acc[rb][fb] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a[rb], blo, acc[rb][fb], 0, 0, 0);
        }
      }
    }
    };
    if constexpr (STORED) {
      if (more) {
        load_b(bnext, jn);
        cnext = fetch(jn);  // in flight during this step's products
      }
      products();
      if (more) put(buf ^ 1, cnext);
    } else if (w < GB_NW / 2) {
      // the two waves of a SIMD draw and multiply in opposite order (as in the BF16 form)
      if (more) draw(buf ^ 1, jn);
      __builtin_amdgcn_sched_barrier(0);
      if (more) load_b(bnext, jn);
      products();
    } else {
      if (more) load_b(bnext, jn);
      products();
      __builtin_amdgcn_sched_barrier(0);
      if (more) draw(buf ^ 1, jn);
    }
    __syncthreads();
#pragma unroll
    for (int fb = 0; fb < NFB; ++fb) {
      bcur[fb][0] = bnext[fb][0];
      bcur[fb][1] = bnext[fb][1];
    }
  }
  float* out = part + (int64_t)s * m * p;
#pragma unroll
  for (int fb = 0; fb < NFB; ++fb) {
    const int64_t t = t0 + 32 * NFB * w + 32 * fb + lc;
    if (t >= m) continue;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = r0 + 32 * rb + 8 * (e >> 2) + 4 * h + (e & 3);
        if (r < p) out[t * p + r] = acc[rb][fb][e];
      }
  }
}

// ------------------------------------------------------------------------ stored C
// The entries the FP8 sketch draws, written once: row r at Cm + r ldc (ldc a multiple of
// 8), pixels j >= n zero.  Each thread item: eight pixels of one row, from the same Philox
// words, Box-Muller and rounding as the draw in the sketch kernel.
__global__ __launch_bounds__(256) void k_gauss_fill_fp8(uint8_t* __restrict__ Cm, int64_t ldc, int64_t n, int p,
                                                        uint64_t seed) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const int64_t groups = ldc / 8, total = (int64_t)p * groups;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(it / groups);
    const int64_t j = (it % groups) * 8;
    uint32_t q[2] = {0u, 0u};
    if (j < n) {
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const Words4 wd = philox4x32_10((uint32_t)((j >> 2) + half), (uint32_t)r, k0, k1);
        float z[4];
        box_muller_f32(wd.w0, wd.w1, z[0], z[1]);
        box_muller_f32(wd.w2, wd.w3, z[2], z[3]);
        uint32_t word = 0u;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t c = j + 4 * half + e >= n ? 0u : e4m3_rne(z[e]);
          word |= c << (8 * e);
        }
        q[half] = word;
      }
    }
    *reinterpret_cast<uint2*>(Cm + (int64_t)r * ldc + j) = make_uint2(q[0], q[1]);
  }
}

// ------------------------------------------------------------------------ FP32 form
constexpr int GF_ROWS = 64;  // sketch rows per workgroup (4 MFMA row blocks of 16)
constexpr int GF_KT = 16;    // pixels per step (4 MFMA k-steps)
constexpr int GF_AS = 20;    // LDS row stride of the C tile (floats)

// Each wave: 64 rows x 64 frames (16 accumulator blocks of 16 x 16); workgroup 256
// frames.  K order inside a step: lane quarter q (= l / 16) reads pixels 4q .. 4q + 3 of
// its frame; k-step ks takes pixel 4q + ks.  Tin: uint8 (raw 0..255) or float.
// SRFT: the rows are the real and imaginary parts of the subsampled randomised Fourier
// transform C = R F D (Section 3.3): row 2r + 0 / 1 holds the cosine / sine of the phase
// 2 pi (u_j - (f_r j mod n) / n) of entry (r, j), with f_r = freq[r] the DFT row kept by R
// and u_j the uniform of D's entry j: word j mod 4 of Philox4x32-10 on the counter
// (j >> 2, 0, 0, 1) with the model's key, times 2^-32.  The phase is formed in float64
// from the exact integer f_r j mod n and rounded once, as a cosine or sine, to float32.
template <typename Tin, bool VEC, bool SRFT>
__global__ __launch_bounds__(256) void k_sketch_gauss_f32(const Tin* __restrict__ D, int64_t ld,
                                                         int64_t n, int64_t m, int p, uint64_t seed,
                                                         int64_t pps, int nft, int nsplit,
                                                         const int32_t* __restrict__ freq,
                                                         float* __restrict__ part) {
  constexpr int FRAMES = 256;
  __shared__ __attribute__((aligned(16))) float sA[2][GF_ROWS * GF_AS];
  const int combos = nft * nsplit;
  const int cidx = blockIdx.x % combos, rt = blockIdx.x / combos;
  const int s = cidx / nft, ft = cidx % nft;
  const int r0 = rt * GF_ROWS;
  const int64_t t0 = (int64_t)ft * FRAMES;
  const int64_t jb = (int64_t)s * pps;
  int64_t je = jb + pps;
  if (je > n) je = n;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int q = l >> 4, lc = l & 15;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const int gr = tid >> 2, gg = tid & 3;
  const int grow = r0 + gr;

  auto draw = [&](int buf, int64_t j0) {
    const int64_t j = j0 + 4 * gg;
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    if (grow < p && j < je) {
      if constexpr (SRFT) {
        const Words4 wd = philox4x32_10((uint32_t)(j >> 2), 0u, k0, k1, 1u);
        const uint32_t wv[4] = {wd.w0, wd.w1, wd.w2, wd.w3};
        const int64_t f = freq[grow >> 1];
        int64_t q = (f * j) % n;  // j is a multiple of 4: entry e is pixel j + e, word e
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (j + e < je) {
            const double frac = (double)wv[e] * 0x1p-32 - (double)q / (double)n;
            double sv, cv;
            sincospi(2.0 * frac, &sv, &cv);
            z[e] = (float)((grow & 1) ? sv : cv);
          }
          q += f;
          if (q >= n) q -= n;
        }
      } else {
        const Words4 wd = philox4x32_10((uint32_t)(j >> 2), (uint32_t)grow, k0, k1);
        box_muller_f64(wd.w0, wd.w1, z[0], z[1]);
        box_muller_f64(wd.w2, wd.w3, z[2], z[3]);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (j + e >= je) z[e] = 0.f;
      }
    }
    *reinterpret_cast<float4*>(&sA[buf][gr * GF_AS + 4 * gg]) = make_float4(z[0], z[1], z[2], z[3]);
  };

  float4 bcur[4], bnext[4];
  auto load_b = [&](float4* dst, int64_t j0) {
    const int64_t j = j0 + 4 * q;
#pragma unroll
    for (int fb = 0; fb < 4; ++fb) {
      const int64_t t = t0 + 64 * w + 16 * fb + lc;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (t < m && j < je) {
        const Tin* src = D + t * ld + j;
        if (VEC && j + 4 <= je) {
          if constexpr (sizeof(Tin) == 1) {
            const uint32_t u = *reinterpret_cast<const uint32_t*>(src);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (float)((u >> (8 * e)) & 0xffu);
          } else {
            const float4 f = *reinterpret_cast<const float4*>(src);
            v[0] = f.x;
            v[1] = f.y;
            v[2] = f.z;
            v[3] = f.w;
          }
        } else {
          for (int e = 0; e < 4 && j + e < je; ++e) v[e] = (float)src[e];
        }
      }
      dst[fb] = make_float4(v[0], v[1], v[2], v[3]);
    }
  };

  f32x4_t acc[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int fb = 0; fb < 4; ++fb) acc[rb][fb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const int64_t nsteps = je > jb ? (je - jb + GF_KT - 1) / GF_KT : 0;
  if (nsteps > 0) {
    draw(0, jb);
    load_b(bcur, jb);
  }
  __syncthreads();
  for (int64_t st = 0; st < nsteps; ++st) {
    const int buf = (int)(st & 1);
    const int64_t jn = jb + (st + 1) * GF_KT;
    const bool more = st + 1 < nsteps;
    if (more) load_b(bnext, jn);
    float4 a[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) a[rb] = *reinterpret_cast<const float4*>(&sA[buf][(16 * rb + lc) * GF_AS + 4 * q]);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int fb = 0; fb < 4; ++fb) {
        const float b = ks == 0 ? bcur[fb].x : ks == 1 ? bcur[fb].y : ks == 2 ? bcur[fb].z : bcur[fb].w;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          const float av = ks == 0 ? a[rb].x : ks == 1 ? a[rb].y : ks == 2 ? a[rb].z : a[rb].w;
          acc[rb][fb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b, acc[rb][fb], 0, 0, 0);
        }
      }
    if (more) draw(buf ^ 1, jn);
    __syncthreads();
#pragma unroll
    for (int fb = 0; fb < 4; ++fb) bcur[fb] = bnext[fb];
  }
  // accumulators: lane l, register e -> row 16 rb + 4 q + e, frame lc
  float* out = part + (int64_t)s * m * p;
#pragma unroll
  for (int fb = 0; fb < 4; ++fb) {
    const int64_t t = t0 + 64 * w + 16 * fb + lc;
    if (t >= m) continue;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + 16 * rb + 4 * q + e;
        if (r < p) out[t * p + r] = acc[rb][fb][e];
      }
  }
}

// Y[t][r] = scale * sum_s part[s][t][r], float64, slices in order
__global__ __launch_bounds__(256) void k_reduce_gauss(const float* __restrict__ part, int nsplit,
                                                     int64_t count, double scale, double* __restrict__ Y) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int s = 0; s < nsplit; ++s) acc += (double)part[(int64_t)s * count + e];
    Y[e] = acc * scale;
  }
}

// The BF16 form's C for the library GEMM, stored pixel-major: Ct[j][r] for j < jn (rows
// j >= n zero), the entries of the drawn form (k_sketch_gauss_bf16) bit for bit.  Thread e
// takes row r = e mod p of pixel quad e / p, so a wave writes consecutive rows of a pixel.
__global__ __launch_bounds__(256) void k_gauss_fill_bf16_t(uint16_t* __restrict__ Ct, int64_t jn, int64_t n, int p,
                                                           uint64_t seed) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const int64_t total = (jn / 4) * p;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(it % p);
    const int64_t j0 = (it / p) * 4;
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    if (j0 < n) {
      const Words4 wd = philox4x32_10((uint32_t)(j0 >> 2), (uint32_t)r, k0, k1);
      box_muller_f32(wd.w0, wd.w1, z[0], z[1]);
      box_muller_f32(wd.w2, wd.w3, z[2], z[3]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      Ct[(j0 + e) * p + r] = j0 + e < n ? (uint16_t)bf16_bits_rne(z[e]) : (uint16_t)0;
  }
}

// The FP8 form's C for the library GEMM, pixel-major e4m3 codes Ct[j][r] (rows j >= n zero),
// the drawn form's entries bit for bit.
__global__ __launch_bounds__(256) void k_gauss_fill_fp8_t(uint8_t* __restrict__ Ct, int64_t jn, int64_t n, int p,
                                                          uint64_t seed) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const int64_t total = (jn / 4) * p;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(it % p);
    const int64_t j0 = (it / p) * 4;
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    if (j0 < n) {
      const Words4 wd = philox4x32_10((uint32_t)(j0 >> 2), (uint32_t)r, k0, k1);
      box_muller_f32(wd.w0, wd.w1, z[0], z[1]);
      box_muller_f32(wd.w2, wd.w3, z[2], z[3]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) Ct[(j0 + e) * p + r] = j0 + e < n ? (uint8_t)e4m3_rne(z[e]) : (uint8_t)0;
  }
}

// Video bytes u = 16 hi + lo as two exact e4m3 parts in the GEMM's split layout:
// Xh[s][t][i] = code(16 hi), Xl[s][t][i] = code(lo) of pixel s Ks + i (zero past the frame).
__global__ __launch_bounds__(256) void k_video_fp8_split(const uint8_t* __restrict__ D, int64_t ld, int64_t n,
                                                         int64_t m, int64_t Ks, int S, uint8_t* __restrict__ Xh,
                                                         uint8_t* __restrict__ Xl) {
  const int64_t per = Ks / 8, total = (int64_t)S * m * per;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int64_t st = it / per, i = (it % per) * 8;
    const int64_t s = st / m, t = st % m, j = s * Ks + i;
    const uint8_t* src = D + t * ld + j;
    uint32_t b[2] = {0u, 0u};
    if (j + 8 <= n) {
      const uint2 v = *reinterpret_cast<const uint2*>(src);
      b[0] = v.x;
      b[1] = v.y;
    } else {
      for (int e = 0; e < 8 && j + e < n; ++e) b[e >> 2] |= (uint32_t)src[e] << (8 * (e & 3));
    }
    uint32_t hw[2] = {0u, 0u}, lw[2] = {0u, 0u};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t u = (b[e >> 2] >> (8 * (e & 3))) & 0xffu;
      hw[e >> 2] |= e4m3_rne(16.0f * (float)(u >> 4)) << (8 * (e & 3));
      lw[e >> 2] |= e4m3_rne((float)(u & 15u)) << (8 * (e & 3));
    }
    *reinterpret_cast<uint2*>(Xh + st * Ks + i) = make_uint2(hw[0], hw[1]);
    *reinterpret_cast<uint2*>(Xl + st * Ks + i) = make_uint2(lw[0], lw[1]);
  }
}

// Video bytes to exact bfloat16 in the GEMM's split layout: Xs[s][t][i] = x(t, s Ks + i),
// zero past the frame.  8 pixels per thread (frames 16-byte aligned, Ks a multiple of 64).
__global__ __launch_bounds__(256) void k_video_bf16_split(const uint8_t* __restrict__ D, int64_t ld, int64_t n,
                                                          int64_t m, int64_t Ks, int S, uint16_t* __restrict__ Xs) {
  const int64_t per = Ks / 8, total = (int64_t)S * m * per;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int64_t st = it / per, i = (it % per) * 8;
    const int64_t s = st / m, t = st % m, j = s * Ks + i;
    const uint8_t* src = D + t * ld + j;
    uint32_t lo = 0u, hi = 0u;
    if (j + 8 <= n) {
      const uint2 v = *reinterpret_cast<const uint2*>(src);
      lo = v.x;
      hi = v.y;
    } else {
      for (int e = 0; e < 8 && j + e < n; ++e) {
        const uint32_t b = src[e];
        if (e < 4) lo |= b << (8 * e);
        else hi |= b << (8 * (e - 4));
      }
    }
    *reinterpret_cast<bf16x8_t*>(Xs + st * Ks + i) = u8x8_to_bf16(lo, hi);
  }
}

// G[a][b] = sum_r conj(Y[a][r]) Y[b][r] over the complex rows of an SRFT sketch stored
// with interleaved (re, im) rows per frame (Y[t][2r], Y[t][2r + 1]): real part to Gr,
// imaginary part to Gi, float64.  A workgroup owns a 16 x 16 tile of (a, b) and steps
// through 16 complex rows at a time in LDS.
__global__ __launch_bounds__(256) void k_gram_cplx(const double* __restrict__ Y, int p, int64_t m,
                                                  double* __restrict__ Gr, double* __restrict__ Gi) {
  __shared__ double sa[16][33], sb[16][33];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t a0 = (int64_t)blockIdx.y * 16, b0 = (int64_t)blockIdx.x * 16;
  const int64_t P2 = 2 * (int64_t)p;
  double re = 0.0, im = 0.0;
  for (int64_t r0 = 0; r0 < P2; r0 += 32) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t col = r0 + tx + 16 * h;
      const int64_t fa = a0 + ty, fb = b0 + ty;
      sa[ty][tx + 16 * h] = (fa < m && col < P2) ? Y[fa * P2 + col] : 0.0;
      sb[ty][tx + 16 * h] = (fb < m && col < P2) ? Y[fb * P2 + col] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const double ar = sa[ty][2 * c], ai = sa[ty][2 * c + 1];
      const double br = sb[tx][2 * c], bi = sb[tx][2 * c + 1];
      re += ar * br + ai * bi;
      im += ar * bi - ai * br;
    }
    __syncthreads();
  }
  const int64_t a = a0 + ty, b = b0 + tx;
  if (a < m && b < m) {
    Gr[a * m + b] = re;
    Gi[a * m + b] = im;
  }
}

}  // namespace

GaussPlan gauss_plan(int64_t n, int64_t m, int p, int prec, int target) {
  GaussPlan g{};
  const bool bf = prec == 1 || prec == 2;
  const int kt = bf ? GB_KT : GF_KT;
  int frames = 256;
  // BF16 / FP8: frame tiles of at most 512 frames.  At 1024 frames (four 32-frame blocks
  // per wave) the tile leaves no registers for the wave-paired draw and products (it
  // spills): a BF16 4K x 1000 sketch with p = 4000 takes 204 ms there and 107 ms in two
  // 512-frame tiles, though each C entry is then drawn twice.
  if (bf) frames = m <= 256 ? 256 : 512;
  int rows = bf ? GB_ROWS : GF_ROWS;
  if (prec == 1) {
    // BF16: 32 RB rows.  RB = 4 for 512-frame tiles: one workgroup per CU either way, and
    // twice the products per drawn entry and converted fragment (1080p-class videos of 400
    // frames: 130 -> 96 ms).  RB = 2 otherwise: at 256 frames RB = 4 or 8 costs the second
    // resident workgroup and measured slower.
    int rb = frames == 512 ? 4 : 2;
    if (rb > 2 && 32 * (rb / 2) >= p) rb /= 2;  // a small p fills fewer rows
    rows = 32 * rb;
  }
  g.frames = frames;
  g.rows = rows;
  g.nrt = (p + rows - 1) / rows;
  g.nft = (int)((m + frames - 1) / frames);
  // about `target` workgroups, slices of at least 64 steps
  const int64_t tiles = (int64_t)g.nrt * g.nft;
  int64_t ns = (target + tiles - 1) / tiles;
  const int64_t maxs = (n + 64 * kt - 1) / (64 * kt);
  if (ns > maxs) ns = maxs;
  if (ns < 1) ns = 1;
  // BF16 / FP8: whole groups of eight combinations where the slices allow it
  while (bf && (g.nft * ns) % 8 != 0 && ns < maxs) ++ns;
  const int64_t steps = (n + kt - 1) / kt;
  const int64_t sps = (steps + ns - 1) / ns;
  g.pps = sps * kt;
  g.nsplit = (int)((n + g.pps - 1) / g.pps);
  if (bf) g.blocks = (int64_t)g.nrt * ((g.nft * g.nsplit + 7) / 8) * 8;
  else g.blocks = (int64_t)g.nrt * g.nft * g.nsplit;
  return g;
}

int64_t gauss_ldc(int64_t n) { return (n + 63) / 64 * 64; }

hipError_t gauss_fill(void* Cm, int64_t ldc, int64_t n, int p, uint64_t seed, int prec, hipStream_t stream) {
  if (prec != 2) return hipErrorInvalidValue;  // the BF16 form stores C pixel-major (gauss_fill_t)
  if (ldc % 8 != 0 || ldc < n) return hipErrorInvalidValue;
  const int64_t total = (int64_t)p * (ldc / 8);
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_gauss_fill_fp8, dim3((unsigned)blocks), dim3(256), 0, stream, static_cast<uint8_t*>(Cm), ldc,
                     n, p, seed);
  return hipGetLastError();
}

hipError_t sketch_gauss(const void* D, int dtype, int64_t ld, int64_t n, int64_t m, int p,
                        uint64_t seed, int prec, const GaussPlan& g, const void* Cm, int64_t ldc, float* part,
                        double* Y, hipStream_t stream) {
  const dim3 grid((unsigned)g.blocks), block(256);
  if (prec == 1) {
    const uint8_t* d = static_cast<const uint8_t*>(D);
    if (Cm != nullptr) return hipErrorInvalidValue;  // a stored BF16 C goes to the library GEMM
    const dim3 bb(64 * GB_NW);
    auto go = [&](auto nfb, auto rb) {
      constexpr int NFB = decltype(nfb)::value, RB = decltype(rb)::value;
      hipLaunchKernelGGL((k_sketch_gauss_bf16<NFB, RB>), grid, bb, 0, stream, d, ld, n, m, p, seed, g.pps, g.nft,
                         g.nsplit, part);
    };
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I4 = std::integral_constant<int, 4>;
    const int rb = g.rows / 32;
    if (g.frames == 256 && rb == 2) go(I1{}, I2{});
    else if (g.frames == 512 && rb == 4) go(I2{}, I4{});
    else if (g.frames == 512 && rb == 2) go(I2{}, I2{});
    else return hipErrorInvalidValue;
  } else if (prec == 2) {
    const uint8_t* d = static_cast<const uint8_t*>(D);
    const uint8_t* c = static_cast<const uint8_t*>(Cm);
    const dim3 bb(64 * GB_NW);
    auto go = [&](auto nfb) {
      constexpr int NFB = decltype(nfb)::value;
      if (c != nullptr)
        hipLaunchKernelGGL((k_sketch_gauss_fp8<NFB, true>), grid, bb, 0, stream, d, ld, n, m, p, seed, g.pps, g.nft,
                           g.nsplit, c, ldc, part);
      else
        hipLaunchKernelGGL((k_sketch_gauss_fp8<NFB, false>), grid, bb, 0, stream, d, ld, n, m, p, seed, g.pps, g.nft,
                           g.nsplit, c, ldc, part);
    };
    if (g.frames == 256) go(std::integral_constant<int, 1>{});
    else if (g.frames == 512) go(std::integral_constant<int, 2>{});
    else return hipErrorInvalidValue;
  } else if (dtype == 0) {
    const uint8_t* d = static_cast<const uint8_t*>(D);
    const bool vec = ld % 4 == 0 && (reinterpret_cast<uintptr_t>(D) & 3) == 0;
    if (vec)
      hipLaunchKernelGGL((k_sketch_gauss_f32<uint8_t, true, false>), grid, block, 0, stream, d, ld, n, m, p, seed,
                         g.pps, g.nft, g.nsplit, nullptr, part);
    else
      hipLaunchKernelGGL((k_sketch_gauss_f32<uint8_t, false, false>), grid, block, 0, stream, d, ld, n, m, p, seed,
                         g.pps, g.nft, g.nsplit, nullptr, part);
  } else {
    const float* d = static_cast<const float*>(D);
    const bool vec = ld % 4 == 0 && (reinterpret_cast<uintptr_t>(D) & 15) == 0;
    if (vec)
      hipLaunchKernelGGL((k_sketch_gauss_f32<float, true, false>), grid, block, 0, stream, d, ld, n, m, p, seed,
                         g.pps, g.nft, g.nsplit, nullptr, part);
    else
      hipLaunchKernelGGL((k_sketch_gauss_f32<float, false, false>), grid, block, 0, stream, d, ld, n, m, p, seed,
                         g.pps, g.nft, g.nsplit, nullptr, part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t count = m * (int64_t)p;
  int64_t nb = (count + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_reduce_gauss, dim3((unsigned)nb), dim3(256), 0, stream, part, g.nsplit, count,
                     1.0 / sqrt((double)p), Y);
  return hipGetLastError();
}

hipError_t sketch_srft(const void* D, int dtype, int64_t ld, int64_t n, int64_t m, int p, uint64_t seed,
                       const GaussPlan& g, const int32_t* freq, float* part, double* Y, hipStream_t stream) {
  // g: gauss_plan(n, m, 2 p, FP32); Y: m x 2p, frame-major, (re, im) interleaved
  const dim3 grid((unsigned)g.blocks), block(256);
  const int p2 = 2 * p;
  if (dtype == 0) {
    const uint8_t* d = static_cast<const uint8_t*>(D);
    const bool vec = ld % 4 == 0 && (reinterpret_cast<uintptr_t>(D) & 3) == 0;
    if (vec)
      hipLaunchKernelGGL((k_sketch_gauss_f32<uint8_t, true, true>), grid, block, 0, stream, d, ld, n, m, p2, seed,
                         g.pps, g.nft, g.nsplit, freq, part);
    else
      hipLaunchKernelGGL((k_sketch_gauss_f32<uint8_t, false, true>), grid, block, 0, stream, d, ld, n, m, p2, seed,
                         g.pps, g.nft, g.nsplit, freq, part);
  } else {
    const float* d = static_cast<const float*>(D);
    const bool vec = ld % 4 == 0 && (reinterpret_cast<uintptr_t>(D) & 15) == 0;
    if (vec)
      hipLaunchKernelGGL((k_sketch_gauss_f32<float, true, true>), grid, block, 0, stream, d, ld, n, m, p2, seed,
                         g.pps, g.nft, g.nsplit, freq, part);
    else
      hipLaunchKernelGGL((k_sketch_gauss_f32<float, false, true>), grid, block, 0, stream, d, ld, n, m, p2, seed,
                         g.pps, g.nft, g.nsplit, freq, part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t count = m * (int64_t)p2;
  int64_t nb = (count + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_reduce_gauss, dim3((unsigned)nb), dim3(256), 0, stream, part, g.nsplit, count,
                     1.0 / sqrt((double)p), Y);
  return hipGetLastError();
}

hipError_t gauss_fill_t(void* Ct, int64_t jn, int64_t n, int p, uint64_t seed, hipStream_t stream) {
  if (jn % 4 != 0 || jn < n) return hipErrorInvalidValue;
  int64_t blocks = ((jn / 4) * p + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_gauss_fill_bf16_t, dim3((unsigned)blocks), dim3(256), 0, stream, static_cast<uint16_t*>(Ct), jn,
                     n, p, seed);
  return hipGetLastError();
}

hipError_t gauss_fill_fp8_t(void* Ct, int64_t jn, int64_t n, int p, uint64_t seed, hipStream_t stream) {
  if (jn % 4 != 0 || jn < n) return hipErrorInvalidValue;
  int64_t blocks = ((jn / 4) * p + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_gauss_fill_fp8_t, dim3((unsigned)blocks), dim3(256), 0, stream, static_cast<uint8_t*>(Ct),
                     jn, n, p, seed);
  return hipGetLastError();
}

hipError_t video_fp8_split(const void* D, int64_t ld, int64_t n, int64_t m, int64_t Ks, int S, void* Xh, void* Xl,
                           hipStream_t stream) {
  if (Ks % 64 != 0 || ld % 16 != 0 || (reinterpret_cast<uintptr_t>(D) & 15) != 0) return hipErrorInvalidValue;
  int64_t blocks = ((int64_t)S * m * (Ks / 8) + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_video_fp8_split, dim3((unsigned)blocks), dim3(256), 0, stream,
                     static_cast<const uint8_t*>(D), ld, n, m, Ks, S, static_cast<uint8_t*>(Xh),
                     static_cast<uint8_t*>(Xl));
  return hipGetLastError();
}

hipError_t video_bf16_split(const void* D, int64_t ld, int64_t n, int64_t m, int64_t Ks, int S, void* Xs,
                            hipStream_t stream) {
  if (Ks % 64 != 0 || ld % 16 != 0 || (reinterpret_cast<uintptr_t>(D) & 15) != 0) return hipErrorInvalidValue;
  int64_t blocks = ((int64_t)S * m * (Ks / 8) + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_video_bf16_split, dim3((unsigned)blocks), dim3(256), 0, stream,
                     static_cast<const uint8_t*>(D), ld, n, m, Ks, S, static_cast<uint16_t*>(Xs));
  return hipGetLastError();
}

hipError_t reduce_gauss(const float* part, int nsplit, int64_t count, double scale, double* Y, hipStream_t stream) {
  int64_t nb = (count + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_reduce_gauss, dim3((unsigned)nb), dim3(256), 0, stream, part, nsplit, count, scale, Y);
  return hipGetLastError();
}

hipError_t gram_cplx(const double* Y, int p, int64_t m, double* Gr, double* Gi, hipStream_t stream) {
  const unsigned t = (unsigned)((m + 15) / 16);
  hipLaunchKernelGGL(k_gram_cplx, dim3(t, t), dim3(256), 0, stream, Y, p, m, Gr, Gi);
  return hipGetLastError();
}

}  // namespace k
}  // namespace cdmd
