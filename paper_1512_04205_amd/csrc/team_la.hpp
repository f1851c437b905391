// Small float64 linear algebra of the cDMD fit written once for a "team" of threads:
// the whole thread block on the GPU (one workgroup per fit), or a single thread on the
// host (where the same code is tested against LAPACK).  Covers the truncated SVD (eq.
// svd), A~ and its eigendecomposition (Section 3.2) and the lift operator G = V S^-1 W:
//
//   * Lanczos with full (twice classical Gram-Schmidt) reorthogonalisation for the
//     top-k eigenpairs of the Gram Y^T Y (the right singular vectors of Y, eq. svd);
//   * cyclic Jacobi (parallel round-robin ordering) on the Lanczos tridiagonal matrix for
//     the Ritz pairs and their residuals;
//   * A~ = S^-1 V^T (Y^T Y') V S^-1 (Section 3.2);
//   * eig(A~) (Section 3.2): Householder reduction to Hessenberg form, Francis double-shift QR
//     (conjugate pairs from 2x2 blocks are exact conjugates), inverse iteration on
//     A~ - lambda I for the eigenvectors (a pair's second member is the conjugate);
//   * unit-norm eigenvectors with the largest-modulus entry real and positive;
//   * G = V S^-1 W.
//
// Every routine is called by all threads of the team with identical arguments; work is
// split with `for (i = tm.tid; i < n; i += tm.nt)` loops and tm.sync() barriers, and
// scalar decisions are computed redundantly by every thread from shared data, so
// control flow stays uniform.  Reductions run in a fixed order (deterministic).
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define TLA_HD __host__ __device__
#else
#define TLA_HD
#endif
// for the Lanczos loop and its per-step routines: a device call would keep the team in
// scratch memory and spill the caller's registers there
#define TLA_INLINE inline __attribute__((always_inline))

namespace cdmd {
namespace tla {

struct cpx {
  double re, im;
};
TLA_HD inline cpx cmk(double r, double i) { return cpx{r, i}; }
TLA_HD inline cpx cadd(cpx a, cpx b) { return cpx{a.re + b.re, a.im + b.im}; }
TLA_HD inline cpx csub(cpx a, cpx b) { return cpx{a.re - b.re, a.im - b.im}; }
TLA_HD inline cpx cmul(cpx a, cpx b) { return cpx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
TLA_HD inline cpx cconj(cpx a) { return cpx{a.re, -a.im}; }
TLA_HD inline double cabs2(cpx a) { return a.re * a.re + a.im * a.im; }
TLA_HD inline double cabsv(cpx a) { return hypot(a.re, a.im); }
TLA_HD inline cpx cscale(cpx a, double s) { return cpx{a.re * s, a.im * s}; }
// a / b, scaled (Smith) so that conj(a)/conj(b) == conj(a/b) bitwise
TLA_HD inline cpx cdiv(cpx a, cpx b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return cpx{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return cpx{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

constexpr double kEps = 2.220446049250313e-16;

// --------------------------------------------------------------------------- teams
// Host team: one thread.
struct HostTeam {
  int tid = 0, nt = 1, lane = 0, wsize = 1, wave = 0, nwaves = 1;
  void sync() {}
  void stamp(int) {}  // phase timing hook (device only)
  double wave_sum(double v) { return v; }
  void half_sums(double v, double& lo, double& hi) { lo = v, hi = 0.0; }  // (wsize 64 only)
  double wave_max(double v) { return v; }
  void wave_argmax(double&, int&) {}
  double sum(double v) { return v; }
  double maxv(double v) { return v; }
  int wave_first(bool b) { return b ? 0 : 1; }  // lowest lane with b set, or wsize
  double recip(double x) { return 1.0 / x; }
  void tick(int) {}                             // sub-phase timing hook (device only)
  HostTeam wave_team() { return *this; }        // the team of this thread's wave
};

// --------------------------------------------------------------------------- Lanczos
struct LanczosWork {
  double* q;      // N        current vector (shared)
  double* w;      // N        (shared)
  double* h;      // Jmax+2   projections (shared)
  double* alpha;  // Jmax+1   (shared)
  double* beta;   // Jmax+1   (shared)
  double* T;      // Jmax + k + 6 Jmax k: tridiagonal eigen-solve work (global scratch)
  double* fast;   // fast (LDS) region of fast_doubles doubles, or nullptr: the tridiagonal
  int64_t fast_doubles;  // work when it fits, and later scratch
  double* qc;     // fast (LDS) copy of the group's rows of the first basis vectors, or nullptr
  int64_t qc_doubles;
};
// Sizes (doubles) of the fast regions of a Lanczos workgroup: the work region and the copy
// of the group's rows of the basis (120 vectors of 32 rows).
constexpr int kLaFast = 13440, kLaQCache = 3840;

// Deterministic start vectors.  The first (salt 0) is the smooth profile
// 1 + sin(0.7 (i + 1)) / 4: the Gram is indexed by frames and its leading eigenvectors are
// slow functions of time, which such a vector overlaps well.  Restart vectors (salt > 0)
// take entry i as 1 + u - 1/2 with u in [0, 1) from an integer hash of (i, salt) (the
// splitmix64 finaliser), so each restart brings a fresh independent direction; host and
// device produce the same bits.
TLA_HD inline double lanczos_start(int i, int salt) {
  if (salt == 0) return 1.0 + 0.25 * sin(0.7 * (i + 1));
  uint64_t x = (uint64_t)(uint32_t)i * 0x9E3779B97F4A7C15ull + (uint64_t)(uint32_t)salt * 0xD1B54A32D192ED03ull;
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return 0.5 + (double)(x >> 11) * 0x1p-53;
}

// Number of eigenvalues smaller than x of the symmetric tridiagonal matrix with diagonal a
// and squared off-diagonal b2 (Sylvester's law of inertia on the LDL^T pivots; a pivot
// smaller than pivmin in modulus is replaced by -pivmin).
// The count is insensitive to small relative errors in each pivot (they amount to tiny
// perturbations of the matrix), so the team may supply a fast reciprocal.
template <class TM>
TLA_HD inline int sturm_count(TM& tm, const double* a, const double* b2, int J, double x,
                              double pivmin) {
  double q = a[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = q < 0.0 ? 1 : 0;
  int i = 1;
  for (; i + 4 <= J; i += 4) {  // operands of four steps loaded ahead of the pivot chain
    double av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = a[i + u] - x;
      bv[u] = b2[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      q = av[u] - bv[u] * tm.recip(q);
      if (fabs(q) < pivmin) q = -pivmin;
      c += q < 0.0 ? 1 : 0;
    }
  }
  for (; i < J; ++i) {
    q = (a[i] - x) - b2[i - 1] * tm.recip(q);
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0 ? 1 : 0;
  }
  return c;
}

// Modulus of the last component of the unit eigenvector of the symmetric tridiagonal
// (a, b2 = squared off-diagonals) for its eigenvalue th: z_J^2 = d_{J-1}(th) / d_J'(th)
// with d_i the characteristic polynomial of the leading i x i block (the residue of
// ((x - T)^-1)_{JJ} = d_{J-1}(x) / d_J(x) at th).  Forward three-term recurrences for d
// and d', rescaled together (the ratio is unchanged) to stay in range.
TLA_HD inline double tridiag_last_component(const double* a, const double* b2, int J, double th) {
  double dm = 1.0, d = th - a[0];   // d_{i-1}, d_i
  double pm = 0.0, pd = 1.0;        // d'_{i-1}, d'_i
  for (int i = 1; i < J; ++i) {
    const double xa = th - a[i], bb = b2[i - 1];
    const double dn = xa * d - bb * dm;
    const double pn = d + xa * pd - bb * pm;
    dm = d;
    d = dn;
    pm = pd;
    pd = pn;
    const double big = fmax(fmax(fabs(d), fabs(dm)), fmax(fabs(pd), fabs(pm)));
    if (big > 1e150) {
      dm *= 1e-150; d *= 1e-150; pm *= 1e-150; pd *= 1e-150;
    } else if (big < 1e-150 && big > 0.0) {
      dm *= 1e150; d *= 1e150; pm *= 1e150; pd *= 1e150;
    }
  }
  if (!(pd != 0.0)) return 1.0;  // repeated eigenvalue: no estimate, not converged
  const double z2 = fabs(dm / pd);
  return z2 >= 1.0 ? 1.0 : sqrt(z2);
}

// The kk largest eigenvalues (descending) of the symmetric tridiagonal (a, b), J x J,
// b[i] coupling i and i+1; b2 holds b[i]^2.  One wave per eigenvalue: its lanes evaluate
// the Sturm count at wsize interior points of the current bracket at once (multisection),
// shrinking the bracket by wsize + 1 per round, down to a width of 2 eps |x| + pivmin.
// With nparts > 1 only ranks r = part (mod nparts), and rank 0, are computed (theta[r] of
// the other ranks is left as it is).
template <class TM>
TLA_HD void tridiag_topk_values(TM& tm, const double* a, const double* b, const double* b2,
                                int J, int kk, double* theta, double* tnorm_out, int part = 0,
                                int nparts = 1) {
  double gl = a[0], gu = a[0], bmax2 = 0.0;
  for (int i = 0; i < J; ++i) {
    const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < J ? fabs(b[i]) : 0.0);
    gl = fmin(gl, a[i] - r);
    gu = fmax(gu, a[i] + r);
    if (i + 1 < J) bmax2 = fmax(bmax2, b2[i]);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, bmax2);
  const double fud = 2.1 * kEps * tnorm * J + 2.1 * pivmin;
  gl -= fud;
  gu += fud;
  *tnorm_out = tnorm;
  const double np1 = (double)(tm.wsize + 1);
  // slot s -> rank: part 0 takes 0, nparts, 2 nparts, ...; part p > 0 takes 0, p, p + nparts, ...
  const int own = part < kk ? (kk - 1 - part) / nparts + 1 : 0;
  const int nslots = part == 0 ? own : 1 + own;
  for (int s0 = 0; s0 < nslots; s0 += tm.nwaves) {
    const int sl = s0 + tm.wave;
    const int r = part == 0 ? sl * nparts : (sl == 0 ? 0 : part + (sl - 1) * nparts);
    if (sl < nslots) {  // uniform over the wave
      const int s = J - 1 - r;  // rank from the smallest; bracket: cnt(lo) <= s < cnt(hi)
      double lo = gl, hi = gu;
      for (int it = 0; it < 256; ++it) {
        if (hi - lo <= 2.0 * kEps * fmax(fabs(lo), fabs(hi)) + pivmin) break;
        const double x = lo + (hi - lo) * ((double)(tm.lane + 1) / np1);
        const int f = tm.wave_first(sturm_count(tm, a, b2, J, x, pivmin) > s);
        const double nhi = f < tm.wsize ? lo + (hi - lo) * ((double)(f + 1) / np1) : hi;
        const double nlo = f > 0 ? lo + (hi - lo) * ((double)f / np1) : lo;
        if (nhi == hi && nlo == lo) break;
        lo = nlo;
        hi = nhi;
      }
      if (tm.lane == 0) theta[r] = 0.5 * (lo + hi);
    }
  }
  tm.sync();
}

template <class TM>
TLA_HD void tridiag_orthonormalise(TM& tm, int J, int kk, double* work, double* Z);
template <class TM>
TLA_HD void tridiag_sign_columns(TM& tm, int J, int kk, double* Z);

// Eigenvectors of the symmetric tridiagonal (a, b) for theta[0..kk-1] (descending) by three
// steps of inverse iteration from hashed start vectors (a different one per eigenvector),
// each a solve with the LU factors (row interchanges) of T - theta I, one thread per
// eigenvector, all at once: unit vectors.  Vectors of nearly
// equal eigenvalues can come out with a small mutual component (of order eps ||T|| / gap);
// with orth set, the columns are then orthonormalised in order (which keeps each in the
// span of the computed vectors of its cluster) and signed so that the largest-modulus
// component is positive.  work: 5 J kk doubles; Z: J x kk, element (i, r) at Z[i*kk + r].
template <class TM>
TLA_HD void tridiag_vectors(TM& tm, const double* a, const double* b, int J, int kk,
                            const double* theta, double tnorm, bool orth, double* work, double* Z) {
  const double tiny = kEps * (tnorm > 0.0 ? tnorm : 1.0);
  for (int r = tm.tid; r < kk; r += tm.nt) {
    const double th = theta[r];
    double* W = work + r;  // element (i, f) at W[(i*5 + f) * kk]
    const int64_t st = kk, ys = 5 * st;
    // factor: pending row (p0, p1) at columns i, i+1; the pivots are kept as reciprocals
    double p0 = a[0] - th, p1 = J > 1 ? b[0] : 0.0;
    for (int i = 0; i + 1 < J; ++i) {
      const double bi = b[i], dn = a[i + 1] - th, bn = i + 2 < J ? b[i + 1] : 0.0;
      double* w = W + i * ys;
      if (fabs(bi) > fabs(p0)) {  // interchange rows i and i+1
        const double inv = tm.recip(bi), l = p0 * inv;
        w[0] = inv;
        w[st] = dn;
        w[2 * st] = 1.0;
        w[3 * st] = l;
        p0 = p1 - l * dn;
        p1 = -l * bn;
      } else {
        if (fabs(p0) < tiny) p0 = p0 < 0.0 ? -tiny : tiny;
        const double inv = tm.recip(p0), l = bi * inv;
        w[0] = inv;
        w[st] = p1;
        w[2 * st] = 0.0;
        w[3 * st] = l;
        p0 = dn - l * p1;
        p1 = bn;
      }
    }
    if (fabs(p0) < tiny) p0 = p0 < 0.0 ? -tiny : tiny;
    W[(J - 1) * ys] = tm.recip(p0);
    double* y = W + 4 * st;  // y_i at y[i*ys]
    for (int i = 0; i < J; ++i) y[i * ys] = lanczos_start(i, 1 + r);  // a different start per vector
    for (int it = 0; it < 3; ++it) {
      // forward (L, with the interchanges): four steps per round, their loads first (step
      // i reads y_{i+1} before step i+1 overwrites it)
      double rp = y[0];
      int i = 0;
      for (; i + 4 < J; i += 4) {
        double xn[4], lv[4], fv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double* w = W + (i + u) * ys;
          xn[u] = y[(i + u + 1) * ys];
          lv[u] = w[3 * st];
          fv[u] = w[2 * st];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (fv[u] != 0.0) {
            y[(i + u) * ys] = xn[u];
            rp -= lv[u] * xn[u];
          } else {
            y[(i + u) * ys] = rp;
            rp = xn[u] - lv[u] * rp;
          }
        }
      }
      for (; i + 1 < J; ++i) {
        const double* w = W + i * ys;
        const double xn = y[(i + 1) * ys], l = w[3 * st];
        if (w[2 * st] != 0.0) {
          y[i * ys] = xn;
          rp -= l * xn;
        } else {
          y[i * ys] = rp;
          rp = xn - l * rp;
        }
      }
      // backward (U), y_{i+1} and y_{i+2} carried in registers
      double y1 = rp * W[(J - 1) * ys], y2 = 0.0;
      y[(J - 1) * ys] = y1;
      i = J - 2;
      for (; i >= 3; i -= 4) {
        double yv[4], sv[4], fv[4], pv[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ii = i - u;
          const double* w = W + ii * ys;
          yv[u] = y[ii * ys];
          sv[u] = w[st];
          fv[u] = w[2 * st];
          pv[u] = w[0];
          bv[u] = ii + 2 < J ? b[ii + 1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ii = i - u;
          double v = yv[u] - sv[u] * y1;
          if (fv[u] != 0.0 && ii + 2 < J) v -= bv[u] * y2;
          v *= pv[u];
          y[ii * ys] = v;
          y2 = y1;
          y1 = v;
        }
      }
      for (; i >= 0; --i) {
        const double* w = W + i * ys;
        double v = y[i * ys] - w[st] * y1;
        if (w[2 * st] != 0.0 && i + 2 < J) v -= b[i + 1] * y2;
        v *= w[0];
        y[i * ys] = v;
        y2 = y1;
        y1 = v;
      }
      double big = 0.0;
      for (int i = 0; i < J; ++i) big = fmax(big, fabs(y[i * ys]));
      // rescale first so that the squares cannot overflow
      const double sc = big > 0.0 ? 1.0 / big : 1.0;
      double nr = 0.0;
      for (int i = 0; i < J; ++i) {
        const double v = y[i * ys] * sc;
        y[i * ys] = v;
        nr += v * v;
      }
      const double inv = 1.0 / sqrt(nr);
      for (int i = 0; i < J; ++i) y[i * ys] *= inv;
    }
    for (int i = 0; i < J; ++i) Z[(int64_t)i * kk + r] = y[i * ys];
  }
  tm.sync();
  if (orth) tridiag_orthonormalise(tm, J, kk, work, Z);
}

// The columns of Z (J x kk, element (i, r) at Z[i*kk + r]) orthonormalised in order and
// signed so that the largest-modulus component is positive.  work: kk^2 doubles.
template <class TM>
TLA_HD void tridiag_orthonormalise(TM& tm, int J, int kk, double* work, double* Z) {
  // Columns already orthonormal to within 1e-4 (the eigenvectors of distinct eigenvalues
  // from inverse iteration are, to about eps ||T|| / gap): with Z^T Z = I + E, the Cholesky
  // factor is R = I + U + O(E^2), U the strict upper triangle of E plus half its diagonal,
  // so Z (I - U) is the Q factor of Z (the in-order Gram-Schmidt result) up to O(E^2).  Two
  // such first-order passes take E from 1e-4 to below rounding.  The products run in
  // parallel over all (p, q) and (i, q) pairs instead of the sequential Cholesky below.
  {
    double* E = work;                    // kk x kk, upper triangle
    double* Zn = work + (int64_t)kk * kk;  // J x kk
    bool first_order = true;
    for (int pass = 0; pass < 2 && first_order; ++pass) {
      double big = 0.0;
      for (int e = tm.tid; e < kk * kk; e += tm.nt) {
        const int p = e / kk, q = e % kk;
        if (p > q) continue;
        double d = 0.0;
        for (int i = 0; i < J; ++i) d += Z[(int64_t)i * kk + p] * Z[(int64_t)i * kk + q];
        if (p == q) d -= 1.0;
        E[e] = d;
        if (!(fabs(d) <= 1e-4)) big = 1.0;
      }
      big = tm.sum(big);
      if (big > 0.0) first_order = false;  // the full path below
      if (!first_order) break;
      for (int e = tm.tid; e < J * kk; e += tm.nt) {
        const int i = e / kk, q = e % kk;
        const double* zi = Z + (int64_t)i * kk;
        double v = zi[q] - 0.5 * E[q * kk + q] * zi[q];
        for (int p = 0; p < q; ++p) v -= zi[p] * E[p * kk + q];
        Zn[e] = v;
      }
      tm.sync();
      for (int e = tm.tid; e < J * kk; e += tm.nt) Z[e] = Zn[e];
      tm.sync();
    }
    if (first_order) {
      tridiag_sign_columns(tm, J, kk, Z);
      return;
    }
  }
  // Orthonormalise the columns in order by Cholesky QR, twice: C = Z^T Z = R^T R, then
  // Z <- Z R^-1 (the Q factor of Z, which Gram-Schmidt in column order would also give;
  // the columns are close to orthonormal, so C is well conditioned and the second pass
  // brings them to working accuracy).  C and R share `work` (free after the solves).
  double* C = work;
  for (int pass = 0; pass < 2; ++pass) {
    for (int e = tm.tid; e < kk * kk; e += tm.nt) {
      const int p = e / kk, q = e % kk;
      if (p > q) continue;
      double d = 0.0;
      for (int i = 0; i < J; ++i) d += Z[(int64_t)i * kk + p] * Z[(int64_t)i * kk + q];
      C[p * kk + q] = d;
    }
    tm.sync();
    // R (upper, in C's upper triangle), row by row on one wave: R_pp = sqrt(C_pp - sum
    // R_ip^2), R_pq = (C_pq - sum R_ip R_iq) / R_pp
    if (tm.wave == 0) {
      auto wt = tm.wave_team();
      for (int p = 0; p < kk; ++p) {
        double dg = C[p * kk + p];
        for (int i = 0; i < p; ++i) dg -= C[i * kk + p] * C[i * kk + p];
        const double rpp = sqrt(dg > 0.0 ? dg : 1e-300);
        for (int q = p + 1 + wt.lane; q < kk; q += wt.wsize) {
          double v = C[p * kk + q];
          for (int i = 0; i < p; ++i) v -= C[i * kk + p] * C[i * kk + q];
          C[p * kk + q] = v / rpp;
        }
        wt.sync();
        if (wt.lane == 0) C[p * kk + p] = rpp;
        wt.sync();
      }
    }
    tm.sync();
    // each row z of Z: z <- z R^-1 (forward substitution over the columns)
    for (int i = tm.tid; i < J; i += tm.nt) {
      double* zi = Z + (int64_t)i * kk;
      for (int q = 0; q < kk; ++q) {
        double v = zi[q];
        for (int p = 0; p < q; ++p) v -= zi[p] * C[p * kk + q];
        zi[q] = v / C[q * kk + q];
      }
    }
    tm.sync();
  }
  tridiag_sign_columns(tm, J, kk, Z);
}

// Columns of Z (J x kk) signed so that the largest-modulus component (lowest index on ties)
// is positive; a thread per column.
template <class TM>
TLA_HD void tridiag_sign_columns(TM& tm, int J, int kk, double* Z) {
  for (int r = tm.tid; r < kk; r += tm.nt) {
    double best = -1.0;
    int bi = 0;
    for (int i = 0; i < J; ++i) {
      const double v = fabs(Z[(int64_t)i * kk + r]);
      if (v > best) best = v, bi = i;
    }
    if (Z[(int64_t)bi * kk + r] < 0.0)
      for (int i = 0; i < J; ++i) Z[(int64_t)i * kk + r] = -Z[(int64_t)i * kk + r];
  }
  tm.sync();
}

// --------------------------------------------------------------------------- row groups
// The Lanczos vectors are split by rows over G groups (workgroups of one grid on the
// device; one group on the host).  Group g owns rows [r0, r1) of every vector, computes
// its share of each dot product, and the groups combine their shares through an
// exchange X, which provides
//   int g, G, r0, r1;
//   bool exchange(TM& tm, const double* part, int n, double* sum, const double* slice,
//                 double* full);
// Every group publishes part[0, n) and, when slice is given, slice[r0, r1); once all have,
// sum[i] is the sum over groups, in the order 0..G-1, of their part[i] (the same value in
// every group), and full[0, N) the published rows of every group.  part and sum may be
// the same array, as may slice and full.  False means the exchange could not complete
// (the caller stops).  Rows of group g: la_group_rows.

// Rows per group and the most groups of the device's split.
constexpr int kLaGroupRows = 32, kLaGroupsMax = 32;
TLA_HD inline int la_groups(int N) {
  const int G = (N + kLaGroupRows - 1) / kLaGroupRows;
  return G < 1 ? 1 : (G > kLaGroupsMax ? kLaGroupsMax : G);
}
// Row stride of the Lanczos basis Q: N rounded up to 16 doubles (128 bytes), so that with
// group boundaries at multiples of 16 rows no cache line holds rows of two groups (the
// groups may run behind different, non-coherent caches).
TLA_HD inline int la_ldq(int N) { return (N + 15) & ~15; }
// Stride of a group's partial array in the exchange buffers (Jmax + 2 rounded to 16).
TLA_HD inline int la_xps(int Jmax) { return (Jmax + 2 + 15) & ~15; }
// Rows [r0, r1) of group g of G: blocks of a multiple of 16 rows (the last shorter or
// empty).
TLA_HD inline void la_group_rows(int N, int G, int g, int* r0, int* r1) {
  const int per = (((N + G - 1) / G) + 15) & ~15;
  const int a = g * per, b = (g + 1) * per;
  *r0 = a < N ? a : N;
  *r1 = b < N ? b : N;
}

// The exchange of a single group.
struct LocalX {
  int g = 0, G = 1, r0 = 0, r1 = 0;
  template <class TM>
  TLA_HD bool exchange(TM& tm, const double* part, int n, double* sum, const double* slice, double* full) {
    tm.sync();
    if (sum != part)
      for (int i = tm.tid; i < n; i += tm.nt) sum[i] = part[i];
    if (slice != nullptr && full != slice)
      for (int t = r0 + tm.tid; t < r1; t += tm.nt) full[t] = slice[t];
    tm.sync();
    return true;
  }
};

// y[r] = sum_{i < n} x[i] A[i*lda + r] (or y[r] -= that sum) for r in [r0, r1): thread
// (r, group of i), eight loads in flight; the groups' partial sums (in `part`) combine in
// the order of the groups.  Rows i < acap of A are read from the copy Ac (element (i, r)
// at Ac[i*(r1 - r0) + r - r0]) instead.
template <class TM>
TLA_HD TLA_INLINE void colsum_rows(TM& tm, const double* A, int64_t lda, const double* x, int n, int r0, int r1, double* y,
                        bool subtract, double* part, int64_t part_doubles, int gmax = 32,
                        const double* Ac = nullptr, int acap = 0) {
  const int nr = r1 - r0;
  if (nr <= 0) {
    tm.sync();
    return;
  }
  int G = tm.nt / nr;
  if (G > gmax) G = gmax;
  if (G < 1 || part == nullptr || (int64_t)G * nr > part_doubles) G = 1;
  for (int e = tm.tid; e < G * nr; e += tm.nt) {
    const int r = r0 + e % nr, g = e / nr;
    const int i0 = (int)((int64_t)n * g / G), i1 = (int)((int64_t)n * (g + 1) / G);
    const double* col = A + r;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0, a5 = 0.0, a6 = 0.0, a7 = 0.0;
    int i = i0;
    if (Ac != nullptr) {
      const double* cc = Ac + (r - r0);
      const int ic = i1 < acap ? i1 : acap;
      for (; i + 8 <= ic; i += 8) {
        a0 += cc[(int64_t)i * nr] * x[i];
        a1 += cc[(int64_t)(i + 1) * nr] * x[i + 1];
        a2 += cc[(int64_t)(i + 2) * nr] * x[i + 2];
        a3 += cc[(int64_t)(i + 3) * nr] * x[i + 3];
        a4 += cc[(int64_t)(i + 4) * nr] * x[i + 4];
        a5 += cc[(int64_t)(i + 5) * nr] * x[i + 5];
        a6 += cc[(int64_t)(i + 6) * nr] * x[i + 6];
        a7 += cc[(int64_t)(i + 7) * nr] * x[i + 7];
      }
      for (; i < ic; ++i) a0 += cc[(int64_t)i * nr] * x[i];
    }
    for (; i + 8 <= i1; i += 8) {
      a0 += col[(int64_t)i * lda] * x[i];
      a1 += col[(int64_t)(i + 1) * lda] * x[i + 1];
      a2 += col[(int64_t)(i + 2) * lda] * x[i + 2];
      a3 += col[(int64_t)(i + 3) * lda] * x[i + 3];
      a4 += col[(int64_t)(i + 4) * lda] * x[i + 4];
      a5 += col[(int64_t)(i + 5) * lda] * x[i + 5];
      a6 += col[(int64_t)(i + 6) * lda] * x[i + 6];
      a7 += col[(int64_t)(i + 7) * lda] * x[i + 7];
    }
    for (; i < i1; ++i) a0 += col[(int64_t)i * lda] * x[i];
    const double acc = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
    if (G == 1) y[r] = subtract ? y[r] - acc : acc;
    else part[(int64_t)g * nr + (r - r0)] = acc;
  }
  tm.sync();
  if (G > 1) {
    for (int r = r0 + tm.tid; r < r1; r += tm.nt) {
      double acc = part[r - r0];
      for (int g = 1; g < G; ++g) acc += part[(int64_t)g * nr + (r - r0)];
      y[r] = subtract ? y[r] - acc : acc;
    }
    tm.sync();
  }
}

// y[r] = sum_{c < n} M[r*ldm + c] x[c] for r in [r0, r1), M symmetric (so this is also the
// column sum of colsum_rows).  With 64-lane waves: each wave takes four rows at a time,
// its lanes over the columns (coalesced rows, eight loads in flight per lane), then a wave
// sum per row; otherwise colsum_rows.
template <class TM>
TLA_HD TLA_INLINE void symv_rows(TM& tm, const double* M, int64_t ldm, const double* x, int n, int r0, int r1, double* y,
                      double* part, int64_t part_doubles) {
  if (tm.wsize != 64) {
    colsum_rows(tm, M, ldm, x, n, r0, r1, y, false, part, part_doubles);
    return;
  }
  for (int rb = r0 + 4 * tm.wave; rb < r1; rb += 4 * tm.nwaves) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const double* row[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) row[u] = M + (int64_t)(rb + u < r1 ? rb + u : rb) * ldm;
    int c = tm.lane;
    for (; c + 64 < n; c += 128) {
      const double x0 = x[c], x1 = x[c + 64];
      double v[8];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v[2 * u] = row[u][c];
        v[2 * u + 1] = row[u][c + 64];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += v[2 * u] * x0 + v[2 * u + 1] * x1;
    }
    if (c < n) {
      const double x0 = x[c];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += row[u][c] * x0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double sum = tm.wave_sum(acc[u]);
      if (tm.lane == 0 && rb + u < r1) y[rb + u] = sum;
    }
  }
  tm.sync();
}

// h[i] = sum over the group's rows of Q[i*ldq + t] w[t], i < n (this group's share), and
// with `self` also h[n] = the group's share of |w|^2: a wave (or half-wave) per i, lanes
// over the rows.  Rows i < qcap of Q are read from the copy Qc (element (i, t) at
// Qc[i*(r1 - r0) + t - r0]) instead.
template <class TM>
TLA_HD TLA_INLINE void dots_rows(TM& tm, const double* Q, int ldq, const double* w, int n, int r0, int r1, double* h,
                      const double* Qc = nullptr, int qcap = 0, bool self = false) {
  const int nr = r1 - r0, nd = n + (self ? 1 : 0);
  if (Qc == nullptr) qcap = 0;
  if (tm.wsize == 64 && nr <= 32) {
    // a half-wave per vector, lanes over the rows; four vectors' loads in flight per lane
    const int half = tm.lane >> 5, t = r0 + (tm.lane & 31);
    const bool rv = t < r1;
    const double wt = rv ? w[t] : 0.0;
    const int slots = 2 * tm.nwaves;
    for (int i0 = 0; i0 < nd; i0 += 4 * slots) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * slots + 2 * tm.wave + half;
        double x = 0.0;
        if (rv && i < n) x = i < qcap ? Qc[(int64_t)i * nr + (t - r0)] : Q[(int64_t)i * ldq + t];
        else if (rv && i == n && self) x = wt;
        v[u] = x * wt;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double lo, hi;
        tm.half_sums(v[u], lo, hi);
        const int ib = i0 + u * slots + 2 * tm.wave;
        if (tm.lane == 0 && ib < nd) h[ib] = lo;
        if (tm.lane == 0 && ib + 1 < nd) h[ib + 1] = hi;
      }
    }
    tm.sync();
    return;
  }
  for (int i = tm.wave; i < nd; i += tm.nwaves) {
    double s = 0.0;
    for (int t = r0 + tm.lane; t < r1; t += tm.wsize) {
      const double x = i == n ? w[t] : (i < qcap ? Qc[(int64_t)i * nr + (t - r0)] : Q[(int64_t)i * ldq + t]);
      s += x * w[t];
    }
    s = tm.wave_sum(s);
    if (tm.lane == 0) h[i] = s;
  }
  tm.sync();
}

// Top-k eigenpairs of the symmetric N x N matrix M (element (r, c) at M[r*ldm + c]) by
// Lanczos with full reorthogonalisation (classical Gram-Schmidt, twice), the rows split
// over the groups of X.  Q: Jmax+1 vectors of stride la_ldq(N) (each group touches its
// rows).  ws.q, ws.w: N (the group's own copies), ws.h: Jmax+2, ws.alpha, ws.beta: Jmax+1.
// Converged when every top-k Ritz residual beta_J |z_J| <= rtol * theta_1, or J = N.  The
// convergence checks run on group 0, which alone writes evals[k] (descending) and Z (J x k,
// the Ritz vectors of T_J, element (i, c) at i*k + c).  Returns J, -1 on failure, -2 when
// an exchange could not complete.
template <class TM, class X>
TLA_HD TLA_INLINE int lanczos_topk(TM& tm, X& xg, const double* M, int ldm, int N, int k, double rtol, int Jmax,
                        double* Q, const LanczosWork& ws, double* evals, double* Z) {
  if (Jmax > N) Jmax = N;
  double* q = ws.q;
  double* w = ws.w;
  double* h = ws.h;
  const int r0 = xg.r0, r1 = xg.r1, ldq = la_ldq(N);
  const bool lead = xg.g == 0;
  // the group's rows of the first qcap basis vectors are also kept in fast memory
  // (element (i, t) at qc[i*(r1 - r0) + t - r0]); the products read them from there
  double* qc = ws.qc;
  int qcap = 0;
  if (qc != nullptr && r1 > r0) {
    const int64_t c = ws.qc_doubles / (r1 - r0);
    qcap = c < Jmax + 1 ? (int)c : Jmax + 1;
  }
  auto store_q = [&](int i, int t, double v) {
    Q[(int64_t)i * ldq + t] = v;
    if (i < qcap) qc[(int64_t)i * (r1 - r0) + (t - r0)] = v;
  };
  // q_0: every group forms the whole (deterministic) start vector
  {
    double s = 0.0;
    for (int i = tm.tid; i < N; i += tm.nt) {
      const double v = lanczos_start(i, 0);
      s += v * v;
    }
    s = tm.sum(s);
    const double inv = 1.0 / sqrt(s);
    for (int i = tm.tid; i < N; i += tm.nt) q[i] = lanczos_start(i, 0) * inv;
    // (recomputed rather than read back from q: another thread wrote q[i])
    for (int i = r0 + tm.tid; i < r1; i += tm.nt) store_q(0, i, lanczos_start(i, 0) * inv);
    tm.sync();
  }
  int J = 0;
  int check = 2 * k > k + 16 ? 2 * k : k + 16;
  if (check > Jmax) check = Jmax;
  double anorm = 0.0;
  int restarts = 0;
  // One classical Gram-Schmidt pass of w[rows] against the first n vectors; the
  // coefficients stay in h[0, n).
  // h[n - 1] is returned in *last (read before the pass's final synchronisation, so that
  // the next writes of h cannot overtake it).
  auto orth_pass = [&](int n, double* last) -> bool {
    dots_rows(tm, Q, ldq, w, n, r0, r1, h, qc, qcap);
    if (!xg.exchange(tm, h, n, h, nullptr, nullptr)) return false;
    if (last != nullptr) *last = h[n - 1];
    colsum_rows(tm, Q, ldq, h, n, r0, r1, w, true, ws.fast, ws.fast_doubles, 8, qc, qcap);
    return true;
  };
  // The squared norm of w and the whole of w, in every group
  auto gather_norm = [&](double* nrm) -> bool {
    double s = 0.0;
    for (int t = r0 + tm.tid; t < r1; t += tm.nt) s += w[t] * w[t];
    s = tm.sum(s);
    if (tm.tid == 0) h[0] = s;
    if (!xg.exchange(tm, h, 1, h, w, w)) return false;
    *nrm = sqrt(h[0]);
    tm.sync();
    return true;
  };
  // Each step exchanges twice: the first Gram-Schmidt pass, then the second pass together
  // with the squared norm and the rows of w as they are before the second pass (w^).  The
  // stored basis vector q_{j+1} = (w^ - Q h2) / beta takes the second-pass correction on
  // the group's own rows; the next product is formed from x = w^ / beta, which differs
  // from q_{j+1} by Q h2 / beta.  By the Lanczos relation M q_i = beta_{i-1} q_{i-1} +
  // alpha_i q_i + beta_i q_{i+1}, M x - M q_{j+1} lies in the span of q_0..q_{j+1} (so the
  // first pass removes it) with component h2_j on q_{j+1}, which is taken off alpha_{j+1}
  // (corr).  beta^2 = |w^|^2 - |h2|^2 since Q^T w^ = h2 and Q^T Q = I.
  double corr = 0.0;
  for (int j = 0; j < Jmax; ++j) {
    tm.tick(-1);
    // w = M x over the group's rows
    symv_rows(tm, M, ldm, q, N, r0, r1, w, ws.fast, ws.fast_doubles);
    tm.tick(10);
    double h1j = 0.0;
    if (!orth_pass(j + 1, &h1j)) return -2;
    double aj = h1j - corr;
    // second pass coefficients and the squared norm of w^ (h[j + 1])
    dots_rows(tm, Q, ldq, w, j + 1, r0, r1, h, qc, qcap, true);
    if (!xg.exchange(tm, h, j + 2, h, w, q)) return -2;  // q <- w^ (every row)
    aj += h[j];
    corr = h[j];
    double h2sq = 0.0;  // |h2|^2: lanes over the coefficients, the same bits in every wave
    for (int i = tm.lane; i <= j; i += tm.wsize) h2sq += h[i] * h[i];
    h2sq = tm.wave_sum(h2sq);
    const double nsq = h[j + 1] - h2sq;
    double nr = sqrt(nsq > 0.0 ? nsq : 0.0);
    colsum_rows(tm, Q, ldq, h, j + 1, r0, r1, w, true, ws.fast, ws.fast_doubles, 8, qc, qcap);
    tm.tick(11);
    if (tm.tid == 0) {
      ws.alpha[j] = aj;  // the same value in every group
      ws.beta[j] = nr;
    }
    tm.sync();
    J = j + 1;
    {
      const double an = fabs(aj) + nr + (j ? ws.beta[j - 1] : 0.0);
      if (an > anorm) anorm = an;
    }
    const bool breakdown = nr <= 64.0 * kEps * anorm;
    if (J >= check || breakdown || J == N) {
      // Ritz values of T_J by multisection, Ritz vectors of T_J by inverse iteration; the
      // residual of Ritz pair i is beta_J |z_{J-1,i}|.  Decision: 0 go on, 1 converged (or
      // J = N), 2 failed.  When the work fits in fast memory every group computes the Ritz
      // values of its share of the ranks (and rank 0, the scale), they meet in one
      // exchange, and every group then reaches the same decision; otherwise group 0 alone
      // checks and sends its decision.
      const int kk = k < J ? k : J;
      const int64_t need = J + kk + 6 * (int64_t)J * kk;
      const bool spread = ws.fast != nullptr && need <= ws.fast_doubles;  // the same in every group
      double* b2 = spread ? ws.fast : ws.T;
      double* theta = b2 + J;
      double* work = theta + kk;
      double* Zm = work + 5 * (int64_t)J * kk;
      double tnorm = 0.0;
      int decision = 0;
      bool have_z = false;  // Zm holds the (not yet orthonormalised) Ritz vectors of T_J
      // The closed form of the last components is exact where they are large but has an
      // absolute floor near sqrt(eps): it can show that a pair has not converged, not that
      // it has.  Only when it cannot decide are the Ritz vectors of T_J computed (inverse
      // iteration).
      if (spread) {
        tm.stamp(0);
        tm.tick(12);
        for (int i = tm.tid; i + 1 < J; i += tm.nt) b2[i] = ws.beta[i] * ws.beta[i];
        for (int r = tm.tid; r < kk; r += tm.nt) theta[r] = 0.0;
        tm.sync();
        tridiag_topk_values(tm, ws.alpha, ws.beta, b2, J, kk, theta, &tnorm, xg.g, xg.G);
        tm.tick(13);
        const double scale = fabs(theta[0]) > 0 ? fabs(theta[0]) : 1e-300;
        double open = 0.0;
        for (int r = xg.g + tm.tid * xg.G; r < kk; r += tm.nt * xg.G) {
          const double zl = tridiag_last_component(ws.alpha, b2, J, theta[r]);
          if (zl > 1e-6 && nr * zl > rtol * scale) open = 1.0;
        }
        open = tm.sum(open);
        for (int r = tm.tid; r < kk; r += tm.nt) h[r] = r % xg.G == xg.g ? theta[r] : 0.0;
        if (tm.tid == 0) h[kk] = open;
        if (!xg.exchange(tm, h, kk + 1, h, nullptr, nullptr)) return -2;
        for (int r = tm.tid; r < kk; r += tm.nt) theta[r] = h[r];
        bool conv = J >= k && h[kk] == 0.0;
        tm.sync();
        if (conv) {
          tridiag_vectors(tm, ws.alpha, ws.beta, J, kk, theta, tnorm, false, work, Zm);
          have_z = true;
          for (int i = 0; i < k; ++i)
            if (nr * fabs(Zm[(int64_t)(J - 1) * kk + i]) > rtol * scale) conv = false;
        }
        tm.tick(14);
        tm.stamp(1);
        if (conv || J == N) decision = J >= k ? 1 : 2;
        else if (J == Jmax) decision = 2;
      } else {
        if (lead) {
          tm.stamp(0);
          tm.tick(12);
          for (int i = tm.tid; i + 1 < J; i += tm.nt) b2[i] = ws.beta[i] * ws.beta[i];
          tm.sync();
          tridiag_topk_values(tm, ws.alpha, ws.beta, b2, J, kk, theta, &tnorm);
          tm.tick(13);
          const double scale = fabs(theta[0]) > 0 ? fabs(theta[0]) : 1e-300;
          double* zl = Zm;
          for (int r = tm.tid; r < kk; r += tm.nt) zl[r] = tridiag_last_component(ws.alpha, b2, J, theta[r]);
          tm.sync();
          bool conv = J >= k;
          for (int i = 0; i < kk && conv; ++i)
            if (zl[i] > 1e-6 && nr * zl[i] > rtol * scale) conv = false;
          tm.sync();
          if (conv) {
            tridiag_vectors(tm, ws.alpha, ws.beta, J, kk, theta, tnorm, false, work, Zm);
            have_z = true;
            for (int i = 0; i < k; ++i)
              if (nr * fabs(Zm[(int64_t)(J - 1) * kk + i]) > rtol * scale) conv = false;
          }
          tm.tick(14);
          tm.stamp(1);
          if (conv || J == N) decision = J >= k ? 1 : 2;
          else if (J == Jmax) decision = 2;
          if (tm.tid == 0) h[0] = (double)decision;
        } else if (tm.tid == 0) {
          h[0] = 0.0;
        }
        if (!xg.exchange(tm, h, 1, h, nullptr, nullptr)) return -2;
        decision = (int)h[0];
        tm.sync();
      }
      if (decision == 2) return -1;
      if (decision == 1) {
        if (lead) {
          // final Ritz vectors: members of eigenvalue clusters orthogonalised (kk = k)
          if (have_z) tridiag_orthonormalise(tm, J, kk, work, Zm);
          else tridiag_vectors(tm, ws.alpha, ws.beta, J, kk, theta, tnorm, true, work, Zm);
          tm.tick(1);
          for (int i = tm.tid; i < k; i += tm.nt) evals[i] = theta[i];
          for (int e = tm.tid; e < J * k; e += tm.nt) Z[e] = Zm[e];
          tm.sync();
          tm.tick(15);
        }
        return J;
      }
      check = J + 8;
      if (check > Jmax) check = Jmax;
      if (breakdown) {
        // invariant subspace found before k pairs converged: restart orthogonally
        // (bounded by the Krylov limit: a matrix of low rank restarts once per null vector)
        if (++restarts > Jmax) return -1;
        for (int t = r0 + tm.tid; t < r1; t += tm.nt) w[t] = lanczos_start(t, J + 17 * restarts);
        tm.sync();
        if (!orth_pass(J, nullptr) || !orth_pass(J, nullptr)) return -2;
        double n2 = 0.0;
        if (!gather_norm(&n2)) return -2;  // w: every row
        if (n2 <= 1e-8) return -1;
        if (tm.tid == 0) ws.beta[j] = 0.0;
        nr = n2;
        corr = 0.0;
        for (int t = tm.tid; t < N; t += tm.nt) q[t] = w[t];
        tm.sync();
      }
    }
    const double inv = 1.0 / nr;
    for (int t = tm.tid; t < N; t += tm.nt) q[t] *= inv;
    for (int t = r0 + tm.tid; t < r1; t += tm.nt) store_q(J, t, w[t] * inv);
    tm.sync();
    tm.tick(12);
  }
  return -1;
}

// --------------------------------------------------------------------------- eig(A~)
// Work: H (k*k), v (4), ev (2k doubles: re, im), status (int shared via scal[0]).
// The reflector I - 2 v v^T / vv applied to rows r0..r0+len-1 (columns c0..c1) from the
// left, then to those columns (rows rr0..rr1) from the right.  With zcol >= 0, the
// entries of column zcol below row r0, which the reflector annihilates, are set to zero.
template <class TM>
TLA_HD void hess_reflect(TM& tm, double* H, int k, int r0, int len, const double* v, double vv,
                         int c0, int c1, int rr0, int rr1, int zcol = -1) {
  const double tv = 2.0 / vv;
  // left: rows r0..r0+len-1, columns c0..c1
  for (int c = c0 + tm.tid; c <= c1; c += tm.nt) {
    double t = 0.0;
    for (int i = 0; i < len; ++i) t += v[i] * H[(r0 + i) * k + c];
    const double f = t * tv;
    H[r0 * k + c] -= f * v[0];
    for (int i = 1; i < len; ++i) H[(r0 + i) * k + c] = c == zcol ? 0.0 : H[(r0 + i) * k + c] - f * v[i];
  }
  tm.sync();
  // right: columns r0..r0+len-1, rows rr0..rr1
  for (int r = rr0 + tm.tid; r <= rr1; r += tm.nt) {
    double t = 0.0;
    for (int i = 0; i < len; ++i) t += H[r * k + r0 + i] * v[i];
    const double f = t * tv;
    for (int i = 0; i < len; ++i) H[r * k + r0 + i] -= f * v[i];
  }
  tm.sync();
}

// Eigenvalues of the real k x k matrix A (row-major); H: k*k scratch.  ev[2k] receives
// (re, im) pairs.  Returns false on failure.
template <class TM>
TLA_HD bool eigvals_general(TM& tm, const double* A, int k, double* H, double* ev) {
  for (int e = tm.tid; e < k * k; e += tm.nt) H[e] = A[e];
  tm.sync();
  double v[3];
  // Householder reduction to Hessenberg form
  for (int j = 0; j < k - 2; ++j) {
    double tail = 0.0;  // sum of squares below the subdiagonal
    for (int i = j + 2 + tm.lane; i < k; i += tm.wsize) tail += H[i * k + j] * H[i * k + j];
    tail = tm.wave_sum(tail);
    const double x0 = H[(j + 1) * k + j];
    const double alpha = sqrt(x0 * x0 + tail);
    if (alpha == 0.0) continue;
    // reflector on rows/cols j+1..k-1; long vector kept in H's column below the diagonal
    // is not reused, so compute the update directly
    const double sg = x0 >= 0 ? 1.0 : -1.0;
    const double v0 = x0 + sg * alpha;
    const double vv = v0 * v0 + tail;
    // snapshot of the vector (column j below the diagonal) before it is overwritten
    // left update of columns j..k-1
    for (int c = j + tm.tid; c < k; c += tm.nt) {
      if (c == j) continue;
      double t = v0 * H[(j + 1) * k + c];
      for (int i = j + 2; i < k; ++i) t += H[i * k + j] * H[i * k + c];
      const double f = 2.0 * t / vv;
      H[(j + 1) * k + c] -= f * v0;
      for (int i = j + 2; i < k; ++i) H[i * k + c] -= f * H[i * k + j];
    }
    tm.sync();
    // right update of all rows, columns j+1..k-1
    for (int r = tm.tid; r < k; r += tm.nt) {
      double t = H[r * k + j + 1] * v0;
      for (int i = j + 2; i < k; ++i) t += H[r * k + i] * H[i * k + j];
      const double f = 2.0 * t / vv;
      H[r * k + j + 1] -= f * v0;
      for (int i = j + 2; i < k; ++i) H[r * k + i] -= f * H[i * k + j];
    }
    tm.sync();
    if (tm.tid == 0) {
      H[(j + 1) * k + j] = -sg * alpha;
      for (int i = j + 2; i < k; ++i) H[i * k + j] = 0.0;
    }
    tm.sync();
  }
  // Francis double-shift QR
  double hnorm = 0.0;
  for (int e = tm.lane; e < k * k; e += tm.wsize) hnorm = fmax(hnorm, fabs(H[e]));
  hnorm = tm.wave_max(hnorm);
  int hi = k - 1, its = 0, total = 0, nev = 0;
  while (hi >= 0) {
    // l = largest index <= hi with a negligible subdiagonal entry H[l][l-1] (0 if none);
    // the lanes test hi - lane, hi - lane - wsize, ... together
    int l = 0;
    for (int top = hi; top > 0; top -= tm.wsize) {
      const int c = top - tm.lane;
      bool small = false;
      if (c > 0) {
        double s = fabs(H[(c - 1) * k + c - 1]) + fabs(H[c * k + c]);
        if (s == 0.0) s = hnorm;
        small = fabs(H[c * k + c - 1]) <= kEps * s;
      }
      const int f = tm.wave_first(small);
      if (f < tm.wsize && top - f > 0) {
        l = top - f;
        break;
      }
    }
    tm.sync();
    if (l > 0 && tm.tid == 0) H[l * k + l - 1] = 0.0;
    tm.sync();
    if (l == hi) {
      ev[2 * nev] = H[hi * k + hi];
      ev[2 * nev + 1] = 0.0;
      ++nev;
      --hi;
      its = 0;
      continue;
    }
    if (l == hi - 1) {
      const double a = H[(hi - 1) * k + hi - 1], b = H[(hi - 1) * k + hi];
      const double c = H[hi * k + hi - 1], d = H[hi * k + hi];
      const double p = 0.5 * (a - d), qq = p * p + b * c, mid = 0.5 * (a + d);
      if (qq >= 0.0) {
        const double z = sqrt(qq);
        const double l1 = mid + (p >= 0 ? z : -z);
        const double det = a * d - b * c;
        const double l2 = (l1 != 0.0) ? det / l1 : mid - (p >= 0 ? z : -z);
        ev[2 * nev] = l1;
        ev[2 * nev + 1] = 0.0;
        ev[2 * nev + 2] = l2;
        ev[2 * nev + 3] = 0.0;
      } else {
        const double im = sqrt(-qq);
        ev[2 * nev] = mid;
        ev[2 * nev + 1] = im;
        ev[2 * nev + 2] = mid;
        ev[2 * nev + 3] = -im;
      }
      nev += 2;
      hi -= 2;
      its = 0;
      continue;
    }
    if (++its > 60 || ++total > 60 * k) return false;
    double s, t;
    if (its == 10 || its == 20) {
      const double wv = fabs(H[hi * k + hi - 1]) + fabs(H[(hi - 1) * k + hi - 2]);
      s = 1.5 * wv;
      t = wv * wv;
    } else {
      s = H[(hi - 1) * k + hi - 1] + H[hi * k + hi];
      t = H[(hi - 1) * k + hi - 1] * H[hi * k + hi] - H[(hi - 1) * k + hi] * H[hi * k + hi - 1];
    }
    double x = H[l * k + l] * H[l * k + l] + H[l * k + l + 1] * H[(l + 1) * k + l] - s * H[l * k + l] + t;
    double y = H[(l + 1) * k + l] * (H[l * k + l] + H[(l + 1) * k + l + 1] - s);
    double z = H[(l + 1) * k + l] * H[(l + 2) * k + l + 1];
    for (int kk = l; kk <= hi - 2; ++kk) {
      const double alpha = sqrt(x * x + y * y + z * z);
      if (alpha != 0.0) {
        v[0] = x + (x >= 0 ? alpha : -alpha);
        v[1] = y;
        v[2] = z;
        const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const int c0 = kk - 1 > l ? kk - 1 : l;
        const int rr1 = kk + 3 < hi ? kk + 3 : hi;
        hess_reflect(tm, H, k, kk, 3, v, vv, c0, hi, l, rr1, kk > l ? kk - 1 : -1);
      }
      x = H[(kk + 1) * k + kk];
      y = H[(kk + 2) * k + kk];
      z = (kk < hi - 2) ? H[(kk + 3) * k + kk] : 0.0;
    }
    {
      const int kk = hi - 1;
      const double alpha = hypot(x, y);
      if (alpha != 0.0) {
        v[0] = x + (x >= 0 ? alpha : -alpha);
        v[1] = y;
        const double vv = v[0] * v[0] + v[1] * v[1];
        const int c0 = kk - 1 > l ? kk - 1 : l;
        hess_reflect(tm, H, k, kk, 2, v, vv, c0, hi, l, hi, kk > l ? kk - 1 : -1);
      }
    }
  }
  return nev == k;
}

// Eigenvector of the real k x k matrix A for the eigenvalue (lre, lim) by three steps of
// inverse iteration, done by one wave team: the complex LU with partial pivoting of
// A - lambda I and the triangular solves are split over the lanes.  LU: k*k, b, y: k
// complex, piv: k ints.  Unnormalised result in out (column of W).  Returns false when
// an iterate is zero or not finite.
template <class TW>
TLA_HD bool eigvec_wave(TW& wt, const double* A, int k, double lre, double lim, cpx* LU, cpx* b,
                        cpx* y, int* piv, cpx* out) {
  const int L = wt.lane, WS = wt.wsize;
  double amax = 0.0;
  for (int e = L; e < k * k; e += WS) {
    const int r = e / k, c = e % k;
    LU[e] = cmk(A[e] - (r == c ? lre : 0.0), r == c ? -lim : 0.0);
    amax = fmax(amax, cabsv(LU[e]));
  }
  amax = wt.wave_max(amax);
  wt.sync();
  const double tiny = (amax > 1e-300 ? amax : 1e-300) * kEps;
  for (int jj = 0; jj < k; ++jj) {
    double best = -1.0;
    int bi = jj;
    for (int i = jj + L; i < k; i += WS) {
      const double a = cabsv(LU[i * k + jj]);
      if (a > best) best = a, bi = i;
    }
    wt.wave_argmax(best, bi);
    if (L == 0) piv[jj] = bi;
    if (bi != jj)
      for (int c = L; c < k; c += WS) {
        const cpx t = LU[jj * k + c];
        LU[jj * k + c] = LU[bi * k + c];
        LU[bi * k + c] = t;
      }
    wt.sync();
    cpx pv = LU[jj * k + jj];
    if (cabsv(pv) < tiny) pv = cmk(tiny, 0.0);
    wt.sync();
    if (L == 0) LU[jj * k + jj] = pv;
    for (int i = jj + 1 + L; i < k; i += WS) {
      const cpx f = cdiv(LU[i * k + jj], pv);
      LU[i * k + jj] = f;
      for (int c = jj + 1; c < k; ++c) LU[i * k + c] = csub(LU[i * k + c], cmul(f, LU[jj * k + c]));
    }
    wt.sync();
  }
  for (int i = L; i < k; i += WS) b[i] = cmk(1.0, 0.0);
  wt.sync();
  bool ok = true;
  for (int it = 0; it < 3; ++it) {
    if (L == 0)
      for (int jj = 0; jj < k; ++jj)
        if (piv[jj] != jj) {
          const cpx t = b[jj];
          b[jj] = b[piv[jj]];
          b[piv[jj]] = t;
        }
    wt.sync();
    for (int i = L; i < k; i += WS) y[i] = b[i];
    wt.sync();
    // forward substitution with the unit lower factor, by columns
    for (int c = 0; c + 1 < k; ++c) {
      const cpx yc = y[c];
      for (int i = c + 1 + L; i < k; i += WS) y[i] = csub(y[i], cmul(LU[i * k + c], yc));
      wt.sync();
    }
    // back substitution with the upper factor, by columns
    for (int c = k - 1; c >= 0; --c) {
      const cpx yc = cdiv(y[c], LU[c * k + c]);
      wt.sync();
      if (L == 0) y[c] = yc;
      for (int i = L; i < c; i += WS) y[i] = csub(y[i], cmul(LU[i * k + c], yc));
      wt.sync();
    }
    double nr = 0.0;
    for (int i = L; i < k; i += WS) nr += cabs2(y[i]);
    nr = sqrt(wt.wave_sum(nr));
    if (!(nr > 0.0 && nr < 1e300)) {
      ok = false;
      break;
    }
    for (int i = L; i < k; i += WS) b[i] = cscale(y[i], 1.0 / nr);
    wt.sync();
  }
  if (ok)
    for (int i = L; i < k; i += WS) out[i] = b[i];
  wt.sync();
  return ok;
}

// Eigenvectors of the real k x k matrix A for the eigenvalues ev (re, im pairs): the
// waves take eigenvalues in turn, each with its own slice of `region` (fast memory,
// 2k^2 + 5k doubles per wave) and no block-wide synchronisation.  The second member of a
// conjugate pair is skipped (the caller conjugates its partner).  W: column j at j*k.
// Returns false on failure.
template <class TM>
TLA_HD bool eigvecs_team(TM& tm, const double* A, int k, const double* ev, cpx* W, double* region,
                         int64_t region_doubles, int* flag) {
  const int64_t per = 2 * (int64_t)k * k + 5 * (int64_t)k;
  int wl = (int)(region_doubles / per);
  if (wl > tm.nwaves) wl = tm.nwaves;
  if (wl < 1) return false;
  if (tm.tid == 0) flag[0] = 0;
  tm.sync();
  if (tm.wave < wl) {
    auto wt = tm.wave_team();
    cpx* LU = reinterpret_cast<cpx*>(region + tm.wave * per);
    cpx* b = LU + (int64_t)k * k;
    cpx* y = b + k;
    int* piv = reinterpret_cast<int*>(y + k);
    for (int j = tm.wave; j < k; j += wl) {
      if (ev[2 * j + 1] < 0.0 && j > 0 && ev[2 * j - 2] == ev[2 * j] && ev[2 * j - 1] == -ev[2 * j + 1])
        continue;
      if (!eigvec_wave(wt, A, k, ev[2 * j], ev[2 * j + 1], LU, b, y, piv, W + (int64_t)j * k) &&
          wt.lane == 0)
        flag[0] = 1;
    }
  }
  tm.sync();
  return flag[0] == 0;
}

// Unit norm, largest-modulus entry (lowest index on ties) real and positive.
TLA_HD inline void normalise_vec(cpx* w, int k) {
  double nr = 0.0;
  int piv = 0;
  double best = -1.0;
  for (int i = 0; i < k; ++i) {
    nr += cabs2(w[i]);
    const double a = cabsv(w[i]);
    if (a > best) best = a, piv = i;
  }
  nr = sqrt(nr);
  const double am = cabsv(w[piv]);
  const cpx ph = cmk(w[piv].re / am * nr, w[piv].im / am * nr);
  for (int i = 0; i < k; ++i) w[i] = cdiv(w[i], ph);
  w[piv].im = 0.0;
}

}  // namespace tla
}  // namespace cdmd

namespace cdmd {
namespace tla {

// Scratch of one small-LA solve (float64 unless noted).
struct SmallLAWork {
  LanczosWork lz;
  double* Q;    // (Jmax+1) x N
  double* V;    // N x k
  double* Z;    // Jmax x k  Ritz vectors of T_J
  double* TV;   // N x k
  double* P;    // nblk x (k*k + k)  block partials of V^T M12 V and |v_i|^2
  double* nu;   // 2k  column norms of V, then sqrt(mu)
  double* At;   // k x k
  double* Hs;   // k x k
  cpx* LU;      // k x k x k
  cpx* bb;      // k x k
  cpx* yy;      // k x k
  int* piv;     // k x k
  int* flag;    // 1 (shared)
};

// Rows per block of the row-range steps below (the device runs a workgroup per block).
constexpr int kLaRows = 64;

// V[c*N + t] = sum_{i < J} Q[i*ldq + t] Z[i*k + c] (ldq = la_ldq(N)) for rows t in
// [t0, t1): the Ritz vectors of M from those of T_J (not normalised).  Thread (t, block of 8 columns); each
// entry is one sum in the order of i, whatever the team.
template <class TM>
TLA_HD void ritz_rows(TM& tm, const double* Q, int N, int J, const double* Z, int k, double* V, int t0,
                      int t1) {
  constexpr int KB = 8;
  const int nr = t1 - t0, CB = (k + KB - 1) / KB;
  for (int e = tm.tid; e < nr * CB; e += tm.nt) {
    const int t = t0 + e % nr, c0 = (e / nr) * KB;
    double acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c] = 0.0;
    const int ldq = la_ldq(N);
    for (int i = 0; i < J; ++i) {
      const double q = Q[(int64_t)i * ldq + t];
      const double* zi = Z + (int64_t)i * k + c0;
#pragma unroll
      for (int c = 0; c < KB; ++c)
        if (c0 + c < k) acc[c] += q * zi[c];
    }
#pragma unroll
    for (int c = 0; c < KB; ++c)
      if (c0 + c < k) V[(int64_t)(c0 + c) * N + t] = acc[c];
  }
  tm.sync();
}

// TV[c*N + a] = sum_b M12[a][b] V[c*N + b] for rows a in [a0, a1), M12[a][b] =
// Mfull[(b+1)*ldm + a] (symmetric Gram): thread (a, block of 8 columns), eight Gram loads
// in flight; the rows b of V pass through `stage` in chunks.  Each entry is one sum in the
// order of b, whatever the team.
template <class TM>
TLA_HD void m12v_rows(TM& tm, const double* Mfull, int ldm, int N, int k, const double* V, double* TV,
                      int a0, int a1, double* stage, int64_t stage_doubles) {
  constexpr int KB = 8;
  const int CB = (k + KB - 1) / KB;
  int chunk = (int)(stage_doubles / (k > 0 ? k : 1));
  if (chunk > 256) chunk = 256;
  const int nr = a1 - a0;
  const int tasks = nr * CB;
  for (int base = 0; base < tasks; base += tm.nt) {
    const int e = base + tm.tid;
    const bool act = e < tasks;
    const int a = act ? a0 + e % nr : a0, c0 = act ? (e / nr) * KB : 0;
    double acc[KB];
#pragma unroll
    for (int c = 0; c < KB; ++c) acc[c] = 0.0;
    for (int b0 = 0; b0 < N; b0 += chunk) {
      const int nb = N - b0 < chunk ? N - b0 : chunk;
      tm.sync();
      for (int f = tm.tid; f < nb * k; f += tm.nt) {
        const int bb = f / k, c = f % k;
        stage[f] = V[(int64_t)c * N + b0 + bb];
      }
      tm.sync();
      if (act) {
        int bb = 0;
        for (; bb + 8 <= nb; bb += 8) {
          double mv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) mv[u] = Mfull[(int64_t)(b0 + bb + u + 1) * ldm + a];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const double* sv = stage + (bb + u) * k + c0;
#pragma unroll
            for (int c = 0; c < KB; ++c)
              if (c0 + c < k) acc[c] += mv[u] * sv[c];
          }
        }
        for (; bb < nb; ++bb) {
          const double mv = Mfull[(int64_t)(b0 + bb + 1) * ldm + a];
          const double* sv = stage + bb * k + c0;
#pragma unroll
          for (int c = 0; c < KB; ++c)
            if (c0 + c < k) acc[c] += mv * sv[c];
        }
      }
    }
    if (act)
#pragma unroll
      for (int c = 0; c < KB; ++c)
        if (c0 + c < k) TV[(int64_t)(c0 + c) * N + a] = acc[c];
  }
  tm.sync();
}

// The block [a0, a1) share of V^T M12 V and of the squared column norms of V:
// P[i*k + j] = sum_a V[i*N + a] TV[j*N + a], P[k*k + i] = sum_a V[i*N + a]^2 over a in the
// block, in the order of a.  The block's rows of V and TV pass through `stage`.
template <class TM>
TLA_HD void block_gram(TM& tm, const double* V, const double* TV, int N, int k, int a0, int a1, double* P,
                       double* stage, int64_t stage_doubles) {
  int rc = (int)(stage_doubles / (2 * (int64_t)k));
  const int nr = a1 - a0;
  if (rc > nr) rc = nr;
  const int ne = k * k + k;
  for (int base = 0; base < ne; base += tm.nt) {
    const int e = base + tm.tid;
    const int i = e < k * k ? e / k : e - k * k, j = e < k * k ? e % k : i;
    const bool act = e < ne;
    const bool sq = e >= k * k;
    double acc = 0.0;
    for (int r0 = 0; r0 < nr; r0 += rc) {
      const int nb = nr - r0 < rc ? nr - r0 : rc;
      tm.sync();
      for (int f = tm.tid; f < nb * k; f += tm.nt) {
        const int c = f / nb, r = f % nb;
        stage[c * rc + r] = V[(int64_t)c * N + a0 + r0 + r];
        stage[(k + c) * rc + r] = TV[(int64_t)c * N + a0 + r0 + r];
      }
      tm.sync();
      if (act) {
        const double* vi = stage + i * rc;
        const double* tj = sq ? stage + i * rc : stage + (k + j) * rc;
        for (int r = 0; r < nb; ++r) acc += vi[r] * tj[r];
      }
    }
    if (act) P[e] = acc;
  }
  tm.sync();
}

// G[t*k + j] = sum_i (V[i*N + t] / nu[i] / sigma[i]) W[j*k + i] for rows t in [t0, t1):
// G = V S^-1 W with the columns of V normalised by nu.
template <class TM>
TLA_HD void g_rows(TM& tm, const double* V, int N, int k, const double* nu, const double* sigma, const cpx* W,
                   cpx* G, int t0, int t1) {
  const int nr = t1 - t0;
  for (int64_t e = tm.tid; e < (int64_t)nr * k; e += tm.nt) {
    const int t = t0 + (int)(e / k), j = (int)(e % k);
    double re = 0.0, im = 0.0;
    for (int i = 0; i < k; ++i) {
      const double v = V[(int64_t)i * N + t] / nu[i] / sigma[i];
      const cpx wv = W[(int64_t)j * k + i];
      re += v * wv.re;
      im += v * wv.im;
    }
    G[(int64_t)t * k + j] = cmk(re, im);
  }
  tm.sync();
}

// Status codes (match cdmd_status).
constexpr int kOk = 0, kDevice = 4, kRankDeficient = 5, kNumeric = 6;

// Truncated SVD (eq. svd), first part: the top-k eigenpairs of the Gram Gr[0:N, 0:N] (N = m-1)
// of the unscaled sketch by Lanczos, the rows split over the groups of X; group 0 holds
// mu[k] the eigenvalues and Z (J x k) the Ritz vectors of T_J (V = Q_J Z is formed by
// ritz_rows).  Returns the status (the same in every group); *Jout = Krylov size.
template <class TM, class X>
TLA_HD TLA_INLINE int small_la_phase_a(TM& tm, X& xg, const double* Gr, int m, int k, double rtol, int Jmax,
                            const SmallLAWork& ws, double* mu, double* Z, int* Jout) {
  const int N = m - 1;
  {
    double bad = 0.0;
    const int64_t mm = (int64_t)m * m;
    const int64_t e0 = mm * xg.g / xg.G, e1 = mm * (xg.g + 1) / xg.G;
    for (int64_t e = e0 + tm.tid; e < e1; e += tm.nt)
      if (!(fabs(Gr[e]) < 1e300)) bad = 1.0;
    bad = tm.sum(bad);
    if (tm.tid == 0) ws.lz.h[0] = bad;
    if (!xg.exchange(tm, ws.lz.h, 1, ws.lz.h, nullptr, nullptr)) return kDevice;
    const bool any = ws.lz.h[0] > 0.0;
    tm.sync();
    if (any) return kNumeric;
  }
  tm.stamp(2);
  const int J = lanczos_topk(tm, xg, Gr, m, N, k, rtol, Jmax, ws.Q, ws.lz, mu, Z);
  tm.stamp(3);
  *Jout = J;
  if (J == -2) return kDevice;
  if (J < 0) return kNumeric;
  if (xg.g != 0) return kOk;
  if (!(mu[0] > 0.0) || !(mu[k - 1] > 1e-12 * mu[0])) return kRankDeficient;
  return kOk;
}

// End of the truncated SVD and A~ (Section 3.2), given the block partials P (nblk blocks of k*k + k,
// from block_gram over V = Q_J Z and TV = M12 V): nu the column norms of V, sigma =
// sqrt(mu) * sketch_scale, A~ = S^-1 Vn^T M12 Vn S^-1 with Vn = V diag(1/nu), and its
// eigenvalues lam (the first part of eig(A~)).
template <class TM>
TLA_HD int small_la_phase_b1(TM& tm, int N, int k, double sketch_scale, const SmallLAWork& ws, int nblk,
                             const double* mu, double* sigma, cpx* lam) {
  double* nu = ws.nu;
  double* s = ws.nu + k;  // sqrt(mu)
  const int64_t ne = (int64_t)k * k + k;
  for (int i = tm.tid; i < k; i += tm.nt) {
    s[i] = sqrt(mu[i]);
    sigma[i] = s[i] * sketch_scale;
    double q = 0.0;
    for (int b = 0; b < nblk; ++b) q += ws.P[b * ne + (int64_t)k * k + i];
    nu[i] = sqrt(q);
  }
  tm.sync();
  for (int e = tm.tid; e < k * k; e += tm.nt) {
    const int i = e / k, j = e % k;
    double a0 = 0.0;
    for (int b = 0; b < nblk; ++b) a0 += ws.P[b * ne + e];
    ws.At[e] = a0 / (nu[i] * nu[j] * s[i] * s[j]);
  }
  tm.sync();
  tm.stamp(4);
  double* fastr = ws.lz.fast;
  const int64_t fastd = ws.lz.fast_doubles;
  double* ev = ws.lz.w;  // reuse: 2k doubles
  if (tm.tid == 0) ws.flag[0] = 0;
  tm.sync();
  if (tm.wave == 0) {  // one wave: the QR sweeps are short and strictly sequential
    auto wt = tm.wave_team();
    const bool ok = eigvals_general(wt, ws.At, k, (int64_t)k * k <= fastd ? fastr : ws.Hs, ev);
    if (!ok && wt.lane == 0) ws.flag[0] = 1;
  }
  tm.sync();
  if (ws.flag[0] != 0) return kNumeric;
  tm.stamp(5);
  for (int j = tm.tid; j < k; j += tm.nt) lam[j] = cmk(ev[2 * j], ev[2 * j + 1]);
  tm.sync();
  return kOk;
}

// True when lam[j] is the second member of a conjugate pair (its eigenvector is the
// conjugate of its partner's).
TLA_HD inline bool conj_second(const cpx* lam, int j) {
  return lam[j].im < 0.0 && j > 0 && lam[j - 1].re == lam[j].re && lam[j - 1].im == -lam[j].im;
}

// eig(A~), end: the second members of conjugate pairs take their partners' conjugates, and
// every column of W is made unit with its largest entry real and positive.
template <class TM>
TLA_HD void small_la_phase_b3(TM& tm, int k, const cpx* lam, cpx* W) {
  for (int j = tm.tid; j < k; j += tm.nt)
    if (conj_second(lam, j))
      for (int i = 0; i < k; ++i) W[(int64_t)j * k + i] = cconj(W[(int64_t)(j - 1) * k + i]);
  tm.sync();
  for (int j = tm.tid; j < k; j += tm.nt) normalise_vec(W + (int64_t)j * k, k);
  tm.sync();
  tm.stamp(6);
}

// End of the truncated SVD, A~ and eig(A~) by one team: phase B1, the eigenvectors W of A~ (column j at
// j*k), phase B3.
template <class TM>
TLA_HD int small_la_phase_b(TM& tm, int N, int k, double sketch_scale, const SmallLAWork& ws, int nblk,
                            const double* mu, double* sigma, cpx* lam, cpx* W) {
  const int st = small_la_phase_b1(tm, N, k, sketch_scale, ws, nblk, mu, sigma, lam);
  if (st != kOk) return st;
  if (!eigvecs_team(tm, ws.At, k, reinterpret_cast<const double*>(lam), W, ws.lz.fast, ws.lz.fast_doubles,
                    ws.flag))
    return kNumeric;
  small_la_phase_b3(tm, k, lam, W);
  return kOk;
}

// After phase A (Krylov size J, Ritz vectors Z of T_J in ws.Z): V = Q Z, TV = M12 V and
// the block partials, phase B, then G, over row blocks of kLaRows.
template <class TM>
TLA_HD int small_la_tail(TM& tm, const double* Gr, int m, int k, int J, double sketch_scale,
                         const SmallLAWork& ws, const double* mu, double* sigma, cpx* lam, cpx* W, cpx* G) {
  const int N = m - 1;
  const int nblk = (N + kLaRows - 1) / kLaRows;
  const int64_t ne = (int64_t)k * k + k;
  for (int b = 0; b < nblk; ++b) {
    const int t1 = (b + 1) * kLaRows < N ? (b + 1) * kLaRows : N;
    ritz_rows(tm, ws.Q, N, J, ws.Z, k, ws.V, b * kLaRows, t1);
  }
  for (int b = 0; b < nblk; ++b) {
    const int t1 = (b + 1) * kLaRows < N ? (b + 1) * kLaRows : N;
    m12v_rows(tm, Gr, m, N, k, ws.V, ws.TV, b * kLaRows, t1, ws.lz.fast, ws.lz.fast_doubles);
    block_gram(tm, ws.V, ws.TV, N, k, b * kLaRows, t1, ws.P + b * ne, ws.lz.fast, ws.lz.fast_doubles);
  }
  const int st = small_la_phase_b(tm, N, k, sketch_scale, ws, nblk, mu, sigma, lam, W);
  if (st != kOk) return st;
  g_rows(tm, ws.V, N, k, ws.nu, sigma, W, G, 0, N);
  tm.stamp(7);
  return kOk;
}

// Truncated SVD, A~, eig(A~) (Section 3.2) and G = V S^-1 W from the Gram Gr (m x m, symmetric) of the
// unscaled sketch, by one team: phase A (one row group), then the tail.  sketch_scale
// multiplies the sketch (so sigma = sqrt(mu) * scale).  Outputs: mu[k] (Gram eigenvalues),
// sigma[k], lam[k] and W (k x k, column j at j*k) as cpx, G (N x k, row t at t*k) as cpx.
// Returns the status; *Jout = Krylov size.  (The device runs the same steps as separate
// kernels, the row-range steps on many workgroups.)
template <class TM>
TLA_HD int small_la_run(TM& tm, const double* Gr, int m, int k, double rtol, int Jmax,
                        double sketch_scale, const SmallLAWork& ws, double* mu, double* sigma,
                        cpx* lam, cpx* W, cpx* G, int* Jout) {
  LocalX xg;
  xg.r1 = m - 1;
  const int st = small_la_phase_a(tm, xg, Gr, m, k, rtol, Jmax, ws, mu, ws.Z, Jout);
  if (st != kOk) return st;
  return small_la_tail(tm, Gr, m, k, *Jout, sketch_scale, ws, mu, sigma, lam, W, G);
}


}  // namespace tla
}  // namespace cdmd

namespace cdmd {
namespace tla {

// Offsets (in doubles) of the global scratch of one small-LA solve.
struct SmallLALayout {
  int64_t Q, T, V, Z, TV, P, nu, At, Hs, LU, bb, yy, piv, X, total;
};
TLA_HD inline SmallLALayout small_la_layout(int N, int k, int Jmax) {
  SmallLALayout L;
  int64_t o = 0;
  L.Q = o;  o += (int64_t)(Jmax + 1) * la_ldq(N);
  L.T = o;  o += (int64_t)Jmax + k + 6 * (int64_t)Jmax * k;
  L.V = o;  o += (int64_t)N * k;
  L.Z = o;  o += (int64_t)Jmax * k;
  L.TV = o; o += (int64_t)N * k;
  L.P = o;  o += (int64_t)((N + kLaRows - 1) / kLaRows) * ((int64_t)k * k + k);
  L.nu = o; o += 2 * (int64_t)k;
  L.At = o; o += (int64_t)k * k;
  L.Hs = o; o += (int64_t)k * k;
  L.LU = o; o += 2 * (int64_t)k * k * k;
  L.bb = o; o += 2 * (int64_t)k * k;
  L.yy = o; o += 2 * (int64_t)k * k;
  L.piv = o; o += (int64_t)k * k;  // ints stored in double slots
  // exchange of the row groups, 128-byte aligned: an arrival counter (a line of its own),
  // then two buffers of kLaGroupsMax partial arrays (la_xps) and a vector (la_ldq)
  o = (o + 15) & ~(int64_t)15;
  L.X = o;  o += 16 + 2 * ((int64_t)kLaGroupsMax * la_xps(Jmax) + la_ldq(N));
  L.total = o;
  return L;
}

// Offsets (in doubles) of the small-LA output block: status, J, mu[k], sigma[k],
// lam[2k], W[2k*k], G[2Nk].
struct SmallLAOutLayout {
  int64_t status, J, mu, sigma, lam, W, G, timing, total;
};
TLA_HD inline SmallLAOutLayout small_la_out_layout(int N, int k) {
  SmallLAOutLayout L;
  L.status = 0;
  L.J = 1;
  L.mu = 2;
  L.sigma = L.mu + k;
  L.lam = L.sigma + k;
  L.W = L.lam + 2 * k;
  L.G = L.W + 2 * (int64_t)k * k;
  L.timing = L.G + 2 * (int64_t)N * k;  // 16 phase-clock slots (device)
  L.total = L.timing + 16;
  return L;
}

}  // namespace tla
}  // namespace cdmd
