// Small float64 linear algebra of the cDMD fit written once for a "team" of threads:
// the whole thread block on the GPU (one workgroup per fit), or a single thread on the
// host (where the same code is tested against LAPACK).  Covers Algorithm 1 steps 4, 6
// and 7 and the lift operator G = V S^-1 W:
//
//   * Lanczos with full (twice classical Gram-Schmidt) reorthogonalisation for the
//     top-k eigenpairs of the Gram Y^T Y (the right singular vectors of Y, step 4);
//   * cyclic Jacobi (parallel round-robin ordering) on the Lanczos tridiagonal matrix for
//     the Ritz pairs and their residuals;
//   * A~ = S^-1 V^T (Y^T Y') V S^-1 (step 6);
//   * eig(A~) (step 7): Householder reduction to Hessenberg form, Francis double-shift QR
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
  double wave_max(double v) { return v; }
  void wave_argmax(double&, int&) {}
  double sum(double v) { return v; }
  double maxv(double v) { return v; }
};

// --------------------------------------------------------------------------- Lanczos
struct LanczosWork {
  double* q;      // N        current vector (shared)
  double* w;      // N        (shared)
  double* h;      // Jmax+1   projections (shared)
  double* alpha;  // Jmax+1   (shared)
  double* beta;   // Jmax+1   (shared)
  double* T;      // Jmax*Jmax  Jacobi matrix (global scratch)
  double* Z;      // Jmax*Jmax  Jacobi eigenvectors (global scratch)
  double* scal;   // 8        shared scalars
  int* pairs;     // 2*(Jmax+2) round-robin pairing / ranking (shared)
  double* rot;    // Jmax+2   rotation (c, s) per pair (shared)
  double* fast;   // fast (LDS) region of fast_doubles doubles, or nullptr: used for the
  int64_t fast_doubles;  // Jacobi T and Z when 2 J^2 fits, and as later scratch
};

// Deterministic start vector.
TLA_HD inline double lanczos_start(int i, int salt) {
  return 1.0 + 0.25 * sin(0.7 * (i + 1) + 1.3 * salt);
}

// Symmetric eigenproblem of the J x J matrix A (row-major, overwritten by its diagonal
// form) by cyclic Jacobi with the round-robin parallel ordering: each step applies J/2
// rotations on disjoint index pairs, first to rows, then to columns, and to the
// eigenvector matrix Z (J x J, column j = eigenvector of A[j][j]).  Sweeps until the
// off-diagonal Frobenius norm is <= eps * ||A||_F.  Returns the number of sweeps, or
// -1 if 40 sweeps did not converge.
template <class TM>
TLA_HD int jacobi_sym(TM& tm, double* A, double* Z, int J, double* cs, int* pr) {
  for (int e = tm.tid; e < J * J; e += tm.nt) Z[e] = (e / J == e % J) ? 1.0 : 0.0;
  tm.sync();
  const int Je = J + (J & 1);  // even player count (a dummy when J is odd)
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tm.tid; e < J * J; e += tm.nt) {
      const double v = A[e] * A[e];
      tot += v;
      if (e / J != e % J) off += v;
    }
    off = tm.sum(off);
    tot = tm.sum(tot);
    if (off <= kEps * kEps * tot || J < 2) break;
    for (int step = 0; step < Je - 1; ++step) {
      // pairs of this step (round robin: player Je-1 fixed, others rotate)
      for (int s = tm.tid; s < Je / 2; s += tm.nt) {
        int a, b;
        if (s == 0) {
          a = Je - 1;
          b = step;
        } else {
          a = (step + s) % (Je - 1);
          b = (step - s + (Je - 1)) % (Je - 1);
        }
        if (a > b) {
          const int t = a;
          a = b;
          b = t;
        }
        pr[2 * s] = a;
        pr[2 * s + 1] = b;
      }
      tm.sync();
      // rotation parameters per pair
      for (int s = tm.tid; s < Je / 2; s += tm.nt) {
        const int a = pr[2 * s], b = pr[2 * s + 1];
        double c = 1.0, sn = 0.0;
        if (b < J) {
          const double apq = A[a * J + b];
          if (apq != 0.0) {
            const double app = A[a * J + a], aqq = A[b * J + b];
            const double theta = (aqq - app) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
          }
        }
        cs[2 * s] = c;
        cs[2 * s + 1] = sn;
      }
      tm.sync();
      // rows: A <- R^T A for each pair (rows a, b), R = [[c, s], [-s, c]]
      for (int e = tm.tid; e < (Je / 2) * J; e += tm.nt) {
        const int s = e / J, col = e % J;
        const int a = pr[2 * s], b = pr[2 * s + 1];
        if (b >= J) continue;
        const double c = cs[2 * s], sn = cs[2 * s + 1];
        const double xa = A[a * J + col], xb = A[b * J + col];
        A[a * J + col] = c * xa - sn * xb;
        A[b * J + col] = sn * xa + c * xb;
      }
      tm.sync();
      // columns: A <- A R, Z <- Z R
      for (int e = tm.tid; e < (Je / 2) * J; e += tm.nt) {
        const int s = e / J, row = e % J;
        const int a = pr[2 * s], b = pr[2 * s + 1];
        if (b >= J) continue;
        const double c = cs[2 * s], sn = cs[2 * s + 1];
        const double xa = A[row * J + a], xb = A[row * J + b];
        A[row * J + a] = c * xa - sn * xb;
        A[row * J + b] = sn * xa + c * xb;
        const double za = Z[row * J + a], zb = Z[row * J + b];
        Z[row * J + a] = c * za - sn * zb;
        Z[row * J + b] = sn * za + c * zb;
      }
      tm.sync();
    }
  }
  return sweep < 40 ? sweep : -1;
}

// Top-k eigenpairs of the symmetric N x N matrix M (element (r, c) at M[r*ldm + c]).
// Q: (Jmax+1) x N scratch (vector-contiguous).  On return evals[k] descending and
// V (N x k, column-major) the unit Ritz vectors; the return value is the Krylov
// dimension J, or -1 on failure.  Converged when every top-k Ritz residual
// beta_J |z_J| <= rtol * theta_1, or J = N.
template <class TM>
TLA_HD int lanczos_topk(TM& tm, const double* M, int ldm, int N, int k, double rtol, int Jmax,
                        double* Q, const LanczosWork& ws, double* evals, double* V) {
  if (Jmax > N) Jmax = N;
  double* q = ws.q;
  double* w = ws.w;
  double* h = ws.h;
  // q_0
  {
    double s = 0.0;
    for (int i = tm.tid; i < N; i += tm.nt) {
      const double v = lanczos_start(i, 0);
      s += v * v;
    }
    s = tm.sum(s);
    const double inv = 1.0 / sqrt(s);
    for (int i = tm.tid; i < N; i += tm.nt) {
      q[i] = lanczos_start(i, 0) * inv;
      Q[i] = q[i];
    }
    tm.sync();
  }
  int J = 0;
  int check = 2 * k > k + 16 ? 2 * k : k + 16;
  if (check > Jmax) check = Jmax;
  double anorm = 0.0;
  int restarts = 0;
  for (int j = 0; j < Jmax; ++j) {
    // w = M q: a wave per group of 4 rows, lanes over columns (coalesced, independent)
    for (int r0 = 4 * tm.wave; r0 < N; r0 += 4 * tm.nwaves) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      const double* m0 = M + (int64_t)r0 * ldm;
      const bool h1 = r0 + 1 < N, h2 = r0 + 2 < N, h3 = r0 + 3 < N;
      for (int c = tm.lane; c < N; c += tm.wsize) {
        const double qc = q[c];
        s0 += m0[c] * qc;
        if (h1) s1 += m0[ldm + c] * qc;
        if (h2) s2 += m0[2 * (int64_t)ldm + c] * qc;
        if (h3) s3 += m0[3 * (int64_t)ldm + c] * qc;
      }
      s0 = tm.wave_sum(s0);
      s1 = tm.wave_sum(s1);
      s2 = tm.wave_sum(s2);
      s3 = tm.wave_sum(s3);
      if (tm.lane == 0) {
        w[r0] = s0;
        if (h1) w[r0 + 1] = s1;
        if (h2) w[r0 + 2] = s2;
        if (h3) w[r0 + 3] = s3;
      }
    }
    tm.sync();
    double aj = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = tm.wave; i <= j; i += tm.nwaves) {
        const double* qi = Q + (int64_t)i * N;
        double s = 0.0;
        for (int t = tm.lane; t < N; t += tm.wsize) s += qi[t] * w[t];
        s = tm.wave_sum(s);
        if (tm.lane == 0) h[i] = s;
      }
      tm.sync();
      aj += h[j];
      for (int t = tm.tid; t < N; t += tm.nt) {
        double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
        int i = 0;
        for (; i + 4 <= j + 1; i += 4) {
          v0 += h[i] * Q[(int64_t)i * N + t];
          v1 += h[i + 1] * Q[(int64_t)(i + 1) * N + t];
          v2 += h[i + 2] * Q[(int64_t)(i + 2) * N + t];
          v3 += h[i + 3] * Q[(int64_t)(i + 3) * N + t];
        }
        for (; i <= j; ++i) v0 += h[i] * Q[(int64_t)i * N + t];
        w[t] -= (v0 + v1) + (v2 + v3);
      }
      tm.sync();
    }
    double nr = 0.0;
    for (int t = tm.tid; t < N; t += tm.nt) nr += w[t] * w[t];
    nr = sqrt(tm.sum(nr));
    ws.alpha[j] = aj;  // identical value on every thread
    ws.beta[j] = nr;
    J = j + 1;
    {
      const double an = fabs(aj) + nr + (j ? ws.beta[j - 1] : 0.0);
      if (an > anorm) anorm = an;
    }
    const bool breakdown = nr <= 64.0 * kEps * anorm;
    if (J >= check || breakdown || J == N) {
      // Ritz pairs of T_J by Jacobi; residual of Ritz pair i is beta_J |Z[J-1][i]|
      const bool fastTZ = ws.fast != nullptr && 2 * (int64_t)J * J <= ws.fast_doubles;
      double* Tm = fastTZ ? ws.fast : ws.T;
      double* Zm = fastTZ ? ws.fast + (int64_t)J * J : ws.Z;
      for (int e = tm.tid; e < J * J; e += tm.nt) {
        const int r = e / J, c = e % J;
        double v = 0.0;
        if (r == c) v = ws.alpha[r];
        else if (c == r + 1) v = ws.beta[r];
        else if (r == c + 1) v = ws.beta[c];
        Tm[e] = v;
      }
      tm.sync();
      tm.stamp(0);
      if (jacobi_sym(tm, Tm, Zm, J, ws.rot, ws.pairs) < 0) return -1;
      tm.stamp(1);
      // order of the top-k (descending): selection by repeated max, computed redundantly
      bool conv = J >= k;
      double th1 = 0.0;
      {
        // rank of each diagonal entry; stored as pairs[] = index of i-th largest
        for (int i = tm.tid; i < J; i += tm.nt) {
          const double di = Tm[i * J + i];
          int rank = 0;
          for (int c = 0; c < J; ++c) {
            const double dc = Tm[c * J + c];
            if (dc > di || (dc == di && c < i)) ++rank;
          }
          ws.pairs[rank] = i;
        }
        tm.sync();
        th1 = Tm[ws.pairs[0] * J + ws.pairs[0]];
        const double scale = fabs(th1) > 0 ? fabs(th1) : 1e-300;
        if (conv)
          for (int i = 0; i < k; ++i) {
            const int col = ws.pairs[i];
            if (nr * fabs(Zm[(J - 1) * J + col]) > rtol * scale) conv = false;
          }
      }
      if (conv || J == N || J == Jmax) {
        if (J < k) return -1;
        for (int i = tm.tid; i < k; i += tm.nt) {
          const int col = ws.pairs[i];
          evals[i] = Tm[col * J + col];
        }
        // V = Q_J Z_k
        for (int e = tm.tid; e < N * k; e += tm.nt) {
          const int c = e / N, t = e % N;
          const int col = ws.pairs[c];
          double s0 = 0.0, s1 = 0.0;
          int i = 0;
          for (; i + 2 <= J; i += 2) {
            s0 += Q[(int64_t)i * N + t] * Zm[i * J + col];
            s1 += Q[(int64_t)(i + 1) * N + t] * Zm[(i + 1) * J + col];
          }
          if (i < J) s0 += Q[(int64_t)i * N + t] * Zm[i * J + col];
          V[(int64_t)c * N + t] = s0 + s1;
        }
        tm.sync();
        // renormalise columns
        for (int c = 0; c < k; ++c) {
          double s = 0.0;
          for (int t = tm.tid; t < N; t += tm.nt) s += V[(int64_t)c * N + t] * V[(int64_t)c * N + t];
          s = tm.sum(s);
          const double inv = 1.0 / sqrt(s);
          for (int t = tm.tid; t < N; t += tm.nt) V[(int64_t)c * N + t] *= inv;
          tm.sync();
        }
        return conv || J == N ? J : -1;
      }
      check = J + (J / 4 > 16 ? J / 4 : 16);
      if (check > Jmax) check = Jmax;
      if (breakdown) {
        // invariant subspace found before k pairs converged: restart orthogonally
        if (++restarts > 8) return -1;
        for (int t = tm.tid; t < N; t += tm.nt) w[t] = lanczos_start(t, J + 17 * restarts);
        tm.sync();
        for (int pass = 0; pass < 2; ++pass) {
          for (int i = tm.wave; i < J; i += tm.nwaves) {
            const double* qi = Q + (int64_t)i * N;
            double s = 0.0;
            for (int t = tm.lane; t < N; t += tm.wsize) s += qi[t] * w[t];
            s = tm.wave_sum(s);
            if (tm.lane == 0) h[i] = s;
          }
          tm.sync();
          for (int t = tm.tid; t < N; t += tm.nt) {
            double v = w[t];
            for (int i = 0; i < J; ++i) v -= h[i] * Q[(int64_t)i * N + t];
            w[t] = v;
          }
          tm.sync();
        }
        double n2 = 0.0;
        for (int t = tm.tid; t < N; t += tm.nt) n2 += w[t] * w[t];
        n2 = sqrt(tm.sum(n2));
        if (n2 <= 1e-8) return -1;
        ws.beta[j] = 0.0;
        nr = n2;
      }
    }
    const double inv = 1.0 / nr;
    for (int t = tm.tid; t < N; t += tm.nt) {
      const double v = w[t] * inv;
      q[t] = v;
      Q[(int64_t)J * N + t] = v;
    }
    tm.sync();
  }
  return -1;
}

// --------------------------------------------------------------------------- A~
// At = S^-1 V^T M12 V S^-1 with M12[a][b] = Mfull[a*ldm + b + 1] (a, b < N), s = sqrt(mu).
// TV: N x k scratch (column-major).
template <class TM>
TLA_HD void reduced_operator(TM& tm, const double* Mfull, int ldm, int N, int k, const double* V,
                             const double* s, double* TV, double* At, double* stage,
                             int64_t stage_doubles) {
  // TV = M12 V, element (a, c) = sum_b M12[a][b] V[b][c].  The Gram is symmetric, so
  // M12[a][b] = Mfull[(b+1)*ldm + a]: one thread per row a reads coalesced columns; the
  // rows b of V pass through `stage` (fast memory) in chunks, k accumulators per thread.
  constexpr int KM = 40;
  int chunk = (int)(stage_doubles / (k > 0 ? k : 1));
  if (chunk > 256) chunk = 256;
  for (int a0 = 0; a0 < N; a0 += tm.nt) {
    const int a = a0 + tm.tid;
    double acc[KM];
#pragma unroll
    for (int c = 0; c < KM; ++c) acc[c] = 0.0;
    for (int b0 = 0; b0 < N; b0 += chunk) {
      const int nb = N - b0 < chunk ? N - b0 : chunk;
      tm.sync();
      for (int e = tm.tid; e < nb * k; e += tm.nt) {
        const int bb = e / k, c = e % k;
        stage[e] = V[(int64_t)c * N + b0 + bb];
      }
      tm.sync();
      if (a < N)
        for (int bb = 0; bb < nb; ++bb) {
          const double mv = Mfull[(int64_t)(b0 + bb + 1) * ldm + a];
          const double* sv = stage + bb * k;
#pragma unroll
          for (int c = 0; c < KM; ++c)
            if (c < k) acc[c] += mv * sv[c];
        }
    }
    if (a < N)
#pragma unroll
      for (int c = 0; c < KM; ++c)
        if (c < k) TV[(int64_t)c * N + a] = acc[c];
  }
  tm.sync();
  for (int e = tm.tid; e < k * k; e += tm.nt) {
    const int i = e / k, j = e % k;
    const double* vi = V + (int64_t)i * N;
    const double* tj = TV + (int64_t)j * N;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int a = 0;
    for (; a + 4 <= N; a += 4) {
      a0 += vi[a] * tj[a];
      a1 += vi[a + 1] * tj[a + 1];
      a2 += vi[a + 2] * tj[a + 2];
      a3 += vi[a + 3] * tj[a + 3];
    }
    for (; a < N; ++a) a0 += vi[a] * tj[a];
    At[i * k + j] = ((a0 + a1) + (a2 + a3)) / (s[i] * s[j]);
  }
  tm.sync();
}

// --------------------------------------------------------------------------- eig(A~)
// Work: H (k*k), v (4), ev (2k doubles: re, im), status (int shared via scal[0]).
template <class TM>
TLA_HD void hess_reflect(TM& tm, double* H, int k, int r0, int len, const double* v, double vv,
                         int c0, int c1, int rr0, int rr1) {
  // left: rows r0..r0+len-1, columns c0..c1
  for (int c = c0 + tm.tid; c <= c1; c += tm.nt) {
    double t = 0.0;
    for (int i = 0; i < len; ++i) t += v[i] * H[(r0 + i) * k + c];
    const double f = 2.0 * t / vv;
    for (int i = 0; i < len; ++i) H[(r0 + i) * k + c] -= f * v[i];
  }
  tm.sync();
  // right: columns r0..r0+len-1, rows rr0..rr1
  for (int r = rr0 + tm.tid; r <= rr1; r += tm.nt) {
    double t = 0.0;
    for (int i = 0; i < len; ++i) t += H[r * k + r0 + i] * v[i];
    const double f = 2.0 * t / vv;
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
    double alpha = 0.0;
    for (int i = j + 1; i < k; ++i) alpha += H[i * k + j] * H[i * k + j];
    alpha = sqrt(alpha);
    if (alpha == 0.0) continue;
    // reflector on rows/cols j+1..k-1; long vector kept in H's column below the diagonal
    // is not reused, so compute the update directly
    const double x0 = H[(j + 1) * k + j];
    const double sg = x0 >= 0 ? 1.0 : -1.0;
    const double v0 = x0 + sg * alpha;
    double vv = v0 * v0;
    for (int i = j + 2; i < k; ++i) vv += H[i * k + j] * H[i * k + j];
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
  for (int e = 0; e < k * k; ++e) hnorm = fmax(hnorm, fabs(H[e]));
  int hi = k - 1, its = 0, total = 0, nev = 0;
  while (hi >= 0) {
    int l = hi;
    while (l > 0) {
      double s = fabs(H[(l - 1) * k + l - 1]) + fabs(H[l * k + l]);
      if (s == 0.0) s = hnorm;
      if (fabs(H[l * k + l - 1]) <= kEps * s) break;
      --l;
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
        hess_reflect(tm, H, k, kk, 3, v, vv, c0, hi, l, rr1);
        if (kk > l && tm.tid == 0) {
          H[(kk + 1) * k + kk - 1] = 0.0;
          H[(kk + 2) * k + kk - 1] = 0.0;
        }
        tm.sync();
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
        hess_reflect(tm, H, k, kk, 2, v, vv, c0, hi, l, hi);
        if (kk > l && tm.tid == 0) H[(kk + 1) * k + kk - 1] = 0.0;
        tm.sync();
      }
    }
  }
  return nev == k;
}

// Eigenvector of A for eigenvalue lam by three steps of inverse iteration with a
// complex LU (partial pivoting) of A - lam I, done by one thread.  LU: k*k cpx scratch,
// b, y: k cpx scratch.  Unit 2-norm result in w.
TLA_HD inline bool inverse_iteration(const double* A, int k, cpx lam, cpx* LU, cpx* b, cpx* y,
                                     int* piv, cpx* w) {
  double amax = 0.0;
  for (int r = 0; r < k; ++r)
    for (int c = 0; c < k; ++c) {
      LU[r * k + c] = cmk(A[r * k + c] - (r == c ? lam.re : 0.0), r == c ? -lam.im : 0.0);
      amax = fmax(amax, cabsv(LU[r * k + c]));
    }
  const double tiny = (amax > 1e-300 ? amax : 1e-300) * kEps;
  for (int j = 0; j < k; ++j) {
    int p = j;
    double best = cabsv(LU[j * k + j]);
    for (int i = j + 1; i < k; ++i) {
      const double a = cabsv(LU[i * k + j]);
      if (a > best) best = a, p = i;
    }
    piv[j] = p;
    if (p != j)
      for (int c = 0; c < k; ++c) {
        const cpx t = LU[j * k + c];
        LU[j * k + c] = LU[p * k + c];
        LU[p * k + c] = t;
      }
    if (cabsv(LU[j * k + j]) < tiny) LU[j * k + j] = cmk(tiny, 0.0);
    for (int i = j + 1; i < k; ++i) {
      const cpx f = cdiv(LU[i * k + j], LU[j * k + j]);
      LU[i * k + j] = f;
      for (int c = j + 1; c < k; ++c) LU[i * k + c] = csub(LU[i * k + c], cmul(f, LU[j * k + c]));
    }
  }
  for (int i = 0; i < k; ++i) b[i] = cmk(1.0, 0.0);
  for (int it = 0; it < 3; ++it) {
    for (int j = 0; j < k; ++j)
      if (piv[j] != j) {
        const cpx t = b[j];
        b[j] = b[piv[j]];
        b[piv[j]] = t;
      }
    for (int i = 0; i < k; ++i) {
      cpx s = b[i];
      for (int c = 0; c < i; ++c) s = csub(s, cmul(LU[i * k + c], y[c]));
      y[i] = s;
    }
    for (int i = k - 1; i >= 0; --i) {
      cpx s = y[i];
      for (int c = i + 1; c < k; ++c) s = csub(s, cmul(LU[i * k + c], y[c]));
      y[i] = cdiv(s, LU[i * k + i]);
    }
    double nr = 0.0;
    for (int i = 0; i < k; ++i) nr += cabs2(y[i]);
    nr = sqrt(nr);
    if (!(nr > 0.0) || !(nr < 1e300)) return false;
    for (int i = 0; i < k; ++i) b[i] = cscale(y[i], 1.0 / nr);
  }
  for (int i = 0; i < k; ++i) w[i] = b[i];
  return true;
}


// Eigenvectors of the real k x k matrix A for the eigenvalues ev (re, im pairs) by three
// steps of inverse iteration each, one wave per eigenvalue: the complex LU with partial
// pivoting of A - lambda I and the triangular solves are split over the wave's lanes,
// in `region` (fast memory; each active wave needs 2k^2 + 5k doubles; waves take
// eigenvalues in rounds).  The second member of a conjugate pair is skipped (the caller
// conjugates its partner).  W: column j at j*k.  Returns false on failure.
template <class TM>
TLA_HD bool eigvecs_team(TM& tm, const double* A, int k, const double* ev, cpx* W, double* region,
                         int64_t region_doubles, int* flag) {
  const int64_t per = 2 * (int64_t)k * k + 5 * (int64_t)k;
  int wl = (int)(region_doubles / per);
  if (wl > tm.nwaves) wl = tm.nwaves;
  if (wl < 1) return false;
  if (tm.tid == 0) flag[0] = 0;
  tm.sync();
  const int L = tm.lane, WS = tm.wsize;
  for (int base = 0; base < k; base += wl) {
    const int j = base + tm.wave;
    bool active = tm.wave < wl && j < k;
    if (active && ev[2 * j + 1] < 0.0 && j > 0 && ev[2 * j - 2] == ev[2 * j] &&
        ev[2 * j - 1] == -ev[2 * j + 1])
      active = false;
    const int wv = tm.wave < wl ? tm.wave : 0;
    cpx* LU = reinterpret_cast<cpx*>(region + wv * per);
    cpx* b = LU + (int64_t)k * k;
    cpx* y = b + k;
    int* piv = reinterpret_cast<int*>(y + k);
    const double lre = active ? ev[2 * j] : 0.0, lim = active ? ev[2 * j + 1] : 0.0;
    double amax = 0.0;
    if (active)
      for (int e = L; e < k * k; e += WS) {
        const int r = e / k, c = e % k;
        LU[e] = cmk(A[e] - (r == c ? lre : 0.0), r == c ? -lim : 0.0);
        amax = fmax(amax, cabsv(LU[e]));
      }
    amax = tm.wave_max(amax);
    tm.sync();
    const double tiny = (amax > 1e-300 ? amax : 1e-300) * kEps;
    for (int jj = 0; jj < k; ++jj) {
      double best = -1.0;
      int bi = jj;
      if (active)
        for (int i = jj + L; i < k; i += WS) {
          const double a = cabsv(LU[i * k + jj]);
          if (a > best) best = a, bi = i;
        }
      tm.wave_argmax(best, bi);
      if (active && L == 0) piv[jj] = bi;
      if (active && bi != jj)
        for (int c = L; c < k; c += WS) {
          const cpx t = LU[jj * k + c];
          LU[jj * k + c] = LU[bi * k + c];
          LU[bi * k + c] = t;
        }
      tm.sync();
      if (active && L == 0 && cabsv(LU[jj * k + jj]) < tiny) LU[jj * k + jj] = cmk(tiny, 0.0);
      tm.sync();
      if (active) {
        const cpx pv = LU[jj * k + jj];
        for (int i = jj + 1 + L; i < k; i += WS) {
          const cpx f = cdiv(LU[i * k + jj], pv);
          LU[i * k + jj] = f;
          for (int c = jj + 1; c < k; ++c) LU[i * k + c] = csub(LU[i * k + c], cmul(f, LU[jj * k + c]));
        }
      }
      tm.sync();
    }
    if (active)
      for (int i = L; i < k; i += WS) b[i] = cmk(1.0, 0.0);
    tm.sync();
    for (int it = 0; it < 3; ++it) {
      if (active && L == 0)
        for (int jj = 0; jj < k; ++jj)
          if (piv[jj] != jj) {
            const cpx t = b[jj];
            b[jj] = b[piv[jj]];
            b[piv[jj]] = t;
          }
      tm.sync();
      for (int i = 0; i < k; ++i) {
        double sr = 0.0, si = 0.0;
        if (active)
          for (int c = L; c < i; c += WS) {
            const cpx pr = cmul(LU[i * k + c], y[c]);
            sr += pr.re;
            si += pr.im;
          }
        sr = tm.wave_sum(sr);
        si = tm.wave_sum(si);
        if (active && L == 0) y[i] = csub(b[i], cmk(sr, si));
        tm.sync();
      }
      for (int i = k - 1; i >= 0; --i) {
        double sr = 0.0, si = 0.0;
        if (active)
          for (int c = i + 1 + L; c < k; c += WS) {
            const cpx pr = cmul(LU[i * k + c], y[c]);
            sr += pr.re;
            si += pr.im;
          }
        sr = tm.wave_sum(sr);
        si = tm.wave_sum(si);
        if (active && L == 0) y[i] = cdiv(csub(y[i], cmk(sr, si)), LU[i * k + i]);
        tm.sync();
      }
      double nr = 0.0;
      if (active)
        for (int i = L; i < k; i += WS) nr += cabs2(y[i]);
      nr = sqrt(tm.wave_sum(nr));
      if (active && !(nr > 0.0 && nr < 1e300) && L == 0) flag[0] = 1;
      if (active && nr > 0.0)
        for (int i = L; i < k; i += WS) b[i] = cscale(y[i], 1.0 / nr);
      tm.sync();
    }
    if (active)
      for (int i = L; i < k; i += WS) W[(int64_t)j * k + i] = b[i];
    tm.sync();
  }
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
  double* TV;   // N x k
  double* At;   // k x k
  double* Hs;   // k x k
  cpx* LU;      // k x k x k
  cpx* bb;      // k x k
  cpx* yy;      // k x k
  int* piv;     // k x k
  int* flag;    // 1 (shared)
};

// Status codes (match cdmd_status).
constexpr int kOk = 0, kRankDeficient = 5, kNumeric = 6;

// Algorithm 1 steps 4, 6, 7 and G = V S^-1 W from the Gram Gr (m x m, symmetric) of the
// unscaled sketch.  sketch_scale multiplies the sketch (so sigma = sqrt(mu) * scale).
// Outputs: mu[k] (Gram eigenvalues), sigma[k], lam[k] and W (k x k, column j at j*k)
// as cpx, G (N x k, row t at t*k) as cpx.  Returns the status; *Jout = Krylov size.
template <class TM>
TLA_HD int small_la_run(TM& tm, const double* Gr, int m, int k, double rtol, int Jmax,
                        double sketch_scale, const SmallLAWork& ws, double* mu, double* sigma,
                        cpx* lam, cpx* W, cpx* G, int* Jout) {
  const int N = m - 1;
  // non-finite input
  {
    double bad = 0.0;
    for (int64_t e = tm.tid; e < (int64_t)m * m; e += tm.nt)
      if (!(fabs(Gr[e]) < 1e300)) bad = 1.0;
    if (tm.sum(bad) > 0.0) return kNumeric;
  }
  tm.stamp(2);
  const int J = lanczos_topk(tm, Gr, m, N, k, rtol, Jmax, ws.Q, ws.lz, mu, ws.V);
  tm.stamp(3);
  *Jout = J;
  if (J < 0) return kNumeric;
  if (!(mu[0] > 0.0) || !(mu[k - 1] > 1e-12 * mu[0])) return kRankDeficient;
  double* s = ws.lz.h;  // reuse: sqrt(mu)
  for (int i = tm.tid; i < k; i += tm.nt) s[i] = sqrt(mu[i]);
  tm.sync();
  for (int i = tm.tid; i < k; i += tm.nt) sigma[i] = s[i] * sketch_scale;
  double* fastr = ws.lz.fast;
  const int64_t fastd = ws.lz.fast_doubles;
  reduced_operator(tm, Gr, m, N, k, ws.V, s, ws.TV, ws.At, fastr, fastd);
  tm.stamp(4);
  double* ev = ws.lz.w;  // reuse: 2k doubles
  if (!eigvals_general(tm, ws.At, k, (int64_t)k * k <= fastd ? fastr : ws.Hs, ev)) return kNumeric;
  tm.stamp(5);
  tm.sync();
  for (int j = tm.tid; j < k; j += tm.nt) lam[j] = cmk(ev[2 * j], ev[2 * j + 1]);
  if (!eigvecs_team(tm, ws.At, k, ev, W, fastr, fastd, ws.flag)) return kNumeric;
  for (int j = tm.tid; j < k; j += tm.nt) {
    const bool second = ev[2 * j + 1] < 0.0 && j > 0 && ev[2 * j - 2] == ev[2 * j] &&
                        ev[2 * j - 1] == -ev[2 * j + 1];
    if (second)
      for (int i = 0; i < k; ++i) W[(int64_t)j * k + i] = cconj(W[(int64_t)(j - 1) * k + i]);
  }
  tm.sync();
  for (int j = tm.tid; j < k; j += tm.nt) normalise_vec(W + (int64_t)j * k, k);
  tm.sync();
  tm.stamp(6);
  // G = V diag(1/sigma) W
  for (int64_t e = tm.tid; e < (int64_t)N * k; e += tm.nt) {
    const int t = (int)(e / k), j = (int)(e % k);
    double re = 0.0, im = 0.0;
    for (int i = 0; i < k; ++i) {
      const double v = ws.V[(int64_t)i * N + t] / sigma[i];
      const cpx wv = W[(int64_t)j * k + i];
      re += v * wv.re;
      im += v * wv.im;
    }
    G[e] = cmk(re, im);
  }
  tm.sync();
  tm.stamp(7);
  return kOk;
}

}  // namespace tla
}  // namespace cdmd

namespace cdmd {
namespace tla {

// Offsets (in doubles) of the global scratch of one small-LA solve.
struct SmallLALayout {
  int64_t Q, T, Z, V, TV, At, Hs, LU, bb, yy, piv, total;
};
TLA_HD inline SmallLALayout small_la_layout(int N, int k, int Jmax) {
  SmallLALayout L;
  int64_t o = 0;
  L.Q = o;  o += (int64_t)(Jmax + 1) * N;
  L.T = o;  o += (int64_t)Jmax * Jmax;
  L.Z = o;  o += (int64_t)Jmax * Jmax;
  L.V = o;  o += (int64_t)N * k;
  L.TV = o; o += (int64_t)N * k;
  L.At = o; o += (int64_t)k * k;
  L.Hs = o; o += (int64_t)k * k;
  L.LU = o; o += 2 * (int64_t)k * k * k;
  L.bb = o; o += 2 * (int64_t)k * k;
  L.yy = o; o += 2 * (int64_t)k * k;
  L.piv = o; o += (int64_t)k * k;  // ints stored in double slots
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
