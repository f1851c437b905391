// Small dense float64 linear algebra of the cDMD fit (host side).  See smallla.hpp.
#include "smallla.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <numeric>

namespace cdmd {
namespace la {

static inline double sgn1(double x) { return x >= 0.0 ? 1.0 : -1.0; }

static inline double dot(const double* a, const double* b, int n) {
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int i = 0;
  for (; i + 4 <= n; i += 4) {
    s0 += a[i] * b[i];
    s1 += a[i + 1] * b[i + 1];
    s2 += a[i + 2] * b[i + 2];
    s3 += a[i + 3] * b[i + 3];
  }
  for (; i < n; ++i) s0 += a[i] * b[i];
  return (s0 + s1) + (s2 + s3);
}

// ---------------------------------------------------------------------------
// Symmetric tridiagonal eigenproblem: implicit QR sweeps, Wilkinson shift.
// A rotation acting on indices (k, k+1) is R = [[c, s], [-s, c]]; the similarity
// T <- R^T T R is applied to the 2x2 block, the coupling to k-1 (where it annihilates
// the bulge) and to k+2 (where it creates the next bulge); Z <- Z R.
bool tridiag_eig(double* d, double* e, int n, double* Z, int R, int row0) {
  if (n <= 0) return true;
  for (int r = 0; r < R; ++r)
    for (int j = 0; j < n; ++j) Z[(size_t)r * n + j] = (row0 + r == j) ? 1.0 : 0.0;
  const double eps = DBL_EPSILON;
  int hi = n - 1;
  long iter = 0;
  const long maxit = 64L * n + 64;
  while (hi > 0) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    if (lo > 0) e[lo - 1] = 0.0;
    if (++iter > maxit) return false;
    const double a = d[hi - 1], b = d[hi], ee = e[hi - 1];
    const double delta = 0.5 * (a - b);
    const double den = delta + sgn1(delta) * std::hypot(delta, ee);
    const double mu = b - ee * (ee / den);
    double bulge = 0.0;
    for (int k = lo; k < hi; ++k) {
      const double u = (k == lo) ? d[lo] - mu : e[k - 1];
      const double v = (k == lo) ? e[lo] : bulge;
      const double r = std::hypot(u, v);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = u / r;
        s = -v / r;
      }
      if (k > lo) e[k - 1] = r;
      const double a0 = d[k], b0 = d[k + 1], e0 = e[k];
      const double cc = c * c, ss = s * s, cs = c * s;
      d[k] = cc * a0 - 2.0 * cs * e0 + ss * b0;
      d[k + 1] = ss * a0 + 2.0 * cs * e0 + cc * b0;
      e[k] = cs * (a0 - b0) + (cc - ss) * e0;
      if (k + 1 < hi) {
        const double f = e[k + 1];
        bulge = -s * f;
        e[k + 1] = c * f;
      }
      for (int rr = 0; rr < R; ++rr) {
        double* zr = Z + (size_t)rr * n;
        const double zk = zr[k], zk1 = zr[k + 1];
        zr[k] = c * zk - s * zk1;
        zr[k + 1] = s * zk + c * zk1;
      }
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// Lanczos with full reorthogonalisation for the top-k eigenpairs.
// Conjugate-linear and plain inner products; for double both are `dot`.
static inline double dotc(const double* a, const double* b, int n) { return dot(a, b, n); }
static inline double dotu(const double* a, const double* b, int n) { return dot(a, b, n); }
static inline cplx dotc(const cplx* a, const cplx* b, int n) {
  cplx s0 = 0.0, s1 = 0.0;
  int i = 0;
  for (; i + 2 <= n; i += 2) {
    s0 += std::conj(a[i]) * b[i];
    s1 += std::conj(a[i + 1]) * b[i + 1];
  }
  for (; i < n; ++i) s0 += std::conj(a[i]) * b[i];
  return s0 + s1;
}
static inline cplx dotu(const cplx* a, const cplx* b, int n) {
  cplx s0 = 0.0, s1 = 0.0;
  int i = 0;
  for (; i + 2 <= n; i += 2) {
    s0 += a[i] * b[i];
    s1 += a[i + 1] * b[i + 1];
  }
  for (; i < n; ++i) s0 += a[i] * b[i];
  return s0 + s1;
}
static inline double re(double x) { return x; }
static inline double re(cplx z) { return z.real(); }

// Lanczos with full reorthogonalisation for a real symmetric (T = double) or complex
// Hermitian (T = cplx) matrix: alpha_j = q_j^H M q_j is real and beta_j = |w| >= 0, so the
// projected matrix is the same real symmetric tridiagonal in both cases.
template <typename T>
static int topk_lanczos(const T* M, int n, int k, double rtol, double* evals, T* evecs) {
  if (k < 1 || k > n || n < 1) return -1;
  std::vector<T> Q((size_t)n * (n + 1), T(0.0));
  std::vector<double> alpha(n + 1, 0.0), beta(n + 1, 0.0);
  std::vector<T> w(n), h(n + 1);
  auto newvec = [&](T* q, int salt) {
    for (int i = 0; i < n; ++i) q[i] = T(1.0 + 0.25 * std::sin(0.7 * (i + 1) + 1.3 * salt));
  };
  auto orth = [&](T* v, int J) -> double {  // twice CGS against Q[0..J)
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < J; ++i) h[i] = dotc(&Q[(size_t)i * n], v, n);
      for (int i = 0; i < J; ++i) {
        const T* qi = &Q[(size_t)i * n];
        const T hi = h[i];
        for (int t = 0; t < n; ++t) v[t] -= hi * qi[t];
      }
    }
    return std::sqrt(re(dotc(v, v, n)));
  };
  {
    T* q0 = Q.data();
    newvec(q0, 0);
    const double nr = std::sqrt(re(dotc(q0, q0, n)));
    for (int i = 0; i < n; ++i) q0[i] /= nr;
  }
  double anorm = 0.0;
  int J = 0;
  int next_check = std::min(n, std::max(2 * k, k + 16));
  std::vector<double> dd, ee, zl;
  std::vector<int> idx;
  int restarts = 0;
  for (int j = 0; j < n; ++j) {
    const T* qj = &Q[(size_t)j * n];
    for (int i = 0; i < n; ++i) w[i] = dotu(M + (size_t)i * n, qj, n);
    // projections on all previous vectors, twice; alpha_j is the q_j component
    double aj = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i <= j; ++i) h[i] = dotc(&Q[(size_t)i * n], w.data(), n);
      aj += re(h[j]);
      for (int i = 0; i <= j; ++i) {
        const T* qi = &Q[(size_t)i * n];
        const T hi = h[i];
        for (int t = 0; t < n; ++t) w[t] -= hi * qi[t];
      }
    }
    alpha[j] = aj;
    beta[j] = std::sqrt(re(dotc(w.data(), w.data(), n)));
    J = j + 1;
    anorm = std::max(anorm, std::fabs(alpha[j]) + beta[j] + (j ? beta[j - 1] : 0.0));
    const bool breakdown = beta[j] <= 64.0 * DBL_EPSILON * anorm;
    if (J == next_check || breakdown || J == n) {
      dd.assign(alpha.begin(), alpha.begin() + J);
      ee.assign(beta.begin(), beta.begin() + J);
      zl.assign(J, 0.0);
      if (!tridiag_eig(dd.data(), ee.data(), J, zl.data(), 1, J - 1)) return -1;
      idx.resize(J);
      std::iota(idx.begin(), idx.end(), 0);
      std::sort(idx.begin(), idx.end(), [&](int a, int b) { return dd[a] > dd[b]; });
      bool conv = J >= k;
      if (conv) {
        const double scale = std::max(std::fabs(dd[idx[0]]), DBL_MIN);
        for (int i = 0; i < k; ++i)
          if (beta[j] * std::fabs(zl[idx[i]]) > rtol * scale) conv = false;
      }
      if (conv || J == n) break;
      if (breakdown) {
        // invariant subspace smaller than k: continue from a fresh orthogonal vector
        if (++restarts > 8) return -1;
        T* qn = &Q[(size_t)J * n];
        newvec(qn, J + 17 * restarts);
        const double nr = orth(qn, J);
        if (nr <= 1e-8) return -1;
        for (int i = 0; i < n; ++i) qn[i] /= nr;
        beta[j] = 0.0;
        next_check = std::min(n, J + std::max(16, J / 4));
        continue;
      }
      next_check = std::min(n, J + std::max(16, J / 4));
    }
    T* qn = &Q[(size_t)J * n];
    const double inv = 1.0 / beta[j];
    for (int i = 0; i < n; ++i) qn[i] = w[i] * inv;
  }
  // full eigenvectors of T_J
  dd.assign(alpha.begin(), alpha.begin() + J);
  ee.assign(beta.begin(), beta.begin() + J);
  std::vector<double> Z((size_t)J * J);
  if (!tridiag_eig(dd.data(), ee.data(), J, Z.data(), J, 0)) return -1;
  idx.resize(J);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return dd[a] > dd[b]; });
  if (J < k) return -1;
  for (int c = 0; c < k; ++c) {
    const int col = idx[c];
    evals[c] = dd[col];
    T* v = evecs + (size_t)c * n;
    std::fill(v, v + n, T(0.0));
    for (int i = 0; i < J; ++i) {
      const double zi = Z[(size_t)i * J + col];
      const T* qi = &Q[(size_t)i * n];
      for (int t = 0; t < n; ++t) v[t] += zi * qi[t];
    }
    const double nr = std::sqrt(re(dotc(v, v, n)));
    for (int t = 0; t < n; ++t) v[t] /= nr;
  }
  return J;
}

int sym_topk(const double* M, int n, int k, double rtol, double* evals, double* evecs) {
  return topk_lanczos<double>(M, n, k, rtol, evals, evecs);
}

int herm_topk(const cplx* M, int n, int k, double rtol, double* evals, cplx* evecs) {
  return topk_lanczos<cplx>(M, n, k, rtol, evals, evecs);
}

// ---------------------------------------------------------------------------
// General complex eigenproblem: Hessenberg reduction by Householder reflections, then
// shifted QR with Givens rotations (Wilkinson shift of the trailing 2x2 block, an
// exceptional shift after 10 and 20 steps without deflation) to upper triangular Schur
// form T = Z^H A Z; eigenvectors of T by back substitution, W = Z x.
bool eig_complex(const cplx* A, int k, cplx* lam, cplx* W) {
  if (k < 1) return false;
  std::vector<cplx> H(A, A + (size_t)k * k), Z((size_t)k * k, cplx(0.0));
  for (int i = 0; i < k; ++i) Z[(size_t)i * k + i] = 1.0;
  for (size_t e = 0; e < H.size(); ++e)
    if (!std::isfinite(H[e].real()) || !std::isfinite(H[e].imag())) return false;
  auto h = [&](int i, int j) -> cplx& { return H[(size_t)i * k + j]; };
  auto z = [&](int i, int j) -> cplx& { return Z[(size_t)i * k + j]; };
  // Hessenberg: P = I - 2 v v^H on rows / columns c+1..k-1
  std::vector<cplx> v(k);
  for (int c = 0; c + 2 < k; ++c) {
    const int len = k - c - 1;
    double xn = 0.0;
    for (int i = 0; i < len; ++i) xn += std::norm(h(c + 1 + i, c));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const cplx x0 = h(c + 1, c);
    const cplx ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cplx(1.0);
    const cplx alpha = -ph * xn;
    for (int i = 0; i < len; ++i) v[i] = h(c + 1 + i, c);
    v[0] -= alpha;
    double vn = 0.0;
    for (int i = 0; i < len; ++i) vn += std::norm(v[i]);
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = 0; i < len; ++i) v[i] /= vn;
    for (int j = 0; j < k; ++j) {  // left: rows c+1..
      cplx s = 0.0;
      for (int i = 0; i < len; ++i) s += std::conj(v[i]) * h(c + 1 + i, j);
      for (int i = 0; i < len; ++i) h(c + 1 + i, j) -= 2.0 * v[i] * s;
    }
    for (int i = 0; i < k; ++i) {  // right: columns c+1.. of H and Z
      cplx s = 0.0, t = 0.0;
      for (int l = 0; l < len; ++l) {
        s += h(i, c + 1 + l) * v[l];
        t += z(i, c + 1 + l) * v[l];
      }
      for (int l = 0; l < len; ++l) {
        h(i, c + 1 + l) -= 2.0 * s * std::conj(v[l]);
        z(i, c + 1 + l) -= 2.0 * t * std::conj(v[l]);
      }
    }
    for (int i = 1; i < len; ++i) h(c + 1 + i, c) = 0.0;
  }
  // shifted QR on the active window [lo, hi]
  std::vector<cplx> gc(k), gs(k);
  int hi = k - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    for (; l > 0; --l) {
      const double tol = DBL_EPSILON * (std::abs(h(l, l)) + std::abs(h(l - 1, l - 1)));
      if (std::abs(h(l, l - 1)) <= tol) {
        h(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 60 * k) return false;
    ++iter;
    cplx mu;
    if (iter % 10 == 0) {
      mu = h(hi, hi) + std::abs(h(hi, hi - 1)) * 0.75;  // exceptional shift
    } else {
      const cplx a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
      const cplx half = 0.5 * (a - d);
      const cplx disc = std::sqrt(half * half + b * c);
      const cplx m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
      mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    }
    for (int i = l; i <= hi; ++i) h(i, i) -= mu;
    // H - mu I = Q R: rotations R_i = [[conj c, conj s], [-s, c]] on rows i, i+1
    for (int i = l; i < hi; ++i) {
      const cplx x = h(i, i), y = h(i + 1, i);
      const double r = std::hypot(std::abs(x), std::abs(y));
      cplx c = 1.0, s = 0.0;
      if (r > 0.0) {
        c = x / r;
        s = y / r;
      }
      gc[i] = c;
      gs[i] = s;
      for (int j = i; j < k; ++j) {
        const cplx u = h(i, j), w2 = h(i + 1, j);
        h(i, j) = std::conj(c) * u + std::conj(s) * w2;
        h(i + 1, j) = -s * u + c * w2;
      }
      h(i + 1, i) = 0.0;
    }
    // R Q + mu I: columns i, i+1 times R_i^H = [[c, -conj s], [s, conj c]]
    for (int i = l; i < hi; ++i) {
      const cplx c = gc[i], s = gs[i];
      const int rmax = std::min(i + 1, hi);
      for (int r = 0; r <= rmax; ++r) {
        const cplx u = h(r, i), w2 = h(r, i + 1);
        h(r, i) = u * c + w2 * s;
        h(r, i + 1) = -u * std::conj(s) + w2 * std::conj(c);
      }
      for (int r = 0; r < k; ++r) {
        const cplx u = z(r, i), w2 = z(r, i + 1);
        z(r, i) = u * c + w2 * s;
        z(r, i + 1) = -u * std::conj(s) + w2 * std::conj(c);
      }
    }
    for (int i = l; i <= hi; ++i) h(i, i) += mu;
  }
  double tn = 0.0;
  for (int i = 0; i < k; ++i)
    for (int j = i; j < k; ++j) tn = std::max(tn, std::abs(h(i, j)));
  const double small = DBL_EPSILON * std::max(tn, DBL_MIN);
  std::vector<cplx> x(k);
  for (int j = 0; j < k; ++j) {
    lam[j] = h(j, j);
    std::fill(x.begin(), x.end(), cplx(0.0));
    x[j] = 1.0;
    for (int i = j - 1; i >= 0; --i) {
      cplx s = 0.0;
      for (int l2 = i + 1; l2 <= j; ++l2) s += h(i, l2) * x[l2];
      cplx den = h(i, i) - lam[j];
      if (std::abs(den) < small) den = small;
      x[i] = -s / den;
    }
    double nr = 0.0;
    cplx* wj = W + (size_t)j * k;
    for (int r = 0; r < k; ++r) {
      cplx acc = 0.0;
      for (int l2 = 0; l2 <= j; ++l2) acc += z(r, l2) * x[l2];
      wj[r] = acc;
      nr += std::norm(acc);
    }
    nr = std::sqrt(nr);
    if (!(nr > 0.0) || !std::isfinite(nr)) return false;
    for (int r = 0; r < k; ++r) wj[r] /= nr;
  }
  return true;
}

// ---------------------------------------------------------------------------
// General real eigenproblem.
bool lu_solve(const cplx* A, int n, const cplx* c, cplx* x) {
  std::vector<cplx> M(A, A + (size_t)n * n);
  std::vector<cplx> b(c, c + n);
  double amax = 0;
  for (int i = 0; i < n * n; ++i) amax = std::max(amax, std::abs(M[i]));
  const double tiny = std::max(amax, 1e-300) * DBL_EPSILON;
  for (int j = 0; j < n; ++j) {
    int piv = j;
    double best = std::abs(M[(size_t)j * n + j]);
    for (int i = j + 1; i < n; ++i)
      if (std::abs(M[(size_t)i * n + j]) > best) best = std::abs(M[(size_t)i * n + j]), piv = i;
    if (piv != j) {
      for (int t = 0; t < n; ++t) std::swap(M[(size_t)j * n + t], M[(size_t)piv * n + t]);
      std::swap(b[j], b[piv]);
    }
    cplx p = M[(size_t)j * n + j];
    if (std::abs(p) < tiny) p = M[(size_t)j * n + j] = cplx(tiny, 0.0);
    for (int i = j + 1; i < n; ++i) {
      const cplx f = M[(size_t)i * n + j] / p;
      if (f == cplx(0.0, 0.0)) continue;
      M[(size_t)i * n + j] = 0.0;
      for (int t = j + 1; t < n; ++t) M[(size_t)i * n + t] -= f * M[(size_t)j * n + t];
      b[i] -= f * b[j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    cplx s = b[i];
    for (int t = i + 1; t < n; ++t) s -= M[(size_t)i * n + t] * x[t];
    x[i] = s / M[(size_t)i * n + i];
    if (!std::isfinite(x[i].real()) || !std::isfinite(x[i].imag())) return false;
  }
  return true;
}

static void hessenberg(std::vector<double>& H, int k) {
  std::vector<double> v(k);
  for (int j = 0; j < k - 2; ++j) {
    double alpha = 0.0;
    for (int i = j + 1; i < k; ++i) alpha += H[(size_t)i * k + j] * H[(size_t)i * k + j];
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    const double x0 = H[(size_t)(j + 1) * k + j];
    std::fill(v.begin(), v.end(), 0.0);
    for (int i = j + 1; i < k; ++i) v[i] = H[(size_t)i * k + j];
    v[j + 1] += sgn1(x0) * alpha;
    double vv = 0.0;
    for (int i = j + 1; i < k; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int c = 0; c < k; ++c) {  // left
      double t = 0.0;
      for (int i = j + 1; i < k; ++i) t += v[i] * H[(size_t)i * k + c];
      const double f = 2.0 * t / vv;
      for (int i = j + 1; i < k; ++i) H[(size_t)i * k + c] -= f * v[i];
    }
    for (int r = 0; r < k; ++r) {  // right
      double t = 0.0;
      for (int i = j + 1; i < k; ++i) t += H[(size_t)r * k + i] * v[i];
      const double f = 2.0 * t / vv;
      for (int i = j + 1; i < k; ++i) H[(size_t)r * k + i] -= f * v[i];
    }
    for (int i = j + 2; i < k; ++i) H[(size_t)i * k + j] = 0.0;
  }
}

// Apply the reflector I - 2 v v^T / (v^T v) (v of length len at index kk) from the left
// to columns [c0, c1] and from the right to rows [r0, r1] of H.
static void reflect(std::vector<double>& H, int k, int kk, int len, const double* v, double vv,
                    int c0, int c1, int r0, int r1) {
  for (int c = c0; c <= c1; ++c) {
    double t = 0.0;
    for (int i = 0; i < len; ++i) t += v[i] * H[(size_t)(kk + i) * k + c];
    const double f = 2.0 * t / vv;
    for (int i = 0; i < len; ++i) H[(size_t)(kk + i) * k + c] -= f * v[i];
  }
  for (int r = r0; r <= r1; ++r) {
    double t = 0.0;
    for (int i = 0; i < len; ++i) t += H[(size_t)r * k + kk + i] * v[i];
    const double f = 2.0 * t / vv;
    for (int i = 0; i < len; ++i) H[(size_t)r * k + kk + i] -= f * v[i];
  }
}

static bool francis_eigvals(std::vector<double>& H, int k, std::vector<cplx>& ev) {
  const double eps = DBL_EPSILON;
  auto at = [&](int i, int j) -> double& { return H[(size_t)i * k + j]; };
  double hnorm = 0.0;
  for (double x : H) hnorm = std::max(hnorm, std::fabs(x));
  int hi = k - 1, its = 0;
  long total = 0;
  ev.clear();
  while (hi >= 0) {
    int l = hi;
    while (l > 0) {
      double s = std::fabs(at(l - 1, l - 1)) + std::fabs(at(l, l));
      if (s == 0.0) s = hnorm;
      if (std::fabs(at(l, l - 1)) <= eps * s) {
        at(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {
      ev.push_back(cplx(at(hi, hi), 0.0));
      --hi;
      its = 0;
      continue;
    }
    if (l == hi - 1) {
      const double a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
      const double p = 0.5 * (a - d), q = p * p + b * c, mid = 0.5 * (a + d);
      if (q >= 0.0) {
        const double z = std::sqrt(q);
        const double l1 = mid + sgn1(p) * z;
        const double det = a * d - b * c;
        const double l2 = (l1 != 0.0) ? det / l1 : mid - sgn1(p) * z;
        ev.push_back(cplx(l1, 0.0));
        ev.push_back(cplx(l2, 0.0));
      } else {
        const double im = std::sqrt(-q);
        ev.push_back(cplx(mid, im));
        ev.push_back(cplx(mid, -im));
      }
      hi -= 2;
      its = 0;
      continue;
    }
    if (++its > 60 || ++total > 60L * k) return false;
    double s, t;
    if (its == 10 || its == 20) {
      const double wv = std::fabs(at(hi, hi - 1)) + std::fabs(at(hi - 1, hi - 2));
      s = 1.5 * wv;
      t = wv * wv;
    } else {
      s = at(hi - 1, hi - 1) + at(hi, hi);
      t = at(hi - 1, hi - 1) * at(hi, hi) - at(hi - 1, hi) * at(hi, hi - 1);
    }
    double x = at(l, l) * at(l, l) + at(l, l + 1) * at(l + 1, l) - s * at(l, l) + t;
    double y = at(l + 1, l) * (at(l, l) + at(l + 1, l + 1) - s);
    double z = at(l + 1, l) * at(l + 2, l + 1);
    for (int kk = l; kk <= hi - 2; ++kk) {
      const double alpha = std::sqrt(x * x + y * y + z * z);
      if (alpha != 0.0) {
        double v[3] = {x + sgn1(x) * alpha, y, z};
        const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        reflect(H, k, kk, 3, v, vv, std::max(l, kk - 1), hi, l, std::min(kk + 3, hi));
        if (kk > l) {
          at(kk + 1, kk - 1) = 0.0;
          at(kk + 2, kk - 1) = 0.0;
        }
      }
      x = at(kk + 1, kk);
      y = at(kk + 2, kk);
      z = (kk < hi - 2) ? at(kk + 3, kk) : 0.0;
    }
    {
      const int kk = hi - 1;
      const double alpha = std::hypot(x, y);
      if (alpha != 0.0) {
        double v[2] = {x + sgn1(x) * alpha, y};
        const double vv = v[0] * v[0] + v[1] * v[1];
        reflect(H, k, kk, 2, v, vv, std::max(l, kk - 1), hi, l, hi);
        if (kk > l) at(kk + 1, kk - 1) = 0.0;
      }
    }
  }
  return (int)ev.size() == k;
}

bool eig_general(const double* A, int k, cplx* lam, cplx* W) {
  if (k < 1) return false;
  for (int i = 0; i < k * k; ++i)
    if (!std::isfinite(A[i])) return false;
  std::vector<double> H(A, A + (size_t)k * k);
  std::vector<cplx> ev;
  if (k == 1) {
    ev.push_back(cplx(A[0], 0.0));
  } else {
    hessenberg(H, k);
    if (!francis_eigvals(H, k, ev)) return false;
  }
  if (k == 1) {
    lam[0] = ev[0];
    W[0] = cplx(1.0, 0.0);
    return true;
  }
  std::vector<cplx> M((size_t)k * k), b(k), y(k);
  for (int j = 0; j < k; ++j) {
    const cplx lj = ev[j];
    lam[j] = lj;
    cplx* wj = W + (size_t)j * k;
    if (lj.imag() < 0.0 && j > 0 && ev[j - 1] == std::conj(lj)) {
      for (int i = 0; i < k; ++i) wj[i] = std::conj(W[(size_t)(j - 1) * k + i]);
      continue;
    }
    for (int r = 0; r < k; ++r)
      for (int c = 0; c < k; ++c) M[(size_t)r * k + c] = cplx(A[(size_t)r * k + c], 0.0) - (r == c ? lj : 0.0);
    for (int i = 0; i < k; ++i) b[i] = cplx(1.0, 0.0);
    for (int it = 0; it < 3; ++it) {
      if (!lu_solve(M.data(), k, b.data(), y.data())) return false;
      double nr = 0.0;
      for (int i = 0; i < k; ++i) nr += std::norm(y[i]);
      nr = std::sqrt(nr);
      if (!(nr > 0.0) || !std::isfinite(nr)) return false;
      for (int i = 0; i < k; ++i) b[i] = y[i] / nr;
    }
    for (int i = 0; i < k; ++i) wj[i] = b[i];
  }
  return true;
}

// ---------------------------------------------------------------------------
bool herm_pd_solve(const cplx* H, int ldh, int n, const cplx* c, cplx* x) {
  std::vector<cplx> L((size_t)n * n, cplx(0.0, 0.0));
  double dmax = 0.0;
  for (int i = 0; i < n; ++i) dmax = std::max(dmax, H[(size_t)i * ldh + i].real());
  if (!(dmax > 0.0)) return false;
  for (int j = 0; j < n; ++j) {
    double djj = H[(size_t)j * ldh + j].real();
    for (int p = 0; p < j; ++p) djj -= std::norm(L[(size_t)j * n + p]);
    if (!(djj > 1e-14 * dmax)) return false;
    const double ljj = std::sqrt(djj);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      cplx s = H[(size_t)i * ldh + j];
      for (int p = 0; p < j; ++p) s -= L[(size_t)i * n + p] * std::conj(L[(size_t)j * n + p]);
      L[(size_t)i * n + j] = s / ljj;
    }
  }
  std::vector<cplx> yv(n);
  for (int i = 0; i < n; ++i) {
    cplx s = c[i];
    for (int p = 0; p < i; ++p) s -= L[(size_t)i * n + p] * yv[p];
    yv[i] = s / L[(size_t)i * n + i].real();
  }
  for (int i = n - 1; i >= 0; --i) {
    cplx s = yv[i];
    for (int p = i + 1; p < n; ++p) s -= std::conj(L[(size_t)p * n + i]) * x[p];
    x[i] = s / L[(size_t)i * n + i].real();
  }
  return true;
}

std::vector<int> conj_partners(const cplx* lam, int k) {
  std::vector<int> partner(k, -1);
  for (int a = 0; a < k; ++a) {
    if (!(lam[a].imag() > 0.0) || partner[a] >= 0) continue;
    int best = -1;
    double bd = 0.0;
    for (int b = 0; b < k; ++b) {
      if (!(lam[b].imag() < 0.0) || partner[b] >= 0) continue;
      const double d = std::abs(lam[b] - std::conj(lam[a]));
      if (d <= 1e-12 * std::abs(lam[a]) && (best < 0 || d < bd)) best = b, bd = d;
    }
    if (best >= 0) partner[a] = best, partner[best] = a;
  }
  return partner;
}

bool omp_gram(const cplx* H, int k, const cplx* c, double x1n2, int K, const cplx* lam,
              double stop_rel, std::vector<int>& S, std::vector<cplx>& beta, double* resid2) {
  S.clear();
  beta.clear();
  std::vector<char> used(k, 0);
  std::vector<cplx> Hs, cs;
  const std::vector<int> partner = lam ? conj_partners(lam, k) : std::vector<int>(k, -1);
  double r2 = x1n2;
  const int steps = std::min(K, k);
  for (int it = 0; it < steps; ++it) {
    // correlations alpha_j = c_j - sum_s H[j, S_s] beta_s, normalised by ||phi_j||
    int pick = -1;
    double best = -1.0;
    for (int j = 0; j < k; ++j) {
      if (used[j]) continue;
      cplx a = c[j];
      for (size_t s = 0; s < S.size(); ++s) a -= H[(size_t)j * k + S[s]] * beta[s];
      const double hj = H[(size_t)j * k + j].real();
      const double corr = std::abs(a) / std::sqrt(std::max(hj, DBL_MIN));
      if (corr > best) best = corr, pick = j;
    }
    if (pick >= 0 && partner[pick] >= 0 && !used[partner[pick]]) {
      bool closed = true;  // every selected pair member has its partner selected
      for (int s : S)
        if (partner[s] >= 0 && !used[partner[s]]) closed = false;
      const int q = partner[pick];
      if (closed && lam[q].imag() > 0.0) pick = q;
    }
    if (pick < 0) break;
    used[pick] = 1;
    S.push_back(pick);
    const int ns = (int)S.size();
    Hs.assign((size_t)ns * ns, cplx(0.0, 0.0));
    cs.assign(ns, cplx(0.0, 0.0));
    for (int a = 0; a < ns; ++a) {
      cs[a] = c[S[a]];
      for (int b = 0; b < ns; ++b) Hs[(size_t)a * ns + b] = H[(size_t)S[a] * k + S[b]];
    }
    beta.assign(ns, cplx(0.0, 0.0));
    if (!herm_pd_solve(Hs.data(), ns, ns, cs.data(), beta.data()))
      if (!lu_solve(Hs.data(), ns, cs.data(), beta.data())) return false;
    double proj = 0.0;
    for (int a = 0; a < ns; ++a) proj += (std::conj(cs[a]) * beta[a]).real();
    r2 = std::max(x1n2 - proj, 0.0);
    if (r2 <= stop_rel * stop_rel * x1n2) break;
  }
  if (resid2) *resid2 = r2;
  return true;
}

// --------------------------------------------------------------------------- spectra
namespace {
// Number of eigenvalues of the symmetric tridiagonal (d, e2 = squared off-diagonals)
// smaller than x (inertia of the LDL^T pivots; a pivot too small in modulus counts as
// negative).
int tri_count_below(const std::vector<double>& d, const std::vector<double>& e2, double x, double pivmin) {
  const int n = (int)d.size();
  int cnt = 0;
  double q = d[0] - x;
  if (std::fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}
}  // namespace

// The symmetric tridiagonal form of A (Householder), with what bisection on it needs.
struct SymTri {
  int n = 0;
  std::vector<double> d, e2;
  double lo = 0.0, hi = 0.0, pivmin = 0.0;
  int count_below(double x) const { return tri_count_below(d, e2, x, pivmin); }
  // the r-th smallest eigenvalue: count(a) <= r < count(b)
  double kth(int r) const {
    double a = lo, b = hi;
    for (int it = 0; it < 200 && b - a > 2.0 * DBL_EPSILON * std::max(std::fabs(a), std::fabs(b)) + pivmin; ++it) {
      const double mid = 0.5 * (a + b);
      if (mid <= a || mid >= b) break;
      if (count_below(mid) > r) b = mid;
      else a = mid;
    }
    return 0.5 * (a + b);
  }
};

static bool sym_tridiagonal(const double* Ain, int n, int lda, SymTri& t) {
  t.n = n;
  std::vector<double> A((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double v = Ain[(size_t)i * lda + j];
      if (!std::isfinite(v)) return false;
      A[(size_t)i * n + j] = 0.5 * (v + Ain[(size_t)j * lda + i]);
    }
  // Householder: for column k, the reflector H = I - 2 v v^T (unit v) zeroes A[k+2.., k];
  // the trailing block becomes H A22 H = A22 - v w^T - w v^T with w = 2 (p - (v^T p) v),
  // p = A22 v.
  std::vector<double> v(n), pv(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // size of the trailing block, rows/cols k+1..n-1
    double xnorm2 = 0.0;
    for (int i = 0; i < m; ++i) {
      v[i] = A[(size_t)(k + 1 + i) * n + k];
      xnorm2 += v[i] * v[i];
    }
    const double xnorm = std::sqrt(xnorm2);
    if (xnorm == 0.0) continue;
    const double alpha = v[0] > 0.0 ? -xnorm : xnorm;
    v[0] -= alpha;
    double vn2 = 0.0;
    for (int i = 0; i < m; ++i) vn2 += v[i] * v[i];
    if (vn2 == 0.0) continue;
    const double vinv = 1.0 / std::sqrt(vn2);
    for (int i = 0; i < m; ++i) v[i] *= vinv;
    double vtp = 0.0;
    for (int i = 0; i < m; ++i) {
      const double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
      // eight independent partial sums (a fixed order), so the loop is not one long
      // chain of dependent additions
      double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int j = 0;
      for (; j + 8 <= m; j += 8)
        for (int u = 0; u < 8; ++u) a[u] += row[j + u] * v[j + u];
      for (; j < m; ++j) a[j & 7] += row[j] * v[j];
      const double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
      pv[i] = acc;
      vtp += v[i] * acc;
    }
    for (int i = 0; i < m; ++i) w[i] = 2.0 * (pv[i] - vtp * v[i]);
    for (int i = 0; i < m; ++i) {
      double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
      for (int j = 0; j < m; ++j) row[j] -= v[i] * w[j] + w[i] * v[j];
    }
    A[(size_t)(k + 1) * n + k] = alpha;
    A[(size_t)k * n + k + 1] = alpha;
    for (int i = 1; i < m; ++i) A[(size_t)(k + 1 + i) * n + k] = A[(size_t)k * n + (k + 1 + i)] = 0.0;
  }
  t.d.assign(n, 0.0);
  t.e2.assign(n > 1 ? n - 1 : 1, 0.0);
  double e2max = 0.0;
  for (int i = 0; i < n; ++i) t.d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) {
    const double e = A[(size_t)(i + 1) * n + i];
    t.e2[i] = e * e;
    e2max = std::max(e2max, t.e2[i]);
  }
  // Gershgorin interval
  t.lo = t.d[0], t.hi = t.d[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::sqrt(t.e2[i - 1]) : 0.0) + (i + 1 < n ? std::sqrt(t.e2[i]) : 0.0);
    t.lo = std::min(t.lo, t.d[i] - r);
    t.hi = std::max(t.hi, t.d[i] + r);
  }
  const double tnorm = std::max(std::fabs(t.lo), std::fabs(t.hi));
  t.pivmin = DBL_MIN * std::max(1.0, e2max);
  t.lo -= 4.0 * DBL_EPSILON * tnorm * n + 2.0 * t.pivmin;
  t.hi += 4.0 * DBL_EPSILON * tnorm * n + 2.0 * t.pivmin;
  return true;
}

bool sym_eigvals(const double* Ain, int n, int lda, std::vector<double>& ev) {
  ev.assign(n, 0.0);
  if (n < 1) return true;
  SymTri t;
  if (!sym_tridiagonal(Ain, n, lda, t)) return false;
  for (int r = 0; r < n; ++r) ev[r] = t.kth(r);
  return true;
}

bool sym_rank_threshold(const double* A, int n, int lda, int r, double scale, double omega, int* k, double* tau) {
  SymTri t;
  if (n < 1 || r < 1 || r > n || !sym_tridiagonal(A, n, lda, t)) return false;
  // singular value q (descending, 0-based) = scale sqrt(eigenvalue of ascending rank n-1-q)
  auto sigma = [&](int q) { return scale * std::sqrt(std::max(t.kth(n - 1 - q), 0.0)); };
  const double med = (r & 1) ? sigma(r / 2) : 0.5 * (sigma(r / 2 - 1) + sigma(r / 2));
  const double th = omega * med;
  const double x = (th / scale) * (th / scale);
  const int above = n - t.count_below(x);
  *k = std::max(0, std::min(r, above));
  *tau = th;
  return true;
}

double gd_lambda_star(double beta) {
  return std::sqrt(2.0 * (beta + 1.0) + 8.0 * beta / ((beta + 1.0) + std::sqrt(beta * beta + 14.0 * beta + 1.0)));
}

double mp_median(double beta) {
  // t(theta) = a + (b - a)(1 - cos theta)/2 on [0, pi] turns the density
  // sqrt((b - t)(t - a)) / (2 pi beta t) dt into the smooth ((b - a)^2/4) sin^2(theta) /
  // (2 pi beta t(theta)) dtheta; its integral (composite Simpson) is the distribution
  // function, and the median is found by bisection on theta.
  const double sb = std::sqrt(beta), a = (1.0 - sb) * (1.0 - sb), b = (1.0 + sb) * (1.0 + sb);
  const double h2 = 0.25 * (b - a) * (b - a);
  auto f = [&](double th) {
    const double s = std::sin(th);
    const double t = a + 0.5 * (b - a) * (1.0 - std::cos(th));
    // a = 0 (beta = 1): sin^2 / t = (1 + cos) / (b / 2), finite at theta = 0
    if (t <= 0.0) return a == 0.0 ? h2 * (1.0 + std::cos(th)) / (M_PI * beta * b) : 0.0;
    return h2 * s * s / (2.0 * M_PI * beta * t);
  };
  auto cdf = [&](double th1) {
    const int panels = 2048;
    const double hh = th1 / panels;
    double acc = f(0.0) + f(th1);
    for (int i = 1; i < panels; ++i) acc += (i & 1 ? 4.0 : 2.0) * f(i * hh);
    return acc * hh / 3.0;
  };
  double lo = 0.0, hi = M_PI;
  for (int it = 0; it < 80; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (cdf(mid) < 0.5) lo = mid;
    else hi = mid;
  }
  const double th = 0.5 * (lo + hi);
  return a + 0.5 * (b - a) * (1.0 - std::cos(th));
}

double gd_omega(double beta) { return gd_lambda_star(beta) / std::sqrt(mp_median(beta)); }

}  // namespace la
}  // namespace cdmd
