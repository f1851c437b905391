// Small dense float64 linear algebra of the cDMD fit (host side).
//
// These are the k x k and (m-1) x (m-1) problems of Algorithm 1: the truncated SVD of
// the sketch Y (eq. svd, computed as the top-k eigenpairs of the Gram Y^T Y), the
// eigendecomposition of A~ (Section 3.2), the amplitude least squares (eq. (eq:b)) and the
// sparsity-constrained amplitudes by orthogonal matching pursuit (Section 2.3).
// All in float64 / complex<double>; none of it touches the video.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace cdmd {
namespace la {

using cplx = std::complex<double>;

// Eigenvalues (and optionally vector rows) of the symmetric tridiagonal matrix with
// diagonal d[0..n-1] and off-diagonal e[0..n-2], by implicit QR sweeps with the
// Wilkinson shift.  Z is R x n row-major holding rows [row0, row0+R) of the
// accumulated rotation matrix (start: the same rows of the identity); on return
// column j of the full matrix is the unit eigenvector of d[j].  R = 0 skips vectors.
// d, e are overwritten (d = eigenvalues, unsorted).  Returns false if an eigenvalue
// failed to converge.
bool tridiag_eig(double* d, double* e, int n, double* Z, int R, int row0);

// Top-k eigenpairs of the symmetric n x n matrix M (row-major) by Lanczos with full
// (twice classical Gram-Schmidt) reorthogonalisation.  Steps are added until every
// one of the top-k Ritz pairs has residual <= rtol * theta_1, or the Krylov space is
// the whole space.  evals[k] descending, evecs n x k column-major (unit columns).
// Returns the Krylov dimension used, or -1 on failure.
int sym_topk(const double* M, int n, int k, double rtol, double* evals, double* evecs);

// The same for a complex Hermitian n x n matrix M (row-major): complex Lanczos vectors,
// a real symmetric tridiagonal projection.  evecs n x k column-major.
int herm_topk(const cplx* M, int n, int k, double rtol, double* evals, cplx* evecs);

// Eigenvalues and unit eigenvectors of a complex general k x k matrix A (row-major):
// Householder reduction to Hessenberg form, shifted QR to triangular Schur form, back
// substitution for the eigenvectors.  W is k x k column-major.  False on failure.
bool eig_complex(const cplx* A, int k, cplx* lam, cplx* W);

// Eigenvalues and unit eigenvectors of a real general k x k matrix A (row-major):
// Householder reduction to Hessenberg form, Francis double-shift QR to real Schur form
// (conjugate pairs from 2x2 blocks are exact conjugates), then inverse iteration on
// A - lambda I for each eigenvector (the partner of a complex pair is its conjugate).
// W is k x k column-major (column j belongs to lam[j]).  Returns false on failure.
bool eig_general(const double* A, int k, cplx* lam, cplx* W);

// Solve H x = c for Hermitian positive definite H (n x n, row-major, leading
// dimension ldh) by Cholesky.  Returns false if H is not numerically positive
// definite (a pivot <= tiny * max diagonal).
bool herm_pd_solve(const cplx* H, int ldh, int n, const cplx* c, cplx* x);

// Solve A x = c for general complex A (n x n row-major) by LU with partial pivoting.
bool lu_solve(const cplx* A, int n, const cplx* c, cplx* x);

// Conjugate partners of the eigenvalues: partner[a] = b when lambda_b = conj(lambda_a) to
// 1e-12 relative (each lambda with Im > 0 takes the closest qualifying unpaired lambda with
// Im < 0), else -1.
std::vector<int> conj_partners(const cplx* lam, int k);

// Orthogonal matching pursuit in coefficient space on the Gram H = Phi^H Phi (k x k),
// c = Phi^H x_1 and x1n2 = ||x_1||^2 for a real x_1: per step alpha = c - H[:,S] beta_S,
// pick the unselected j maximising |alpha_j| / sqrt(H_jj) (the first maximum on exact
// ties), then beta_S = H[S,S]^-1 c[S].  With the eigenvalues lam (nullable): while the
// support holds both members of each of its conjugate pairs the residual is real, the
// two members of an unselected pair tie by symmetry, and a pick of either goes to the one
// with Im lambda > 0.  Stops after K atoms or when ||x_1 - Phi_S beta_S||^2 =
// x1n2 - Re(c_S^H beta_S) <= (stop_rel^2) x1n2.  Returns false if a subsystem is singular.
bool omp_gram(const cplx* H, int k, const cplx* c, double x1n2, int K, const cplx* lam,
              double stop_rel, std::vector<int>& S, std::vector<cplx>& beta,
              double* resid2);

// All eigenvalues (ascending) of the symmetric n x n matrix A (row-major, leading
// dimension lda): Householder reduction to tridiagonal form, then bisection with Sturm
// counts.  Returns false on non-finite input.
bool sym_eigvals(const double* A, int n, int lda, std::vector<double>& ev);
// Remark 2's rank from the Gram A (n x n): with sigma_q = scale sqrt(mu_q) the r largest
// singular values, tau = omega * median(sigma_0..sigma_{r-1}) and k = #{sigma_q > tau}; only
// the median and one count are computed (bisection on the tridiagonal form).  False for a
// non-finite A.
bool sym_rank_threshold(const double* A, int n, int lda, int r, double scale, double omega, int* k, double* tau);

// The optimal hard threshold of Gavish and Donoho for an aspect ratio beta = (smaller
// dimension) / (larger dimension) in (0, 1]: lambda*(beta) for a known noise level, the
// median mu_beta of the Marchenko-Pastur law of ratio beta, and omega(beta) =
// lambda*(beta) / sqrt(mu_beta), the coefficient of the median singular value.
double gd_lambda_star(double beta);
double mp_median(double beta);
double gd_omega(double beta);

}  // namespace la
}  // namespace cdmd
