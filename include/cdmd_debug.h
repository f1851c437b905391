/*
 * cdmd_debug.h -- test entry points of libcdmd.so.  The cdmd_dbg_* linear-algebra calls
 * expose the float64 small linear algebra of the fit for testing without a GPU: they
 * run on the calling thread and touch no device.  cdmd_dbg_force_valu_lift selects the
 * float32 vector-ALU lift instead of the MFMA lift so tests can compare the two.  None
 * of these is part of the hot path's public API.
 */
#ifndef CDMD_DEBUG_H
#define CDMD_DEBUG_H

#include <stdint.h>

#include "cdmd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Top-k eigenpairs of the symmetric n x n matrix M (host, row-major) by Lanczos with
   full reorthogonalisation (the route to the truncated SVD, eq. svd).
   evals[k] descending; evecs n x k column-major.  *steps = Krylov dimension used.
   Errors: INVALID_ARG, NUMERIC. */
cdmd_status cdmd_dbg_sym_topk(const double* M, int32_t n, int32_t k, double rtol,
                              double* evals, double* evecs, int32_t* steps);

/* Eigenvalues and unit eigenvectors of a real k x k matrix A (host, row-major)
   (Section 3.2).  lam[2k] (re, im); W[2k*k] column-major complex (re, im).
   Errors: INVALID_ARG, NUMERIC. */
cdmd_status cdmd_dbg_eig_general(const double* A, int32_t k, double* lam, double* W);

/* The complex counterparts used with a complex measurement matrix (the SRFT sketch of
   Section 3.3): top-k eigenpairs of the Hermitian n x n matrix M (host, row-major, re/im
   interleaved) by complex Lanczos with full reorthogonalisation (evecs n x k column-major
   complex), and eigenvalues / unit eigenvectors of a complex k x k matrix A (row-major,
   re/im interleaved; lam[2k], W[2k*k] column-major) by Hessenberg reduction, shifted QR
   and back substitution.  Errors: INVALID_ARG, NUMERIC. */
cdmd_status cdmd_dbg_herm_topk(const double* M, int32_t n, int32_t k, double rtol,
                               double* evals, double* evecs, int32_t* steps);
cdmd_status cdmd_dbg_eig_complex(const double* A, int32_t k, double* lam, double* W);

/* Orthogonal matching pursuit in coefficient space (Section 2.3, eq. (eq:sparsecoding))
   on H = Phi^H Phi (k x k complex, row-major, re/im interleaved), c = Phi^H x_1 (k
   complex) for a real x_1, and x1n2 = ||x_1||^2.  lam (nullable; k complex, re/im
   interleaved) gives the conjugate pairs: while the support is closed under conjugation
   a pick of either member of an unselected pair goes to the one with Im lambda > 0.
   S[k] receives the support in selection order, beta[2k] the amplitudes, *ns = |S|,
   *resid2 = ||x_1 - Phi_S beta||^2.  Errors: INVALID_ARG, NUMERIC. */
cdmd_status cdmd_dbg_omp_gram(const double* H, int32_t k, const double* c, double x1n2,
                              int32_t K, const double* lam, int32_t* S, double* beta,
                              int32_t* ns, double* resid2);

/* All eigenvalues (ascending, ev[n]) of the symmetric n x n row-major matrix A, as the
   automatic target rank computes them on the host (Householder tridiagonalisation, Sturm
   bisection).  Errors: INVALID_ARG, NUMERIC (non-finite input). */
cdmd_status cdmd_dbg_sym_eigvals(const double* A, int32_t n, double* ev);

/* The hard-threshold coefficients of the automatic target rank for aspect ratio beta in
   (0, 1]: lambda*(beta), the Marchenko-Pastur median mu_beta and omega(beta) (each output
   optional).  Errors: INVALID_ARG. */
cdmd_status cdmd_dbg_gd_threshold(double beta, double* lambda_star, double* mp_median, double* omega);

/* Remark 2's rank from a Gram A (n x n, row-major) the way cdmd_process_video computes it
   (the median singular value and one count, no full spectrum): the r largest singular
   values sigma_q = scale sqrt(mu_q), tau = omega * median, k = #{sigma_q > tau}.
   Errors: INVALID_ARG, NUMERIC (non-finite input). */
cdmd_status cdmd_dbg_rank_threshold(const double* A, int32_t n, int32_t r, double scale, double omega, int32_t* k,
                                    double* tau);

/* The device small linear algebra (truncated SVD, A~, eig(A~) and G = V S^-1 W from the
   m x m Gram Gr of the unscaled sketch), run on the host with the same code the GPU runs:
   groups = 1 by one thread; groups = 2..32 with the Lanczos vectors split by rows over that
   many host threads, which exchange their shares as the GPU's workgroups do.  Outputs:
   mu[k] Gram eigenvalues (descending), sigma[k], lam[2k] (re, im), W[2k*k] (column j at
   2*j*k, re/im interleaved), G[2(m-1)k] (row t at 2*t*k), *steps Krylov dimension.
   Returns OK, RANK_DEFICIENT, NUMERIC, or INVALID_ARG for a bad argument. */
cdmd_status cdmd_dbg_team_small_la(const double* Gr, int32_t m, int32_t k, double rtol,
                                   double sketch_scale, int32_t groups, double* mu, double* sigma,
                                   double* lam, double* W, double* G, int32_t* steps);

/* Phase times (ms) of the last device small-LA solve (group 0's clock): [0] Lanczos incl.
   convergence checks, [1] of which the checks, [2] Ritz vectors V = Q Z, M12 V and A~
   (from the end of [0]), [3] eigenvalues of A~, [4] eigenvectors, [5] G, and of [0]:
   [6] waits at the exchanges between the row groups, [7] matrix-vector products, [8]
   Gram-Schmidt work, [9] norm and next vector, [10] multisection of the checks, [11]
   the rest of the checks (closed-form test, tridiagonal inverse iteration), [12] hand-over
   of the Ritz vectors of T_J, [13] loads of the exchanged shares, [14] orthonormalisation
   of the final Ritz vectors of T_J; [15] unused.
   Errors: INVALID_ARG. */
cdmd_status cdmd_dbg_la_phases(const cdmd_model* mdl, double* ms16);

/* Force (1) or release (0) the gather form of the sparse sketch of a uint8 video (one
   byte load per triple and frame) where the streaming form (coalesced 16-byte loads of
   every frame, 16-byte aligned frames) would run.  Takes effect at the next cdmd_fit.
   Errors: INVALID_ARG. */
cdmd_status cdmd_dbg_force_gather_sketch(cdmd_model* mdl, int32_t on);

/* Choose the form of the sparse sketch of a uint8 video as the autotuner would: -1 the
   gather form, or 10 F + V for the streaming form with F frames per workgroup and V
   16-byte vectors per thread (the candidates are 41, 21, 22, 11, 12 and 14).  Takes effect
   at the next cdmd_fit; a later cdmd_autotune replaces it.  Errors: INVALID_ARG (a form
   that does not fit the table), UNSUPPORTED (not a uint8 sparse sketch). */
cdmd_status cdmd_dbg_sparse_form(cdmd_model* mdl, int32_t form);

/* Force (1) or release (0) the float64 small linear algebra on the host instead of the
   device workgroup solve (which runs for 16-byte aligned uint8 videos with m <= 1025).
   Takes effect at the next cdmd_fit.  Errors: INVALID_ARG. */
cdmd_status cdmd_dbg_force_host_la(cdmd_model* mdl, int32_t on);

/* Split the Lanczos vectors of the device small-LA solve over `groups` row groups
   (workgroups, at most m - 1; 0 = as many as the rows call for: one per 32 rows, at most
   32).  Takes effect at the next cdmd_fit.  Errors: INVALID_ARG (groups outside [0, 32]). */
cdmd_status cdmd_dbg_la_groups(cdmd_model* mdl, int32_t groups);

/* Force (1) or release (0) the float32 vector-ALU lift for a uint8 video whose FP32
   lift would otherwise run on MFMA (bf16 terms).  Takes effect at the next cdmd_fit.
   Errors: INVALID_ARG. */
cdmd_status cdmd_dbg_force_valu_lift(cdmd_model* mdl, int32_t on);

#ifdef __cplusplus
}
#endif

#endif /* CDMD_DEBUG_H */
