"""Plain FP64 CPU oracle for compressed DMD background modeling.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and bench.py's CPU
baseline may import this module.  It shares no code with the HIP path and must never
be used to produce a product result.

Follows Erichson, Brunton and Kutz, "Compressed Dynamic Mode Decomposition for
Background Modeling":

* snapshot split X, X' (Section 2.1, eq. FullData);
* sketch Y = C X, Y' = C X' (Section 3.2, eq. (eq:YCX)) with Gaussian, sparse +/-1,
  single-pixel or SRFT C (Section 3.3; the SRFT sketch is complex and every later step
  takes conjugate transposes);
* the least-squares operator on the sketched snapshots, projected on the leading left
  singular vectors: Y = U S V* truncated to rank k (eq. svd), A~ = U* Y' V S^-1 and its
  eigenpairs A~ W = W Lambda (Section 3.2);
* full modes Phi = X' V S^-1 W (eq. Eq:cDMDModes) and amplitudes b, the least-squares
  fit of the first frame x_1 (Section 2.2, eq. (eq:b));
* Vandermonde matrix lambda_j^(t-1) (Section 2.1, the factorisation Phi B V);
* background L = Re(sum over selected modes b_p phi_p lambda_p^(t-1)) (Section 2.2,
  eq. (equ:DMDTerms) and its footnote on the real part);
* sparsity-constrained amplitudes by orthogonal matching pursuit (Section 2.3,
  eq. (eq:sparsecoding)), on the full modes or, by Remark 3 of Section 3.2, on the
  compressed modes Phi_Y = Y' V S^-1 W and the first compressed frame y_1;
* foreground mask |x_jt - xhat_jt| > tau (Section 4, eq. (eq:thres)), and its median
  filtering (Section 4, BMC evaluation);
* recall, precision, F-measure (Section 4).

Numerical route: direct SVD of Y, LAPACK eig, direct least squares and explicit-
residual OMP, all in float64 / complex128.  Where the paper is silent the readings
adopted are stated at each function (eigenvector normalisation, canonical mode order,
OMP ties, rank tolerance, strict threshold).

Pixel values: uint8 frames are scaled by 1/255; float frames are used as they are.
Frames are given frame-major, D of shape (m, n) (frame t is row t); X = D^T.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

from . import philox

# rank test: sigma_k <= RANK_TOL * sigma_1 is rank deficient (the paper sets no
# tolerance; 1e-6 is what a Gram-based route can still resolve in float64)
RANK_TOL = 1e-6
# conjugate partners: lambda_b = conj(lambda_a) to this relative distance
PAIR_REL = 1e-12
# OMP stops early when ||r|| <= OMP_STOP_REL * ||x_1||
OMP_STOP_REL = 1e-12
# |lambda|^(m-1) above this overflows the Vandermonde matrix
VANDER_MAX = 1e30


class RankDeficient(ValueError):
    pass


class NumericError(ValueError):
    pass


# ---------------------------------------------------------------- data access
def pixel_rows(D: np.ndarray, scale: float, i0: int = 0, i1: Optional[int] = None,
               pixels: Optional[np.ndarray] = None) -> np.ndarray:
    """Rows of the snapshot matrix [x_1 ... x_m] (pixels x frames) in float64:
    pixel range [i0, i1) or an explicit pixel index list."""
    if pixels is not None:
        blk = D[:, np.asarray(pixels)]
    else:
        blk = D[:, i0:(D.shape[1] if i1 is None else i1)]
    return blk.T.astype(np.float64) * scale


# ---------------------------------------------------------------- sketches
def sketch_sparse(D: np.ndarray, scale: float, idx: np.ndarray, sign: np.ndarray):
    """Y^ = C D for a sparse +/-1 (or single-pixel, weight +1) C given by its index
    table idx (p, nnz) and signs (p, nnz); index -1 marks an empty slot (rows of the
    i.i.d. sparse C of Section 3.3 hold different numbers of nonzeros).  Integer frames
    are summed exactly in int64 before scaling.  Returns (Y^ float64 (p, m), integer sums
    or None)."""
    m, n = D.shape
    p, nnz = idx.shape
    used = idx >= 0
    safe = np.where(used, idx, 0)
    w = np.where(used, sign, 0)
    if np.issubdtype(D.dtype, np.integer):
        acc = np.zeros((m, p), dtype=np.int64)
        for j in range(nnz):
            acc += D[:, safe[:, j]].astype(np.int64) * w[:, j].astype(np.int64)[None, :]
        return acc.T.astype(np.float64) * scale, acc.T.copy()
    acc = np.zeros((m, p), dtype=np.float64)
    for j in range(nnz):
        acc += D[:, safe[:, j]].astype(np.float64) * w[:, j].astype(np.float64)[None, :]
    return acc.T * scale, None


def gaussian_C(seed: int, p: int, j0: int, j1: int, quantise=None) -> np.ndarray:
    """Dense Gaussian C restricted to pixel columns [j0, j1): entries N(0, 1/p).
    ``quantise`` (a callable on float64 arrays) rounds the N(0,1) draws to a storage
    format before the 1/sqrt(p) scale (the quantised-C reading of a low-precision
    sketch)."""
    z = philox.gaussian_block(seed, 0, p, j0, j1)
    if quantise is not None:
        z = quantise(z)
    return z / np.sqrt(p)


def sketch_gaussian(D: np.ndarray, scale: float, seed: int, p: int, chunk: int = 8192,
                    quantise=None, rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """Y^ = C D with dense Gaussian C, accumulated over pixel chunks in float64.
    ``rows`` restricts the output to a subset of sketch rows."""
    m, n = D.shape
    Y = np.zeros((p if rows is None else len(rows), m))
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        if rows is None:
            C = gaussian_C(seed, p, j0, j1, quantise)
        else:  # only the requested rows of C (each entry is a function of its row and pixel)
            C = np.concatenate([philox.gaussian_block(seed, r, r + 1, j0, j1) for r in rows])
            if quantise is not None:
                C = quantise(C)
            C = C / np.sqrt(p)
        Y += C @ pixel_rows(D, scale, j0, j1)
    return Y


def srft_diagonal(seed: int, n: int) -> np.ndarray:
    """The random diagonal D of the SRFT (Section 3.3): unit-modulus entries
    exp(2 pi i u_j), u_j from ``philox.srft_uniforms``."""
    return np.exp(2j * np.pi * philox.srft_uniforms(seed, 0, n))


def sketch_srft(D: np.ndarray, scale: float, freqs: np.ndarray, seed: int) -> np.ndarray:
    """Y^ = C X with the subsampled randomised Fourier transform C = R F D / sqrt(p)
    (Section 3.3): D = ``srft_diagonal``, F the unnormalised n-point DFT with entries
    exp(-2 pi i f j / n) (the paper's F(j, k) with the 1/m of the printed exponent read as
    1/n, the transform's own length), R the p rows ``freqs``.  Frame by frame through the
    FFT: (F (D x_t))[freqs].  Complex p x m."""
    m, n = D.shape
    d = srft_diagonal(seed, n)
    freqs = np.asarray(freqs, dtype=np.int64).reshape(-1)
    Y = np.empty((len(freqs), m), dtype=np.complex128)
    for t in range(m):
        Y[:, t] = np.fft.fft(d * (D[t].astype(np.float64) * scale))[freqs]
    return Y / np.sqrt(len(freqs))


def _round_sig(z: np.ndarray, mant_bits: int, emin: int) -> np.ndarray:
    """Round to nearest with ties to even onto a binary format with ``mant_bits``
    stored mantissa bits and minimum normal exponent ``emin`` (subnormals below),
    in one rounding step from float64."""
    z = np.asarray(z, dtype=np.float64)
    a = np.abs(z)
    _, E = np.frexp(a)                     # a = f 2^E, f in [0.5, 1)
    e = np.maximum(E - 1, emin)
    q = np.ldexp(1.0, e - mant_bits)
    return np.sign(z) * (np.round(a / q) * q)


def round_bf16(z: np.ndarray) -> np.ndarray:
    """Round float64 to the nearest bfloat16 (8-bit exponent, 7 stored mantissa
    bits), ties to even."""
    return _round_sig(z, 7, -126)


def round_e4m3(z: np.ndarray) -> np.ndarray:
    """Round float64 to OCP FP8 e4m3fn (bias 7, 3 mantissa bits, no infinities,
    largest finite 448), ties to even, saturating to +/-448."""
    return np.clip(_round_sig(z, 3, -6), -448.0, 448.0)


# ---------------------------------------------------------------- fit
@dataclasses.dataclass
class Model:
    lam: np.ndarray          # (k,) complex eigenvalues, canonical order
    W: np.ndarray            # (k, k) eigenvectors of A~ (columns), normalised
    sigma: np.ndarray        # (k,) singular values of Y
    V: np.ndarray            # (m-1, k) right singular vectors of Y
    Atilde: np.ndarray       # (k, k)
    G: np.ndarray            # (m-1, k) complex V S^-1 W: Phi = X' G
    Phi: Optional[np.ndarray]   # (n, k) complex full modes (None when not formed)
    b: Optional[np.ndarray]     # (k,) complex amplitudes
    phi_norm: Optional[np.ndarray]


def normalise_eigvecs(W: np.ndarray) -> np.ndarray:
    """Unit 2-norm columns; the largest-modulus entry of each column (lowest index on
    ties) is made real and positive."""
    W = W / np.linalg.norm(W, axis=0, keepdims=True)
    piv = np.argmax(np.abs(W), axis=0)
    ph = W[piv, np.arange(W.shape[1])]
    return W * (np.abs(ph) / ph)[None, :]


def conjugate_partners(lam: np.ndarray) -> np.ndarray:
    """partner[a] = b when lambda_b is the conjugate of lambda_a (to PAIR_REL relative),
    else -1.  Each lambda with Im > 0 is paired with the closest unpaired lambda with
    Im < 0 that qualifies; real eigenvalues have no partner."""
    k = len(lam)
    partner = np.full(k, -1, dtype=np.int64)
    for a in range(k):
        if lam[a].imag > 0 and partner[a] < 0:
            cand = [b for b in range(k) if lam[b].imag < 0 and partner[b] < 0
                    and abs(lam[b] - np.conj(lam[a])) <= PAIR_REL * abs(lam[a])]
            if cand:
                b = min(cand, key=lambda q: abs(lam[q] - np.conj(lam[a])))
                partner[a], partner[b] = b, a
    return partner


def canonical_order(lam: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Mode order: descending key = |b_j| * ||phi_j||.  The two members of a conjugate
    pair share one key, the larger of their two, so they are always adjacent, and the
    member with Im lambda > 0 comes first.  Remaining ties keep the eigensolver's
    order."""
    k = len(lam)
    partner = conjugate_partners(lam)
    pk = np.array(key, dtype=np.float64)
    for a in range(k):
        if partner[a] >= 0:
            pk[a] = max(key[a], key[partner[a]])
    return np.array(sorted(range(k), key=lambda j: (-pk[j], lam[j].imag <= 0, j)), dtype=np.int64)


def reduced_operator(Yhat: np.ndarray, k: int):
    """The rank-k reduced operator of the sketched snapshots (Section 3.2): with
    Y = Y^[:, :m-1], Y' = Y^[:, 1:] (eq. (eq:YCX)) and the truncated SVD Y = U S V*
    (eq. svd), A~ = U* Y' V S^-1 and its eigenpairs A~ W = W Lambda (unit-norm W,
    normalised as in ``normalise_eigvecs``).  Returns (lam, W, sigma, V, Atilde).
    Raises RankDeficient if sigma_k <= RANK_TOL sigma_1."""
    p, m = Yhat.shape
    if not (m >= 2 and 1 <= k <= min(p, m - 1)):
        raise ValueError("need m >= 2 and 1 <= k <= min(p, m-1)")
    Y, Yp = Yhat[:, :m - 1], Yhat[:, 1:]
    U, s, Vh = np.linalg.svd(Y, full_matrices=False)
    if not s[0] > 0 or s[k - 1] <= RANK_TOL * s[0]:
        raise RankDeficient(f"sigma_k/sigma_1 = {s[k-1] / max(s[0], 1e-300):.3e}")
    U, s, V = U[:, :k], s[:k], Vh[:k].conj().T
    Atilde = U.conj().T @ Yp @ (V / s[None, :])
    lam, W = np.linalg.eig(Atilde)
    W = normalise_eigvecs(W)
    return lam, W, s, V, Atilde


def lift(D: np.ndarray, scale: float, G: np.ndarray, pixels: Optional[np.ndarray] = None,
         chunk: int = 65536) -> np.ndarray:
    """Full modes Phi = X' G (eq. Eq:cDMDModes with G = V S^-1 W), for all pixels or a
    pixel subset; X' = [x_2 ... x_m]."""
    if pixels is not None:
        return pixel_rows(D, scale, pixels=pixels)[:, 1:] @ G
    n = D.shape[1]
    out = np.empty((n, G.shape[1]), dtype=np.complex128)
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        Xp = pixel_rows(D, scale, i0, i1)[:, 1:]
        out[i0:i1] = Xp @ G.real + 1j * (Xp @ G.imag)
    return out


def fit(D: np.ndarray, scale: float, Yhat: np.ndarray, k: int, form_phi: bool = True) -> Model:
    """Compressed DMD given the sketch Y^ = C D (Section 3.2, Algorithm 1): the reduced
    operator and its eigenpairs, the full modes Phi = X' V S^-1 W (eq. Eq:cDMDModes) and
    the amplitudes b = argmin ||Phi b - x_1|| (eq. (eq:b)); modes in canonical order."""
    lam, W, s, V, At = reduced_operator(Yhat, k)
    G = (V / s[None, :]) @ W
    if not form_phi:
        return Model(lam, W, s, V, At, G, None, None, None)
    Phi = lift(D, scale, G)
    x1 = D[0].astype(np.float64) * scale
    b = np.linalg.lstsq(Phi, x1.astype(np.complex128), rcond=None)[0]
    nrm = np.linalg.norm(Phi, axis=0)
    o = canonical_order(lam, np.abs(b) * nrm)
    return Model(lam[o], W[:, o], s, V, At, G[:, o], Phi[:, o], b[o], nrm[o])


def fit_compressed(Yhat: np.ndarray, k: int) -> Model:
    """Algorithm 1 with the amplitudes of Remark 3 (Section 3.2): the compressed modes
    Phi_Y = Y' V S^-1 W (the eigenvector matrix applied to the compressed snapshots) and
    b = argmin ||y_1 - Phi_Y b|| with y_1 the first compressed frame (column 0 of the
    sketch); the same OMP on (Phi_Y, y_1) gives the sparse amplitudes.  Modes in canonical
    order by |b_j| ||phi_Y,j||; the returned Phi is Phi_Y (p x k), phi_norm its column
    norms.  The full modes of the background are still X' G with the returned G."""
    lam, W, s, V, At = reduced_operator(Yhat, k)
    G = (V / s[None, :]) @ W
    PhiY = Yhat[:, 1:] @ G
    y1 = Yhat[:, 0].astype(np.complex128)
    b = np.linalg.lstsq(PhiY, y1, rcond=None)[0]
    nrm = np.linalg.norm(PhiY, axis=0)
    o = canonical_order(lam, np.abs(b) * nrm)
    return Model(lam[o], W[:, o], s, V, At, G[:, o], PhiY[:, o], b[o], nrm[o])


# ---------------------------------------------------------------- exact DMD (pins)
def dmd_bruteforce(X: np.ndarray, Xp: np.ndarray):
    """A^ = X' X^+ formed explicitly (n x n), Section 2.1; returns (eigvals, A^)."""
    Ahat = Xp @ np.linalg.pinv(X)
    return np.linalg.eigvals(Ahat), Ahat


def dmd_exact(x: np.ndarray, k: int):
    """Exact DMD on the full snapshot matrix x (n x m): the cDMD steps with C = I."""
    X, Xp = x[:, :-1], x[:, 1:]
    U, s, Vh = np.linalg.svd(X, full_matrices=False)
    U, s, V = U[:, :k], s[:k], Vh[:k].conj().T
    At = U.conj().T @ Xp @ (V / s[None, :])
    lam, W = np.linalg.eig(At)
    W = normalise_eigvecs(W)
    Phi = Xp @ (V / s[None, :]) @ W
    b = np.linalg.lstsq(Phi, x[:, 0].astype(np.complex128), rcond=None)[0]
    return lam, Phi, b


# ---------------------------------------------------------------- automatic target rank
def gd_lambda_star(beta: float) -> float:
    """The optimal hard threshold coefficient for a known noise level (Gavish and Donoho,
    "The optimal hard threshold for singular values is 4/sqrt(3)", 2014), aspect ratio
    beta = (smaller dimension) / (larger dimension) in (0, 1]:
    lambda*(beta) = sqrt(2 (beta + 1) + 8 beta / ((beta + 1) + sqrt(beta^2 + 14 beta + 1)))."""
    b = float(beta)
    return float(np.sqrt(2.0 * (b + 1.0) + 8.0 * b / ((b + 1.0) + np.sqrt(b * b + 14.0 * b + 1.0))))


def mp_median(beta: float) -> float:
    """Median of the Marchenko-Pastur law of ratio beta in (0, 1] (variance 1): the mu with
    int_a^mu sqrt((b - t)(t - a)) / (2 pi beta t) dt = 1/2, a, b = (1 -+ sqrt(beta))^2, by
    numerical quadrature and root finding."""
    from scipy.integrate import quad
    from scipy.optimize import brentq
    b_ = float(beta)
    lo, hi = (1.0 - np.sqrt(b_)) ** 2, (1.0 + np.sqrt(b_)) ** 2
    def dens(t):
        # the density; at beta = 1 it is integrable like t^(-1/2) at t = a = 0
        return np.sqrt(max((hi - t) * (t - lo), 0.0)) / (2.0 * np.pi * b_ * t) if t > 0.0 else 0.0

    def cdf(x):
        return quad(dens, lo, x, limit=200, epsabs=1e-14, epsrel=1e-13)[0] if x > lo else 0.0
    return float(brentq(lambda x: cdf(x) - 0.5, lo, hi, xtol=1e-14, rtol=1e-14))


def gd_omega(beta: float) -> float:
    """The threshold coefficient for an unknown noise level: omega(beta) =
    lambda*(beta) / sqrt(mu_beta), applied to the median singular value."""
    return gd_lambda_star(beta) / np.sqrt(mp_median(beta))


def optimal_rank(Yhat: np.ndarray):
    """Automatic target rank (Section 3.2, Remark 2): the optimal hard threshold of Gavish
    and Donoho on the singular values of Y = Y^[:, :m-1] with the noise level unknown:
    tau* = omega(beta) * median(sigma), beta = min(p, m-1) / max(p, m-1), and k the number of
    singular values above tau*.  Returns (k, tau*, sigma) with sigma all min(p, m-1)
    singular values in descending order."""
    p, m = Yhat.shape
    s = np.linalg.svd(Yhat[:, :m - 1], compute_uv=False)
    beta = min(p, m - 1) / max(p, m - 1)
    tau = gd_omega(beta) * float(np.median(s))
    return int(np.count_nonzero(s > tau)), tau, s


# ---------------------------------------------------------------- selection
def omp(Phi: np.ndarray, x1: np.ndarray, K: int, lam: Optional[np.ndarray] = None,
        margins: Optional[list] = None):
    """Orthogonal matching pursuit for eq. (eq:sparsecoding), explicit residual form:
    r = x_1; repeat: pick the unselected mode maximising |phi_j^H r| / ||phi_j||,
    project x_1 onto the selected modes by least squares, recompute r; stop after
    min(K, k) atoms or when ||r|| <= OMP_STOP_REL ||x_1||.

    Ties (reading of the paper, which is silent on them).  With a real x_1 and a support
    that holds both members of every conjugate pair in it, the least-squares amplitudes
    of a pair are conjugates, the residual is real, and the two members of any pair not
    yet selected have equal correlations: |phi_b^H r| = |conj(phi_a)^H r| = |phi_a^H r|.
    When ``lam`` is given (conjugate pairs by ``conjugate_partners``), such a pick goes to
    the member with Im lambda > 0 whichever member rounding favours.  Any other exact
    tie goes to the lowest index.

    ``margins``, when a list, receives per pick the relative gap (best - next) / best
    between the picked correlation and the best correlation outside the picked mode and
    its tied partner: a small gap marks a near tie, on which a computation in another
    precision may pick differently.  Returns (support in selection order, beta_S)."""
    n, k = Phi.shape
    real_x = not np.iscomplexobj(x1) or not np.any(np.imag(x1))
    x1 = x1.astype(np.complex128)
    nrm = np.linalg.norm(Phi, axis=0)
    partner = conjugate_partners(np.asarray(lam)) if lam is not None else np.full(k, -1)
    S: list = []
    beta = np.zeros(0, dtype=np.complex128)
    r = x1.copy()
    x1n = np.linalg.norm(x1)
    for _ in range(min(K, k)):
        corr = np.abs(Phi.conj().T @ r) / nrm
        corr[S] = -1.0
        j = int(np.argmax(corr))
        closed = all(partner[s] < 0 or partner[s] in S for s in S)
        q = int(partner[j])
        tied = real_x and closed and q >= 0 and q not in S
        if tied and lam[q].imag > 0:
            j, q = q, j
        if margins is not None:
            rest = corr.copy()
            rest[j] = -1.0
            if tied:
                rest[q] = -1.0
            top = corr[j] if corr[j] > 0 else 1.0
            margins.append(float((corr[j] - rest.max()) / top) if rest.max() >= 0 else 1.0)
        S.append(j)
        beta = np.linalg.lstsq(Phi[:, S], x1, rcond=None)[0]
        r = x1 - Phi[:, S] @ beta
        if np.linalg.norm(r) <= OMP_STOP_REL * x1n:
            break
    return np.array(S, dtype=np.int64), beta


def select_zero_mode(lam: np.ndarray) -> np.ndarray:
    """The single mode with continuous-time eigenvalue closest to the origin,
    |omega| = |log lambda| with dt = 1 (Section 2.2)."""
    return np.array([int(np.argmin(np.abs(np.log(lam.astype(np.complex128)))))])


def select_omega(lam: np.ndarray, thr: float) -> np.ndarray:
    """The modes whose continuous-time eigenvalue omega_j = log(lambda_j) / dt (Section
    2.2, eq. omegaj; dt = 1, principal branch) lies strictly inside the disc |omega| < thr,
    in index order.  Conjugate partners have conjugate omega and are kept or dropped
    together."""
    return np.flatnonzero(np.abs(np.log(lam.astype(np.complex128))) < thr)


def refit(Phi_S: np.ndarray, x1: np.ndarray) -> np.ndarray:
    """Amplitudes of x_1 on a fixed support: argmin over beta of ||x_1 - Phi_S beta||_2
    (the least-squares problem of eq. (eq:b) restricted to the selected modes)."""
    return np.linalg.lstsq(Phi_S, x1.astype(np.complex128), rcond=None)[0]


# ---------------------------------------------------------------- reconstruction
def vandermonde(lam: np.ndarray, t0: int, t1: int) -> np.ndarray:
    """V[j, t] = lambda_j^(t-1) for frames t = t0+1 .. t1 (1-based), by repeated
    multiplication (0^0 = 1)."""
    lam = np.asarray(lam, dtype=np.complex128)
    if np.any(np.abs(lam) > 1.0) and np.max(np.abs(lam)) ** max(t1 - 1, 0) > VANDER_MAX:
        raise NumericError("|lambda|^(m-1) overflows")
    V = np.empty((lam.size, t1), dtype=np.complex128)
    if t1:
        V[:, 0] = 1.0
    for t in range(1, t1):
        V[:, t] = V[:, t - 1] * lam
    return V[:, t0:t1]


def background(Phi_S: np.ndarray, beta: np.ndarray, lam_S: np.ndarray, t0: int, t1: int,
               static: bool = False) -> np.ndarray:
    """L = Re(Phi_S diag(beta) V_S) for frames [t0, t1) (eq. equ:DMDTerms, real part),
    or the static model Re(Phi_S beta) (Section 2.3) when ``static``."""
    if static:
        return (Phi_S @ beta).real
    return (Phi_S @ (beta[:, None] * vandermonde(lam_S, t0, t1))).real


def foreground(x: np.ndarray, L: np.ndarray, tau: float) -> np.ndarray:
    """eq. (eq:thres): 1 where |x - xhat| > tau (strict); NaN gives 0."""
    with np.errstate(invalid="ignore"):
        return np.abs(x - L) > tau


def median3(mask: np.ndarray, H: int, W: int) -> np.ndarray:
    """Post-processing of the foreground masks (Section 4, the BMC evaluation: the
    thresholded masks are in addition median filtered; the paper gives no window, the
    reading here is 3x3 with the border replicated): per frame of the frame-major (m, H W)
    binary mask, the median of each pixel's nine neighbours, which for binary values is
    their majority."""
    m = mask.shape[0]
    f = np.asarray(mask).reshape(m, H, W).astype(np.int32)
    g = np.pad(f, ((0, 0), (1, 1), (1, 1)), mode="edge")
    cnt = sum(g[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W] for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    return (cnt >= 5).reshape(m, H * W)


def prf(mask: np.ndarray, gt: np.ndarray):
    """Recall TP/(TP+FN), precision TP/(TP+FP), F = 2PR/(P+R); 0 on empty
    denominators (Section 4)."""
    mask = np.asarray(mask, bool)
    gt = np.asarray(gt, bool)
    tp = float(np.count_nonzero(mask & gt))
    fp = float(np.count_nonzero(mask & ~gt))
    fn = float(np.count_nonzero(~mask & gt))
    R = tp / (tp + fn) if tp + fn else 0.0
    P = tp / (tp + fp) if tp + fp else 0.0
    F = 2 * P * R / (P + R) if P + R else 0.0
    return R, P, F


# ---------------------------------------------------------------- driver
@dataclasses.dataclass
class Pipeline:
    model: Model
    Yhat: np.ndarray
    support: np.ndarray
    beta: np.ndarray


def run(D: np.ndarray, scale: float, k: int, *, sketch: str, p: int = 0,
        idx: Optional[np.ndarray] = None, sign: Optional[np.ndarray] = None,
        seed: int = 0, K: int = 10, selector: str = "omp") -> Pipeline:
    """Sketch -> fit -> selection, all in float64 (the stages before the mask).  For
    the SRFT sketch ``idx`` holds the kept DFT rows."""
    if sketch in ("sparse", "spixel"):
        Yhat, _ = sketch_sparse(D, scale, idx, sign)
    elif sketch == "gaussian":
        Yhat = sketch_gaussian(D, scale, seed, p)
    elif sketch == "srft":
        Yhat = sketch_srft(D, scale, idx, seed)
    else:
        raise ValueError(sketch)
    mdl = fit(D, scale, Yhat, k)
    x1 = D[0].astype(np.float64) * scale
    if selector == "omp":
        S, beta = omp(mdl.Phi, x1, K, lam=mdl.lam)
    elif selector == "zero_mode":
        S = select_zero_mode(mdl.lam)
        beta = mdl.b[S]
    elif selector == "all":
        S = np.arange(k)
        beta = mdl.b
    else:
        raise ValueError(selector)
    return Pipeline(mdl, Yhat, S, beta)


def f_measure(mask: np.ndarray, gt: np.ndarray) -> float:
    """F-measure of a foreground mask against ground truth (Section "Results" evaluation:
    recall TP/(TP+FN), precision TP/(TP+FP), F = 2PR/(P+R)); a zero denominator gives 0."""
    mask = np.asarray(mask, dtype=bool)
    gt = np.asarray(gt, dtype=bool)
    tp = float(np.count_nonzero(mask & gt))
    fp = float(np.count_nonzero(mask & ~gt))
    fn = float(np.count_nonzero(~mask & gt))
    rec = tp / (tp + fn) if tp + fn > 0 else 0.0
    pre = tp / (tp + fp) if tp + fp > 0 else 0.0
    return 2 * pre * rec / (pre + rec) if pre + rec > 0 else 0.0
