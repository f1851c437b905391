"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a brute-force
construction, a closed form, a known input decomposition, an invariance, a textbook
property or an independent library routine.
"""
import os

import numpy as np
import pytest
import scipy.stats
import torch

import synthvideo as sv
from oracle import cdmd_ref as R
from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ helpers (inputs)
def lowrank_video(n, m, n_pairs, reals=(), seed=0, static=True):
    """x_t = s + sum_j Re(psi_j mu_j^(t-1)) + sum_r d_r nu_r^(t-1), exactly DMD-
    representable.  Returns D (m, n), true eigenvalues, true b_j phi_j columns."""
    rng = np.random.default_rng(seed)
    lam, cols = [], []
    X = np.zeros((n, m))
    t = np.arange(m)
    if static:
        s = rng.uniform(0.2, 0.6, n)
        X += s[:, None]
        lam.append(1.0 + 0j)
        cols.append(s.astype(complex))
    for _ in range(n_pairs):
        psi = rng.normal(size=n) + 1j * rng.normal(size=n)
        mu = rng.uniform(0.9, 1.0) * np.exp(1j * rng.uniform(0.05, 1.0))
        X += (psi[:, None] * mu ** t[None, :]).real
        lam += [mu, np.conj(mu)]
        cols += [psi / 2, np.conj(psi) / 2]
    for nu in reals:
        d = rng.normal(size=n)
        X += d[:, None] * nu ** t[None, :]
        lam.append(complex(nu))
        cols.append(d.astype(complex))
    return X.T.copy(), np.array(lam), np.stack(cols, axis=1)


def match(a, b):
    """Optimal matching of two eigenvalue lists (Hungarian on |a_i - b_j|)."""
    from scipy.optimize import linear_sum_assignment
    C = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(C)
    return r, c, C[r, c]


def dense_from_table(idx, sign, n):
    C = np.zeros((idx.shape[0], n))
    for r in range(idx.shape[0]):
        for j in range(idx.shape[1]):
            if idx[r, j] >= 0:
                C[r, idx[r, j]] = sign[r, j]
    return C


# ------------------------------------------------------------------ P9: Philox KAT
def test_philox_kat_golden():
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        out = philox.philox4x32_10(*w[0:4], w[4], w[5])
        assert [int(o) for o in out] == w[6:10]


def test_box_muller_moments_and_ks():
    z = philox.gaussian_block(seed=12345, r0=0, r1=200, j0=0, j1=5000).ravel()
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # neighbouring pixels / rows are uncorrelated
    Z = philox.gaussian_block(seed=7, r0=0, r1=400, j0=0, j1=400)
    assert abs(np.corrcoef(Z[:, :-1].ravel(), Z[:, 1:].ravel())[0, 1]) < 0.02
    assert abs(np.corrcoef(Z[:-1].ravel(), Z[1:].ravel())[0, 1]) < 0.02


def test_gaussian_block_subranges_consistent():
    full = philox.gaussian_block(99, 0, 9, 0, 37)
    part = philox.gaussian_block(99, 3, 7, 5, 30)
    np.testing.assert_array_equal(full[3:7, 5:30], part)


# ------------------------------------------------------------------ rounding formats
def test_round_bf16_matches_torch():
    z = np.random.default_rng(0).normal(size=20000) * 3.0
    z = z.astype(np.float32).astype(np.float64)     # torch rounds from float32
    ref = torch.from_numpy(z.astype(np.float32)).to(torch.bfloat16).float().double().numpy()
    np.testing.assert_array_equal(R.round_bf16(z), ref)


def test_round_e4m3_matches_torch():
    z = np.random.default_rng(1).normal(size=20000) * 40.0
    z = z[np.abs(z) < 448]
    z = np.concatenate([z, [2.0 ** -9, 1.5 * 2.0 ** -9, 0.0, 1.0625, 1.1875]])
    z = z.astype(np.float32).astype(np.float64)     # torch rounds from float32
    ref = torch.from_numpy(z.astype(np.float32)).to(torch.float8_e4m3fn).float().double().numpy()
    np.testing.assert_array_equal(R.round_e4m3(z), ref)
    assert list(R.round_e4m3(np.array([1e4, -1e4]))) == [448.0, -448.0]
    # one rounding step from float64 (no detour through float32)
    assert R.round_e4m3(np.array([2.87499996]))[0] == 2.75
    assert R.round_bf16(np.array([1.0 + 2.0 ** -8 + 2.0 ** -30]))[0] == 1.0 + 2.0 ** -7


# ------------------------------------------------------------------ sketches
def test_sparse_sketch_equals_dense_product():
    rng = np.random.default_rng(3)
    D = rng.integers(0, 256, size=(17, 300), dtype=np.uint8)
    idx, sign = sv.sparse_table(300, 23, 32, seed=4)
    Y, Yint = R.sketch_sparse(D, 1 / 255, idx, sign)
    C = dense_from_table(idx, sign, 300)
    Yref = C @ D.T.astype(np.float64)
    np.testing.assert_array_equal(Yint, Yref.astype(np.int64))
    np.testing.assert_allclose(Y, Yref / 255, rtol=1e-15)


def test_iid_sparse_sketch_equals_dense_product():
    """The i.i.d. very sparse C of Section 3.3 (s = n / ln n, rows padded with -1): the
    sketch is the explicit dense product, and the entries have the stated law (mean
    nonzeros per row n/s, symmetric signs)."""
    rng = np.random.default_rng(4)
    n, m, p = 5000, 12, 400
    D = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
    s = n / np.log(n)
    idx, sign = sv.iid_sparse_table(n, p, s, seed=11)
    assert (idx < 0).any() and (idx >= 0).sum(axis=1).min() >= 0
    C = dense_from_table(idx, sign, n)
    Yf, Yi = R.sketch_sparse(D, 1.0, idx, sign)
    np.testing.assert_array_equal(Yi, (C @ D.T.astype(np.float64)).astype(np.int64))
    nz = (idx >= 0).sum()
    assert abs(nz / p - np.log(n)) < 5 * np.sqrt(np.log(n) / p)
    sg = sign[idx >= 0]
    assert abs((sg == 1).mean() - 0.5) < 5 * 0.5 / np.sqrt(nz)
    for r in range(p):
        row = idx[r][idx[r] >= 0]
        assert len(np.unique(row)) == len(row)


def test_gaussian_sketch_equals_dense_product():
    rng = np.random.default_rng(5)
    D = rng.random((9, 1000)).astype(np.float32)
    Y = R.sketch_gaussian(D, 1.0, seed=77, p=30, chunk=128)
    C = philox.gaussian_block(77, 0, 30, 0, 1000) / np.sqrt(30)
    np.testing.assert_allclose(Y, C @ D.T.astype(np.float64), rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ P1: brute-force DMD
def test_bruteforce_dmd_tiny():
    rng = np.random.default_rng(11)
    n, m = 12, 8
    D = rng.normal(size=(m, n))
    x = D.T
    idx = np.arange(n, dtype=np.int32)[:, None]           # C = I
    Y, _ = R.sketch_sparse(D, 1.0, idx, np.ones((n, 1), np.int8))
    k = m - 1
    mdl = R.fit(D, 1.0, Y, k)
    ev, Ahat = R.dmd_bruteforce(x[:, :-1], x[:, 1:])
    ev = ev[np.argsort(-np.abs(ev))][:k]                  # the nonzero ones
    _, _, err = match(mdl.lam, ev)
    assert err.max() < 1e-10
    for j in range(k):                                    # A^ phi = lambda phi
        ph = mdl.Phi[:, j]
        assert np.linalg.norm(Ahat @ ph - mdl.lam[j] * ph) < 1e-9 * np.linalg.norm(ph)


def test_single_pixel_full_permutation_equals_identity():
    D, lam_true, _ = lowrank_video(60, 15, 3, seed=2)
    k = 7
    I = np.arange(60, dtype=np.int32)[:, None]
    Pm, sgn = sv.single_pixel_table(60, 60, seed=9)
    a = R.fit(D, 1.0, R.sketch_sparse(D, 1.0, I, np.ones((60, 1), np.int8))[0], k)
    b = R.fit(D, 1.0, R.sketch_sparse(D, 1.0, Pm, sgn)[0], k)
    np.testing.assert_allclose(a.lam, b.lam, atol=1e-12)
    np.testing.assert_allclose(a.Phi * a.b, b.Phi * b.b, atol=1e-10)


# ------------------------------------------------------------------ P4: low rank
@pytest.mark.parametrize("kind", ["gaussian", "sparse"])
@pytest.mark.parametrize("mult", [1, 2, 10])
def test_cdmd_equals_dmd_on_exactly_low_rank(kind, mult):
    n, m = 400, 30
    D, lam_true, _ = lowrank_video(n, m, 3, reals=(0.97,), seed=21)
    r = len(lam_true)
    p = mult * r
    if kind == "gaussian":
        Y = R.sketch_gaussian(D, 1.0, seed=5, p=p)
    else:
        idx, sign = sv.sparse_table(n, p, 32, seed=6)
        Y = R.sketch_sparse(D, 1.0, idx, sign)[0]
    mdl = R.fit(D, 1.0, Y, r)
    ev, _ = R.dmd_bruteforce(D.T[:, :-1], D.T[:, 1:])
    ev = ev[np.argsort(-np.abs(ev))][:r]
    _, _, err = match(mdl.lam, ev)
    assert err.max() < 1e-9
    lam_d, Phi_d, b_d = R.dmd_exact(D.T, r)
    ri, ci, _ = match(mdl.lam, lam_d)
    np.testing.assert_allclose(mdl.Phi[:, ri] * mdl.b[ri], Phi_d[:, ci] * b_d[ci], atol=1e-8)


# ------------------------------------------------------------------ SRFT (Section 3.3)
def test_srft_sketch_fft_route_equals_the_definition():
    """The FFT route of the SRFT sketch equals C X with C = R F D / sqrt(p) built entry
    by entry from the definition, F(f, j) = exp(-2 pi i f j / n)."""
    rng = np.random.default_rng(3)
    n, m, p, seed = 45, 7, 11, 12345
    D = rng.integers(0, 256, size=(m, n)).astype(np.uint8)
    freqs = rng.choice(n, size=p, replace=False)
    d = R.srft_diagonal(seed, n)
    F = np.array([[np.exp(-2j * np.pi * f * j / n) for j in range(n)] for f in range(n)])
    C = F[freqs] * d[None, :] / np.sqrt(p)
    np.testing.assert_allclose(R.sketch_srft(D, 1 / 255, freqs, seed), C @ (D.T / 255.0), atol=1e-13)


def test_srft_full_transform_is_unitary():
    """With every DFT row kept (p = n), C = F D / sqrt(n) is unitary: each frame keeps its
    norm (Parseval), and the sketch's Gram equals the video's."""
    rng = np.random.default_rng(4)
    n, m = 64, 9
    D = rng.normal(size=(m, n))
    Y = R.sketch_srft(D, 1.0, np.arange(n), 77)
    np.testing.assert_allclose(np.linalg.norm(Y, axis=0), np.linalg.norm(D, axis=1), rtol=1e-13)
    np.testing.assert_allclose(Y.conj().T @ Y, D @ D.T, atol=1e-11)


def test_srft_diagonal_unit_modulus_and_uniform_phases():
    d = R.srft_diagonal(9, 40000)
    np.testing.assert_allclose(np.abs(d), 1.0, rtol=1e-15)
    u = np.angle(d) / (2 * np.pi) % 1.0
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-3
    # sub-ranges draw the same entries as the whole
    np.testing.assert_array_equal(philox.srft_uniforms(9, 13, 101), philox.srft_uniforms(9, 0, 200)[13:101])


@pytest.mark.parametrize("mult", [1, 2, 5])
def test_srft_cdmd_recovers_real_dynamics(mult):
    """A complex sketch of an exactly low-rank real video: the cDMD eigenvalues are the
    video's (conjugate pairs included) and b_j phi_j its mode columns, to 1e-9."""
    n, m = 500, 30
    D, lam_true, cols = lowrank_video(n, m, 3, reals=(0.97,), seed=22)
    r = len(lam_true)
    freqs = np.random.default_rng(5).choice(n, size=mult * r, replace=False)
    Y = R.sketch_srft(D, 1.0, freqs, 31)
    assert np.iscomplexobj(Y)
    mdl = R.fit(D, 1.0, Y, r)
    ri, ci, err = match(mdl.lam, lam_true)
    assert err.max() < 1e-9
    np.testing.assert_allclose(mdl.Phi[:, ri] * mdl.b[ri], cols[:, ci], atol=1e-8)


# ------------------------------------------------------------------ P5: known modes
def test_recovers_known_modes_from_generator():
    spec = sv.preset("cfg1", exact=True, out="f64", H=60, W=80, m=60, bump_sigma=6.0,
                     blur_sigma=3.0, seed=31, drift=(0.97, 0.99))
    v = sv.make_video(spec)
    D = v.D.numpy()
    k = len(v.bg_lambda)
    Y = R.sketch_gaussian(D, 1.0, seed=8, p=60)
    mdl = R.fit(D, 1.0, Y, k)
    ri, ci, err = match(mdl.lam, v.bg_lambda)
    assert err.max() < 1e-10
    got = mdl.Phi[:, ri] * mdl.b[ri]
    np.testing.assert_allclose(got, v.bg_modes[:, ci], atol=1e-9)
    L = R.background(mdl.Phi, mdl.b, mdl.lam, 0, spec.m)
    np.testing.assert_allclose(L, D.T, atol=1e-9)


def test_recovers_known_modes_lowrank_sparse_sketch():
    D, lam_true, cols = lowrank_video(3000, 40, 4, reals=(0.95,), seed=41)
    idx, sign = sv.sparse_table(3000, 120, 32, seed=3)
    mdl = R.fit(D, 1.0, R.sketch_sparse(D, 1.0, idx, sign)[0], len(lam_true))
    ri, ci, err = match(mdl.lam, lam_true)
    assert err.max() < 1e-10
    np.testing.assert_allclose(mdl.Phi[:, ri] * mdl.b[ri], cols[:, ci], atol=1e-9)


# ------------------------------------------------------------------ Remark 3: compressed modes
def test_compressed_amplitudes_identity_sketch_equal_full():
    """With C = I (p = n, every pixel sampled once, sign +1) the compressed modes are the
    full modes and y_1 = x_1, so Remark 3 changes nothing: same order, modes, amplitudes
    and OMP support as the full fit."""
    D, _, _ = lowrank_video(80, 20, 3, reals=(0.96,), seed=61)
    D = D + 1e-3 * np.random.default_rng(1).normal(size=D.shape)
    I = np.arange(80, dtype=np.int32)[:, None]
    Y = R.sketch_sparse(D, 1.0, I, np.ones((80, 1), np.int8))[0]
    full = R.fit(D, 1.0, Y, 9)
    comp = R.fit_compressed(Y, 9)
    np.testing.assert_allclose(comp.lam, full.lam, atol=1e-12)
    np.testing.assert_allclose(comp.Phi, full.Phi, atol=1e-10)
    np.testing.assert_allclose(comp.b, full.b, atol=1e-10)
    Sf, bf = R.omp(full.Phi, D[0], 4, lam=full.lam)
    Sc, bc = R.omp(comp.Phi, Y[:, 0], 4, lam=comp.lam)
    assert list(Sf) == list(Sc)
    np.testing.assert_allclose(bc, bf, atol=1e-10)


def test_compressed_modes_are_sketched_full_modes():
    """Phi_Y = Y' V S^-1 W = C X' V S^-1 W = C Phi for the same V, S, W, and on exactly
    DMD-representable data b_j phi_Y,j = C (b_j phi_j) for the generator's modes (the
    sketch of a mode's contribution to x_1)."""
    n, m = 3000, 40
    D, lam_true, cols = lowrank_video(n, m, 4, reals=(0.95,), seed=41)
    idx, sign = sv.sparse_table(n, 120, 32, seed=3)
    C = dense_from_table(idx, sign, n)
    Y = R.sketch_sparse(D, 1.0, idx, sign)[0]
    r = len(lam_true)
    comp = R.fit_compressed(Y, r)   # (its canonical order may differ from the full fit's)
    ri, ci, err = match(comp.lam, lam_true)
    assert err.max() < 1e-10
    np.testing.assert_allclose(comp.Phi[:, ri] * comp.b[ri], C @ cols[:, ci], atol=1e-8)
    # the compressed modes are C times the full modes built from the same G
    Phi_full_same_G = D.T[:, 1:] @ comp.G
    np.testing.assert_allclose(comp.Phi, C @ Phi_full_same_G, atol=1e-8)


# ------------------------------------------------------------------ P7: invariances
def test_invariance_to_sketch_scale():
    D, lam_true, _ = lowrank_video(500, 25, 2, seed=51)
    D = D + 1e-3 * np.random.default_rng(0).normal(size=D.shape)   # full rank
    Y = R.sketch_gaussian(D, 1.0, seed=3, p=50)
    a = R.fit(D, 1.0, Y, 8)
    b = R.fit(D, 1.0, 37.5 * Y, 8)
    np.testing.assert_allclose(a.lam, b.lam, rtol=1e-12)
    np.testing.assert_allclose(a.Phi * a.b, b.Phi * b.b, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(a.Phi, 37.5 * b.Phi, rtol=1e-9, atol=1e-12)
    La = R.background(a.Phi, a.b, a.lam, 0, 25)
    Lb = R.background(b.Phi, b.b, b.lam, 0, 25)
    np.testing.assert_allclose(La, Lb, atol=1e-11)


def test_rank_deficient_constant_video():
    D = np.full((10, 200), 100, dtype=np.uint8)
    idx, sign = sv.sparse_table(200, 20, 8, seed=1)
    Y = R.sketch_sparse(D, 1 / 255, idx, sign)[0]
    with pytest.raises(R.RankDeficient):
        R.fit(D, 1 / 255, Y, 2)
    R.fit(D, 1 / 255, Y, 1)        # rank one is fine


# ------------------------------------------------------------------ P6: OMP
def test_omp_full_support_equals_lstsq():
    D, lam_true, _ = lowrank_video(800, 30, 3, seed=61)
    D = D + 1e-2 * np.random.default_rng(1).normal(size=D.shape)
    mdl = R.fit(D, 1.0, R.sketch_gaussian(D, 1.0, 2, 60), 10)
    x1 = D[0]
    S, beta = R.omp(mdl.Phi, x1, K=10)
    full = np.zeros(10, complex)
    full[S] = beta
    np.testing.assert_allclose(full, mdl.b, rtol=1e-8, atol=1e-10)


def test_omp_orthonormal_dictionary_picks_largest_coefficients():
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.normal(size=(200, 12)) + 1j * rng.normal(size=(200, 12)))
    coef = rng.normal(size=12) + 1j * rng.normal(size=12)
    x = Q @ coef
    S, beta = R.omp(Q * 3.0, x, K=4)           # column scaling must not matter
    assert set(S) == set(np.argsort(-np.abs(coef))[:4])
    np.testing.assert_allclose(3.0 * beta, coef[S], rtol=1e-10)


def test_omp_exact_sparse_recovery():
    rng = np.random.default_rng(8)
    A = rng.normal(size=(300, 40)) + 1j * rng.normal(size=(300, 40))
    true = np.array([3, 17, 29])
    coef = np.array([2.0, -1.5 + 0.5j, 1.0j])
    x = A[:, true] @ coef
    S, beta = R.omp(A, x, K=3)
    assert sorted(S) == sorted(true)
    np.testing.assert_allclose(beta[np.argsort(S)], coef[np.argsort(true)], rtol=1e-10)


def test_omp_tie_rule_lowest_index():
    e = np.eye(4, dtype=complex)
    x = np.array([1.0, 1.0, 0.5, 0.0])
    S, _ = R.omp(e, x, K=1)
    assert list(S) == [0]


def test_omp_conjugate_pair_tie_goes_to_positive_imaginary_member():
    """Real x_1 and a conjugate pair of atoms: the first correlations are equal by
    symmetry (|conj(a)^H x| = |a^H x| for real x), and the pick goes to the member with
    Im lambda > 0 wherever it sits; once one member is in, the residual is complex and
    the partner is an ordinary candidate.  Without eigenvalues no pairing is known and
    the first maximum wins."""
    rng = np.random.default_rng(12)
    n = 400
    a = rng.normal(size=n) + 1j * rng.normal(size=n)
    c = rng.normal(size=n)
    x1 = (1.5 * a).real + 0.05 * c
    mu = 0.97 * np.exp(0.4j)
    for order in ([0, 1, 2], [1, 0, 2], [2, 1, 0]):
        cols = [a, np.conj(a), c + 0j]
        lams = [mu, np.conj(mu), 0.5 + 0j]
        Phi = np.stack([cols[i] for i in order], axis=1)
        lam = np.array([lams[i] for i in order])
        gaps = []
        S, _ = R.omp(Phi, x1, K=3, lam=lam, margins=gaps)
        first = order.index(0)                 # where the Im > 0 member sits
        assert S[0] == first, (order, S)
        assert S[1] == order.index(1)          # its partner completes the pair next
        assert gaps[0] > 0.1                   # the real atom is far behind the pair
    # the partners' correlations really are equal to rounding
    corr = np.abs(np.stack([a, np.conj(a)]).conj() @ x1) / np.linalg.norm(a)
    assert abs(corr[0] - corr[1]) <= 1e-12 * corr[0]


def test_omp_margins_flag_a_near_tie():
    """Two atoms with correlations 1 and 1 - 1e-7: the first pick's margin is 1e-7."""
    e = np.eye(3, dtype=complex)
    x = np.array([1.0, 1.0 - 1e-7, 0.25])
    gaps = []
    S, _ = R.omp(e, x, K=2, margins=gaps)
    assert list(S) == [0, 1]
    np.testing.assert_allclose(gaps[0], 1e-7, rtol=1e-6)
    np.testing.assert_allclose(gaps[1], 1.0 - 0.25 / (1.0 - 1e-7), rtol=1e-9)


# ------------------------------------------------------------------ omega selector, refit
def test_select_omega_hand_values():
    """|omega| = |log lambda| with the principal branch, worked by hand for each lambda:
    1 -> 0; exp(+-0.25i) -> 0.25 (conjugates go together); 0.9 -> -ln 0.9 = 0.1053605...;
    -1 -> |i pi| = pi; 0.8 exp(+-0.3i) -> sqrt(ln(0.8)^2 + 0.09) = 0.3738891; 2i -> |ln 2 +
    i pi/2| = 1.7169316; e^0.5 -> 0.5.  Thresholds just below and above each value,
    and the strict inequality at 0 (lambda = 1 has |omega| = 0, not < 0)."""
    lam = np.array([1.0, np.exp(0.25j), np.exp(-0.25j), 0.9, -1.0, 0.8 * np.exp(0.3j),
                    0.8 * np.exp(-0.3j), 2j, np.exp(0.5)], dtype=np.complex128)
    d = 1e-9
    cases = {
        0.0: [],
        d: [0],
        0.1053605 - d: [0],
        0.1053606: [0, 3],
        0.25 - d: [0, 3],
        0.25 + d: [0, 1, 2, 3],
        0.3738890: [0, 1, 2, 3],
        0.3738891: [0, 1, 2, 3, 5, 6],
        0.5 + d: [0, 1, 2, 3, 5, 6, 8],
        1.7169316: [0, 1, 2, 3, 5, 6, 7, 8],
        np.pi - d: [0, 1, 2, 3, 5, 6, 7, 8],
        np.pi + d: list(range(9)),
    }
    for thr, want in cases.items():
        assert list(R.select_omega(lam, thr)) == want, (thr, R.select_omega(lam, thr))


def test_refit_hand_solved_and_conjugate_transpose():
    """Two cases worked by hand.  Phi = [[1, i], [0, 1], [0, 0]], x = (1, 2, 3):
    Phi beta = (b1 + i b2, b2, 0), so b2 = 2, b1 = 1 - 2i (residual (0, 0, 3)).
    phi = (1, i, 1), x = (1, 1, 0): beta = phi^H x / phi^H phi = (1 - i) / 3; the plain
    transpose would give phi^T x / phi^T phi = (1 + i) / 1."""
    Phi = np.array([[1, 1j], [0, 1], [0, 0]], dtype=np.complex128)
    np.testing.assert_allclose(R.refit(Phi, np.array([1.0, 2.0, 3.0])), [1 - 2j, 2], atol=1e-14)
    phi = np.array([[1], [1j], [1]], dtype=np.complex128)
    np.testing.assert_allclose(R.refit(phi, np.array([1.0, 1.0, 0.0])), [(1 - 1j) / 3], atol=1e-15)


def test_refit_orthogonal_dictionary_closed_form():
    """Orthogonal complex columns of norms d_j: beta_j = phi_j^H x / d_j^2, and a
    component of x outside the span does not move beta."""
    rng = np.random.default_rng(31)
    Q, _ = np.linalg.qr(rng.normal(size=(60, 6)) + 1j * rng.normal(size=(60, 6)))
    d = np.array([0.5, 1.0, 2.0, 3.0, 7.0])
    Phi = Q[:, :5] * d[None, :]
    beta_true = np.array([1 + 1j, -2, 0.5j, 3 - 1j, 0.25])
    x = (Phi @ beta_true + 4.0 * Q[:, 5]).real        # complex x would be fine too
    beta_true = Phi.conj().T @ x / d ** 2             # the closed form for the real x
    np.testing.assert_allclose(R.refit(Phi, x), beta_true, atol=1e-12)
    np.testing.assert_allclose(R.refit(Phi[:, [4, 1]], x), beta_true[[4, 1]], atol=1e-12)


# ------------------------------------------------------------------ P11: Vandermonde
def test_vandermonde_closed_form():
    rng = np.random.default_rng(3)
    lam = np.concatenate([np.exp(1j * rng.uniform(0, np.pi, 5)),
                          rng.uniform(0.99, 1.0, 3) * np.exp(1j * rng.uniform(0, 3, 3)), [0.0, 1.0]])
    V = R.vandermonde(lam, 0, 1000)
    np.testing.assert_array_equal(V[:, 0], np.ones(lam.size))
    np.testing.assert_allclose(np.abs(V[:5]), 1.0, rtol=1e-12)
    t = np.arange(1000)
    cf = np.abs(lam)[:, None] ** t[None, :] * np.exp(1j * np.angle(lam)[:, None] * t[None, :])
    cf[-2, 0] = 1.0
    np.testing.assert_allclose(V, cf, rtol=1e-11, atol=1e-300)
    np.testing.assert_array_equal(R.vandermonde(lam, 10, 20), V[:, 10:20])
    with pytest.raises(R.NumericError):
        R.vandermonde(np.array([1.2]), 0, 1000)


# ------------------------------------------------------------------ P10: mask and metrics
def test_mask_zero_on_noise_free_background():
    spec = sv.preset("cfg1", exact=True, out="f64", H=40, W=50, m=30, bump_sigma=5.0,
                     blur_sigma=2.0, seed=3)
    v = sv.make_video(spec)
    D = v.D.numpy()
    mdl = R.fit(D, 1.0, R.sketch_gaussian(D, 1.0, 1, 40), len(v.bg_lambda))
    L = R.background(mdl.Phi, mdl.b, mdl.lam, 0, spec.m)
    assert not R.foreground(D.T, L, 1e-8).any()


def test_mask_strict_and_nan():
    x = np.array([[0.5, 0.6, np.nan, 0.2]])
    L = np.array([[0.4, 0.5, 0.3, 0.2]])
    m = R.foreground(x, L, 0.1)
    # |0.5-0.4| is 0.09999999999999998 in binary, |0.6-0.5| is 0.09999999999999998 too
    assert list(m[0]) == [abs(0.5 - 0.4) > 0.1, abs(0.6 - 0.5) > 0.1, False, False]
    assert list(R.foreground(np.array([0.25]), np.array([0.0]), 0.25)) == [False]


def test_median3_equals_library_median_filter():
    """The mask median filter against scipy's median filter (3x3 window within each
    frame, border replicated), on masks of several densities and odd shapes."""
    import scipy.ndimage
    rng = np.random.default_rng(6)
    for H, W, dens in ((7, 9, 0.5), (16, 33, 0.2), (1, 5, 0.6), (5, 1, 0.4)):
        mk = rng.random((3, H * W)) < dens
        want = scipy.ndimage.median_filter(mk.reshape(3, H, W).astype(np.uint8), size=(1, 3, 3),
                                           mode="nearest").reshape(3, H * W).astype(bool)
        np.testing.assert_array_equal(R.median3(mk, H, W), want)


def test_prf_identities():
    gt = np.array([1, 1, 0, 0, 1], bool)
    assert R.prf(gt, gt) == (1.0, 1.0, 1.0)
    R_, P_, F_ = R.prf(np.array([1, 0, 1, 0, 0], bool), gt)
    assert (R_, P_) == (1 / 3, 1 / 2)
    assert abs(F_ - 2 * (1 / 3) * (1 / 2) / (1 / 3 + 1 / 2)) < 1e-15
    assert R.prf(np.zeros(5, bool), np.zeros(5, bool)) == (0.0, 0.0, 0.0)


# ------------------------------------------------------------------ P13: zero mode
def test_zero_mode_selector_static_video():
    spec = sv.preset("cfg1", exact=True, out="f64", H=30, W=40, m=20, n_pairs=0, seed=4,
                     blur_sigma=2.0)
    v = sv.make_video(spec)
    D = v.D.numpy() + 1e-4 * np.random.default_rng(0).normal(size=(20, 1200))
    mdl = R.fit(D, 1.0, R.sketch_gaussian(D, 1.0, 3, 20), 3)
    S = R.select_zero_mode(mdl.lam)
    assert abs(mdl.lam[S[0]] - 1.0) < 1e-4
    L = R.background(mdl.Phi[:, S], mdl.b[S], mdl.lam[S], 0, 20)
    xhat = R.background(mdl.Phi[:, S], mdl.b[S], mdl.lam[S], 0, 20, static=True)
    assert np.abs(L - xhat[:, None]).max() < 1e-3
    np.testing.assert_allclose(xhat, v.D.numpy()[0], atol=1e-3)


# ------------------------------------------------------------------ canonical order
def test_canonical_order_pairs_positive_imag_first():
    lam = np.array([0.9 - 0.1j, 1.0, 0.9 + 0.1j, 0.5])
    # conjugate members share the larger key even when their keys differ
    key = np.array([2.0, 3.0, 2.0 * (1 - 1e-6), 1.0])
    assert list(R.canonical_order(lam, key)) == [1, 2, 0, 3]
    # a mode whose key falls between the two members does not split the pair
    lam2 = np.array([0.9 - 0.1j, 0.7 + 0j, 0.9 + 0.1j])
    key2 = np.array([2.0, 1.9, 1.8])
    assert list(R.canonical_order(lam2, key2)) == [2, 0, 1]


def test_eigvec_normalisation():
    rng = np.random.default_rng(2)
    W = rng.normal(size=(6, 6)) + 1j * rng.normal(size=(6, 6))
    Wn = R.normalise_eigvecs(W * np.exp(1j * 0.3))
    np.testing.assert_allclose(np.linalg.norm(Wn, axis=0), 1.0)
    piv = np.argmax(np.abs(Wn), axis=0)
    assert np.all(Wn[piv, range(6)].real > 0) and np.allclose(Wn[piv, range(6)].imag, 0)
    # same column up to phase
    ratio = Wn / W
    assert np.allclose(np.abs(ratio / ratio[0:1]), 1.0)


def test_f_measure_definition():
    """Recall, precision and F on a hand-counted example; degenerate cases give 0."""
    gt = np.array([1, 1, 1, 0, 0, 0, 0, 1], dtype=bool)
    mk = np.array([1, 1, 0, 1, 0, 0, 0, 0], dtype=bool)
    # TP 2, FP 1, FN 2: P = 2/3, R = 1/2, F = 2 (1/3) / (7/6) = 4/7
    assert abs(R.f_measure(mk, gt) - 4 / 7) < 1e-15
    assert R.f_measure(np.zeros(8, bool), gt) == 0.0
    assert R.f_measure(gt, gt) == 1.0


# ------------------------------------------------------------------ automatic target rank (Remark 2)
def test_gd_lambda_star_square_case_is_4_over_sqrt3():
    """beta = 1: lambda* = sqrt(4 + 8 / (2 + 4)) = sqrt(16/3) = 4 / sqrt(3)."""
    assert abs(R.gd_lambda_star(1.0) - 4.0 / np.sqrt(3.0)) < 1e-15
    assert abs(R.gd_lambda_star(1e-12) - np.sqrt(2.0)) < 1e-9      # beta -> 0: sqrt(2)


def test_mp_median_against_monte_carlo():
    """The median eigenvalue of W^T W / n for an n x mm Gaussian W (beta = mm / n) converges
    to the Marchenko-Pastur median; at n = 4000 the sample median is within 1e-2."""
    rng = np.random.default_rng(2024)
    for n, mm in ((4000, 1000), (3000, 3000)):
        W = rng.normal(size=(n, mm))
        ev = np.linalg.eigvalsh(W.T @ W / n)
        assert abs(np.median(ev) - R.mp_median(mm / n)) < 1e-2, (n, mm, np.median(ev), R.mp_median(mm / n))


def test_gd_omega_against_the_published_cubic():
    """Gavish and Donoho give omega(beta) ~ 0.56 beta^3 - 0.95 beta^2 + 1.82 beta + 1.43 as an
    approximation; the exact coefficient stays within 0.02 of it over (0, 1], and
    omega(1) = 2.858 (to three decimals)."""
    for beta in (0.05, 0.1, 0.25, 0.5, 0.75, 1.0):
        cubic = 0.56 * beta ** 3 - 0.95 * beta ** 2 + 1.82 * beta + 1.43
        assert abs(R.gd_omega(beta) - cubic) < 0.02, (beta, R.gd_omega(beta), cubic)
    assert abs(R.gd_omega(1.0) - 2.858) < 1e-3


def test_optimal_rank_recovers_planted_rank():
    """A rank-r matrix with singular values far above the noise bulk plus i.i.d. noise: the
    threshold keeps exactly the r planted directions, at two aspect ratios."""
    rng = np.random.default_rng(7)
    for p, m, r in ((2000, 500, 12), (600, 401, 7)):
        U, _ = np.linalg.qr(rng.normal(size=(p, r)))
        V, _ = np.linalg.qr(rng.normal(size=(m, r)))
        sig = np.linspace(400.0, 120.0, r)
        Y = (U * sig) @ V.T + rng.normal(size=(p, m))
        k, tau, s = R.optimal_rank(Y)
        assert k == r, (k, r, tau, s[:r + 2])
        assert s[r - 1] > tau > s[r]
