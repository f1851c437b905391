"""The SRFT measurement matrix C = R F D / sqrt(p) (Section 3.3) on the GPU against the
FP64 oracle, through the C ABI.

The device draws D's phases from the counter-based definition both sides implement
(Philox4x32-10 on (j >> 2, 0, 0, 1)), forms each entry's phase 2 pi (u_j - (f_r j mod n)/n)
in float64 from the exact integer f_r j mod n, and rounds its cosine and sine once to
float32; products and sums are float32 within a pixel slice (FP32 MFMA), float64 across
slices.  The sketch is complex; the Gram, Lanczos, A~ and its eigenpairs are complex float64
on the host.

Tolerances
* sketch, per entry and part: |Y_gpu - Y_q| <= 2^-16 ((|Re C_q| + |Im C_q|) |X|)_rt against
  the sketch of the float32-rounded C_q built entry by entry (the bound of the Gaussian FP32
  form, whose accumulation is the same kernel), and ||Y_gpu - Y_ref||_F <= 1e-6 ||Y_ref||_F
  against the oracle's float64 FFT route;
* the small linear algebra on the device's own sketch against LAPACK's SVD and eig
  (the oracle's reduced_operator on that sketch): sigma within 1e-10, eigenvalues within
  1e-8, relative;
* eigenvalues against the FP64 oracle: <= 1e-6 (the FP32 form's target); masks with the
  oracle's support >= 99.9% identical;
* the automatic rank: singular values within 1e-9 of LAPACK on the device's sketch, tau*
  within Weyl's bound omega(beta) ||E||_2 of the oracle's.
"""
import numpy as np
import pytest
import torch

import synthvideo as sv
from oracle import cdmd_ref as R
from tests.cdmd_testutil import eig_rel_err

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1512_04205_amd")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _freqs(n, p, seed):
    return np.random.default_rng(seed).choice(n, size=p, replace=False).astype(np.int32)


def _quantised_C(n, freqs, seed):
    """C_q: the definition's entries, real and imaginary parts rounded to float32."""
    d = R.srft_diagonal(seed, n)
    j = np.arange(n, dtype=np.int64)
    C = np.exp(-2j * np.pi * ((freqs.astype(np.int64)[:, None] * j[None, :]) % n) / n) * d[None, :]
    return C.real.astype(np.float32).astype(np.float64) + 1j * C.imag.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("case", [
    ("u8", 40, 60, 30, 50),         # dtype, H, W, m, p: 2400 pixels
    ("u8", 37, 53, 21, 70),         # ragged pixel tail, m below one frame tile
    ("f32", 30, 64, 40, 64),
    ("u8", 64, 96, 300, 40),        # two frame tiles
])
def test_srft_sketch(case):
    kind, H, W, m, p = case
    _say("srft sketch", case)
    rng = np.random.default_rng(8)
    n = H * W
    seed = 0xABCDEF0123
    if kind == "f32":
        D = rng.random((m, n), dtype=np.float32)
        dtype, scale = P.F32, 1.0
    else:
        D = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
        dtype, scale = P.U8, 1 / 255
    fr = _freqs(n, p, 3)
    mdl = P.Model(n, m, min(5, m - 1), p, sketch=P.SKETCH_SRFT, dtype=dtype, idx=fr.reshape(p, 1), seed=seed)
    mdl.fit(torch.from_numpy(D).cuda())
    Yg = mdl.sketch()
    assert Yg.shape == (p, m) and np.iscomplexobj(Yg)
    Cq = _quantised_C(n, fr, seed)
    X = D.astype(np.float64).T * scale
    Yq = Cq @ X / np.sqrt(p)
    Yabs = (np.abs(Cq.real) + np.abs(Cq.imag)) @ np.abs(X) / np.sqrt(p)
    for part in (np.real, np.imag):
        err = np.abs(part(Yg) - part(Yq))
        assert (err <= 2.0 ** -16 * Yabs + 1e-300).all(), (err / Yabs).max()
    Yref = R.sketch_srft(D, scale, fr, seed)
    assert np.linalg.norm(Yg - Yref) <= 1e-6 * np.linalg.norm(Yref)


def _video(H=48, W=64, m=60, seed=17, out="u8"):
    spec = sv.preset("cfg1", H=H, W=W, m=m, bump_sigma=6.0, blur_sigma=3.0, seed=seed, rect_side=(8, 8), out=out)
    return sv.make_video(spec)


@pytest.mark.parametrize("out", ["u8", "f32"])
def test_srft_fit_mask_parity(out):
    """A small video: the complex small linear algebra on the device's own sketch against
    LAPACK, the modes against the FP64 oracle, OMP support and masks."""
    _say("srft fit", out)
    v = _video(out=out)
    D = v.D.numpy()
    m, n = D.shape
    k, p, K, seed, tau = 10, 200, 6, 77, 0.1
    fr = _freqs(n, p, 9)
    mdl = P.Model(n, m, k, p, sketch=P.SKETCH_SRFT, dtype=P.U8 if out == "u8" else P.F32, idx=fr.reshape(p, 1),
                  seed=seed)
    Dg = torch.from_numpy(D).cuda()
    mdl.fit(Dg)
    md = mdl.modes()
    # the host solve on the device's sketch against LAPACK
    lam_d, _, s_d, _, _ = R.reduced_operator(mdl.sketch(), k)
    np.testing.assert_allclose(md["sigma"], s_d, rtol=1e-10)
    rel, _, _ = eig_rel_err(md["lam"], lam_d)
    assert rel.max() <= 1e-8, rel.max()
    # against the FP64 oracle
    ref = R.run(D, v.scale, k, sketch="srft", idx=fr, seed=seed, K=K)
    rel, _, _ = eig_rel_err(md["lam"], ref.model.lam)
    assert rel.max() <= 1e-6, rel.max()
    S, beta = mdl.select(P.SEL_OMP, K=K)
    assert sorted(S) == sorted(ref.support)
    mdl.select(P.SEL_EXPLICIT, explicit=ref.support)
    mk = torch.zeros((m, P.mask_words(n)), dtype=torch.int32, device="cuda")
    mdl.foreground(Dg, mk, tau)
    L = R.background(ref.model.Phi[:, ref.support], ref.beta, ref.model.lam[ref.support], 0, m)
    mr = R.foreground(D.T.astype(np.float64) * v.scale, L, tau)
    mg = P.unpack_mask(mk.cpu().numpy().view(np.uint32), n).T
    agree = 1.0 - (mg != mr).mean()
    assert agree >= 0.999, agree


def test_srft_automatic_rank():
    """Remark 2's rank for the complex SRFT sketch (its Hermitian Gram enters the host
    spectrum code as the real symmetric embedding of twice the order, every eigenvalue
    twice): the singular values equal LAPACK's SVD of the device's own sketch within 1e-9;
    tau* lies within Weyl's bound omega(beta) ||E||_2 of the oracle's (E the device sketch's
    float32 rounding); the rank equals the oracle's unless a singular value lies within
    twice that bound of tau*.  The long-video executor's per-batch rank (the median and one
    Sturm count, without the full spectrum) equals cdmd_optimal_rank's."""
    _say("srft rank")
    v = _video(H=48, W=64, m=150, seed=23)
    D = v.D.numpy()
    m, n = D.shape
    p, seed = 300, 91
    fr = _freqs(n, p, 4).reshape(p, 1)
    Dg = torch.from_numpy(D).cuda()
    k, tau, sig = P.optimal_rank(Dg, n, m, p, sketch=P.SKETCH_SRFT, idx=fr, seed=seed)
    mdl = P.Model(n, m, 5, p, sketch=P.SKETCH_SRFT, idx=fr, seed=seed)
    mdl.fit(Dg)
    Yd = mdl.sketch()
    Yr = R.sketch_srft(D, v.scale, fr.reshape(-1), seed)
    mm = m - 1
    np.testing.assert_allclose(sig, np.linalg.svd(Yd[:, :mm], compute_uv=False), rtol=1e-9,
                               atol=1e-9 * sig[0])
    kr, taur, sr = R.optimal_rank(Yr)
    e2 = np.linalg.norm(Yd[:, :mm] - Yr[:, :mm], 2)
    beta = min(p, mm) / max(p, mm)
    tol = R.gd_omega(beta) * e2 * (1 + 1e-9) + 1e-9 * taur
    assert abs(tau - taur) <= tol, (tau, taur, tol)
    gap = np.min(np.abs(sr - taur))
    _say("k", k, "oracle k", kr, "||E||_2 / sigma_1", e2 / sr[0], "closest sigma to tau", gap / taur)
    if gap > 2 * tol:
        assert k == kr
    assert 1 <= k < min(p, mm)
    # the executor's rank per batch
    mk = torch.zeros((m, P.mask_words(n)), dtype=torch.int32, device="cuda")
    used = P.process_video(Dg, n, m, p, mk, batch_frames=75, k=0, K=4, tau=0.1, workers=1, sketch=P.SKETCH_SRFT,
                           idx=fr, seed=seed)
    for b, t0 in enumerate((0, 75)):
        kb = P.optimal_rank(Dg[t0:t0 + 75], n, 75, p, sketch=P.SKETCH_SRFT, idx=fr, seed=seed)[0]
        assert used[b] == max(1, min(kb, 74, p, 40)), (b, used[b], kb)


@pytest.mark.timeout(600)
def test_srft_at_the_sweep_size():
    """The SRFT fit at the size the sensing sweep times (720x480x200 uint8, p = 1000).  The
    sketch: per entry and part within 2^-16 ((|Re C_q| + |Im C_q|) |X|) of the oracle's
    float64 FFT route (|C_q| accumulated in pixel chunks; float32 sums over slices of about
    10^4 pixels put the Frobenius error near u sqrt(L), about 2e-6 here).  The small linear
    algebra: eigenvalues within 1e-8 of the oracle's reduced operator on the device's own
    sketch, and within 1e-6 (the FP32 form's target) of the oracle on its own sketch
    (measured 4e-7)."""
    _say("srft sweep size")
    v = sv.make_video(sv.PRESETS["ctxB"])
    D = v.D.numpy()
    m, n = D.shape
    p, k, seed = 1000, 20, 31017
    fr = _freqs(n, p, 5)
    mdl = P.Model(n, m, k, p, sketch=P.SKETCH_SRFT, idx=fr.reshape(p, 1), seed=seed)
    mdl.fit(torch.from_numpy(D).cuda())
    Yg = mdl.sketch()
    Yr = R.sketch_srft(D, v.scale, fr, seed)
    d = R.srft_diagonal(seed, n)
    Yabs = np.zeros((p, m))
    for j0 in range(0, n, 16384):
        j1 = min(n, j0 + 16384)
        j = np.arange(j0, j1, dtype=np.int64)
        C = np.exp(-2j * np.pi * ((fr.astype(np.int64)[:, None] * j[None, :]) % n) / n) * d[None, j0:j1]
        Yabs += (np.abs(C.real) + np.abs(C.imag)) @ (D[:, j0:j1].astype(np.float64).T * v.scale)
    Yabs /= np.sqrt(p)
    for part in (np.real, np.imag):
        err = np.abs(part(Yg) - part(Yr))
        assert (err <= 2.0 ** -16 * Yabs).all(), (err / Yabs).max()
    _say("sketch Frobenius rel err", np.linalg.norm(Yg - Yr) / np.linalg.norm(Yr))
    lam = mdl.modes()["lam"]
    lam_d, _, _, _, _ = R.reduced_operator(Yg, k)
    erel, _, _ = eig_rel_err(lam, lam_d)
    assert erel.max() <= 1e-8, erel.max()
    lam_r, _, _, _, _ = R.reduced_operator(Yr, k)
    erel, _, _ = eig_rel_err(lam, lam_r)
    _say("eig rel err against the FP64 oracle", float(erel.max()))
    assert erel.max() <= 1e-6, erel.max()
