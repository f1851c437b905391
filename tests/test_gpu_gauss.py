"""Dense Gaussian sketch on the GPU vs the FP64 oracle, through the C ABI.

C is drawn on the device from the same counter-based definition the oracle uses
(Philox4x32-10 + Box-Muller).  Comparisons use the oracle's quantised-C sketch: the
FP64 normals rounded to the form's storage type, then Y^ = C X in float64.

Tolerances
* FP32 form: the device computes the normals in float64 and rounds once to float32, so
  C is the oracle's; products and sums are float32 within a pixel slice of <= 1024 steps
  of 4, float64 across slices.  Per entry |Y_gpu - Y_ref| <= 2^-16 (|C| |X|)_rt, the
  worst-case float32 accumulation bound for 256 additions (256 * 2^-24), with margin.
* BF16 form: the device computes the normals in float32 with the hardware
  transcendentals (relative error ~1e-6), so about 1 in 4000 entries rounds to the
  neighbouring bfloat16 (2^-8 relative); ||Y_gpu - Y_ref||_F <= 1e-4 ||Y_ref||_F.
* eigenvalues against the unquantised FP64 oracle: <= 1e-6 (FP32 form), <= 1e-3
  (BF16 form), the per-form targets.
"""
import numpy as np
import pytest
import torch

import synthvideo as sv
from oracle import cdmd_ref as R
from oracle import philox
from tests.cdmd_testutil import eig_rel_err, mask_agreement

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1512_04205_amd")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _round_f32(z):
    return np.asarray(z, dtype=np.float64).astype(np.float32).astype(np.float64)


def _ref_sketch(D, scale, seed, p, quant):
    m, n = D.shape
    C = quant(philox.gaussian_block(seed, 0, p, 0, n))
    X = D.astype(np.float64).T * scale
    Y = C @ X / np.sqrt(p)
    Yabs = np.abs(C) @ np.abs(X) / np.sqrt(p)
    return Y, Yabs


@pytest.mark.parametrize("case", [
    ("u8", 90, 160, 40, 100),        # dtype, H, W, m, p: 14400 pixels, ragged row tile
    ("u8", 37, 53, 21, 70),          # ragged pixel tail (1961 pixels), m < frame tile
    ("f32", 60, 80, 50, 300),
    ("u8_ld", 30, 50, 30, 64),       # frames with a stride ld > n, not a multiple of 4
])
def test_gaussian_sketch_fp32_form(case):
    kind, H, W, m, p = case
    _say("gauss fp32 sketch", case)
    rng = np.random.default_rng(3)
    n = H * W
    seed = 0x1234_5678_9ABC
    if kind == "f32":
        D = rng.random((m, n), dtype=np.float32)
        dtype, scale, ld = P.F32, 1.0, n
        Dg = torch.from_numpy(D).cuda()
    else:
        D = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
        dtype, scale = P.U8, 1 / 255
        ld = n + 3 if kind == "u8_ld" else n
        buf = torch.zeros((m, ld), dtype=torch.uint8)
        buf[:, :n] = torch.from_numpy(D)
        Dg = buf.cuda()
    mdl = P.Model(n, m, min(5, m - 1), p, sketch=P.SKETCH_GAUSSIAN, dtype=dtype, ld=ld, seed=seed)
    mdl.fit(Dg)
    Yg = mdl.sketch()
    Y, Yabs = _ref_sketch(D, scale, seed, p, _round_f32)
    err = np.abs(Yg - Y)
    assert (err <= 2.0 ** -16 * Yabs + 1e-300).all(), (err / Yabs).max()


@pytest.mark.parametrize("case", [(90, 160, 40, 100), (37, 64, 21, 70), (48, 96, 300, 130),
                                  (40, 64, 200, 70), (30, 32, 129, 65), (20, 48, 560, 64),
                                  (16, 80, 1000, 130)])
def test_gaussian_sketch_bf16_form(case):
    H, W, m, p = case
    _say("gauss bf16 sketch", case)
    rng = np.random.default_rng(4)
    n = H * W
    seed = 99
    D = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
    mdl = P.Model(n, m, min(5, m - 1), p, sketch=P.SKETCH_GAUSSIAN, dtype=P.U8, seed=seed,
                  sketch_prec=P.PREC_BF16)
    mdl.fit(torch.from_numpy(D).cuda())
    Yg = mdl.sketch()
    Y, _ = _ref_sketch(D, 1 / 255, seed, p, R.round_bf16)
    rel = np.linalg.norm(Yg - Y) / np.linalg.norm(Y)
    assert rel <= 1e-4, rel


@pytest.mark.parametrize("case", [(90, 160, 40, 100), (37, 64, 21, 70), (20, 48, 560, 64)])
def test_gaussian_sketch_fp8_form(case):
    """FP8 form: C rounded to e4m3 (the oracle's round_e4m3 of the float64 normals), pixel
    bytes exact (two e4m3 halves).  About 2e-5 of the entries round to the neighbouring
    e4m3 value (2^-3 relative) because the device normals are float32:
    ||Y_gpu - Y_ref||_F <= 3e-3 ||Y_ref||_F."""
    H, W, m, p = case
    _say("gauss fp8 sketch", case)
    rng = np.random.default_rng(6)
    n = H * W
    D = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
    mdl = P.Model(n, m, min(5, m - 1), p, sketch=P.SKETCH_GAUSSIAN, dtype=P.U8, seed=31,
                  sketch_prec=P.PREC_FP8)
    mdl.fit(torch.from_numpy(D).cuda())
    Yg = mdl.sketch()
    Y, _ = _ref_sketch(D, 1 / 255, 31, p, R.round_e4m3)
    rel = np.linalg.norm(Yg - Y) / np.linalg.norm(Y)
    assert rel <= 3e-3, rel


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("case", [(37, 61, 70, 130), (119, 101, 40, 200), (16, 80, 1000, 65)])
def test_stored_c_sketch_equals_drawn(prec, case):
    """cdmd_store_measurement (frame sizes that are not multiples of 8 or 64, ragged row
    tiles, several pixel slices, up to 1000 frames).  The same quantised entries go through
    the library GEMM (BF16; FP8 as two e4m3 parts of each byte), float32 sums in another
    order, so each entry is within the float32 accumulation bound 2^-16 (|C_q| |X|) of the
    drawn form's; the eigenvalues of A~ of these noise videos move by up to a few 1e-6
    under such a change of the sketch (about 1e-7 relative), and are checked within 1e-4, a
    tenth of the BF16 form's target against the oracle.  The autotuner's pick among the
    library's candidate algorithms keeps the bound.  Switching the copy off again gives the
    drawn sketch bit for bit."""
    H, W, m, p = case
    _say("stored C", prec, case)
    sp = P.PREC_BF16 if prec == "bf16" else P.PREC_FP8
    rng = np.random.default_rng(8)
    n = H * W
    ld = (n + 15) // 16 * 16  # the BF16 / FP8 forms read 16-byte aligned frames
    Dh = np.zeros((m, ld), np.uint8)
    Dh[:, :n] = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
    Dh[:, n:] = 255  # bytes past the frame must not enter the sketch
    D = torch.from_numpy(Dh).cuda()
    k = min(5, m - 1)
    a = P.Model(n, m, k, p, sketch=P.SKETCH_GAUSSIAN, dtype=P.U8, seed=77, sketch_prec=sp, ld=ld)
    b = P.Model(n, m, k, p, sketch=P.SKETCH_GAUSSIAN, dtype=P.U8, seed=77, sketch_prec=sp, ld=ld)
    b.store_measurement(True)
    a.fit(D)
    b.fit(D)
    Ya, Yb = a.sketch(), b.sketch()
    quant = R.round_bf16 if prec == "bf16" else R.round_e4m3
    C = quant(philox.gaussian_block(77, 0, p, 0, n))
    Yabs = np.abs(C) @ (Dh[:, :n].astype(np.float64).T / 255.0) / np.sqrt(p)
    err = np.abs(Ya - Yb)
    assert (err <= 2.0 ** -16 * Yabs).all(), (err / Yabs).max()
    rel, _, _ = eig_rel_err(b.modes()["lam"], a.modes()["lam"])
    assert rel.max() <= 1e-4, rel.max()
    # the autotuner picks among the library's candidate GEMM algorithms: the same bound
    b.autotune(D)
    b.fit(D)
    err = np.abs(b.sketch() - Ya)
    assert (err <= 2.0 ** -16 * Yabs).all(), (err / Yabs).max()
    b.store_measurement(False)
    b.fit(D)
    assert np.array_equal(b.sketch(), Ya)


def test_stored_bf16_c_refused_in_batches():
    """A stored BF16 C is streamed by a library GEMM, which batch graphs do not capture."""
    n, m, p = 64 * 40, 30, 50
    g = P.Model(n, m, 5, p, sketch=P.SKETCH_GAUSSIAN, dtype=P.U8, seed=1, sketch_prec=P.PREC_BF16)
    g.store_measurement(True)
    with pytest.raises(P.CdmdError, match="UNSUPPORTED"):
        P.Batch([g])
    g.store_measurement(False)
    b = P.Batch([g])
    # a C stored after the batch was made is refused at the fit
    g.store_measurement(True)
    D = torch.zeros((m, n), dtype=torch.uint8, device="cuda")
    with pytest.raises(P.CdmdError, match="UNSUPPORTED"):
        b.fit([D])
    b.close()


def test_stored_c_refused_for_other_sketches():
    n, m, p = 64 * 40, 30, 50
    idx, sign = sv.sparse_table(n, p, 8, 1)
    sp = P.Model(n, m, 5, p, idx=idx, sign=sign)
    with pytest.raises(P.CdmdError, match="UNSUPPORTED"):
        sp.store_measurement(True)
    g32 = P.Model(n, m, 5, p, sketch=P.SKETCH_GAUSSIAN, dtype=P.U8, seed=1, sketch_prec=P.PREC_FP32)
    with pytest.raises(P.CdmdError, match="UNSUPPORTED"):
        g32.store_measurement(True)


def test_gaussian_fp8_fit():
    """Eigenvalues of the FP8 form against the oracle on the same e4m3-quantised C
    (arithmetic error only: <= 1e-3), and the error the quantisation itself causes against
    the unquantised float64 oracle (reported; below 5e-2 here)."""
    _say("gauss fp8 fit")
    spec = sv.preset("cfg1", H=60, W=80, m=60, bump_sigma=6.0, blur_sigma=3.0, seed=17, rect_side=(8, 8),
                     out="u8")
    v = sv.make_video(spec)
    D = v.D.numpy()
    n, m = D.shape[1], D.shape[0]
    mdl = P.Model(n, m, 10, 300, sketch=P.SKETCH_GAUSSIAN, dtype=P.U8, seed=5, sketch_prec=P.PREC_FP8)
    mdl.fit(torch.from_numpy(D).cuda())
    lam = mdl.modes()["lam"]
    Yq = R.sketch_gaussian(D, v.scale, 5, 300, quantise=R.round_e4m3)
    lam_q = R.fit(D, v.scale, Yq, 10).lam
    rel_q, _, _ = eig_rel_err(lam, lam_q)
    lam_64 = R.run(D, v.scale, 10, sketch="gaussian", p=300, seed=5).model.lam
    rel_64, _, _ = eig_rel_err(lam, lam_64)
    _say("fp8 eig err vs quantised-C oracle", rel_q.max(), "vs float64 oracle", rel_64.max())
    assert rel_q.max() <= 1e-3
    assert rel_64.max() <= 5e-2


def test_gaussian_bf16_needs_aligned_uint8():
    with pytest.raises(P.CdmdError) as e:
        P.Model(1000, 20, 5, 50, sketch=P.SKETCH_GAUSSIAN, dtype=P.F32, sketch_prec=P.PREC_BF16)
    assert e.value.status == P.E_UNSUPPORTED
    mdl = P.Model(1024, 20, 5, 50, sketch=P.SKETCH_GAUSSIAN, dtype=P.U8, sketch_prec=P.PREC_BF16)
    buf = torch.zeros(20 * 1024 + 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.CdmdError) as e:
        mdl.fit(buf[1:1 + 20 * 1024].view(20, 1024))
    assert e.value.status == P.E_UNSUPPORTED


def _fit_gauss(v, k, p, seed, prec, K=6):
    D = v.D.numpy() if v.D.device.type == "cpu" else v.D.cpu().numpy()
    n, m = D.shape[1], D.shape[0]
    dtype = P.U8 if D.dtype == np.uint8 else P.F32
    Dg = torch.from_numpy(D).cuda()
    mdl = P.Model(n, m, k, p, sketch=P.SKETCH_GAUSSIAN, dtype=dtype, seed=seed, sketch_prec=prec)
    mdl.fit(Dg)
    ref = R.run(D, v.scale, k, sketch="gaussian", p=p, seed=seed, K=K)
    return D, Dg, mdl, ref


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_gaussian_fit_and_mask_parity(prec):
    """Small cfg-1-like video (float32 for the FP32 form, uint8 for the BF16 form): modes
    against the unquantised FP64 oracle, then OMP support and masks."""
    _say("gauss fit", prec)
    out = "f32" if prec == "fp32" else "u8"
    spec = sv.preset("cfg1", H=60, W=80, m=60, bump_sigma=6.0, blur_sigma=3.0, seed=17,
                     rect_side=(8, 8), out=out)
    v = sv.make_video(spec)
    pr = P.PREC_FP32 if prec == "fp32" else P.PREC_BF16
    D, Dg, mdl, ref = _fit_gauss(v, k=10, p=300, seed=5, prec=pr)
    md = mdl.modes()
    rel, _, _ = eig_rel_err(md["lam"], ref.model.lam)
    assert rel.max() <= (1e-6 if prec == "fp32" else 1e-3), rel.max()
    S, beta = mdl.select(P.SEL_OMP, K=6)
    if prec == "fp32":
        assert sorted(S) == sorted(ref.support)
    # masks with the oracle's support
    S, beta = mdl.select(P.SEL_EXPLICIT, explicit=ref.support)
    n, m = D.shape[1], D.shape[0]
    mk = torch.zeros((m, P.mask_words(n)), dtype=torch.int32, device="cuda")
    tau = 0.1
    mdl.foreground(Dg, mk, tau)
    L = R.background(ref.model.Phi[:, ref.support], ref.beta, ref.model.lam[ref.support], 0, m)
    x = D.T.astype(np.float64) * v.scale
    mr = R.foreground(x, L, tau)
    words = mk.cpu().numpy().view(np.uint32)
    pix = np.arange(n)
    mg = ((words[:, pix >> 5] >> (pix & 31).astype(np.uint32)) & 1).astype(bool).T
    agree = 1.0 - (mg != mr).mean()
    assert agree >= 0.999, agree


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_gaussian_cfg1_full_size():
    """The 320x240x200 float32 workload with p = 500, k = 10 (FP32 form): eigenvalues
    within 1e-6 of the FP64 oracle, OMP support identical, masks >= 99.9% identical."""
    _say("gauss cfg1 full size")
    v = sv.make_video(sv.PRESETS["cfg1"])
    D, Dg, mdl, ref = _fit_gauss(v, k=10, p=500, seed=1, prec=P.PREC_FP32, K=10)
    md = mdl.modes()
    rel, _, _ = eig_rel_err(md["lam"], ref.model.lam)
    assert rel.max() <= 1e-6, rel.max()
    S, beta = mdl.select(P.SEL_OMP, K=10)
    assert sorted(S) == sorted(ref.support)
    n, m = D.shape[1], D.shape[0]
    mk = torch.zeros((m, P.mask_words(n)), dtype=torch.int32, device="cuda")
    mdl.foreground(Dg, mk, 0.1)
    L = R.background(ref.model.Phi[:, ref.support], ref.beta, ref.model.lam[ref.support], 0, m)
    mr = R.foreground(D.T.astype(np.float64) * v.scale, L, 0.1)
    words = mk.cpu().numpy().view(np.uint32)
    pix = np.arange(n)
    mg = ((words[:, pix >> 5] >> (pix & 31).astype(np.uint32)) & 1).astype(bool).T
    assert 1.0 - (mg != mr).mean() >= 0.999
