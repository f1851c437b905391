"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerances
* sparse / single-pixel sketch of a uint8 video: integer sums, bit-exact;
* eigenvalues: relative error <= 1e-6 per matched mode (FP32 form);
* b_j phi_j, Phi, L: relative to the largest entry of the oracle quantity, 2e-5
  (float32 products and accumulation over m <= 600 frames, ~sqrt(m) * 2^-24 * growth);
* masks: >= 99.9% identical, and every disagreement inside the band
  ||x - L| - tau| <= 10 * (max |L_gpu - L_oracle|) + 1e-6.
"""
import numpy as np
import pytest
import torch

import synthvideo as sv
from oracle import cdmd_ref as R
from tests.cdmd_testutil import NEAR_TIE_FP32, eig_rel_err, mask_agreement

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1512_04205_amd")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _small_u8(H=72, W=100, m=60, seed=7, **kw):
    spec = sv.preset("cfg2", H=H, W=W, m=m, bump_sigma=8.0, blur_sigma=3.0, n_rects=3,
                     rect_side=(6, 14), speed=(0.5, 2.0), seed=seed, **kw)
    return sv.make_video(spec)


def _fit_both(v, k, p, nnz, K=6, table_seed=3, spixel=False):
    D = v.D.numpy() if v.D.device.type == "cpu" else v.D.cpu().numpy()
    n, m = D.shape[1], D.shape[0]
    if spixel:
        idx, sign = sv.single_pixel_table(n, p, table_seed)
    else:
        idx, sign = sv.sparse_table(n, p, nnz, table_seed)
    dtype = P.U8 if D.dtype == np.uint8 else P.F32
    Dg = torch.from_numpy(D).cuda()
    mdl = P.Model(n, m, k, p, sketch=P.SKETCH_SPIXEL if spixel else P.SKETCH_SPARSE, dtype=dtype,
                  idx=idx, sign=sign)
    mdl.fit(Dg)
    ref = R.run(D, v.scale, k, sketch="sparse", idx=idx, sign=sign, K=K)
    return D, Dg, mdl, ref, idx, sign


# ------------------------------------------------------------------ sketch
@pytest.mark.parametrize("shape", [(40, 50, 33, 700, 32), (48, 64, 64, 300, 7),
                                   (30, 41, 17, 9000, 3), (64, 64, 40, 1000, 32)])
def test_sparse_sketch_bit_exact(shape):
    """Both forms of the uint8 sparse sketch (streaming for 16-byte aligned frames, gather
    otherwise or when forced) give the exact integer sums."""
    H, W, m, p, nnz = shape
    _say("sketch", shape)
    rng = np.random.default_rng(1)
    n = H * W
    D = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
    idx, sign = sv.sparse_table(n, p, nnz, seed=5)
    k = min(4, m - 1)
    Yref, Yiref = R.sketch_sparse(D, 1 / 255, idx, sign)
    for gather in (False, True):
        mdl = P.Model(n, m, k, p, idx=idx, sign=sign)
        mdl.force_gather_sketch(gather)
        mdl.fit(torch.from_numpy(D).cuda())
        Y, Yi = mdl.sketch(integer=True)
        np.testing.assert_array_equal(Yi, Yiref)
        np.testing.assert_allclose(Y, Yref, rtol=1e-15, atol=0)


def test_sparse_sketch_streaming_large_p():
    """Several row blocks (p > 8192), frame groups of one, a pixel count that is not a
    multiple of the 8 KB chunk: streaming form, exact."""
    _say("sketch large p")
    rng = np.random.default_rng(2)
    H, W, m, p, nnz = 96, 176, 37, 9000, 4
    n = H * W
    D = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
    idx, sign = sv.sparse_table(n, p, nnz, seed=8)
    mdl = P.Model(n, m, 4, p, idx=idx, sign=sign)
    mdl.fit(torch.from_numpy(D).cuda())
    _, Yi = mdl.sketch(integer=True)
    _, Yiref = R.sketch_sparse(D, 1 / 255, idx, sign)
    np.testing.assert_array_equal(Yi, Yiref)


def test_single_pixel_sketch_bit_exact():
    _say("spixel sketch")
    rng = np.random.default_rng(2)
    m, n, p = 25, 3000, 500
    D = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
    idx, sign = sv.single_pixel_table(n, p, seed=3)
    mdl = P.Model(n, m, 5, p, sketch=P.SKETCH_SPIXEL, idx=idx, sign=sign)
    mdl.fit(torch.from_numpy(D).cuda())
    _, Yi = mdl.sketch(integer=True)
    np.testing.assert_array_equal(Yi, D[:, idx[:, 0]].T.astype(np.int64))


def test_sketch_with_frame_stride():
    _say("sketch ld > n")
    rng = np.random.default_rng(4)
    m, n, ld, p = 20, 1000, 1088, 200
    Dfull = rng.integers(0, 256, size=(m, ld), dtype=np.uint8)
    idx, sign = sv.sparse_table(n, p, 16, seed=2)
    mdl = P.Model(n, m, 4, p, ld=ld, idx=idx, sign=sign)
    Dg = torch.from_numpy(Dfull).cuda()
    mdl.fit(Dg)
    _, Yi = mdl.sketch(integer=True)
    np.testing.assert_array_equal(Yi, R.sketch_sparse(Dfull[:, :n], 1 / 255, idx, sign)[1])


# ------------------------------------------------------------------ fit
@pytest.mark.parametrize("case", ["u8", "u8_ragged", "f32", "spixel"])
def test_fit_parity(case):
    _say("fit", case)
    if case == "u8":
        v = _small_u8()
        D, Dg, mdl, ref, *_ = _fit_both(v, k=12, p=400, nnz=32)
    elif case == "u8_ragged":
        v = _small_u8(H=37, W=53, m=45, seed=9)
        D, Dg, mdl, ref, *_ = _fit_both(v, k=9, p=300, nnz=17)
    elif case == "f32":
        spec = sv.preset("cfg1", H=60, W=80, m=50, bump_sigma=6.0, blur_sigma=3.0, seed=11,
                         rect_side=(8, 8))
        v = sv.make_video(spec)
        D, Dg, mdl, ref, *_ = _fit_both(v, k=10, p=300, nnz=32)
    else:
        v = _small_u8(seed=13)
        D, Dg, mdl, ref, *_ = _fit_both(v, k=10, p=2000, nnz=1, spixel=True)
    md = mdl.modes()
    rel, r, c = eig_rel_err(md["lam"], ref.model.lam)
    assert rel.max() <= 1e-6, rel
    # canonical order agrees with the oracle's except across near-equal keys
    keys = np.abs(ref.model.b) * ref.model.phi_norm
    perm = np.empty(len(r), dtype=int)
    perm[r] = c
    bad = [j for j in range(len(perm))
           if perm[j] != j and abs(keys[perm[j]] - keys[j]) > 1e-5 * keys.max()]
    assert not bad, (perm, keys)
    np.testing.assert_allclose(md["sigma"], ref.model.sigma, rtol=1e-8)
    # b_j ||phi_j|| (invariant) and phi norms
    scale_ref = np.abs(ref.model.b) * ref.model.phi_norm
    np.testing.assert_allclose(np.abs(md["b"]) * md["phi_norm"], scale_ref, rtol=2e-5, atol=2e-5 * scale_ref.max())


def test_modes_phi_and_background():
    _say("modes+background")
    v = _small_u8(seed=21)
    D, Dg, mdl, ref, *_ = _fit_both(v, k=10, p=400, nnz=32)
    n, m, k = D.shape[1], D.shape[0], 10
    phi = torch.zeros((k, n), dtype=torch.complex64, device="cuda")
    md = mdl.modes(video=Dg, phi=phi)
    Pg = phi.cpu().numpy().T.astype(np.complex128)
    bphi_g = Pg * md["b"][None, :]
    bphi_r = ref.model.Phi * ref.model.b[None, :]
    err = np.abs(bphi_g - bphi_r).max() / np.abs(bphi_r).max()
    assert err < 2e-5, err
    # all modes: background equals the DMD reconstruction
    S, beta = mdl.select(P.SEL_ALL)
    L = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    mdl.background(Dg, L)
    Lr = R.background(ref.model.Phi, ref.model.b, ref.model.lam, 0, m)
    errL = np.abs(L.cpu().numpy().T - Lr).max() / np.abs(Lr).max()
    assert errL < 2e-5, errL
    # static model
    xs = torch.zeros(n, dtype=torch.float32, device="cuda")
    mdl.background(Dg, xs, static=True)
    xr = R.background(ref.model.Phi, ref.model.b, ref.model.lam, 0, 1, static=True)
    assert np.abs(xs.cpu().numpy() - xr).max() / np.abs(xr).max() < 2e-5


@pytest.mark.parametrize("selector", ["omp", "zero_mode", "omega", "explicit"])
def test_select_and_mask_parity(selector):
    _say("select", selector)
    v = _small_u8(seed=31, m=80)
    D, Dg, mdl, ref, *_ = _fit_both(v, k=14, p=500, nnz=32, K=8)
    n, m = D.shape[1], D.shape[0]
    mo = ref.model
    x1 = D[0].astype(np.float64) / 255
    if selector == "omp":
        gaps = []
        Sr, br = R.omp(mo.Phi, x1, 8, lam=mo.lam, margins=gaps)
        if min(gaps) >= NEAR_TIE_FP32:
            S, beta = mdl.select(P.SEL_OMP, K=8)
            assert list(S) == list(Sr)
        else:   # a near tie the float32 lift may resolve either way: the oracle's support
            S, beta = mdl.select(P.SEL_EXPLICIT, explicit=Sr)
    elif selector == "zero_mode":
        S, beta = mdl.select(P.SEL_ZERO_MODE)
        Sr = R.select_zero_mode(mo.lam)
        br = mo.b[Sr]
        assert list(S) == list(Sr)
    elif selector == "omega":
        S, beta = mdl.select(P.SEL_OMEGA, omega_thr=0.3)
        Sr = R.select_omega(mo.lam, 0.3)
        br = mo.b[Sr]
        assert list(S) == list(Sr)
    else:
        Sr = np.array([0, 3, 4])
        S, beta = mdl.select(P.SEL_EXPLICIT, explicit=Sr)
        br = R.refit(mo.Phi[:, Sr], x1)
        assert list(S) == list(Sr)
    # |beta_j| ||phi_j|| is invariant to the sign/phase freedom of each mode
    np.testing.assert_allclose(np.abs(beta) * mo.phi_norm[S], np.abs(br) * mo.phi_norm[Sr],
                               rtol=1e-4, atol=1e-4 * np.abs(br * mo.phi_norm[Sr]).max())
    tau = 0.1
    words = P.mask_words(n)
    mk = torch.zeros((m, words), dtype=torch.int32, device="cuda")
    counts = mdl.foreground(Dg, mk, tau, counts=True)
    mg = P.unpack_mask(mk.cpu().numpy().view(np.uint32), n)
    Lr = R.background(mo.Phi[:, Sr], br, mo.lam[Sr], 0, m)
    x = D.T.astype(np.float64) / 255
    mr = R.foreground(x, Lr, tau).T
    L = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    mdl.background(Dg, L)
    lerr = np.abs(L.cpu().numpy() - Lr.T).max()
    frac, inband, nd = mask_agreement(mg, mr, x.T, Lr.T, tau, 10 * lerr + 1e-6)
    assert frac >= 0.999 and inband, (frac, nd, lerr)
    np.testing.assert_array_equal(counts, mg.sum(axis=1))
    # unpacked mask equals the packed one
    m8 = torch.zeros((m, n), dtype=torch.uint8, device="cuda")
    mdl.foreground(Dg, m8, tau, bitpacked=False)
    np.testing.assert_array_equal(m8.cpu().numpy().astype(bool), mg)


def test_exact_recovery_of_generator_modes():
    _say("exact recovery")
    spec = sv.preset("cfg1", exact=True, out="f32", H=64, W=96, m=60, bump_sigma=6.0,
                     blur_sigma=3.0, seed=41)
    v = sv.make_video(spec)
    D = v.D.numpy()
    k = len(v.bg_lambda)
    idx, sign = sv.sparse_table(D.shape[1], 200, 32, 5)
    mdl = P.Model(D.shape[1], D.shape[0], k, 200, dtype=P.F32, idx=idx, sign=sign)
    mdl.fit(torch.from_numpy(D).cuda())
    lam = mdl.modes()["lam"]
    rel, _, _ = eig_rel_err(lam, v.bg_lambda)
    # float32 storage of the frames perturbs the exact low-rank data at 2^-24
    assert rel.max() < 1e-5, rel


def test_determinism():
    _say("determinism")
    v = _small_u8(seed=51)
    D = v.D.numpy()
    idx, sign = sv.sparse_table(D.shape[1], 300, 32, 5)
    out = []
    for _ in range(2):
        mdl = P.Model(D.shape[1], D.shape[0], 10, 300, idx=idx, sign=sign)
        Dg = torch.from_numpy(D).cuda()
        mdl.fit(Dg)
        md = mdl.modes()
        mdl.select(P.SEL_OMP, K=6)
        mk = torch.zeros((D.shape[0], P.mask_words(D.shape[1])), dtype=torch.int32, device="cuda")
        mdl.foreground(Dg, mk, 0.1)
        out.append((md["lam"], md["b"], mk.cpu().numpy()))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    np.testing.assert_array_equal(out[0][2], out[1][2])


def test_error_paths_on_device():
    _say("errors")
    D = np.full((10, 400), 77, dtype=np.uint8)
    idx, sign = sv.sparse_table(400, 40, 8, 1)
    mdl = P.Model(400, 10, 3, 40, idx=idx, sign=sign)
    Dg = torch.from_numpy(D).cuda()
    with pytest.raises(P.CdmdError) as e:
        mdl.fit(Dg)
    assert e.value.status == P.E_RANK_DEFICIENT
    with pytest.raises(P.CdmdError) as e:
        mdl.select(P.SEL_OMP, K=2)
    assert e.value.status == P.E_STATE
    with pytest.raises(P.CdmdError) as e:
        mdl.foreground(Dg, torch.zeros((10, 13), dtype=torch.int32, device="cuda"), 0.1)
    assert e.value.status == P.E_STATE


# ------------------------------------------------------------------ MFMA lift
@pytest.mark.parametrize("shape", [(40, 52, 45), (72, 100, 60), (30, 64, 130)])
def test_mfma_lift_matches_valu_lift_and_oracle(shape):
    """uint8 video: the MFMA lift (3 bf16 terms of G) and the float32 VALU lift give the
    same amplitudes, Phi and OMP support as the oracle (ragged pixel tiles and frame
    chunks included)."""
    H, W, m = shape
    _say("mfma lift", shape)
    v = _small_u8(H=H, W=W, m=m, seed=61)
    D = v.D.numpy()
    n = D.shape[1]
    k, p = 10, 300
    idx, sign = sv.sparse_table(n, p, 32, 7)
    Dg = torch.from_numpy(D).cuda()
    ref = R.run(D, v.scale, k, sketch="sparse", idx=idx, sign=sign, K=6)
    bphi_r = ref.model.Phi * ref.model.b[None, :]
    out = {}
    for path in ("mfma", "valu"):
        mdl = P.Model(n, m, k, p, idx=idx, sign=sign)
        if path == "valu":
            mdl.force_valu_lift(True)
        mdl.fit(Dg)
        phi = torch.zeros((k, n), dtype=torch.complex64, device="cuda")
        md = mdl.modes(video=Dg, phi=phi)
        S, _ = mdl.select(P.SEL_OMP, K=6)
        bphi = phi.cpu().numpy().T.astype(np.complex128) * md["b"][None, :]
        out[path] = (md, S, bphi)
        rel, _, _ = eig_rel_err(md["lam"], ref.model.lam)
        assert rel.max() <= 1e-6
        err = np.abs(bphi - bphi_r).max() / np.abs(bphi_r).max()
        assert err < 2e-5, (path, err)
        assert list(S) == list(ref.support), (path, S, ref.support)
    km = np.abs(out["mfma"][0]["b"]) * out["mfma"][0]["phi_norm"]
    kv = np.abs(out["valu"][0]["b"]) * out["valu"][0]["phi_norm"]
    assert np.abs(km - kv).max() <= 2e-5 * kv.max()


def test_bf16_lift_form():
    """BF16 lift (G rounded to bfloat16, MFMA, float32 accumulation): eigenvalues are
    those of the exact sketch; amplitudes and masks agree with the FP64 oracle to the
    stated bf16 bounds."""
    _say("bf16 lift")
    v = _small_u8(H=64, W=96, m=80, seed=71)
    D = v.D.numpy()
    n, m = D.shape[1], D.shape[0]
    k, p, K, tau = 12, 400, 8, 0.1
    idx, sign = sv.sparse_table(n, p, 32, 9)
    Dg = torch.from_numpy(D).cuda()
    mdl = P.Model(n, m, k, p, idx=idx, sign=sign, lift_prec=P.PREC_BF16)
    mdl.fit(Dg)
    ref = R.run(D, v.scale, k, sketch="sparse", idx=idx, sign=sign, K=K)
    md = mdl.modes()
    rel, _, _ = eig_rel_err(md["lam"], ref.model.lam)
    assert rel.max() <= 1e-3
    key_r = np.abs(ref.model.b) * ref.model.phi_norm
    np.testing.assert_allclose(np.abs(md["b"]) * md["phi_norm"], key_r, rtol=2e-2, atol=2e-2 * key_r.max())
    mdl.select(P.SEL_EXPLICIT, explicit=ref.support)
    mk = torch.zeros((m, P.mask_words(n)), dtype=torch.int32, device="cuda")
    mdl.foreground(Dg, mk, tau)
    mg = P.unpack_mask(mk.cpu().numpy().view(np.uint32), n)
    Lr = R.background(ref.model.Phi[:, ref.support], ref.beta, ref.model.lam[ref.support], 0, m)
    mr = R.foreground(D.T.astype(np.float64) / 255, Lr, tau).T
    assert (mg == mr).mean() >= 0.999


# ------------------------------------------------------------------ device small LA
def test_device_lanczos_row_groups_agree():
    """The device Lanczos split over 1, 2, 3, 7 or the default number of row groups
    (workgroups exchanging their shares through global memory) gives the same Krylov size,
    singular values and eigenvalues, up to the reordering of float64 sums."""
    _say("device Lanczos row groups")
    v = _small_u8(H=64, W=96, m=300, seed=83)
    D = v.D.numpy()
    n, m, k, p = D.shape[1], D.shape[0], 25, 900
    idx, sign = sv.sparse_table(n, p, 32, 6)
    Dg = torch.from_numpy(D).cuda()
    ref = None
    for groups in (1, 2, 3, 7, 0):
        mdl = P.Model(n, m, k, p, idx=idx, sign=sign)
        mdl.la_groups(groups)
        mdl.fit(Dg)
        md, J = mdl.modes(), mdl.info()["lanczos_steps"]
        if ref is None:
            ref = (md, J)
            continue
        assert J == ref[1], (groups, J, ref[1])
        np.testing.assert_allclose(md["sigma"], ref[0]["sigma"], rtol=1e-12, err_msg=f"groups {groups}")
        rel, _, _ = eig_rel_err(md["lam"], ref[0]["lam"])
        assert rel.max() <= 1e-10, (groups, rel.max())


@pytest.mark.parametrize("shape", [(72, 100, 120, 16), (48, 64, 300, 25)])
def test_device_small_la_matches_host_la_and_oracle(shape):
    """The one-workgroup float64 solve (Lanczos + Jacobi, A~, Francis QR, G) gives the
    oracle's eigenvalues and the same amplitudes and supports as the host solve."""
    H, W, m, k = shape
    _say("device small LA", shape)
    v = _small_u8(H=H, W=W, m=m, seed=81)
    D = v.D.numpy()
    n = D.shape[1]
    p = 600
    idx, sign = sv.sparse_table(n, p, 32, 5)
    Dg = torch.from_numpy(D).cuda()
    ref = R.run(D, v.scale, k, sketch="sparse", idx=idx, sign=sign, K=8)
    res = {}
    for path in ("device", "host"):
        mdl = P.Model(n, m, k, p, idx=idx, sign=sign)
        if path == "host":
            mdl.force_host_la(True)
        mdl.fit(Dg)
        md = mdl.modes()
        S, _ = mdl.select(P.SEL_OMP, K=8)
        res[path] = (md, S)
        rel, _, _ = eig_rel_err(md["lam"], ref.model.lam)
        assert rel.max() <= 1e-9, (path, rel.max())
        np.testing.assert_allclose(md["sigma"], ref.model.sigma, rtol=1e-9)
        key_r = np.abs(ref.model.b) * ref.model.phi_norm
        assert np.abs(np.abs(md["b"]) * md["phi_norm"] - key_r).max() <= 2e-5 * key_r.max(), path
        assert list(S) == list(ref.support), (path, S, ref.support)
    np.testing.assert_allclose(res["device"][0]["lam"], res["host"][0]["lam"], rtol=1e-10, atol=1e-12)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("m", [1025, 1026])
def test_largest_rank_at_the_device_solve_limit(m):
    """k = 40, the largest rank the library builds, at m = 1025 frames (N = 1024: the largest
    device small-LA solve, 32 row groups of 32 rows) and at m = 1026 (past it: the host
    solve): eigenvalues within 1e-9 of the FP64 oracle, sigma within 1e-9, the same OMP
    support; k = 41 is refused."""
    _say("largest rank", m)
    v = _small_u8(H=40, W=64, m=m, seed=29)
    D = v.D.numpy()
    n = D.shape[1]
    k, p = 40, 300
    idx, sign = sv.sparse_table(n, p, 32, 6)
    Dg = torch.from_numpy(D).cuda()
    ref = R.run(D, v.scale, k, sketch="sparse", idx=idx, sign=sign, K=8)
    mdl = P.Model(n, m, k, p, idx=idx, sign=sign)
    mdl.fit(Dg)
    md = mdl.modes()
    rel, _, _ = eig_rel_err(md["lam"], ref.model.lam)
    assert rel.max() <= 1e-9, rel.max()
    np.testing.assert_allclose(md["sigma"], ref.model.sigma, rtol=1e-9)
    S, _ = mdl.select(P.SEL_OMP, K=8)
    assert list(S) == list(ref.support)
    with pytest.raises(P.CdmdError) as e:
        P.Model(n, m, 41, p, idx=idx, sign=sign)
    assert e.value.status == P.E_UNSUPPORTED
