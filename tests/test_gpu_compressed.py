"""Remark 3 (Section 3.2) on the GPU, through the C ABI: amplitudes and OMP on the
compressed modes Phi_Y = Y' V S^-1 W and the first compressed frame y_1, against the FP64
oracle of the same variant (oracle.cdmd_ref.fit_compressed).

Tolerances
* eigenvalues: relative error <= 1e-6 per matched mode (as the full fit);
* |b_j| ||phi_Y,j||, ||phi_Y,j||, ||y_1||^2 and |beta_j| ||phi_Y,j||: everything here is
  float64 from the exact integer sketch (no float32 lift), so 1e-6 relative to the
  largest entry covers the Lanczos-versus-SVD differences of the eigenvectors;
* the OMP support: identical;
* masks (background from the full modes X' G_S): as test_gpu_parity, >= 99.9% identical
  and every disagreement inside the band ||x - L| - tau| <= 10 max|L_gpu - L_ref| + 1e-6.
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


def _video(H=72, W=100, m=80, seed=31):
    spec = sv.preset("cfg2", H=H, W=W, m=m, bump_sigma=8.0, blur_sigma=3.0, n_rects=3,
                     rect_side=(6, 14), speed=(0.5, 2.0), seed=seed)
    return sv.make_video(spec)


def _fit(v, k, p, nnz, seed=3):
    D = v.D.numpy() if v.D.device.type == "cpu" else v.D.cpu().numpy()
    n, m = D.shape[1], D.shape[0]
    idx, sign = sv.sparse_table(n, p, nnz, seed)
    Dg = torch.from_numpy(D).cuda()
    mdl = P.Model(n, m, k, p, sketch=P.SKETCH_SPARSE, dtype=P.U8, idx=idx, sign=sign)
    mdl.set_amplitudes(P.AMP_COMPRESSED)
    mdl.fit(Dg)
    Y = R.sketch_sparse(D, v.scale, idx, sign)[0]
    ref = R.fit_compressed(Y, k)
    return D, Dg, mdl, ref, Y


@pytest.mark.parametrize("shape", [(72, 100, 80, 14, 500, 32), (40, 64, 121, 25, 700, 8),
                                   (32, 50, 33, 6, 300, 32)])
def test_compressed_fit_matches_oracle(shape):
    H, W, m, k, p, nnz = shape
    _say("compressed fit", shape)
    v = _video(H=H, W=W, m=m)
    D, Dg, mdl, ref, Y = _fit(v, k, p, nnz)
    md = mdl.modes()
    rel, _, _ = eig_rel_err(md["lam"], ref.lam)
    assert rel.max() <= 1e-6
    # modes matched by eigenvalue (the canonical order can swap near-equal keys)
    from scipy.optimize import linear_sum_assignment
    ri, ci = linear_sum_assignment(np.abs(md["lam"][:, None] - ref.lam[None, :]))
    key_g = (np.abs(md["b"]) * md["phi_norm"])[ri]
    key_r = (np.abs(ref.b) * ref.phi_norm)[ci]
    np.testing.assert_allclose(key_g, key_r, rtol=0, atol=1e-6 * key_r.max())
    np.testing.assert_allclose(md["phi_norm"][ri], ref.phi_norm[ci], rtol=0, atol=1e-6 * ref.phi_norm.max())
    y1n2 = float(np.vdot(Y[:, 0], Y[:, 0]).real)
    assert abs(mdl.info()["x1_norm2"] - y1n2) <= 1e-9 * y1n2


def test_compressed_omp_and_mask():
    _say("compressed omp + mask")
    v = _video(seed=37, m=80)
    D, Dg, mdl, ref, Y = _fit(v, 14, 500, 32)
    n, m = D.shape[1], D.shape[0]
    gaps = []
    Sr, br = R.omp(ref.Phi, Y[:, 0], 8, lam=ref.lam, margins=gaps)
    if min(gaps) >= NEAR_TIE_FP32:
        S, beta = mdl.select(P.SEL_OMP, K=8)
        assert list(S) == list(Sr)
    else:   # a near tie the device may resolve either way: the oracle's support
        S, beta = mdl.select(P.SEL_EXPLICIT, explicit=Sr)
    np.testing.assert_allclose(np.abs(beta) * ref.phi_norm[S], np.abs(br) * ref.phi_norm[Sr],
                               rtol=0, atol=1e-6 * np.abs(br * ref.phi_norm[Sr]).max())
    # the background and mask use the full modes X' G_S with the compressed amplitudes
    Phi_S = R.lift(D, v.scale, ref.G[:, Sr])
    Lr = R.background(Phi_S, br, ref.lam[Sr], 0, m)
    x = D.T.astype(np.float64) / 255
    tau = 0.1
    mr = R.foreground(x, Lr, tau).T
    mk = torch.zeros((m, P.mask_words(n)), dtype=torch.int32, device="cuda")
    counts = mdl.foreground(Dg, mk, tau, counts=True)
    mg = P.unpack_mask(mk.cpu().numpy().view(np.uint32), n)
    L = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    mdl.background(Dg, L)
    lerr = np.abs(L.cpu().numpy() - Lr.T).max()
    assert lerr <= 2e-5 * np.abs(Lr).max()
    frac, inband, nd = mask_agreement(mg, mr, x.T, Lr.T, tau, 10 * lerr + 1e-6)
    assert frac >= 0.999 and inband, (frac, nd, lerr)
    np.testing.assert_array_equal(counts, mg.sum(axis=1))


def test_compressed_switch_back_and_unsupported():
    """AMP_FULL after AMP_COMPRESSED gives the full fit again, bit for bit; a float32
    video (host small LA) cannot use the compressed modes; batches refuse such models."""
    _say("compressed switch")
    v = _video(H=40, W=64, m=50, seed=5)
    D = v.D.numpy() if v.D.device.type == "cpu" else v.D.cpu().numpy()
    n, m = D.shape[1], D.shape[0]
    idx, sign = sv.sparse_table(n, 300, 32, 4)
    Dg = torch.from_numpy(D).cuda()
    a = P.Model(n, m, 8, 300, sketch=P.SKETCH_SPARSE, dtype=P.U8, idx=idx, sign=sign)
    a.fit(Dg)
    full = a.modes()
    a.set_amplitudes(P.AMP_COMPRESSED)
    with pytest.raises(P.CdmdError):
        a.modes()  # unfitted after the switch
    with pytest.raises(P.CdmdError) as e:
        P.Batch([a])
    assert e.value.status == P.E_UNSUPPORTED
    a.fit(Dg)
    a.set_amplitudes(P.AMP_FULL)
    a.fit(Dg)
    again = a.modes()
    np.testing.assert_array_equal(again["b"], full["b"])
    np.testing.assert_array_equal(again["lam"], full["lam"])
    Df = torch.from_numpy(D.astype(np.float32) / 255).cuda()
    f = P.Model(n, m, 8, 300, sketch=P.SKETCH_SPARSE, dtype=P.F32, idx=idx, sign=sign)
    with pytest.raises(P.CdmdError) as e:
        f.set_amplitudes(P.AMP_COMPRESSED)  # refused here or by the fit
        f.fit(Df)
    assert e.value.status == P.E_UNSUPPORTED
