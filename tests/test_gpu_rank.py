"""Automatic target rank (Section 3.2, Remark 2) on the GPU against the FP64 oracle.

Integer (uint8 sparse) sketches are exact, so the sketch's singular values (device FP64
Gram, host spectrum) agree with the oracle's direct SVD within 1e-9 relative, the threshold
tau* within 1e-9 and the rank k = #{sigma > tau*} exactly (a singular value within the
tolerance of tau* would make the count ill-posed; the test reports the smallest distance).
A float32 Gaussian sketch carries its own rounding E = Yhat_gpu - Yhat_oracle: by Weyl's
inequality each singular value moves by at most ||E||_2, the median by at most ||E||_2 and
tau* = omega * median by at most omega ||E||_2; the singular values must match the SVD of
the device's own sketch within 1e-9."""
import numpy as np
import pytest
import torch

import synthvideo as sv
from oracle import cdmd_ref as R

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1512_04205_amd")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _check(k, tau, sig, Yhat, Yhat_dev=None):
    """``Yhat_dev``: the device's own sketch when it is not exact (else None)."""
    kr, taur, sr = R.optimal_rank(Yhat)
    r = len(sr)
    if Yhat_dev is None:
        np.testing.assert_allclose(sig, sr, rtol=1e-9, atol=1e-9 * sr[0])
        tol = 1e-9 * taur
    else:
        mm = Yhat.shape[1] - 1
        sd = np.linalg.svd(Yhat_dev[:, :mm], compute_uv=False)
        np.testing.assert_allclose(sig, sd, rtol=1e-9, atol=1e-9 * sd[0])
        e2 = np.linalg.norm(Yhat_dev[:, :mm] - Yhat[:, :mm], 2)
        assert np.all(np.abs(sd - sr) <= e2 * (1 + 1e-9) + 1e-12 * sr[0])
        beta = min(Yhat.shape) / max(Yhat.shape)
        tol = R.gd_omega(beta) * e2 * (1 + 1e-9) + 1e-9 * taur
        _say("||E||_2", e2, "rel to sigma_1", e2 / sr[0])
    assert abs(tau - taur) <= tol, (tau, taur, tol)
    gap = np.min(np.abs(sr - taur)) / taur
    _say("k", k, "oracle k", kr, "of", r, "tau", taur, "closest sigma (rel)", gap)
    if gap * taur > 2 * tol:
        assert k == kr, (k, kr)
    return kr


@pytest.mark.parametrize("case", ["sparse_u8", "gauss_f32", "sparse_u8_tall"])
def test_optimal_rank_small(case):
    _say("rank", case)
    if case == "gauss_f32":
        spec = sv.preset("cfg1", H=60, W=80, m=120, bump_sigma=5.0, blur_sigma=3.0, n_rects=3,
                         rect_side=(6, 6), seed=61)
        v = sv.make_video(spec)
        D = v.D.numpy()
        m, n = D.shape
        p = 300
        Dd = torch.from_numpy(D).cuda()
        k, tau, sig = P.optimal_rank(Dd, n, m, p, sketch=P.SKETCH_GAUSSIAN, dtype=P.F32, seed=17)
        mdl = P.Model(n, m, 10, p, sketch=P.SKETCH_GAUSSIAN, dtype=P.F32, seed=17).fit(Dd)
        torch.cuda.synchronize()
        _check(k, tau, sig, R.sketch_gaussian(D, 1.0, 17, p), mdl.sketch())
        mdl.close()
        return
    else:
        H, W, m, p = (72, 128, 150, 600) if case == "sparse_u8" else (48, 64, 300, 200)
        spec = sv.preset("cfg2", H=H, W=W, m=m, bump_sigma=8.0, blur_sigma=3.0, n_rects=4,
                         rect_side=(6, 14), speed=(0.5, 2.0), seed=62)
        v = sv.make_video(spec)
        D = v.D.numpy()
        n = H * W
        idx, sign = sv.sparse_table(n, p, 32, 5)
        k, tau, sig = P.optimal_rank(torch.from_numpy(D).cuda(), n, m, p, idx=idx, sign=sign)
        Yhat = R.sketch_sparse(D, 1 / 255, idx, sign)[0]
    _check(k, tau, sig, Yhat)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("preset,p", [("cfg2", 2000), ("ctxA", 1000)])
def test_optimal_rank_full_size(preset, p):
    """The 1080p headline video and the paper's 1280x720x200 timing shape (where the paper
    chose k by this threshold): the rank the GPU picks equals the oracle's."""
    _say("rank full size", preset)
    spec = sv.PRESETS[preset]
    v = sv.make_video(spec, device="cuda")
    m, n = v.D.shape
    idx, sign = sv.sparse_table(n, p, 32, seed=2002)
    k, tau, sig = P.optimal_rank(v.D, n, m, p, idx=idx, sign=sign)
    Yhat = R.sketch_sparse(v.D.cpu().numpy(), 1 / 255, idx, sign)[0]
    kr = _check(k, tau, sig, Yhat)
    assert 1 <= kr < min(p, m - 1)
