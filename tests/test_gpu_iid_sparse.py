"""The i.i.d. very sparse measurement matrix of Section 3.3 (entries +1 / -1 with
probability 1/(2s) each, s = n / ln n; rows of different weight, padded with -1 in the
table) through the C ABI, against the FP64 oracle.

Tolerances: the uint8 sketch is integer arithmetic, bit-exact in both kernel forms; the
float32-video sketch sums the same terms in the same order in float64 (1e-12 relative);
eigenvalues of the fit 1e-6 relative per matched mode, as for the fixed-weight table.
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


@pytest.mark.parametrize("shape", [(40, 50, 33, 700), (48, 64, 64, 300), (96, 176, 37, 9000)])
def test_iid_sparse_sketch_bit_exact(shape):
    """Streaming form (aligned frames, several row blocks when p > 8192), gather form, and
    the float32-video form, with rows of every weight including empty ones."""
    H, W, m, p = shape
    _say("iid sketch", shape)
    rng = np.random.default_rng(3)
    n = H * W
    D = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
    idx, sign = sv.iid_sparse_table(n, p, n / np.log(n), seed=7)
    idx[::97] = -1  # some rows without any nonzero
    assert (idx < 0).any()
    k = min(4, m - 1)
    Yref, Yiref = R.sketch_sparse(D, 1 / 255, idx, sign)
    Dg = torch.from_numpy(D).cuda()
    for gather in (False, True):
        mdl = P.Model(n, m, k, p, idx=idx, sign=sign)
        mdl.force_gather_sketch(gather)
        mdl.fit(Dg)
        Y, Yi = mdl.sketch(integer=True)
        np.testing.assert_array_equal(Yi, Yiref)
        np.testing.assert_allclose(Y, Yref, rtol=1e-15, atol=0)
    Df = D.astype(np.float32) / 255
    mf = P.Model(n, m, k, p, dtype=P.F32, idx=idx, sign=sign)
    mf.fit(torch.from_numpy(Df).cuda())
    Yf = mf.sketch()
    Yfref, _ = R.sketch_sparse(Df, 1.0, idx, sign)
    np.testing.assert_allclose(Yf, Yfref, rtol=1e-12, atol=1e-12 * np.abs(Yfref).max())


def test_iid_sparse_fit_matches_oracle():
    _say("iid fit")
    spec = sv.preset("cfg2", H=72, W=100, m=80, bump_sigma=8.0, blur_sigma=3.0, n_rects=3,
                     rect_side=(6, 14), speed=(0.5, 2.0), seed=31)
    v = sv.make_video(spec)
    D = v.D.numpy() if v.D.device.type == "cpu" else v.D.cpu().numpy()
    m, n = D.shape
    idx, sign = sv.iid_sparse_table(n, 500, n / np.log(n), seed=9)
    k = 14
    mdl = P.Model(n, m, k, 500, idx=idx, sign=sign)
    mdl.fit(torch.from_numpy(D).cuda())
    ref = R.fit(D, v.scale, R.sketch_sparse(D, v.scale, idx, sign)[0], k)
    rel, _, _ = eig_rel_err(mdl.modes()["lam"], ref.lam)
    assert rel.max() <= 1e-6
