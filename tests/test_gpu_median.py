"""Median filtering of foreground masks (Section 4, BMC evaluation) through the C ABI:
cdmd_mask_median3 against the oracle's median3 (itself pinned to scipy's median filter).
Integer work: bit-exact, for bit-packed and uint8 masks, frame widths that are and are not
multiples of 32 (the word-parallel kernel and the per-bit one), one-pixel-wide frames, and
on a mask the library itself produced."""
import numpy as np
import pytest
import torch

import synthvideo as sv
from oracle import cdmd_ref as R

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1512_04205_amd")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _pack(mk):
    m, n = mk.shape
    w = P.mask_words(n)
    bits = np.zeros((m, 32 * w), dtype=np.uint8)
    bits[:, :n] = mk
    return np.packbits(bits, axis=1, bitorder="little").view(np.uint32).reshape(m, w)


@pytest.mark.parametrize("shape", [(37, 45, 5, 0.3), (64, 64, 3, 0.5), (1, 70, 2, 0.5), (70, 1, 2, 0.4),
                                   (120, 96, 4, 0.1), (1, 64, 2, 0.5), (33, 32, 3, 0.5), (20, 320, 2, 0.5)])
def test_median3_matches_oracle(shape):
    H, W, m, dens = shape
    _say("median3", shape)
    rng = np.random.default_rng(H * 131 + W)
    mk = rng.random((m, H * W)) < dens
    want = R.median3(mk, H, W)
    src = torch.from_numpy(_pack(mk).view(np.int32)).cuda()
    dst = torch.zeros_like(src)
    P.mask_median3(src, dst, H, W, bitpacked=True)
    np.testing.assert_array_equal(P.unpack_mask(dst.cpu().numpy().view(np.uint32), H * W), want)
    s8 = torch.from_numpy(mk.astype(np.uint8)).cuda()
    d8 = torch.zeros_like(s8)
    P.mask_median3(s8, d8, H, W, bitpacked=False)
    np.testing.assert_array_equal(d8.cpu().numpy().astype(bool), want)
    with pytest.raises(P.CdmdError) as e:
        P.mask_median3(src, src, H, W)
    assert e.value.status == P.E_INVALID_ARG


def test_median3_of_a_fitted_mask():
    _say("median3 fitted")
    spec = sv.preset("cfg2", H=72, W=100, m=40, bump_sigma=8.0, blur_sigma=3.0, n_rects=3,
                     rect_side=(6, 14), speed=(0.5, 2.0), seed=11)
    v = sv.make_video(spec)
    D = v.D.numpy() if v.D.device.type == "cpu" else v.D.cpu().numpy()
    m, n = D.shape
    idx, sign = sv.sparse_table(n, 400, 32, 2)
    mdl = P.Model(n, m, 10, 400, idx=idx, sign=sign)
    Dg = torch.from_numpy(D).cuda()
    mdl.fit(Dg)
    mdl.select(P.SEL_OMP, K=6)
    mk = torch.zeros((m, P.mask_words(n)), dtype=torch.int32, device="cuda")
    mdl.foreground(Dg, mk, 0.1)
    out = torch.zeros_like(mk)
    P.mask_median3(mk, out, 72, 100)
    got = P.unpack_mask(out.cpu().numpy().view(np.uint32), n)
    want = R.median3(P.unpack_mask(mk.cpu().numpy().view(np.uint32), n), 72, 100)
    np.testing.assert_array_equal(got, want)
