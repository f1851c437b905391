"""Batched fits (one graph launch for many models) and the autotuner, through the C ABI.

Every model of a batch must give what the same model gives when fitted alone: the
eigenvalues bit for bit (the small linear algebra is the same code on the same Gram),
b_j and ||phi_j|| to 1e-12 relative (the autotuner may change the number of lift
workgroups, which only reorders float64 sums of float32 partials).  One model per kind
is also checked against the FP64 oracle (eigenvalues <= 1e-6 relative).
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


# (kind, H, W, m, k, p): W multiple of 16 so uint8 frames are 16-byte aligned
STREAMS = [
    ("sparse", 48, 64, 60, 8, 400),
    ("sparse", 72, 96, 45, 5, 300),
    ("gauss_fp32", 40, 48, 50, 6, 120),
    ("gauss_bf16", 64, 80, 80, 12, 200),
    ("sparse", 30, 32, 33, 4, 100),
    ("f32", 40, 64, 40, 6, 300),       # host small LA: fitted after the graph
    ("sparse", 90, 128, 70, 10, 500),
]


def _make(i, kind, H, W, m, k, p):
    out = "f32" if kind == "f32" else "u8"
    spec = sv.preset("cfg2", H=H, W=W, m=m, n_pairs=2, bump_sigma=8.0, blur_sigma=3.0, n_rects=2,
                     rect_side=(4, 10), speed=(0.5, 2.0), seed=300 + i, out=out)
    v = sv.make_video(spec, device="cuda")
    n = H * W
    if kind.startswith("gauss"):
        prec = P.PREC_BF16 if kind == "gauss_bf16" else P.PREC_FP32
        mk = lambda: P.Model(n, m, k, p, sketch=P.SKETCH_GAUSSIAN, seed=11 + i, sketch_prec=prec)
        ref = dict(sketch="gaussian", p=p, seed=11 + i)
    else:
        idx, sign = sv.sparse_table(n, p, 32, 50 + i)
        dt = P.F32 if kind == "f32" else P.U8
        mk = lambda: P.Model(n, m, k, p, dtype=dt, idx=idx, sign=sign)
        ref = dict(sketch="sparse", idx=idx, sign=sign)
    return v, mk, ref


def _state(mdl):
    md = mdl.modes()
    return md["lam"], md["b"], md["phi_norm"]


def test_batch_matches_single_fits_and_replays():
    _say("batch fit")
    made = [_make(i, *s) for i, s in enumerate(STREAMS)]
    videos = [v.D for v, _, _ in made]
    singles = []
    for (v, mk, _), s in zip(made, STREAMS):
        mdl = mk()
        mdl.fit(v.D)
        singles.append(_state(mdl))
    models = [mk() for _, mk, _ in made]
    batch = P.Batch(models)
    for rep in range(2):   # capture, then replay
        st = batch.fit(videos)
        assert st == [P.OK] * len(models), st
        for q, (mdl, ref) in enumerate(zip(models, singles)):
            lam, b, pn = _state(mdl)
            np.testing.assert_array_equal(lam, ref[0], err_msg=f"stream {q} rep {rep}")
            np.testing.assert_allclose(np.abs(b) * pn, np.abs(ref[1]) * ref[2], rtol=1e-12,
                                       atol=1e-12 * (np.abs(ref[1]) * ref[2]).max())
    # one model of each kind against the FP64 oracle
    for q in (0, 2, 3, 5):
        v, _, ref = made[q]
        kind, H, W, m, k, p = STREAMS[q]
        D = v.D.cpu().numpy()
        pipe = R.run(D, v.scale, k, **ref)
        rel, _, _ = eig_rel_err(models[q].modes()["lam"], pipe.model.lam)
        assert rel.max() <= (1e-3 if kind == "gauss_bf16" else 1e-6), (q, rel.max())
    # new video buffers: the graph is captured again
    videos2 = [v.clone() for v in videos]
    st = batch.fit(videos2)
    assert st == [P.OK] * len(models)
    for mdl, ref in zip(models, singles):
        np.testing.assert_array_equal(_state(mdl)[0], ref[0])
    # selection and masks work on models fitted by the batch
    S, beta = models[0].select(P.SEL_OMP, K=4)
    mkw = torch.zeros((STREAMS[0][3], P.mask_words(STREAMS[0][1] * STREAMS[0][2])), dtype=torch.int32,
                      device="cuda")
    models[0].foreground(videos2[0], mkw, 0.1)
    batch.close()


def test_batch_reports_per_model_failures():
    _say("batch failures")
    v = sv.make_video(sv.preset("cfg2", H=32, W=64, m=40, n_pairs=1, bump_sigma=6.0, n_rects=2,
                                rect_side=(4, 8), speed=(0.5, 1.0), seed=5), device="cuda")
    n, m = 32 * 64, 40
    idx, sign = sv.sparse_table(n, 200, 32, 1)
    good = P.Model(n, m, 6, 200, idx=idx, sign=sign)
    bad = P.Model(n, m, 6, 200, idx=idx, sign=sign)
    flat = torch.full_like(v.D, 77)     # constant video: rank 1 < k
    batch = P.Batch([good, bad])
    st = batch.statuses([v.D, flat])
    assert st[0] == P.OK and st[1] == P.E_RANK_DEFICIENT, st
    with pytest.raises(P.CdmdError):
        batch.fit([v.D, flat])
    assert batch.fit([v.D, v.D]) == [P.OK, P.OK]
    batch.close()


def test_autotune_keeps_results():
    _say("autotune")
    v, mk, _ = _make(0, "gauss_bf16", 64, 96, 70, 10, 300)
    a = mk()
    a.fit(v.D)
    ref = _state(a)
    b = mk()
    b.autotune(v.D)
    b.fit(v.D)
    inf = b.info()
    assert inf["lift_grid"] > 0 and inf["sketch_slices"] > 0
    lam, bb, pn = _state(b)
    rel, _, _ = eig_rel_err(lam, ref[0])
    # the sketch slices may differ: float32 partial sums regrouped (BF16 products)
    assert rel.max() <= 1e-5


def test_autotune_sparse_sketch_stays_exact():
    """Whichever sparse-sketch form the autotuner picks, the integer sketch is exact."""
    _say("autotune sparse")
    rng = np.random.default_rng(12)
    H, W, m, p = 64, 96, 50, 700
    n = H * W
    D = rng.integers(0, 256, size=(m, n), dtype=np.uint8)
    idx, sign = sv.sparse_table(n, p, 32, seed=9)
    mdl = P.Model(n, m, 6, p, idx=idx, sign=sign)
    Dg = torch.from_numpy(D).cuda()
    mdl.autotune(Dg)
    mdl.fit(Dg)
    assert mdl.info()["sparse_form"] != 0
    _, Yi = mdl.sketch(integer=True)
    _, Yiref = R.sketch_sparse(D, 1 / 255, idx, sign)
    np.testing.assert_array_equal(Yi, Yiref)
