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


# (kind, H, W, ld, m, k, p, lift precision): frame sizes with and without a partial
# 128-pixel tile, padded frames, both reconstruction forms and one float32 video (whose
# reconstruction takes the VALU form, launched on its own)
FG_STREAMS = [
    ("sparse", 48, 60, None, 40, 6, 200, "fp32"),      # 2880 px: 22 full tiles and half a tile
    ("sparse", 40, 48, None, 50, 5, 150, "bf16"),      # 1920 px: full tiles only
    ("sparse", 8, 12, None, 30, 3, 60, "fp32"),        # 96 px: one partial tile only
    ("gauss_bf16", 37, 53, 1968, 45, 6, 120, "fp32"),  # padded frames, a partial tile
    ("f32", 40, 64, None, 40, 6, 300, "fp32"),
    ("sparse", 64, 96, None, 300, 8, 300, "bf16"),     # 300 frames: a larger tile in LDS
    ("sparse", 30, 40, None, 70, 10, 250, "fp32"),
]


def _fg_make(i, kind, H, W, ld, m, k, p, lift):
    n = H * W
    ld = ld or n
    out = "f32" if kind == "f32" else "u8"
    spec = sv.preset("cfg2", H=H, W=W, m=m, n_pairs=2, bump_sigma=max(H, W) / 8.0, blur_sigma=2.0,
                     n_rects=2, rect_side=(2, max(3, W // 6)), speed=(0.5, 2.0), seed=700 + i, out=out)
    D = sv.make_video(spec, device="cuda").D
    if ld != n:
        Dp = torch.zeros((m, ld), dtype=D.dtype, device="cuda")
        Dp[:, :n] = D
        D = Dp
    lp = P.PREC_BF16 if lift == "bf16" else P.PREC_FP32
    if kind.startswith("gauss"):
        mdl = P.Model(n, m, k, p, sketch=P.SKETCH_GAUSSIAN, ld=ld, seed=21 + i, sketch_prec=P.PREC_BF16, lift_prec=lp)
    else:
        idx, sign = sv.sparse_table(n, p, 32, 80 + i)
        mdl = P.Model(n, m, k, p, dtype=P.F32 if kind == "f32" else P.U8, ld=ld, idx=idx, sign=sign, lift_prec=lp)
    return D, mdl


def _masks(models):
    return [torch.full((mdl.m, P.mask_words(mdl.n)), -1, dtype=torch.int32, device="cuda") for mdl in models]


def test_batch_foreground_equals_per_model_masks():
    """cdmd_batch_foreground (one work-queue launch per reconstruction form over every
    model's pixel tiles) gives each model's cdmd_foreground mask bit for bit: full and
    partial tiles, padded frames, both reconstruction forms, the VALU form of a float32
    video, the static model, and two calls back to back with no synchronisation between
    them (the second with another tau)."""
    _say("batch foreground")
    made = [_fg_make(i, *s) for i, s in enumerate(FG_STREAMS)]
    videos = [D for D, _ in made]
    models = [mdl for _, mdl in made]
    batch = P.Batch(models)
    assert batch.fit(videos) == [P.OK] * len(models)
    for mdl in models:
        mdl.select(P.SEL_OMP, K=min(4, mdl.k))
    for static in (False, True):
        taus = (0.1, 0.05)
        got = [_masks(models) for _ in taus]
        for tau, mk in zip(taus, got):
            batch.foreground(videos, mk, tau, static_bg=static)
        torch.cuda.synchronize()
        fg = 0
        for tau, mk in zip(taus, got):
            for q, (mdl, D, g) in enumerate(zip(models, videos, mk)):
                ref = torch.full_like(g, -1)
                mdl.foreground(D, ref, tau, static=static)
                torch.cuda.synchronize()
                assert torch.equal(g, ref), (q, FG_STREAMS[q], tau, static)
                fg += int(ref.ne(0).sum())
        assert fg > 0  # the masks hold foreground


def test_batch_foreground_more_than_64_models():
    """70 models share one video shape: the work list is split into launches of 64 entries;
    every mask equals the model's own cdmd_foreground."""
    _say("batch foreground, 70 models")
    H, W, m = 24, 40, 36
    n = H * W
    spec = sv.preset("cfg2", H=H, W=W, m=m, n_pairs=2, bump_sigma=4.0, blur_sigma=2.0, n_rects=1,
                     rect_side=(2, 5), seed=901)
    D = sv.make_video(spec, device="cuda").D
    models = []
    for i in range(70):
        idx, sign = sv.sparse_table(n, 80, 32, 1000 + i)
        models.append(P.Model(n, m, 4, 80, idx=idx, sign=sign))
    videos = [D] * len(models)
    batch = P.Batch(models)
    assert batch.fit(videos) == [P.OK] * len(models)
    for mdl in models:
        mdl.select(P.SEL_OMP, K=3)
    got = _masks(models)
    batch.foreground(videos, got, 0.1)
    torch.cuda.synchronize()
    for q, (mdl, g) in enumerate(zip(models, got)):
        ref = torch.full_like(g, -1)
        mdl.foreground(D, ref, 0.1)
        torch.cuda.synchronize()
        assert torch.equal(g, ref), q


def test_batch_foreground_refusals():
    _say("batch foreground refusals")
    D, mdl = _fg_make(0, *FG_STREAMS[0])
    batch = P.Batch([mdl])
    assert batch.fit([D]) == [P.OK]
    mk = _masks([mdl])
    with pytest.raises(P.CdmdError) as e:   # not selected
        batch.foreground([D], mk, 0.1)
    assert e.value.status == P.E_STATE
    mdl.select(P.SEL_OMP, K=3)
    with pytest.raises(P.CdmdError) as e:
        batch.foreground([D], mk, -1.0)
    assert e.value.status == P.E_INVALID_ARG
