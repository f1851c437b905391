"""Learned background-mode selector on the GPU vs the FP64 oracle (oracle/mlp_ref.py),
through the C ABI.

Tolerances
* gradient: float32 forward/backward with fixed-order float64 partial sums;
  ||g_gpu - g_ref|| <= 1e-4 ||g_ref|| and every entry within 1e-5 |g_ref,i| + 1e-5 max|g_ref|,
  loss within 1e-5 relative;
* training: 40 Adam steps on the same caller-drawn batches; per-step losses within 1e-3
  relative and ||theta_gpu - theta_ref|| <= 1e-2 ||theta_ref - theta_0|| (Adam divides
  by sqrt(v), so float32 rounding of tiny gradients moves single parameters);
* forward: float32 logits within 1e-5 (1 + |z|); bfloat16 inference (hidden activations
  and the weights after the input layer rounded to 8 significant bits) within
  0.05 (1 + |z|);
* features: within 1e-5 relative of the oracle's (float32 storage).
"""
import numpy as np
import pytest
import torch

import synthvideo as sv
from oracle import cdmd_ref as R
from oracle import mlp_ref as MR

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1512_04205_amd")


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _data(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 6)).astype(np.float32).astype(np.float64)
    y = (X[:, 0] + 0.5 * X[:, 3] - 0.25 * X[:, 5] > 0.1).astype(np.float64)
    return X, y


@pytest.mark.parametrize("n", [1, 37, 300])
def test_mlp_gradient_matches_oracle(n):
    _say("mlp grad", n)
    theta = sv.mlp_init(n)
    X, y = _data(n, n)
    loss, g = P.mlp_grad(_dev(theta), _dev(X), _dev(y))
    Lr, gr = MR.loss_and_grad(theta, X, y)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(loss - Lr) <= 1e-5 * abs(Lr), (loss, Lr)
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr), np.linalg.norm(g - gr) / np.linalg.norm(gr)
    # element by element: float32 products and activations (relative 1e-5 of each entry)
    # plus the absolute rounding floor of sums whose terms cancel (1e-5 of the largest entry)
    err = np.abs(g - gr)
    bound = 1e-5 * np.abs(gr) + 1e-5 * np.abs(gr).max()
    assert (err <= bound).all(), (int(np.argmax(err / bound)), float((err / bound).max()))


def test_mlp_training_follows_oracle():
    _say("mlp train")
    theta0 = sv.mlp_init(21)
    X, y = _data(21, 400)
    rng = np.random.default_rng(22)
    steps, batch = 40, 64
    batches = [rng.permutation(400)[:batch] for _ in range(steps)]
    th = _dev(theta0)
    am = torch.zeros(P.MLP_NPARAM, device="cuda")
    av = torch.zeros(P.MLP_NPARAM, device="cuda")
    bi = _dev(np.concatenate(batches), torch.int32)
    losses = P.mlp_train(th, am, av, _dev(X), _dev(y), bi, batch, lr=1e-3).cpu().numpy()
    # oracle, same batches
    theta = theta0.copy()
    opt = MR.Adam(MR.NPARAM, lr=1e-3)
    ref_losses = []
    for b in batches:
        L, g = MR.loss_and_grad(theta, X[b], y[b])
        ref_losses.append(L)
        theta = opt.step(theta, g)
    np.testing.assert_allclose(losses, ref_losses, rtol=1e-3)
    tg = th.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(tg - theta) <= 1e-2 * np.linalg.norm(theta - theta0)


def test_mlp_forward_fp32_and_bf16():
    _say("mlp forward")
    theta = sv.mlp_init(3)
    X, _ = _data(3, 200)
    z_ref, _ = MR.forward(theta, X)
    z = P.mlp_forward(_dev(theta), _dev(X)).cpu().numpy()
    assert (np.abs(z - z_ref) <= 1e-5 * (1 + np.abs(z_ref))).all()
    zb = P.mlp_forward(_dev(theta), _dev(X), bf16=True).cpu().numpy()
    assert (np.abs(zb - z_ref) <= 0.05 * (1 + np.abs(z_ref))).all()


def _video(seed, H=90, W=120, m=80, n_pairs=None):
    rng = np.random.default_rng(seed)
    n_pairs = int(rng.integers(2, 6)) if n_pairs is None else n_pairs
    spec = sv.preset("cfg2", H=H, W=W, m=m, n_pairs=n_pairs, bump_sigma=10.0, blur_sigma=4.0,
                     n_rects=4, rect_side=(8, 16), speed=(0.5, 2.0), seed=seed)
    return sv.make_video(spec, device="cuda")


def test_mode_features_match_oracle():
    _say("mode features")
    v = _video(5)
    m, n = v.D.shape
    k = 10
    idx, sign = sv.sparse_table(n, 600, 32, 1)
    mdl = P.Model(n, m, k, 600, idx=idx, sign=sign)
    mdl.fit(v.D)
    md = mdl.modes()
    F = mdl.mode_features().cpu().numpy().astype(np.float64)
    Fr = MR.features(md["lam"], md["b"], md["phi_norm"], mdl.info()["x1_norm2"], m)
    np.testing.assert_allclose(F, Fr, rtol=1e-5, atol=1e-6)


def _bits_to_mask(words, n):
    """(m, words) int32 bit-packed mask (bit b of word w = pixel 32 w + b) -> (m, n) bool,
    on the device."""
    sh = torch.arange(32, device=words.device, dtype=torch.int32)
    bits = (words.unsqueeze(-1) >> sh) & 1
    return bits.reshape(words.shape[0], -1)[:, :n].bool()


def _gt_chunk(v, t0, t1):
    """The generator's ground truth (the moving rectangles) of frames [t0, t1) as a
    (t1 - t0, n) bool device tensor."""
    s = v.spec
    gt = torch.zeros((t1 - t0, s.H, s.W), dtype=torch.bool, device="cuda")
    for t in range(t0, t1):
        for (y0, x0, h, w) in v.rects[t]:
            gt[t - t0, y0:y0 + h, x0:x0 + w] = True
    return gt.reshape(t1 - t0, s.n)


def _counts(mask, gt):
    return (float((mask & gt).sum()), float((mask & ~gt).sum()), float((~mask & gt).sum()))


def _f_from_counts(tp, fp, fn):
    rec = tp / (tp + fn) if tp + fn > 0 else 0.0
    pre = tp / (tp + fp) if tp + fp > 0 else 0.0
    return 2 * pre * rec / (pre + rec) if pre + rec > 0 else 0.0


def _f_dev(mask, gt):
    """F-measure (recall, precision and their harmonic mean) counted on the device."""
    return _f_from_counts(*_counts(mask, gt))


def _f_video(words, v, chunk=25):
    """F-measure of a bit-packed (m, words) device mask against the ground truth of v,
    frame chunk by frame chunk (bounded device memory)."""
    n, m = v.spec.n, v.spec.m
    c = np.zeros(3)
    for t0 in range(0, m, chunk):
        t1 = min(m, t0 + chunk)
        c += _counts(_bits_to_mask(words[t0:t1], n), _gt_chunk(v, t0, t1))
    return _f_from_counts(*c)


def test_device_f_measure_matches_oracle():
    rng = np.random.default_rng(4)
    a = rng.random((7, 300)) < 0.3
    b = rng.random((7, 300)) < 0.2
    assert abs(_f_dev(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) - R.f_measure(a, b)) < 1e-12
    # the chunked count over a small generated video equals the oracle's F on its masks
    v = _video(3, H=40, W=64, m=30)
    mw = torch.from_numpy(rng.integers(-2 ** 31, 2 ** 31, size=(30, P.mask_words(40 * 64)),
                                       dtype=np.int64).astype(np.int32)).cuda()
    ref = R.f_measure(P.unpack_mask(mw.cpu().numpy().view(np.uint32), 40 * 64), v.gt_mask())
    assert abs(_f_video(mw, v, chunk=7) - ref) < 1e-12
    words = rng.integers(-2 ** 31, 2 ** 31, size=(5, 4), dtype=np.int64).astype(np.int32)
    got = _bits_to_mask(torch.from_numpy(words).cuda(), 100).cpu().numpy()
    np.testing.assert_array_equal(got, P.unpack_mask(words.view(np.uint32), 100))


@pytest.mark.timeout(900)
def test_learned_selector_at_stated_scale():
    """The learned selector as stated for it: trained on at least 20,000 modes labelled by
    sparse coding (OMP, K = 10, k = 25, sparse p = 2000 x 32) of 640x480 videos of 300
    frames with 5-19 background modes, applied to held-out 1920x1080 videos of 500 frames
    with the 0.9-confidence fallback to OMP.  Reports, on the held-out videos, the
    F-measure of the foreground masks (tau = 0.1) against the generator's ground truth for
    OMP, for the learned selection with fallback and for the network alone, the fallback
    rate at several confidence levels, the network's agreement with the OMP labels and the
    selection times.  Requires: the training loss falls; the network agrees with OMP on at
    least 75% of the held-out modes; the network alone loses at most 0.05 and the learned
    path with fallback at most 0.02 in mean F against OMP; the library's probabilities and
    fallback decision agree with the FP64 oracle's (mlp_ref.predict) up to bfloat16
    inference.  (The measured result is negative: the network is never confident about
    all 25 modes at 0.9, so the learned path falls back to OMP, and the network alone is a
    little below OMP; the numbers are printed.)"""
    import time
    _say("learned selector: training set")
    k, p, K, tau = 25, 2000, 10, 0.1
    rng = np.random.default_rng(2024)
    base = sv.PRESETS["train640"]
    n = base.H * base.W
    idx, sign = sv.sparse_table(n, p, 32, 640)
    mdl = P.Model(n, base.m, k, p, idx=idx, sign=sign)
    feats, labels, vids = [], [], 0
    t_start = time.perf_counter()
    while sum(len(l) for l in labels) < 20000:
        spec = sv.preset("train640", n_pairs=int(rng.integers(2, 10)), seed=50000 + vids)
        vids += 1
        v = sv.make_video(spec, device="cuda")
        try:
            mdl.fit(v.D)
        except P.CdmdError:
            continue
        S, _ = mdl.select(P.SEL_OMP, K=K)
        feats.append(mdl.mode_features().cpu().numpy())
        lab = np.zeros(k, np.float32)
        lab[S] = 1
        labels.append(lab)
        if vids % 100 == 0:
            _say("videos", vids, "modes", sum(len(l) for l in labels), "s", round(time.perf_counter() - t_start, 1))
    mdl.close()
    X = np.concatenate(feats)
    y = np.concatenate(labels)
    _say("training modes", len(y), "from", vids, "videos; positives", int(y.sum()))
    # standardised features for training; the standardisation is folded into the first
    # layer afterwards, so that the network reads the features the library computes
    mu, sd = X.mean(axis=0), X.std(axis=0) + 1e-6
    Xs = (X - mu) / sd
    th = _dev(sv.mlp_init(7))
    am = torch.zeros(P.MLP_NPARAM, device="cuda")
    av = torch.zeros(P.MLP_NPARAM, device="cuda")
    batch, steps = 256, 4000
    bi = _dev(np.concatenate([rng.choice(len(y), batch) for _ in range(steps)]), torch.int32)
    losses = P.mlp_train(th, am, av, _dev(Xs), _dev(y), bi, batch, lr=2e-3).cpu().numpy()
    _say("loss", float(losses[:20].mean()), "->", float(losses[-200:].mean()))
    assert losses[-200:].mean() < 0.7 * losses[:20].mean()
    theta = th.cpu().numpy().astype(np.float64)
    W1 = theta[:384].reshape(64, 6) / sd[None, :]
    theta[384:448] -= W1 @ mu
    theta[:384] = W1.ravel()
    th = _dev(theta)
    pr_train, _, _ = MR.predict(theta, X)
    _say("training agreement with OMP", float(((pr_train >= 0.5) == (y > 0.5)).mean()))

    _say("learned selector: held-out 1080p videos")
    big = sv.PRESETS["cfg2"]
    n2 = big.H * big.W
    idx2, sign2 = sv.sparse_table(n2, p, 32, 1080)
    mdl = P.Model(n2, big.m, k, p, idx=idx2, sign=sign2)
    mk = torch.zeros((big.m, P.mask_words(n2)), dtype=torch.int32, device="cuda")
    f_omp, f_lrn, f_raw, agree, t_omp, t_lrn, minconf = [], [], [], [], [], [], []
    fallbacks = trials = 0
    for s in range(6):
        spec = sv.preset("cfg2", n_pairs=int(rng.integers(2, 10)), seed=90000 + s)
        v = sv.make_video(spec, device="cuda")
        try:
            mdl.fit(v.D)
        except P.CdmdError:
            continue
        trials += 1
        t0 = time.perf_counter()
        S_omp, _ = mdl.select(P.SEL_OMP, K=K)
        t_omp.append(time.perf_counter() - t0)
        mdl.foreground(v.D, mk, tau)
        f_omp.append(_f_video(mk, v))
        t0 = time.perf_counter()
        S_l, _, prob, fb = mdl.select_learned(th, confidence=0.9, K_fallback=K)
        t_lrn.append(time.perf_counter() - t0)
        fallbacks += int(fb)
        mdl.foreground(v.D, mk, tau)
        f_lrn.append(_f_video(mk, v))
        # the library's decision against the FP64 oracle's on the same features
        F = mdl.mode_features().cpu().numpy().astype(np.float64)
        pr, S_ref, conf_ref = MR.predict(theta, F, 0.9)
        z_ref = np.log(pr / (1 - pr))
        z_dev = np.log(prob / (1 - prob))
        tol = 0.05 * (1 + np.abs(z_ref))
        assert (np.abs(z_dev - z_ref) <= tol).all(), np.abs(z_dev - z_ref).max()
        clear = np.abs(z_ref) > tol
        assert ((prob >= 0.5) == (pr >= 0.5))[clear].all()
        z09 = np.log(9.0)
        if (np.abs(np.abs(z_ref) - z09) > 0.05 * (1 + z09)).all():
            assert fb == (not conf_ref or len(S_ref) == 0), (fb, conf_ref)
        lab = np.zeros(k, bool)
        lab[S_omp] = True
        agree.append(float(((prob >= 0.5) == lab).mean()))
        minconf.append(float(np.maximum(prob, 1 - prob).min()))
        # the network alone (confidence 0.5: falls back only when it selects nothing)
        mdl.select_learned(th, confidence=0.5, K_fallback=K)
        mdl.foreground(v.D, mk, tau)
        f_raw.append(_f_video(mk, v))
        _say("video", s, "F omp", round(f_omp[-1], 4), "learned", round(f_lrn[-1], 4), "network",
             round(f_raw[-1], 4), "fallback", fb, "agreement", round(agree[-1], 3))
        del v
    mdl.close()
    _say("mean F: omp", np.mean(f_omp), "learned (0.9 + fallback)", np.mean(f_lrn), "network alone",
         np.mean(f_raw), "| fallbacks", fallbacks, "/", trials, "| agreement with OMP", np.mean(agree),
         "| selection ms omp", 1e3 * np.median(t_omp), "learned", 1e3 * np.median(t_lrn))
    used = {c: int(sum(mc >= c for mc in minconf)) for c in (0.6, 0.7, 0.8, 0.9)}
    _say("videos where the network decides every mode, by confidence level:", used, "of", trials)
    assert trials >= 5
    assert np.mean(agree) >= 0.75
    assert np.mean(f_raw) >= np.mean(f_omp) - 0.05
    assert np.mean(f_lrn) >= np.mean(f_omp) - 0.02
