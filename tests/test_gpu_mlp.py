"""Learned background-mode selector on the GPU vs the FP64 oracle (oracle/mlp_ref.py),
through the C ABI.

Tolerances
* gradient: float32 forward/backward with fixed-order float64 partial sums;
  ||g_gpu - g_ref|| <= 1e-4 ||g_ref||, loss within 1e-5 relative;
* training: 40 Adam steps on the same caller-drawn batches; per-step losses within 1e-3
  relative and ||theta_gpu - theta_ref|| <= 1e-2 ||theta_ref - theta_0|| (Adam divides
  by sqrt(v), so float32 rounding of tiny gradients moves single parameters);
* forward: float32 logits within 1e-5 (1 + |z|); bfloat16 inference (weights, inputs
  and activations rounded to 8 significant bits) within 0.05 (1 + |z|);
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


@pytest.mark.timeout(600)
def test_learned_selector_trained_on_omp_labels():
    """Train on OMP selections of generated videos (features from the GPU fit, labels =
    membership in the OMP support), then select on held-out videos: the learned
    selection (with OMP fallback below 0.9 confidence) is compared with plain OMP by the
    F-measure of the foreground masks against the generator's ground truth.  Reports
    both and the fallback rate; requires training to lower the loss and the learned path
    to lose at most 0.02 in mean F."""
    _say("learned selector")
    k, p, K, tau = 12, 600, 6, 0.1
    feats, labels = [], []
    for s in range(120):
        v = _video(1000 + s)
        m, n = v.D.shape
        idx, sign = sv.sparse_table(n, p, 32, s)
        mdl = P.Model(n, m, k, p, idx=idx, sign=sign)
        try:
            mdl.fit(v.D)
        except P.CdmdError:
            continue
        S, _ = mdl.select(P.SEL_OMP, K=K)
        feats.append(mdl.mode_features().cpu().numpy())
        lab = np.zeros(k, np.float32)
        lab[S] = 1
        labels.append(lab)
    X = np.concatenate(feats)
    y = np.concatenate(labels)
    _say("training modes", len(y), "positives", int(y.sum()))
    # train on standardised features, then fold the standardisation into the first layer
    # so that the network reads the raw features the library computes
    mu, sd = X.mean(axis=0), X.std(axis=0) + 1e-6
    X = (X - mu) / sd
    th = _dev(sv.mlp_init(7))
    am = torch.zeros(P.MLP_NPARAM, device="cuda")
    av = torch.zeros(P.MLP_NPARAM, device="cuda")
    rng = np.random.default_rng(8)
    batch, steps = 128, 1500
    bi = _dev(np.concatenate([rng.choice(len(y), batch) for _ in range(steps)]), torch.int32)
    losses = P.mlp_train(th, am, av, _dev(X), _dev(y), bi, batch, lr=3e-3).cpu().numpy()
    _say("loss", float(losses[:20].mean()), "->", float(losses[-100:].mean()))
    assert losses[-100:].mean() < 0.85 * losses[:20].mean()
    theta = th.cpu().numpy().astype(np.float64)
    W1 = theta[:384].reshape(64, 6) / sd[None, :]
    theta[384:448] -= W1 @ mu
    theta[:384] = W1.ravel()
    th = _dev(theta)
    f_omp, f_lrn, f_raw, fallbacks, trials = [], [], [], 0, 0
    for s in range(12):
        v = _video(9000 + s)
        m, n = v.D.shape
        idx, sign = sv.sparse_table(n, p, 32, 100 + s)
        mdl = P.Model(n, m, k, p, idx=idx, sign=sign)
        try:
            mdl.fit(v.D)
        except P.CdmdError:
            continue
        trials += 1
        gt = v.gt_mask()
        mk = torch.zeros((m, P.mask_words(n)), dtype=torch.int32, device="cuda")
        mdl.select(P.SEL_OMP, K=K)
        mdl.foreground(v.D, mk, tau)
        f_omp.append(R.f_measure(P.unpack_mask(mk.cpu().numpy(), n), gt))
        _, _, _, fb = mdl.select_learned(th, confidence=0.9, K_fallback=K)
        fallbacks += int(fb)
        mdl.foreground(v.D, mk, tau)
        f_lrn.append(R.f_measure(P.unpack_mask(mk.cpu().numpy(), n), gt))
        # the network alone (confidence 0.5: never falls back unless it selects nothing)
        S_raw, _, _, fb_raw = mdl.select_learned(th, confidence=0.5, K_fallback=K)
        mdl.foreground(v.D, mk, tau)
        f_raw.append(R.f_measure(P.unpack_mask(mk.cpu().numpy(), n), gt))
    _say("F omp", np.mean(f_omp), "F learned (0.9 + fallback)", np.mean(f_lrn),
         "F network alone", np.mean(f_raw), "fallbacks", fallbacks, "/", trials)
    assert trials >= 8
    assert np.mean(f_lrn) >= np.mean(f_omp) - 0.02
