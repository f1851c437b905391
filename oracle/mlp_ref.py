"""FP64 reference of the learned background-mode selector: features, MLP, loss, gradients,
Adam.  TEST INFRASTRUCTURE ONLY (tests/, __graft_entry__.smoke(), bench.py's CPU
baseline); the product path never imports anything under oracle/.

The paper suggests learning the profile of background amplitudes instead of fixing a
selection rule (Section 2.2, "DMD for Foreground/Background Separation", its last paragraph).  The
selector here predicts, per DMD mode, whether sparse coding (orthogonal matching pursuit
on x_1, Algorithm 1's background selection) would pick it.

Features of mode j (k modes, m frames; lambda_j, b_j, phi_j of the fit):
  f0 = |lambda_j|
  f1 = |arg lambda_j|                          in [0, pi]
  f2 = log(|b_j| ||phi_j|| / ||x_1||)          (log of max(., 1e-300)): the mode's share
                                               of the first frame
  f3 = ||phi_j||_2 / max_i ||phi_i||_2         (0 if every mode is zero)
  f4 = (1/m) sum_{t=0}^{m-1} |b_j|^2 |lambda_j|^{2t} ||phi_j||^2 / ||x_1||^2
       (mean energy of the mode's contribution over the frames, relative to frame 1)
  f5 = j / k                                   (position in the canonical order)
The amplitude and the mode norm enter relative to the first frame and to the largest
mode, so that the features do not change with the frame size or the scale of C (a
selector trained on small videos is applied to large ones).

Network: h1 = GELU(W1 f + b1) (64), h2 = GELU(W2 h1 + b2) (64), z = w3 . h2 + b3, with
the exact GELU(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2.  Loss: mean binary
cross-entropy with logits, l(z, y) = max(z, 0) - z y + log(1 + exp(-|z|)).
Parameters are one flat vector in the order W1 (64 x 6 row-major), b1, W2 (64 x 64),
b2, w3 (64), b3: 4673 numbers.
Adam (Kingma and Ba, 2015): beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

H = 64
NF = 6
NPARAM = H * NF + H + H * H + H + H + 1   # 4673


def unpack(theta: np.ndarray):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = theta[o:o + H * NF].reshape(H, NF); o += H * NF
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o]
    return W1, b1, W2, b2, w3, b3


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def features(lam, b, phi_norm, x1_norm2: float, m: int) -> np.ndarray:
    """(k, 6) feature matrix of the k modes (canonical order)."""
    lam = np.asarray(lam, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    phi_norm = np.asarray(phi_norm, dtype=np.float64)
    k = len(lam)
    a = np.abs(lam)
    F = np.empty((k, NF))
    F[:, 0] = a
    F[:, 1] = np.abs(np.angle(lam))
    F[:, 2] = np.log(np.maximum(np.abs(b) * phi_norm / math.sqrt(x1_norm2), 1e-300))
    pmax = phi_norm.max() if k else 0.0
    F[:, 3] = phi_norm / pmax if pmax > 0 else 0.0
    t = np.arange(m, dtype=np.float64)
    F[:, 4] = (np.abs(b) ** 2 * phi_norm ** 2 / x1_norm2) * np.mean(a[:, None] ** (2.0 * t[None, :]), axis=1)
    F[:, 5] = np.arange(k) / k
    return F


def forward(theta, X):
    """Logits (N,) and the intermediate values."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = gelu(a1)
    a2 = h1 @ W2.T + b2
    h2 = gelu(a2)
    z = h2 @ w3 + b3
    return z, (X, a1, h1, a2, h2)


def bce_with_logits(z, y):
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))


def loss(theta, X, y) -> float:
    z, _ = forward(theta, X)
    return float(np.mean(bce_with_logits(z, y)))


def loss_and_grad(theta, X, y):
    """Mean BCE loss and its gradient with respect to the flat parameter vector, by the
    chain rule through the two GELU layers."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    z, (X, a1, h1, a2, h2) = forward(theta, X)
    y = np.asarray(y, dtype=np.float64)
    N = len(z)
    L = float(np.mean(bce_with_logits(z, y)))
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / N          # d loss / d z
    g_w3 = h2.T @ dz
    g_b3 = dz.sum()
    d_a2 = (dz[:, None] * w3[None, :]) * gelu_grad(a2)
    g_W2 = d_a2.T @ h1
    g_b2 = d_a2.sum(axis=0)
    d_a1 = (d_a2 @ W2) * gelu_grad(a1)
    g_W1 = d_a1.T @ X
    g_b1 = d_a1.sum(axis=0)
    g = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])
    return L, g


def numerical_grad(theta, X, y, h=1e-6, idx=None):
    """Central differences of the loss for the parameters in idx (all when None)."""
    theta = np.asarray(theta, dtype=np.float64)
    idx = np.arange(len(theta)) if idx is None else np.asarray(idx)
    g = np.empty(len(idx))
    for q, i in enumerate(idx):
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        g[q] = (loss(tp, X, y) - loss(tm, X, y)) / (2.0 * h)
    return g


class Adam:
    """Adam with bias correction, step count starting at 1."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def train(theta0, X, y, batches, lr=1e-3):
    """Adam over the given sequence of index batches (each an array of sample indices)."""
    theta = np.asarray(theta0, dtype=np.float64).copy()
    opt = Adam(len(theta), lr=lr)
    for bi in batches:
        _, g = loss_and_grad(theta, X[bi], y[bi])
        theta = opt.step(theta, g)
    return theta


def predict(theta, X, conf: float = 0.9):
    """Membership probabilities, the predicted support (p >= 1/2) and whether every mode
    is confident (max(p, 1 - p) >= conf)."""
    z, _ = forward(theta, X)
    pr = 1.0 / (1.0 + np.exp(-z))
    return pr, np.flatnonzero(pr >= 0.5), bool(np.all(np.maximum(pr, 1.0 - pr) >= conf))
