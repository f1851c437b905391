"""Seeded synthetic grayscale videos and sketch tables: the inputs only.

This module draws the inputs that both the FP64 oracle and the HIP path consume:
video frames, ground-truth foreground masks, the known background eigenvalues of
the generator, and the random index/sign tables of the sparse and single-pixel
measurement matrices.  It holds none of the cDMD arithmetic.

The videos stand in for the surveillance sequences the paper evaluates on
(ChangeDetection.net and BMC, Section "Evaluation on Real Videos"), which are not
available: a smooth static background, complex-valued oscillatory background
patterns whose temporal factors are exp(i*omega*t) (so that each pair of conjugate
eigenvalues is exactly representable by DMD), an optional slow real illumination
drift, bright moving rectangles as foreground, additive Gaussian noise, clipping and
optional uint8 quantisation.

Layout: ``D`` has shape (m, n) -- frame t is row t, contiguous -- with n = H*W in
row-major pixel order.  The paper's snapshot matrix X (pixels x frames) is D^T.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np
import torch

__all__ = [
    "VideoSpec", "Video", "PRESETS", "make_video", "sparse_table",
    "single_pixel_table", "preset",
]


@dataclasses.dataclass(frozen=True)
class VideoSpec:
    H: int
    W: int
    m: int
    n_pairs: int = 3                       # oscillatory background pairs
    bump_sigma: float = 12.0               # px, spatial Gaussian bumps of the pairs
    amp: Tuple[float, float] = (0.05, 0.10)
    omega: Tuple[float, float] = (0.05, 0.50)
    blur_sigma: float = 8.0                # px, static background smoothing
    bg_range: Tuple[float, float] = (0.2, 0.6)
    drift: Optional[Tuple[float, float]] = None   # (mu_lo, mu_hi): real |lambda| < 1 drift
    drift_amp: float = 0.05
    n_rects: int = 4
    rect_side: Tuple[int, int] = (20, 20)
    rect_value: Tuple[float, float] = (0.9, 0.9)
    speed: Tuple[float, float] = (1.0, 3.0)   # px per frame
    noise_sigma: float = 0.01
    out: str = "f32"                       # "u8" | "f32" | "f64"
    exact: bool = False                    # no foreground, noise, clipping, rounding
    seed: int = 1001

    @property
    def n(self) -> int:
        return self.H * self.W


PRESETS = {
    # 320x240x200 float32, Gaussian sketch p=500, k=10
    "cfg1": VideoSpec(H=240, W=320, m=200, n_pairs=3, bump_sigma=12.0, n_rects=4,
                      rect_side=(20, 20), rect_value=(0.9, 0.9), speed=(1.0, 3.0),
                      noise_sigma=0.01, out="f32", seed=1001),
    # 1920x1080x500 uint8, sparse sketch p=2000 x 32, k=25, tau=0.1
    "cfg2": VideoSpec(H=1080, W=1920, m=500, n_pairs=8, bump_sigma=72.0, n_rects=12,
                      rect_side=(40, 120), rect_value=(0.6, 1.0), speed=(2.0, 6.0),
                      noise_sigma=2.0 / 255.0, out="u8", seed=1002),
    # 3840x2160x1000 uint8, dense Gaussian sketch p=4000, k=40
    "cfg3": VideoSpec(H=2160, W=3840, m=1000, n_pairs=7, bump_sigma=144.0, n_rects=30,
                      rect_side=(60, 240), rect_value=(0.6, 1.0), speed=(2.0, 6.0),
                      drift=(0.995, 1.0), noise_sigma=2.0 / 255.0, out="u8", seed=1003),
    # the paper's timing shape: 1280x720x200, sparse p=1000
    "ctxA": VideoSpec(H=720, W=1280, m=200, n_pairs=8, bump_sigma=48.0, n_rects=12,
                      rect_side=(27, 80), rect_value=(0.6, 1.0), speed=(1.3, 4.0),
                      noise_sigma=2.0 / 255.0, out="u8", seed=1006),
    # 720x480x200 uint8: the shape of the sensing-matrix comparison (fps and F-measure vs p)
    "ctxB": VideoSpec(H=480, W=720, m=200, n_pairs=6, bump_sigma=32.0, n_rects=8,
                      rect_side=(18, 54), rect_value=(0.6, 1.0), speed=(1.0, 3.0),
                      noise_sigma=2.0 / 255.0, out="u8", seed=1007),
    # 640x480x300 uint8 (learned-selector training shape)
    "train640": VideoSpec(H=480, W=640, m=300, n_pairs=5, bump_sigma=24.0, n_rects=8,
                          rect_side=(13, 40), rect_value=(0.6, 1.0), speed=(1.0, 3.0),
                          noise_sigma=2.0 / 255.0, out="u8", seed=1005),
}


def preset(name: str, **overrides) -> VideoSpec:
    return dataclasses.replace(PRESETS[name], **overrides)


@dataclasses.dataclass
class Video:
    spec: VideoSpec
    D: torch.Tensor                 # (m, n) frames, dtype uint8 / float32 / float64
    scale: float                    # pixel value x = D * scale (1/255 for uint8)
    rects: np.ndarray               # (m, n_rects, 4) int: y0, x0, h, w per frame
    bg_lambda: np.ndarray           # known background eigenvalues (complex)
    bg_modes: Optional[np.ndarray]  # (n, len(bg_lambda)) complex b_j*phi_j, exact variant only

    def gt_mask(self, t0: int = 0, t1: Optional[int] = None,
                pixels: Optional[np.ndarray] = None) -> np.ndarray:
        """Ground-truth foreground coverage for frames [t0, t1) as bool (t1-t0, n)
        (or (t1-t0, len(pixels)) for a pixel subset)."""
        s = self.spec
        t1 = s.m if t1 is None else t1
        if pixels is None:
            out = np.zeros((t1 - t0, s.H, s.W), dtype=bool)
            for t in range(t0, t1):
                for (y0, x0, h, w) in self.rects[t]:
                    out[t - t0, y0:y0 + h, x0:x0 + w] = True
            return out.reshape(t1 - t0, s.n)
        py, px = np.divmod(np.asarray(pixels, dtype=np.int64), s.W)
        out = np.zeros((t1 - t0, len(py)), dtype=bool)
        for t in range(t0, t1):
            for (y0, x0, h, w) in self.rects[t]:
                out[t - t0] |= (py >= y0) & (py < y0 + h) & (px >= x0) & (px < x0 + w)
        return out


def _gauss1d(sigma: float, dtype, device) -> torch.Tensor:
    r = int(math.ceil(4.0 * sigma))
    x = torch.arange(-r, r + 1, dtype=dtype, device=device)
    g = torch.exp(-0.5 * (x / sigma) ** 2)
    return g / g.sum()


def _blur(img: torch.Tensor, sigma: float) -> torch.Tensor:
    """Separable Gaussian blur with reflect padding of an (H, W) image."""
    g = _gauss1d(sigma, img.dtype, img.device)
    r = (g.numel() - 1) // 2
    x = img[None, None]
    H, W = img.shape
    # reflect padding needs pad < size; fall back to replicate on tiny images
    mode = "reflect" if (r < H and r < W) else "replicate"
    x = torch.nn.functional.pad(x, (r, r, 0, 0), mode=mode)
    x = torch.nn.functional.conv2d(x, g.view(1, 1, 1, -1))
    x = torch.nn.functional.pad(x, (0, 0, r, r), mode=mode)
    x = torch.nn.functional.conv2d(x, g.view(1, 1, -1, 1))
    return x[0, 0]


def _bump(H: int, W: int, cy: float, cx: float, sigma: float, dtype, device) -> torch.Tensor:
    y = torch.arange(H, dtype=dtype, device=device)[:, None]
    x = torch.arange(W, dtype=dtype, device=device)[None, :]
    return torch.exp(-((y - cy) ** 2 + (x - cx) ** 2) / (2.0 * sigma * sigma))


def _rect_paths(spec: VideoSpec, rng: np.random.Generator) -> np.ndarray:
    """Linear paths reflected at the borders; returns (m, n_rects, 4) int32."""
    s = spec
    out = np.zeros((s.m, s.n_rects, 4), dtype=np.int32)
    for r in range(s.n_rects):
        h = int(rng.integers(s.rect_side[0], s.rect_side[1] + 1))
        w = int(rng.integers(s.rect_side[0], s.rect_side[1] + 1))
        h, w = min(h, s.H), min(w, s.W)
        py = float(rng.uniform(0, s.H - h))
        px = float(rng.uniform(0, s.W - w))
        sp = float(rng.uniform(*s.speed))
        th = float(rng.uniform(0, 2 * math.pi))
        vy, vx = sp * math.sin(th), sp * math.cos(th)
        for t in range(s.m):
            out[t, r] = (int(round(py)), int(round(px)), h, w)
            py += vy
            px += vx
            if py < 0 or py > s.H - h:
                vy = -vy
                py = min(max(py, 0.0), float(s.H - h))
            if px < 0 or px > s.W - w:
                vx = -vx
                px = min(max(px, 0.0), float(s.W - w))
    return out


def make_video(spec: VideoSpec, device: str | torch.device = "cpu",
               frame_chunk: int = 64) -> Video:
    """Draw one video.  Parameters come from a NumPy generator seeded with
    ``spec.seed``; the pixel noise comes from a torch generator on ``device`` with the
    same seed, so a given (spec, device type) always yields the same bytes."""
    s = spec
    device = torch.device(device)
    rng = np.random.default_rng(s.seed)
    fdt = torch.float64 if (s.exact or s.out == "f64") else torch.float32
    tg = torch.Generator(device=device)
    tg.manual_seed(s.seed)

    # static background: blurred uniform noise rescaled to bg_range
    u = torch.rand((s.H, s.W), generator=tg, device=device, dtype=fdt)
    bg = _blur(u, s.blur_sigma)
    lo, hi = bg.min(), bg.max()
    bg = s.bg_range[0] + (bg - lo) * ((s.bg_range[1] - s.bg_range[0]) / (hi - lo))
    bg = bg.reshape(-1)

    # oscillatory pairs: Re(a (g1 + i g2) e^{i w (t-1)})
    pats, lam, modes = [], [1.0 + 0.0j], []
    coeff_cos, coeff_sin = [], []
    omegas = []
    for _ in range(s.n_pairs):
        cy1, cx1 = rng.uniform(0, s.H), rng.uniform(0, s.W)
        cy2, cx2 = rng.uniform(0, s.H), rng.uniform(0, s.W)
        a = float(rng.uniform(*s.amp))
        w = float(rng.uniform(*s.omega))
        g1 = a * _bump(s.H, s.W, cy1, cx1, s.bump_sigma, fdt, device).reshape(-1)
        g2 = a * _bump(s.H, s.W, cy2, cx2, s.bump_sigma, fdt, device).reshape(-1)
        pats += [g1, g2]
        omegas.append(w)
        lam += [complex(math.cos(w), math.sin(w)), complex(math.cos(w), -math.sin(w))]
    drift_mu = None
    drift_field = None
    if s.drift is not None:
        drift_mu = float(rng.uniform(*s.drift))
        dfield = _blur(torch.rand((s.H, s.W), generator=tg, device=device, dtype=fdt),
                       4.0 * s.blur_sigma).reshape(-1)
        dfield = s.drift_amp * (dfield - dfield.min()) / (dfield.max() - dfield.min())
        drift_field = dfield
        lam.append(complex(drift_mu, 0.0))

    rects = _rect_paths(s, rng) if not s.exact else np.zeros((s.m, 0, 4), np.int32)
    rect_vals = rng.uniform(s.rect_value[0], s.rect_value[1], size=s.n_rects)

    P = torch.stack(pats) if pats else torch.zeros((0, s.n), dtype=fdt, device=device)

    out_dtype = {"u8": torch.uint8, "f32": torch.float32, "f64": torch.float64}[s.out]
    if s.exact and s.out == "u8":
        raise ValueError("the exact variant is unquantised; use out='f64' or 'f32'")
    D = torch.empty((s.m, s.n), dtype=out_dtype, device=device)
    om = torch.tensor(omegas, dtype=fdt, device=device)
    for t0 in range(0, s.m, frame_chunk):
        t1 = min(s.m, t0 + frame_chunk)
        tt = torch.arange(t0, t1, dtype=fdt, device=device)[:, None]  # t-1 for frame t
        X = bg[None, :].expand(t1 - t0, s.n).clone()
        if s.n_pairs:
            T = torch.empty((t1 - t0, 2 * s.n_pairs), dtype=fdt, device=device)
            T[:, 0::2] = torch.cos(tt * om[None, :])
            T[:, 1::2] = -torch.sin(tt * om[None, :])
            X += T @ P
        if drift_field is not None:
            X += (drift_mu ** tt) * drift_field[None, :]
        if not s.exact:
            Xv = X.view(t1 - t0, s.H, s.W)
            for t in range(t0, t1):
                for (y0, x0, h, w), val in zip(rects[t], rect_vals):
                    Xv[t - t0, y0:y0 + h, x0:x0 + w] = val
            X += s.noise_sigma * torch.randn(X.shape, generator=tg, device=device, dtype=fdt)
            X.clamp_(0.0, 1.0)
        if s.out == "u8":
            D[t0:t1] = torch.round(X * 255.0).clamp_(0, 255).to(torch.uint8)
        else:
            D[t0:t1] = X.to(out_dtype)
    scale = 1.0 / 255.0 if s.out == "u8" else 1.0

    bg_modes = None
    if s.exact:
        # b_j phi_j of the exact decomposition: static part, then each conjugate half
        cols = [bg.double().cpu().numpy().astype(np.complex128)]
        for j in range(s.n_pairs):
            psi = (pats[2 * j].double() + 1j * pats[2 * j + 1].double()).cpu().numpy()
            cols += [psi / 2.0, np.conj(psi) / 2.0]
        if drift_field is not None:
            cols.append(drift_field.double().cpu().numpy().astype(np.complex128))
        bg_modes = np.stack(cols, axis=1)
    return Video(spec=s, D=D, scale=scale, rects=rects, bg_lambda=np.array(lam),
                 bg_modes=bg_modes)


def sparse_table(n: int, p: int, nnz: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Fixed-row-weight sparse +/-1 measurement matrix: row r holds ``nnz`` distinct
    pixel indices (independent across rows) with Rademacher signs.
    Returns idx (p, nnz) int32 and sign (p, nnz) int8 in {+1, -1}."""
    if nnz > n:
        raise ValueError("nnz must not exceed n")
    rng = np.random.default_rng(seed)
    idx = np.empty((p, nnz), dtype=np.int64)
    # Floyd's sampling, vectorised over rows: for j = n-nnz .. n-1 draw t in [0, j];
    # take t unless already chosen in that row, else take j.
    for c, j in enumerate(range(n - nnz, n)):
        t = rng.integers(0, j + 1, size=p)
        if c:
            dup = (idx[:, :c] == t[:, None]).any(axis=1)
            t = np.where(dup, j, t)
        idx[:, c] = t
    sign = np.where(rng.integers(0, 2, size=(p, nnz)) == 1, 1, -1).astype(np.int8)
    return idx.astype(np.int32), sign


def iid_sparse_table(n: int, p: int, s: float, seed: int, width: int = 32) -> Tuple[np.ndarray, np.ndarray]:
    """Very sparse random projection with i.i.d. entries: +1 and -1 with probability
    1/(2s) each, 0 otherwise (s = n / ln n is the very sparse rate).  Drawn per row as a
    Binomial(n, 1/s) count of distinct, uniformly placed pixels with Rademacher signs (the
    same distribution).  Rows are padded with index -1 (sign +1) to the largest count.
    Returns idx (p, w) int32 and sign (p, w) int8; ValueError if w exceeds ``width``."""
    if not s >= 1.0:
        raise ValueError("need s >= 1")
    rng = np.random.default_rng(seed)
    counts = rng.binomial(n, 1.0 / s, size=p)
    w = max(1, int(counts.max()))
    if w > width:
        raise ValueError(f"a row holds {w} nonzeros, more than the table width {width}")
    idx = np.full((p, w), -1, dtype=np.int32)
    sign = np.ones((p, w), dtype=np.int8)
    for r in range(p):
        c = int(counts[r])
        if c:
            idx[r, :c] = rng.choice(n, size=c, replace=False)
            sign[r, :c] = np.where(rng.integers(0, 2, size=c) == 1, 1, -1)
    return idx, sign


def single_pixel_table(n: int, p: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Single-pixel measurements C = R: p distinct pixels (rows of the identity drawn
    without replacement), weight +1.  Returns idx (p, 1) int32, sign (p, 1) int8."""
    if p > n:
        raise ValueError("single-pixel sketch needs p <= n")
    rng = np.random.default_rng(seed)
    idx = rng.choice(n, size=p, replace=False).astype(np.int32)[:, None]
    return idx, np.ones((p, 1), dtype=np.int8)


def mlp_init(seed: int) -> np.ndarray:
    """Initial parameters of the 6-64-64-1 selector network as one flat vector in the
    order W1 (64 x 6), b1, W2 (64 x 64), b2, w3 (64), b3: weights uniform in
    +-1/sqrt(fan_in), biases zero; float32-representable values in a float64 array."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((6, 64), (64, 64), (64, 1)):
        lim = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)
