#!/usr/bin/env python3
"""Throughput of the cDMD hot path (fit + background-mode selection + foreground mask)
on one MI355X.

Workload (default): 1920x1080 grayscale, m = 500 uint8 frames resident in HBM, sparse
+/-1 sketch with p = 2000 rows x 32 pixels, target rank k = 25, OMP with K = 10
atoms, threshold tau = 0.1, bit-packed mask.  One step = one cdmd_fit + cdmd_select
+ cdmd_foreground over the whole video.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--prec both|fp32|bf16|fp32_compressed]
                    [--no-cpu-baseline]
                    [--workload cfg2|cfg1|cfg3|cfg4|video] [--copy-ref-mib N]
                    [--gauss-prec bf16|fp8] [--draw-c]
    python bench.py --summarize trace|traffic|counters --dir D [--dir D2] --out FILE ...

--workload cfg1 times the FP32 form of the dense Gaussian sketch on the 320x240x200
float32 video (p = 500, k = 10); cfg3 the BF16 form on the 3840x2160x1000 uint8 video
(p = 4000, k = 40; --gauss-prec fp8 the FP8 form; C is kept in device memory unless
--draw-c); cfg4 fits 64 streams of mixed shape and sketch with one graph launch per step;
video runs a 1000-frame 1080p video through cdmd_process_video in 200-frame batches with
the paper's evaluation settings (a step is the whole video).  The default line is the 1080p workload above.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"hbm": 8000.0, "fp32": 157.3, "fp64": 78.6, "bf16": 2500.0, "fp8": 5000.0}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def sector_bytes(idx, n, ld, m, sector=64):
    """Bytes of the distinct 64-byte sectors a sparse gather must fetch over all frames."""
    import numpy as np
    pix = np.unique(idx.ravel()).astype(np.int64)
    total = 0
    if (ld % sector) == 0:
        return int(np.unique(pix // sector).size) * sector * m
    for t in range(m):
        total += int(np.unique((t * ld + pix) // sector).size) * sector
    return total


def cpu_baseline(D_dev, spec, k, p, nnz, K, tau, band_rows, threads=None):
    """The FP64 oracle timed on the host on a horizontal band of the same video (the
    first ``band_rows`` image rows, all frames); stages that scale with the pixel
    count are extrapolated to the full frame, the n-independent SVD/eig stage is not.
    ``threads`` limits the BLAS/OpenMP threads (None: all the library uses)."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    import synthvideo as sv
    from oracle import cdmd_ref as R

    n_s = band_rows * spec.W
    D = D_dev[:, :n_s].contiguous().cpu().numpy()
    idx, sign = sv.sparse_table(n_s, p, nnz, seed=4242)
    scale = 1.0 / 255.0
    t = {}
    with threadpool_limits(limits=threads):
        used = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
        t0 = time.perf_counter()
        Y, _ = R.sketch_sparse(D, scale, idx, sign)
        t["sketch"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        lam, W, s, V, At = R.reduced_operator(Y, k)
        t["svd_eig"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        G = (V / s[None, :]) @ W
        Phi = R.lift(D, scale, G)
        x1 = D[0].astype(np.float64) * scale
        b = np.linalg.lstsq(Phi, x1.astype(np.complex128), rcond=None)[0]
        t["lift_lstsq"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        S, beta = R.omp(Phi, x1, K, lam=lam)
        t["omp"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        m = D.shape[0]
        for i0 in range(0, n_s, 16384):
            i1 = min(n_s, i0 + 16384)
            L = R.background(Phi[i0:i1][:, S], beta, lam[S], 0, m)
            R.foreground(R.pixel_rows(D, scale, i0, i1), L, tau)
        t["bg_mask"] = time.perf_counter() - t0
    f = spec.n / n_s
    total = t["svd_eig"] + f * (t["sketch"] + t["lift_lstsq"] + t["omp"] + t["bg_mask"])
    measured = sum(t.values())
    return {
        "value": m / total, "unit": "frames/s", "cores": int(used), "kind": "oracle",
        "host_cpus": os.cpu_count(),
        "sample": (f"FP64 oracle on rows 0..{band_rows - 1} of the same video ({n_s} of {spec.n} "
                   f"pixels, all {m} frames, p={p} with its own {nnz}-per-row table, k={k}, K={K}); "
                   f"measured {measured:.1f} s on {used} thread(s), pixel-proportional stages "
                   f"scaled x{f:.1f}, SVD/eig stage unscaled"),
        "stages_s": {kk: round(v, 3) for kk, v in t.items()},
    }


def oracle_quality(D_dev, idx, sign, k, K, tau, res, npix=20000, seed=0):
    """Per form: the GPU's eigenvalues, b_j phi_j on sampled pixels and the foreground mask on
    those pixels over all frames, against the FP64 oracle of the whole frame on the same
    (exact integer) sketch.  Mask disagreements must lie in the band ||x - L| - tau| <= band
    (1e-4 for float32-class forms, 2e-2 for the bfloat16 form); the oracle's OMP support is
    used for both (the GPU is given it explicitly when the oracle records a near tie)."""
    import numpy as np
    import torch
    from scipy.optimize import linear_sum_assignment
    import paper_1512_04205_amd as P
    from oracle import cdmd_ref as R

    t0 = time.perf_counter()
    Dh = D_dev.cpu().numpy()
    m, n = Dh.shape
    Yr, _ = R.sketch_sparse(Dh, 1.0 / 255.0, idx, sign)
    mo = R.fit(Dh, 1.0 / 255.0, Yr, k)
    x1 = Dh[0].astype(np.float64) / 255.0
    gaps = []
    Sr, br = R.omp(mo.Phi, x1, K, lam=mo.lam, margins=gaps)
    pix = np.sort(np.random.default_rng(seed).choice(n, npix, replace=False))
    x = Dh[:, pix].T.astype(np.float64) / 255.0
    Lr = R.background(mo.Phi[pix][:, Sr], br, mo.lam[Sr], 0, m)
    mr = R.foreground(x, Lr, tau)
    bphi_r = mo.Phi[pix] * mo.b[None, :]
    oracle_s = time.perf_counter() - t0
    del Dh
    out = {}
    pix_t = torch.from_numpy(pix).to(D_dev.device)
    for f, r in res.items():
        mdl = r["model"]
        q = {}
        lam_g = r["lam"]
        C = np.abs(lam_g[:, None] - mo.lam[None, :])
        a, b = linear_sum_assignment(C)
        q["eig_rel_err_max"] = float((C[a, b] / np.abs(mo.lam[b])).max())
        if f != "fp32_compressed":  # the compressed form's amplitudes answer another problem
            phi = torch.zeros((k, n), dtype=torch.complex64, device=D_dev.device)
            md = mdl.modes(video=D_dev, phi=phi)
            pg = phi[:, pix_t].cpu().numpy().T.astype(np.complex128)
            del phi
            bphi_g = pg * md["b"][None, :]
            err = np.abs(bphi_g[:, a] - bphi_r[:, b]).max() / np.abs(bphi_r).max()
            q["bphi_rel_err_max"] = float(err)
            near = 1e-4 if f == "fp32" else 3e-2
            if min(gaps) >= near:
                S, _ = mdl.select(P.SEL_OMP, K=K)
                q["omp_support_equal"] = bool(list(S) == list(Sr))
            if min(gaps) < near or not q["omp_support_equal"]:
                mdl.select(P.SEL_EXPLICIT, explicit=Sr)
            mk = torch.zeros((m, P.mask_words(n)), dtype=torch.int32, device=D_dev.device)
            mdl.foreground(D_dev, mk, tau)
            words = mk[:, (pix_t >> 5)].cpu().numpy().view(np.uint32)
            mg = ((words >> (pix & 31).astype(np.uint32)[None, :]) & 1).astype(bool).T
            diff = mg != mr
            band = 1e-4 if f == "fp32" else 2e-2
            q["mask_agreement"] = float(1.0 - diff.mean())
            q["mask_disagreements_in_band"] = bool((np.abs(np.abs(x - Lr) - tau)[diff] <= band).all())
            q["mask_band"] = band
        out[f] = q
    return out, {"pixels_sampled": npix, "frames": m, "oracle_s": round(oracle_s, 1),
                 "omp_min_margin": float(min(gaps))}


WORKLOADS = {
    # the headline: sparse sketch of a 1080p uint8 video
    "cfg2": dict(preset="cfg2", sketch="sparse", k=25, p=2000, nnz=32, K=10, tau=0.1,
                 desc="1920x1080 uint8 video, m=500, sparse +/-1 sketch p=2000 x 32, k=25, OMP K=10, "
                      "tau=0.1, fp64 small LA"),
    # FP32 form of the dense Gaussian sketch on the 320x240x200 float32 video
    "cfg1": dict(preset="cfg1", sketch="gaussian", k=10, p=500, nnz=0, K=10, tau=0.1, seed=1,
                 desc="320x240 float32 video, m=200, dense Gaussian sketch p=500 (FP32 form), k=10, "
                      "OMP K=10, tau=0.1, fp64 small LA"),
    # BF16 form of the dense Gaussian sketch on the 3840x2160x1000 uint8 video
    "cfg3": dict(preset="cfg3", sketch="gaussian", k=40, p=4000, nnz=0, K=10, tau=0.1, seed=3,
                 desc="3840x2160 uint8 video, m=1000, dense Gaussian sketch p=4000 (BF16 form), k=40, "
                      "OMP K=10, tau=0.1, fp64 small LA"),
    # the paper's evaluation settings on a long video: consecutive 200-frame batches, very
    # sparse C (s = n / ln n) with p = 1000, automatic rank, OMP K = 10, median-filtered masks
    "video": dict(preset="cfg2", sketch="iid", k=0, p=1000, nnz=32, K=10, tau=0.1, seed=21, frames=1000,
                  batch=200,
                  desc="1920x1080 uint8 video, 1000 frames in batches of 200, i.i.d. very sparse C "
                       "(s = n/ln n) with p=1000, automatic rank per batch, OMP K=10, tau=0.1, "
                       "3x3 median-filtered masks"),
    # Section 4's comparison of sensing matrices: fit time and F-measure against p for the
    # dense Gaussian, the i.i.d. very sparse and the single-pixel C on a 720x480x200 video
    "sensing": dict(preset="ctxB", sketch="sweep", k=0, p=0, nnz=32, K=10, tau=0.1, seed=31,
                    ps=(100, 250, 500, 1000, 2000, 4000), draws=5,
                    desc="720x480 uint8 video, m=200, rank by Remark 2 per draw, OMP K=10, tau=0.1: fit "
                         "frames/s and F-measure "
                         "against the generator's ground truth for p in {100..4000}, Gaussian (BF16 and "
                         "FP32 forms) / i.i.d. very sparse (s = n/ln n) / single-pixel / SRFT C, 5 draws of C "
                         "each"),
    # many independent streams in one graph launch
    "cfg4": dict(preset=None, sketch="mixed", k=0, p=0, nnz=32, K=10, tau=0.1, seed=4,
                 desc="64 uint8 streams in one batch: resolutions 320x240 / 640x480 / 1280x720 / "
                      "1920x1080, m in [100, 600], k in [5, 30], sparse (32 nnz) or dense Gaussian "
                      "(BF16 form) sketch with p in [20k, 100k], FP32 lift; aggregate frames/s of "
                      "batch fit + per-stream OMP + batched mask"),
}


def batch_streams(seed, count=64):
    """Parameters of the streams of the batched workload (seeded)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    res = [(240, 320), (480, 640), (720, 1280), (1080, 1920)]
    out = []
    for i in range(count):
        H, W = res[int(rng.integers(0, 4))]
        out.append(dict(H=H, W=W, m=int(rng.integers(100, 601)), k=int(rng.integers(5, 31)),
                        p=int(rng.integers(20000, 100001)), gauss=bool(rng.integers(0, 2)),
                        seed=9000 + i))
    return out


def run_video(args, wl):
    """A long video in consecutive batches (cdmd_process_video): returns the JSON line.
    A step is the whole video; value is its frames/s with three batches in flight, and the
    same with one and two is reported beside it."""
    import math
    import numpy as np
    import torch
    import paper_1512_04205_amd as P
    import synthvideo as sv
    spec = sv.preset(wl["preset"], m=wl["frames"], seed=1002)
    log(f"generating {spec.W}x{spec.H}x{spec.m} {spec.out} video on the GPU")
    v = sv.make_video(spec, device="cuda")
    n, frames = spec.n, spec.m
    idx, sign = sv.iid_sparse_table(n, wl["p"], n / math.log(n), wl["seed"])
    mask = torch.zeros((frames, P.mask_words(n)), dtype=torch.int32, device="cuda")
    res = {}
    for workers in (1, 2, 3):
        # the executor (streams, per-batch models, mask buffers) is made once, as a model is
        # for the other workloads; the first warmup video creates its models
        ex = P.VideoExecutor(n, wl["p"], batch_frames=wl["batch"], k=wl["k"], K=wl["K"], tau=wl["tau"],
                             workers=workers, median_hw=(spec.H, spec.W), idx=idx, sign=sign)

        def step():
            return ex.run(v.D, frames, mask)
        for _ in range(max(1, args.warmup)):
            used = step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            used = step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        # one-shot cdmd_process_video (executor created and freed inside the call), for context
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P.process_video(v.D, n, frames, wl["p"], mask, batch_frames=wl["batch"], k=wl["k"], K=wl["K"],
                        tau=wl["tau"], workers=workers, median_hw=(spec.H, spec.W), idx=idx, sign=sign)
        torch.cuda.synchronize()
        ms1 = (time.perf_counter() - t1) * 1e3
        ex.close()
        res[workers] = dict(ms=ms, fps=frames / (ms / 1e3), ranks=[int(x) for x in used], one_shot_ms=ms1)
        log(f"workers {workers}: {ms:.2f} ms per video, {frames / (ms / 1e3):.0f} frames/s, ranks {used}; "
            f"one-shot call with set-up {ms1:.2f} ms")
    gt_frac = float(np.mean(v.gt_mask(0, 10)))
    return {
        "metric": "frames/sec cDMD fit+fg mask, long 1080p video in 200-frame batches",
        "value": res[3]["fps"], "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res[3]["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["desc"], "n": n, "frames": frames, "batch": wl["batch"], "p": wl["p"],
                   "K": wl["K"], "tau": wl["tau"]},
        "roofline": None,
        "workers": 3,
        "by_workers": {w: {"ms_per_step": r["ms"], "fps": r["fps"], "one_shot_ms": r["one_shot_ms"]}
                       for w, r in res.items()},
        "ranks_per_batch": res[3]["ranks"],
        "foreground_fraction_first_frames": gt_frac,
        "note": "a step is the whole video: every batch sketched, fitted, selected, thresholded and median "
                "filtered by a reused executor; one_shot_ms: one cdmd_process_video call, set-up included",
    }


def run_sensing(args, wl):
    """fps of the fit (sketch through amplitudes and the OMP selection; the mask excluded) and
    F-measure of the foreground mask against the ground truth, for every sensing matrix and
    p, each over several draws of C; returns the JSON line (value: the i.i.d. very sparse C
    at p = 1000, the paper's evaluation setting)."""
    import math
    import numpy as np
    import torch
    import paper_1512_04205_amd as P
    import synthvideo as sv
    spec = sv.PRESETS[wl["preset"]]
    log(f"generating {spec.W}x{spec.H}x{spec.m} {spec.out} video on the GPU")
    v = sv.make_video(spec, device="cuda")
    m, n = v.D.shape
    k, K, tau = wl["k"], wl["K"], wl["tau"]
    gt = torch.from_numpy(v.gt_mask()).cuda()
    mask = torch.zeros((m, P.mask_words(n)), dtype=torch.int32, device="cuda")
    shifts = torch.arange(32, dtype=torch.int32, device="cuda")

    def f_measure():
        bits = ((mask.unsqueeze(-1) >> shifts) & 1).reshape(m, -1)[:, :n].bool()
        tp = (bits & gt).sum().item()
        fp = (bits & ~gt).sum().item()
        fn = (~bits & gt).sum().item()
        return 2.0 * tp / (2.0 * tp + fp + fn) if tp + fp + fn else 1.0

    def model(kind, p, draw):
        # the rank of each draw by Remark 2 (the paper's evaluation setting), not timed
        seed = wl["seed"] * 1000 + draw
        if kind.startswith("gaussian"):
            sp = P.PREC_BF16 if kind == "gaussian_bf16" else P.PREC_FP32
            kw = dict(sketch=P.SKETCH_GAUSSIAN, dtype=P.U8, seed=seed, sketch_prec=sp)
        elif kind == "sparse":
            idx, sign = sv.iid_sparse_table(n, p, n / math.log(n), seed)
            kw = dict(idx=idx, sign=sign)
        elif kind == "srft":
            fr = np.random.default_rng(seed).choice(n, size=p, replace=False).astype(np.int32)
            kw = dict(sketch=P.SKETCH_SRFT, idx=fr.reshape(p, 1), seed=seed)
        else:
            idx, sign = sv.single_pixel_table(n, p, seed)
            kw = dict(sketch=P.SKETCH_SPIXEL, idx=idx, sign=sign)
        if kind == "srft":  # no automatic rank for a complex sketch: the i.i.d. sparse C's rank
            kd = k if k > 0 else max(1, min(srft_rank[p], p, m - 1, 40))
        else:
            kd = k if k > 0 else max(1, min(P.optimal_rank(v.D, n, m, p, **kw)[0], p, m - 1, 40))
            if kind == "sparse" and draw == 0:
                srft_rank[p] = kd
        return P.Model(n, m, kd, p, **kw), kd

    table = []
    srft_rank = {}
    for kind in ("gaussian_bf16", "gaussian_fp32", "sparse", "spixel", "srft"):
        for p in wl["ps"]:
            ms, fs, ks = [], [], []
            for draw in range(wl["draws"]):
                mdl, kd = model(kind, p, draw)
                ks.append(kd)
                mdl.fit(v.D)  # warm-up: first use of the model's buffers
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                reps = max(1, args.steps // 4)
                for _ in range(reps):
                    mdl.fit(v.D)
                    mdl.select(P.SEL_OMP, K=K)
                torch.cuda.synchronize()
                ms.append((time.perf_counter() - t0) / reps * 1e3)
                mdl.foreground(v.D, mask, tau)
                torch.cuda.synchronize()
                fs.append(f_measure())
                mdl.close()
            row = dict(sensing=kind, p=p, k=[int(x) for x in ks], ms_fit=float(np.median(ms)),
                       fps=float(m / (np.median(ms) / 1e3)),
                       f_mean=float(np.mean(fs)), f_std=float(np.std(fs)), f_min=float(np.min(fs)),
                       f_max=float(np.max(fs)))
            table.append(row)
            log(f"{kind:14s} p={p:5d} k={ks}: {row['ms_fit']:.3f} ms/fit, {row['fps']:.0f} fps, "
                f"F {row['f_mean']:.4f} +- {row['f_std']:.4f} [{row['f_min']:.4f}, {row['f_max']:.4f}]")
    head = next(r for r in table if r["sensing"] == "sparse" and r["p"] == 1000)
    return {
        "metric": "frames/sec cDMD fit (sketch..amplitudes + OMP), 720x480x200, by sensing matrix and p",
        "value": head["fps"], "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": head["ms_fit"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl["desc"], "n": n, "frames": m, "k": k, "K": K, "tau": tau,
                   "value_is": "i.i.d. very sparse C, p = 1000"},
        "roofline": None,
        "sweep": table,
        "note": "fps = frames / median fit time over the draws (sketch, Gram, small LA, lift, amplitudes, "
                "OMP; the mask excluded); F = 2TP / (2TP + FP + FN) of the tau = 0.1 mask over every pixel "
                "and frame against the generator's ground truth",
    }


def run_batch(args, wl):
    """The batched workload: returns the JSON line."""
    import numpy as np
    import torch

    import paper_1512_04205_amd as P
    import synthvideo as sv

    streams = batch_streams(wl["seed"])
    videos, models, masks = [], [], []
    log(f"generating {len(streams)} streams")
    for s in streams:
        spec = sv.preset("cfg2", H=s["H"], W=s["W"], m=s["m"], n_pairs=4, bump_sigma=s["W"] / 30.0,
                         n_rects=6, rect_side=(s["W"] // 50, s["W"] // 16), seed=s["seed"])
        v = sv.make_video(spec, device="cuda")
        n = s["H"] * s["W"]
        if s["gauss"]:
            mdl = P.Model(n, s["m"], s["k"], s["p"], sketch=P.SKETCH_GAUSSIAN, seed=s["seed"],
                          sketch_prec=P.PREC_BF16)
        else:
            idx, sign = sv.sparse_table(n, s["p"], wl["nnz"], seed=s["seed"])
            mdl = P.Model(n, s["m"], s["k"], s["p"], sketch=P.SKETCH_SPARSE, idx=idx, sign=sign)
        videos.append(v.D)
        models.append(mdl)
        masks.append(torch.zeros((s["m"], P.mask_words(n)), dtype=torch.int32, device="cuda"))
    batch = P.Batch(models)
    frames = sum(s["m"] for s in streams)

    def step():
        st = batch.statuses(videos)
        if all(c == P.OK for c in st):
            for mdl in models:
                mdl.select(P.SEL_OMP, K=min(wl["K"], mdl.k))
            batch.foreground(videos, masks, wl["tau"])   # every stream's mask in one work-queue launch
            return st
        for mdl, v, mk, code in zip(models, videos, masks, st):
            if code == P.OK:
                mdl.select(P.SEL_OMP, K=min(wl["K"], mdl.k))
                mdl.foreground(v, mk, wl["tau"])
        return st

    log(f"warmup {args.warmup} (first call: autotuning and graph capture)")
    t0 = time.perf_counter()
    st = step()
    torch.cuda.synchronize()
    log(f"first call {time.perf_counter() - t0:.2f} s, statuses {sorted(set(st))}")
    for _ in range(max(args.warmup - 1, 0)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    ok = sum(1 for c in st if c == P.OK)
    log(f"batch step {ms:.2f} ms, {ok}/{len(st)} streams fitted, {frames} frames")
    # the mask phase alone (selection done): one work-queue launch against a launch per stream
    mask_ms = {}
    if ok == len(st):
        reps = 5

        def one_launch():
            batch.foreground(videos, masks, wl["tau"])

        def per_stream():
            for mdl, v, mk in zip(models, videos, masks):
                mdl.foreground(v, mk, wl["tau"])

        for name, fn in (("work_queue", one_launch), ("per_stream", per_stream)):
            fn()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            mask_ms[name] = (time.perf_counter() - t1) / reps * 1e3
        log(f"mask phase: {mask_ms}")
    return {
        "metric": "frames/sec cDMD fit+fg mask, 1080p, BF16 vs FP32 at stated eig err; HBM GB/s",
        "value": frames / (ms / 1e3), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": wl["desc"], "streams": len(streams), "frames": frames,
                   "sparse_streams": sum(1 for s in streams if not s["gauss"]),
                   "gaussian_streams": sum(1 for s in streams if s["gauss"]),
                   "statuses": [int(c) for c in st]},
        "roofline": None,
        "mask_phase_ms": mask_ms,
        "note": "the fits run inside one graph launch, the masks of all streams in one work-queue launch "
                "(mask_phase_ms: that launch against one cdmd_foreground per stream); per-kernel times "
                "come from rocprofv3",
    }


def sources_sha256():
    """Hash of the HIP/C++ sources of the library (kernels and host code)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1512_04205_amd", "csrc")
    for s in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))
                    + glob.glob(os.path.join(csrc, "*.cpp"))):
        h.update(os.path.basename(s).encode())
        with open(s, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel of known size)
    from the committed counter summary, if it was taken on the current sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        t = json.load(f)
    if t.get("sources_sha256") != sources_sha256():
        return {}
    return {q: d["fetch_bytes"] + d["write_bytes"] for q, d in t["kernels"].items()}


# ---------------------------------------------------------------- profile summaries
# `python bench.py --summarize trace|traffic|counters ...` turns rocprofv3 CSV output into
# the short summaries kept under profiles/ (the traffic summary is what measured_traffic
# reads back).

GROUPS = (("k_sketch", "sketch"), ("k_gram", "gram"), ("k_lift", "lift"), ("k_recon<", "recon"),
          ("k_la_a", "lanczos"))


def short_name(kn):
    kn = kn.replace("void ", "").replace("cdmd::k::", "").replace("(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in kn:  # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def group_of(name):
    for key, g in GROUPS:
        if name.startswith(key):
            return g
    return None


def read_csv(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def find_csv(d, suffix):
    import glob
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def summarize_trace(d, last, title, cmd, out_path, bench_log=None):
    """Per-kernel durations inside the last `last` steps: from the sketch dispatch before the
    first of the last `last` Lanczos dispatches to the end of the reconstruction after the
    last one (earlier dispatches, such as the autotuner's trials of other tile shapes and
    the video generator, are left out)."""
    rows = read_csv(find_csv(d, "kernel_trace.csv"))
    ev = sorted(((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"]))
                 for r in rows), key=lambda e: e[0])
    la = [i for i, e in enumerate(ev) if e[2] == "k_la_a"][-last:]
    i0 = max(i for i in range(la[0]) if group_of(ev[i][2]) == "sketch")
    i1 = min(i for i in range(la[-1], len(ev)) if group_of(ev[i][2]) == "recon")
    per = {}
    for st, en, name in ev[i0:i1 + 1]:
        per.setdefault(name, []).append((en - st) / 1e3)
    span = (ev[i1][1] - ev[i0][0]) / 1e3 / last
    lines = [title, "", "Command (from the repository root, TMPDIR=/tmp):", "  " + cmd, "",
             f"Kernels dispatched in the last {last} steps (warm-up and timed; the autotuner's trials of other",
             "tile shapes and the video generator come before them and are left out): calls per step and",
             "durations.", "",
             f"{'kernel':44s} {'per step':>8s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'us/step':>9s}"]
    tot = 0.0
    for name, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        avg = sum(v) / len(v)
        tot += sum(v) / last
        lines.append(f"{name[:44]:44s} {len(v) / last:8.1f} {avg:9.1f} {min(v):9.1f} {max(v):9.1f} "
                     f"{sum(v) / last:9.1f}")
    lines += ["", f"sum of the kernel times per step: {tot:.1f} us; step span (first sketch to last mask, "
                  f"kernels of the second stream overlapping): {span:.1f} us"]
    if bench_log:
        with open(bench_log) as f:
            js = [l for l in f if l.startswith("{")]
        if js:
            b = json.loads(js[-1])
            lines.append(f"bench ms_per_step under the profiler: {b['ms_per_step']:.3f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counter_table(d):
    """{dispatch: (kernel, {counter: value summed over instances}, duration_ns)}"""
    rows = read_csv(find_csv(d, "counter_collection.csv"))
    disp = {}
    for r in rows:
        did = int(r["Dispatch_Id"])
        e = disp.setdefault(did, [r["Kernel_Name"], {}, int(r["End_Timestamp"]) - int(r["Start_Timestamp"])])
        e[1][r["Counter_Name"]] = e[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return disp


def summarize_traffic(fetch_dir, write_dir, workload, cmds, out_path, ref_mib=1024):
    """HBM bytes per dispatch of each kernel group from FETCH_SIZE and WRITE_SIZE (KiB),
    scaled by what the counters read for the copy of ref_mib MiB (ref_mib read and written);
    the last dispatch of each group."""
    res = {}
    for kind, d in (("fetch", fetch_dir), ("write", write_dir)):
        cname = "FETCH_SIZE" if kind == "fetch" else "WRITE_SIZE"
        tab = counter_table(d)
        ref = [v[1][cname] for k, v in sorted(tab.items()) if "copyBuffer" in v[0] or "copy" in v[0].lower()]
        ref_kib = max(ref) if ref else None
        res[kind + "_ref_kib"] = ref_kib
        # the last step: from the sketch before the last Lanczos dispatch to the first
        # reconstruction after it (dispatch order)
        ids = sorted(tab)
        names = {i: short_name(tab[i][0]) for i in ids}
        la = max(i for i in ids if names[i] == "k_la_a")
        i0 = max(i for i in ids if i < la and group_of(names[i]) == "sketch")
        i1 = min(i for i in ids if i > la and group_of(names[i]) == "recon")
        for did in ids:
            if did < i0 or did > i1:
                continue
            kn, cv, _ = tab[did]
            g = group_of(names[did])
            if g is None or cname not in cv:
                continue
            res.setdefault(g, {})[kind] = (names[did], cv[cname])
    expect = ref_mib * 1024.0
    fs = expect / res["fetch_ref_kib"] if res["fetch_ref_kib"] else 1.0
    ws = expect / res["write_ref_kib"] if res["write_ref_kib"] else 1.0
    out = {"workload": workload, "commands": cmds,
           "reference": {"kernel": f"device-to-device copy of {ref_mib} MiB", "fetch_kib": res["fetch_ref_kib"],
                         "write_kib": res["write_ref_kib"], "fetch_scale": fs, "write_scale": ws},
           "sources_sha256": sources_sha256(), "kernels": {}}
    for _, g in GROUPS:
        if g in res and "fetch" in res[g] and "write" in res[g]:
            out["kernels"][g] = {"kernel": res[g]["fetch"][0],
                                 "fetch_bytes": int(res[g]["fetch"][1] * 1024 * fs),
                                 "write_bytes": int(res[g]["write"][1] * 1024 * ws)}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


def summarize_counters(d, title, cmd, out_path, kernels):
    """The counters of the last dispatch of each kernel whose short name starts with one of
    `kernels`, with the MFMA rate from SQ_INSTS_VALU_MFMA_MOPS_* (512 flops each)."""
    tab = counter_table(d)
    last = {}
    for did, (kn, cv, dur) in sorted(tab.items()):
        nm = short_name(kn)
        if any(nm.startswith(k) for k in kernels):
            last[nm] = (cv, dur)
    lines = [title, "", "Command (from the repository root, TMPDIR=/tmp):", "  " + cmd, ""]
    for nm, (cv, dur) in last.items():
        lines.append(f"{nm}: {dur / 1e3:.1f} us under the profiler")
        for c in sorted(cv):
            lines.append(f"  {c:34s} {cv[c]:.6g}")
        mops = sum(v for c, v in cv.items() if c.startswith("SQ_INSTS_VALU_MFMA_MOPS"))
        if mops:
            lines.append(f"  MFMA work {mops * 512 / 1e9:.2f} GFLOP -> {mops * 512 / dur / 1e3:.1f} TFLOP/s "
                         f"over the dispatch")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in cv and "SQ_BUSY_CU_CYCLES" in cv and cv["SQ_BUSY_CU_CYCLES"]:
            # the busy cycles of the four SIMDs' matrix cores over the CUs' busy cycles
            lines.append(f"  MFMA busy fraction SQ_VALU_MFMA_BUSY_CYCLES / (4 SQ_BUSY_CU_CYCLES): "
                         f"{cv['SQ_VALU_MFMA_BUSY_CYCLES'] / (4 * cv['SQ_BUSY_CU_CYCLES']):.3f}")
        if mops:
            lines.append(f"  MFMA rate / dense BF16 peak (2500 TFLOP/s): {mops * 512 / dur / 1e3 / 2500:.3f}")
        lines.append("")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def lanczos_flops(N, J):
    """Algorithmic float64 work of J Lanczos steps: the matvec with the N x N Gram (2N^2)
    and two classical Gram-Schmidt passes against j vectors (8Nj)."""
    return 2.0 * J * N * N + 4.0 * N * J * J


def la_rest_flops(N, k, J):
    """The rest of the small linear algebra: the Ritz vectors Q Z, M12 V and V^T (M12 V)."""
    return 2.0 * N * J * k + 2.0 * N * N * k + 2.0 * N * k * k


def la_groups(N):
    """Workgroups (one per compute unit) of the device Lanczos: one per 32 rows, at most 32."""
    return max(1, min(32, (N + 31) // 32))


def summarize_main(argv):
    ap = argparse.ArgumentParser(prog="bench.py --summarize")
    ap.add_argument("--summarize", choices=["trace", "traffic", "counters"], required=True)
    ap.add_argument("--dir", action="append", required=True, help="rocprofv3 output directories")
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", default="")
    ap.add_argument("--cmd", action="append", default=[])
    ap.add_argument("--last", type=int, default=4)
    ap.add_argument("--bench-log")
    ap.add_argument("--workload", default="")
    ap.add_argument("--kernels", default="k_lift,k_recon<,k_sketch")
    a = ap.parse_args(argv)
    if a.summarize == "trace":
        summarize_trace(a.dir[0], a.last, a.title, " ".join(a.cmd), a.out, a.bench_log)
    elif a.summarize == "traffic":
        summarize_traffic(a.dir[0], a.dir[1], a.workload, a.cmd, a.out)
    else:
        summarize_counters(a.dir[0], a.title, " ".join(a.cmd), a.out, a.kernels.split(","))


def main():
    if "--summarize" in sys.argv:
        summarize_main(sys.argv[1:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="both", choices=["fp32", "bf16", "fp32_compressed", "both"],
                    help="lift/reconstruction form (cfg2); 'both' times FP32 (the reported value), "
                         "BF16 and FP32 with the amplitudes on the compressed modes side by side")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--gauss-prec", default="bf16", choices=["bf16", "fp8"],
                    help="cfg3: the precision form of the dense Gaussian sketch")
    ap.add_argument("--draw-c", action="store_true",
                    help="cfg3: draw the Gaussian C on the fly instead of storing it in device memory")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip cdmd_autotune before the warm-up (default tile shapes)")
    ap.add_argument("--cpu-band-rows", type=int, default=68)
    ap.add_argument("--cpu-band-rows-1t", type=int, default=17,
                    help="band of the single-thread CPU baseline")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the per-form comparison with the full-frame FP64 oracle (cfg2)")
    ap.add_argument("--copy-ref-mib", type=int, default=1024,
                    help="run a device-to-device copy of this many MiB first (the reference "
                         "kernel for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is pixel sharding, described but not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1512_04205_amd as P
    import synthvideo as sv

    wl = WORKLOADS[args.workload]
    if args.workload == "cfg4":
        print(json.dumps(run_batch(args, wl)), flush=True)
        return
    if args.workload == "video":
        print(json.dumps(run_video(args, wl)), flush=True)
        return
    if args.workload == "sensing":
        print(json.dumps(run_sensing(args, wl)), flush=True)
        return
    copy_gbs = None
    if args.copy_ref_mib > 0:
        # device-to-device copy of a known size: the measured HBM ceiling (read + write bytes
        # over the copy's event time), and the reference kernel for scaling HBM counters
        a = torch.empty(args.copy_ref_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 2.0 * a.numel() * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
        log(f"copy reference: {args.copy_ref_mib} MiB read + {args.copy_ref_mib} MiB written, {copy_gbs:.0f} GB/s")
        del a, b
    spec = sv.PRESETS[wl["preset"]]
    k, p, nnz, K, tau = wl["k"], wl["p"], wl["nnz"], wl["K"], wl["tau"]
    gauss = wl["sketch"] == "gaussian"
    log(f"generating {spec.W}x{spec.H}x{spec.m} {spec.out} video on the GPU")
    v = sv.make_video(spec, device="cuda")
    D = v.D
    m, n = D.shape
    u8 = D.dtype == torch.uint8
    if gauss:
        idx = sign = None
    else:
        idx, sign = sv.sparse_table(n, p, nnz, seed=2002)
    mask = torch.zeros((m, P.mask_words(n)), dtype=torch.int32, device="cuda")
    sect = sector_bytes(idx, n, n, m) if not gauss else 0
    video_bytes = float(n) * m * (1 if u8 else 4)

    def run_form(prec: str):
        # "fp32_compressed": the FP32 form with the amplitudes and the selection on the
        # compressed modes (Remark 3: no lift in the fit)
        lp = P.PREC_BF16 if prec == "bf16" else P.PREC_FP32
        if gauss:
            sp = ({"bf16": P.PREC_BF16, "fp8": P.PREC_FP8}[args.gauss_prec] if args.workload == "cfg3"
                  else P.PREC_FP32)
            mdl = P.Model(n, m, k, p, sketch=P.SKETCH_GAUSSIAN, dtype=P.U8 if u8 else P.F32,
                          seed=wl["seed"], sketch_prec=sp, lift_prec=lp)
            if sp != P.PREC_FP32 and not args.draw_c:
                try:
                    mdl.store_measurement(True)
                    stored_c[prec] = True
                    log(f"[{prec}] C stored in device memory ({p} x {n})")
                except P.CdmdError as e:
                    log(f"[{prec}] C drawn on the fly ({e})")
        else:
            mdl = P.Model(n, m, k, p, sketch=P.SKETCH_SPARSE, dtype=P.U8, idx=idx, sign=sign,
                          lift_prec=lp)
        mdl.set_timing(True)
        if prec == "fp32_compressed":
            mdl.set_amplitudes(P.AMP_COMPRESSED)
        if not args.no_autotune:
            mdl.autotune(D)
            log(f"[{prec}] autotuned: lift workgroups {mdl.info()['lift_grid']}, sparse form "
                f"{mdl.info()['sparse_form']}, Gaussian slices {mdl.info()['sketch_slices']}")

        def step():
            mdl.fit(D)
            mdl.select(P.SEL_OMP, K=K)
            mdl.foreground(D, mask, tau)

        log(f"[{prec}] warmup {args.warmup}")
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        acc = {"sketch": 0.0, "gram": 0.0, "lift": 0.0, "recon": 0.0, "small_la": 0.0, "lanczos": 0.0}
        log(f"[{prec}] timing {args.steps} steps")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
            inf = mdl.info()
            acc["sketch"] += inf["gpu_ms_sketch"]
            acc["gram"] += inf["gpu_ms_gram"]
            acc["lift"] += inf["gpu_ms_lift"]
            acc["recon"] += inf["gpu_ms_recon"]
            acc["small_la"] += inf["ms_small_la"]
            acc["lanczos"] += inf["gpu_ms_lanczos"]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms = (t1 - t0) / args.steps * 1e3
        avg = {kk: vv / args.steps for kk, vv in acc.items()}
        avg["la_rest"] = avg["small_la"] - avg["lanczos"]
        inf = mdl.info()
        log(f"[{prec}] per-step ms", {kk: round(vv, 4) for kk, vv in avg.items()}, "total", round(ms, 3))
        S_n = inf["n_selected"]
        J = inf["lanczos_steps"]
        N = m - 1
        # algorithmic work per launch: (bytes that must cross HBM, useful flops, flop peak).
        # The lift is Phi' = X' (V S^-1) (k real columns) with the fused Gram of [Phi' | x_1],
        # on bf16 MFMA in both forms (the FP32 form splits V S^-1 into three bf16 terms).
        if gauss:
            sk_peak = PEAK["bf16"] if args.workload == "cfg3" else PEAK["fp32"]
            sk = (video_bytes + 4.0 * p * m, 2.0 * p * n * m, sk_peak)
        else:
            sk = (sect + idx.size * 8 + 4.0 * p * m, 2.0 * idx.size * m, PEAK["fp32"])
        work = {
            "sketch": sk,
            "gram": (4.0 * p * m + 8.0 * m * m, 2.0 * p * m * m, PEAK["fp64"]),
            "lift": (video_bytes, 2.0 * n * (m - 1) * k + 2.0 * n * (k + 1) ** 2, PEAK["bf16"]),
            "recon": (2.0 * video_bytes + n * m / 8.0, 8.0 * n * m * S_n, PEAK["fp32"]),
            # the float64 small linear algebra, against the chip's published float64 rate
            "lanczos": (8.0 * m * m, lanczos_flops(N, J), PEAK["fp64"]),
            "la_rest": (8.0 * m * m, la_rest_flops(N, k, J), PEAK["fp64"]),
        }
        kernels = {}
        for q, (byt, fl, fpk) in work.items():
            if avg[q] <= 0.0:  # not run in this form (the lift of the compressed form)
                continue
            sec = avg[q] / 1e3
            gbs, tfs = byt / sec / 1e9, fl / sec / 1e12
            hb, fb = gbs / PEAK["hbm"], tfs / fpk
            if q in ("lanczos", "la_rest"):
                bound = "alu"
            elif hb >= fb:
                bound = "hbm"
            else:
                bound = "mfma" if (q in ("lift", "recon") or fpk >= PEAK["bf16"]) else "alu"
            kernels[q] = {"ms": round(avg[q], 4), "GB/s": round(gbs, 1), "TFLOP/s": round(tfs, 4),
                          "hbm_frac": round(hb, 4), "flop_frac": round(fb, 4), "bound": bound,
                          "bytes": byt, "flops": fl, "flop_peak": fpk}
        lam = mdl.modes()["lam"]
        return {"ms": ms, "fps": m / (ms / 1e3), "avg": avg, "kernels": kernels, "lam": lam, "model": mdl,
                "lanczos": J, "n_sel": S_n,
                "tiles": {"lift_grid": inf["lift_grid"], "sparse_form": inf["sparse_form"],
                          "sketch_slices": inf["sketch_slices"]}}

    if args.workload == "cfg2":
        forms = ["fp32", "bf16", "fp32_compressed"] if args.prec == "both" else [args.prec]
    else:
        forms = ["bf16"] if args.workload == "cfg3" else ["fp32"]
    stored_c = {}
    res = {f: run_form(f) for f in forms}

    from scipy.optimize import linear_sum_assignment
    lam_r, ref_kind = None, None
    if args.workload == "cfg2":
        log("oracle eigenvalues from the exact sketch")
        from oracle import cdmd_ref as R
        Dh = D.cpu().numpy()
        Yr, _ = R.sketch_sparse(Dh, 1.0 / 255.0, idx, sign)
        lam_r = R.reduced_operator(Yr, k)[0]
        ref_kind = "FP64 oracle on the same (exact integer) sketch"
        del Dh
    elif args.workload == "cfg1":
        log("oracle eigenvalues (FP64 Gaussian sketch)")
        from oracle import cdmd_ref as R
        Dh = D.cpu().numpy()
        Yr = R.sketch_gaussian(Dh, v.scale, wl["seed"], p)
        lam_r = R.reduced_operator(Yr, k)[0]
        ref_kind = "FP64 oracle, unquantised Gaussian C"
        del Dh
    else:
        log("FP32-form GPU eigenvalues as the reference (the FP64 oracle would take hours here)")
        ref = P.Model(n, m, k, p, sketch=P.SKETCH_GAUSSIAN, dtype=P.U8, seed=wl["seed"],
                      sketch_prec=P.PREC_FP32)
        ref.fit(D)
        lam_r = ref.modes()["lam"]
        ref_kind = "FP32 form of the same sketch on the GPU (float64 normals)"
        del ref
    for f, r in res.items():
        C = np.abs(r["lam"][:, None] - lam_r[None, :])
        a, b = linear_sum_assignment(C)
        r["eig_rel_err_max"] = float((C[a, b] / np.abs(lam_r[b])).max())

    head = res[forms[0]]
    dom = max(head["kernels"], key=lambda q: head["kernels"][q]["ms"])

    def roof_of(kd):
        if kd["bound"] == "hbm":
            return {"bound": "hbm", "achieved": kd["GB/s"], "peak": PEAK["hbm"], "unit": "GB/s",
                    "frac": kd["hbm_frac"]}
        return {"bound": kd["bound"], "achieved": kd["TFLOP/s"], "peak": kd["flop_peak"],
                "unit": "TFLOP/s", "frac": kd["flop_frac"]}

    traffic = measured_traffic({"cfg2": "1080p_m500"}.get(args.workload, args.workload)) \
        if forms[0] == "fp32" else {}
    roof = roof_of(head["kernels"][dom])
    roof.update({"kernel": dom, "traffic": traffic.get(dom)})
    if dom in ("lanczos", "la_rest"):
        # secondary figure: the share of the float64 rate of the compute units the solve occupies
        cus = la_groups(m - 1) if dom == "lanczos" else 1
        roof["occupied_cus"] = cus
        roof["frac_of_occupied_cus"] = round(roof["achieved"] / (PEAK["fp64"] * cus / 256.0), 5)
    streaming = {q: dict(roof_of(head["kernels"][q]), ms=head["kernels"][q]["ms"], traffic=traffic.get(q))
                 for q in ("sketch", "lift", "recon")}
    out = {
        "metric": "frames/sec cDMD fit+fg mask, 1080p, BF16 vs FP32 at stated eig err; HBM GB/s",
        "value": head["fps"],
        "unit": "frames/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if forms[0] == "fp32" else "bf16",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": n, "m": m, "k": k, "p": p, "nnz": nnz, "K": K,
                   "tau": tau, "lift_prec": forms[0],
                   **({"sketch_prec": args.gauss_prec, "c_stored": bool(stored_c.get(forms[0]))}
                      if args.workload == "cfg3" else {})},
        "roofline": roof,
        "streaming_rooflines": streaming,
        "sketch_hbm_gbps": head["kernels"]["sketch"]["GB/s"],
        "eig_rel_err_max": head["eig_rel_err_max"],
        "eig_reference": ref_kind,
        "eig_note": ("the eigenvalues come from the sketch and the float64 small linear algebra in "
                     "every form; the forms differ in the lift (b_j phi_j) and the reconstruction "
                     "(mask), reported per form"),
        "forms": {f: {"fps": r["fps"], "ms_per_step": r["ms"], "eig_rel_err_max": r["eig_rel_err_max"],
                      "small_la_ms": round(r["avg"]["small_la"], 3), "lanczos_steps": r["lanczos"],
                      "n_selected": r["n_sel"], "tiles": r["tiles"],
                      "kernels": {q: {kk: vv for kk, vv in d.items() if kk not in ("bytes", "flops")}
                                  for q, d in r["kernels"].items()}}
                  for f, r in res.items()},
    }
    if copy_gbs is not None:
        out["hbm_copy_gbps"] = round(copy_gbs, 1)
    if args.workload == "cfg2" and not args.no_quality:
        log("per-form quality against the full-frame FP64 oracle")
        qual, qinfo = oracle_quality(D, idx, sign, k, K, tau, res)
        for f, q in qual.items():
            out["forms"][f].update(q)
        out["quality_reference"] = dict(qinfo, kind="FP64 oracle of the whole frame on the same exact sketch; "
                                                   "b_j phi_j and masks on sampled pixels x all frames")
    if not args.no_cpu_baseline and args.workload == "cfg2":
        log("CPU baseline (FP64 oracle on a band of the video), all threads")
        out["cpu_baseline"] = cpu_baseline(D, spec, k, p, nnz, K, tau, args.cpu_band_rows)
        log("CPU baseline, one thread")
        out["cpu_baseline_1thread"] = cpu_baseline(D, spec, k, p, nnz, K, tau, args.cpu_band_rows_1t, threads=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
