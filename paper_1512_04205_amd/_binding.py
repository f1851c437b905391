"""ctypes binding of libcdmd.so (include/cdmd.h): argument marshalling only.

Every step of the cDMD path runs inside the library; this module turns torch tensors
into raw device pointers and streams, numpy arrays into host pointers, and status codes
into exceptions.  It never computes a result itself and has no fallback: if the library
is missing, importing the package fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcdmd.so")

# enums (include/cdmd.h)
OK, E_INVALID_ARG, E_UNSUPPORTED, E_OUT_OF_MEMORY, E_DEVICE, E_RANK_DEFICIENT, E_NUMERIC, E_STATE = range(8)
U8, F32 = 0, 1
SKETCH_GAUSSIAN, SKETCH_SPARSE, SKETCH_SPIXEL, SKETCH_SRFT = 0, 1, 2, 3
PREC_FP32, PREC_BF16, PREC_FP8 = 0, 1, 2
SEL_OMP, SEL_ZERO_MODE, SEL_OMEGA, SEL_EXPLICIT, SEL_ALL = 0, 1, 2, 3, 4
AMP_FULL, AMP_COMPRESSED = 0, 1

_STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "OUT_OF_MEMORY", 4: "DEVICE",
                 5: "RANK_DEFICIENT", 6: "NUMERIC", 7: "STATE"}

EXPORTED = [
    "cdmd_abi_version", "cdmd_last_error", "cdmd_create", "cdmd_fit", "cdmd_modes",
    "cdmd_select", "cdmd_background", "cdmd_foreground", "cdmd_get_sketch",
    "cdmd_info_get", "cdmd_set_timing", "cdmd_set_amplitudes", "cdmd_mask_median3", "cdmd_free",
    "cdmd_dbg_force_valu_lift",
    "cdmd_dbg_force_host_la", "cdmd_dbg_team_small_la", "cdmd_dbg_la_phases", "cdmd_dbg_la_groups",
    "cdmd_dbg_force_gather_sketch", "cdmd_dbg_sparse_form", "cdmd_dbg_rank_threshold",
    "cdmd_mode_features", "cdmd_mlp_grad", "cdmd_mlp_train", "cdmd_mlp_train_noalloc", "cdmd_mlp_forward",
    "cdmd_select_learned", "cdmd_autotune", "cdmd_batch_create", "cdmd_batch_fit",
    "cdmd_batch_foreground",
    "cdmd_batch_free", "cdmd_optimal_rank", "cdmd_store_measurement", "cdmd_process_video",
    "cdmd_video_create", "cdmd_video_run", "cdmd_video_free", "cdmd_dbg_herm_topk", "cdmd_dbg_eig_complex",
]
MLP_NPARAM = 4673


class CdmdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("m", ctypes.c_int64), ("ld", ctypes.c_int64),
        ("k", ctypes.c_int32), ("p", ctypes.c_int32), ("nnz", ctypes.c_int32),
        ("dtype", ctypes.c_int32), ("sketch", ctypes.c_int32),
        ("sketch_prec", ctypes.c_int32), ("lift_prec", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("sparse_idx", ctypes.POINTER(ctypes.c_int32)),
        ("sparse_sign", ctypes.POINTER(ctypes.c_int8)),
    ]


class VideoPlan(ctypes.Structure):
    _fields_ = [("batch_frames", ctypes.c_int32), ("k", ctypes.c_int32), ("K", ctypes.c_int32),
                ("workers", ctypes.c_int32), ("tau", ctypes.c_double), ("H", ctypes.c_int64),
                ("W", ctypes.c_int64)]


class Info(ctypes.Structure):
    _fields_ = [
        ("fitted", ctypes.c_int32), ("selected", ctypes.c_int32),
        ("warn_few_samples", ctypes.c_int32), ("n_selected", ctypes.c_int32),
        ("sigma_ratio", ctypes.c_double), ("x1_norm2", ctypes.c_double),
        ("omp_residual2", ctypes.c_double),
        ("ms_sketch", ctypes.c_double), ("ms_small_la", ctypes.c_double),
        ("ms_lift", ctypes.c_double), ("ms_host_post", ctypes.c_double),
        ("lanczos_steps", ctypes.c_int32), ("timing", ctypes.c_int32),
        ("gpu_ms_sketch", ctypes.c_double), ("gpu_ms_gram", ctypes.c_double),
        ("gpu_ms_lift", ctypes.c_double), ("gpu_ms_recon", ctypes.c_double),
        ("lift_grid", ctypes.c_int32), ("sketch_slices", ctypes.c_int32),
        ("sparse_form", ctypes.c_int32), ("gpu_ms_lanczos", ctypes.c_double),
    ]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


_lib: Optional[ctypes.CDLL] = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libcdmd.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_1512_04205_amd/build.py`")
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    DP = ctypes.POINTER(ctypes.c_double)
    lib.cdmd_abi_version.restype = I32
    lib.cdmd_last_error.restype = ctypes.c_char_p
    lib.cdmd_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(P)]
    lib.cdmd_fit.argtypes = [P, P, P]
    lib.cdmd_modes.argtypes = [P, DP, DP, DP, DP, P, P, P]
    lib.cdmd_select.argtypes = [P, I32, I32, D, ctypes.POINTER(I32), I32, ctypes.POINTER(I32),
                                ctypes.POINTER(I32), DP]
    lib.cdmd_background.argtypes = [P, P, I64, I64, I32, P, I64, P]
    lib.cdmd_foreground.argtypes = [P, P, ctypes.c_float, I32, I32, P, ctypes.POINTER(I64), P]
    lib.cdmd_get_sketch.argtypes = [P, DP, ctypes.POINTER(I64)]
    lib.cdmd_info_get.argtypes = [P, ctypes.POINTER(Info)]
    lib.cdmd_set_timing.argtypes = [P, I32]
    lib.cdmd_set_amplitudes.argtypes = [P, I32]
    lib.cdmd_store_measurement.argtypes = [P, ctypes.c_int32, ctypes.c_void_p]
    lib.cdmd_process_video.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(VideoPlan), ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.c_void_p]
    lib.cdmd_video_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(VideoPlan), ctypes.POINTER(P)]
    lib.cdmd_video_run.argtypes = [P, P, ctypes.c_int64, P, ctypes.POINTER(ctypes.c_int32), P]
    lib.cdmd_video_free.argtypes = [P]
    lib.cdmd_video_free.restype = None
    lib.cdmd_mask_median3.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, I32, P]
    lib.cdmd_dbg_force_valu_lift.argtypes = [P, I32]
    lib.cdmd_dbg_force_host_la.argtypes = [P, I32]
    lib.cdmd_dbg_la_groups.argtypes = [P, I32]
    lib.cdmd_dbg_force_gather_sketch.argtypes = [P, I32]
    lib.cdmd_optimal_rank.argtypes = [ctypes.POINTER(Config), P, P, ctypes.POINTER(I32), DP, DP]
    lib.cdmd_dbg_sparse_form.argtypes = [P, I32]
    lib.cdmd_dbg_la_phases.argtypes = [P, DP]
    lib.cdmd_mode_features.argtypes = [P, P, P]
    lib.cdmd_mlp_grad.argtypes = [P, P, P, I32, P, P, P]
    lib.cdmd_mlp_train.argtypes = [P, P, P, P, P, I64, P, I32, I32, ctypes.c_float, I64, P, P]
    lib.cdmd_mlp_train_noalloc.argtypes = [P, P, P, P, P, I64, P, I32, I32, ctypes.c_float, I64, P, P]
    lib.cdmd_mlp_forward.argtypes = [P, P, I32, I32, P, P]
    lib.cdmd_select_learned.argtypes = [P, P, D, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), DP, DP,
                                        ctypes.POINTER(I32), P]
    lib.cdmd_autotune.argtypes = [P, P, P]
    lib.cdmd_batch_create.argtypes = [ctypes.POINTER(P), I32, ctypes.POINTER(P)]
    lib.cdmd_batch_fit.argtypes = [P, ctypes.POINTER(P), P, ctypes.POINTER(I32)]
    lib.cdmd_batch_foreground.argtypes = [P, ctypes.POINTER(P), ctypes.c_float, I32, ctypes.POINTER(P), P]
    lib.cdmd_batch_free.argtypes = [P]
    lib.cdmd_batch_free.restype = None
    lib.cdmd_free.argtypes = [P]
    lib.cdmd_free.restype = None
    for name in EXPORTED:
        if name not in ("cdmd_abi_version", "cdmd_last_error", "cdmd_free", "cdmd_batch_free"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        raise CdmdError(status, load_library().cdmd_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


def _video_ptr(video, dtype: int, n: int, m: int, ld: int) -> int:
    import torch
    if not isinstance(video, torch.Tensor) or not video.is_cuda:
        raise TypeError("video must be a CUDA (HIP) torch tensor")
    want = torch.uint8 if dtype == U8 else torch.float32
    if video.dtype != want:
        raise TypeError(f"video dtype {video.dtype} does not match the model ({want})")
    if video.dim() != 2 or video.shape[0] != m or video.shape[1] < n or video.stride(1) != 1 \
            or video.stride(0) != ld:
        raise ValueError("video must be (m, >= n) with unit pixel stride and frame stride ld")
    return video.data_ptr()


def optimal_rank(video, n: int, m: int, p: int, *, sketch: int = SKETCH_SPARSE, dtype: int = U8,
                 ld: Optional[int] = None, idx: Optional[np.ndarray] = None, sign: Optional[np.ndarray] = None,
                 seed: int = 0, sketch_prec: int = PREC_FP32, stream=None):
    """Automatic target rank (Remark 2): the Gavish-Donoho hard threshold on the singular
    values of the sketch.  Returns (k, tau, sigma)."""
    lib = load_library()
    ld = int(ld if ld is not None else n)
    cfg = Config()
    cfg.n, cfg.m, cfg.ld, cfg.k, cfg.p = int(n), int(m), ld, 1, int(p)
    cfg.dtype, cfg.sketch, cfg.seed = dtype, sketch, seed
    cfg.sketch_prec, cfg.lift_prec = sketch_prec, PREC_FP32
    keep = []
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        cfg.nnz = idx.shape[1] if idx.ndim == 2 else 1
        cfg.sparse_idx = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        keep.append(idx)
    if sign is not None:
        sign = np.ascontiguousarray(sign, dtype=np.int8)
        cfg.sparse_sign = sign.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        keep.append(sign)
    r = min(int(p), int(m) - 1)
    sig = np.zeros(r)
    k = ctypes.c_int32(0)
    tau = ctypes.c_double(0.0)
    _check(lib.cdmd_optimal_rank(ctypes.byref(cfg), _video_ptr(video, dtype, int(n), int(m), ld), _stream(stream),
                                 ctypes.byref(k), ctypes.byref(tau), _dptr(sig)))
    return int(k.value), float(tau.value), sig


def _video_setup(n, p, batch_frames, k, K, tau, workers, median_hw, sketch, dtype, ld, idx, sign, seed,
                 sketch_prec, lift_prec):
    cfg = Config()
    cfg.n, cfg.m, cfg.ld, cfg.k, cfg.p = int(n), 2, int(ld), 1, int(p)
    cfg.dtype, cfg.sketch, cfg.seed = dtype, sketch, seed
    cfg.sketch_prec, cfg.lift_prec = sketch_prec, lift_prec
    keep = []
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        cfg.nnz = idx.shape[1] if idx.ndim == 2 else 1
        cfg.sparse_idx = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        keep.append(idx)
    if sign is not None:
        sign = np.ascontiguousarray(sign, dtype=np.int8)
        cfg.sparse_sign = sign.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        keep.append(sign)
    plan = VideoPlan()
    plan.batch_frames, plan.k, plan.K, plan.workers, plan.tau = batch_frames, k, K, workers, tau
    plan.H, plan.W = median_hw if median_hw is not None else (0, 0)
    return cfg, plan, keep


def process_video(video, n: int, frames: int, p: int, mask, *, batch_frames: int = 200, k: int = 0,
                  K: int = 10, tau: float = 0.1, workers: int = 2, median_hw=None,
                  sketch: int = SKETCH_SPARSE, dtype: int = U8, ld: Optional[int] = None,
                  idx: Optional[np.ndarray] = None, sign: Optional[np.ndarray] = None, seed: int = 0,
                  sketch_prec: int = PREC_FP32, lift_prec: int = PREC_FP32, stream=None) -> np.ndarray:
    """A long video in batches of consecutive frames (cdmd_process_video): fills the device
    mask (frames, mask_words(n)) int32 and returns the rank used for each batch."""
    lib = load_library()
    ld = int(ld if ld is not None else n)
    cfg, plan, keep = _video_setup(n, p, batch_frames, k, K, tau, workers, median_hw, sketch, dtype, ld, idx,
                                   sign, seed, sketch_prec, lift_prec)
    nb = max(1, (frames + batch_frames - 1) // batch_frames)
    k_used = np.zeros(nb, dtype=np.int32)
    words = mask_words(n)
    _check(lib.cdmd_process_video(ctypes.byref(cfg), ctypes.byref(plan),
                                  _video_ptr(video, dtype, n, frames, ld),
                                  frames, _tensor_ptr(mask, frames * words),
                                  k_used.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _stream(stream)))
    del keep
    return k_used


class VideoExecutor:
    """A reusable long-video executor (cdmd_video_create / cdmd_video_run / cdmd_video_free):
    the arguments of process_video fixed once; run() processes one video and returns the
    rank used for each batch."""

    def __init__(self, n: int, p: int, *, batch_frames: int = 200, k: int = 0, K: int = 10, tau: float = 0.1,
                 workers: int = 2, median_hw=None, sketch: int = SKETCH_SPARSE, dtype: int = U8,
                 ld: Optional[int] = None, idx: Optional[np.ndarray] = None, sign: Optional[np.ndarray] = None,
                 seed: int = 0, sketch_prec: int = PREC_FP32, lift_prec: int = PREC_FP32):
        lib = load_library()
        self.n, self.dtype, self.batch_frames = int(n), dtype, int(batch_frames)
        self.ld = int(ld if ld is not None else n)
        cfg, plan, keep = _video_setup(n, p, batch_frames, k, K, tau, workers, median_hw, sketch, dtype, self.ld,
                                       idx, sign, seed, sketch_prec, lift_prec)
        h = ctypes.c_void_p()
        _check(lib.cdmd_video_create(ctypes.byref(cfg), ctypes.byref(plan), ctypes.byref(h)))
        del keep  # the executor keeps its own copy of the sparse table
        self._h = h

    def run(self, video, frames: int, mask, stream=None) -> np.ndarray:
        if not self._h:
            raise CdmdError(E_STATE, "executor closed")
        nb = max(1, (frames + self.batch_frames - 1) // self.batch_frames)
        k_used = np.zeros(nb, dtype=np.int32)
        _check(load_library().cdmd_video_run(self._h, _video_ptr(video, self.dtype, self.n, frames, self.ld), frames,
                                             _tensor_ptr(mask, frames * mask_words(self.n)),
                                             k_used.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             _stream(stream)))
        return k_used

    def close(self):
        if getattr(self, "_h", None):
            load_library().cdmd_video_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """One cDMD model: configuration, prepared sketch matrix, device workspace and the
    results of the last fit (a thin owner of a cdmd_model*)."""

    def __init__(self, n: int, m: int, k: int, p: int, *, sketch: int = SKETCH_SPARSE,
                 dtype: int = U8, ld: Optional[int] = None, idx: Optional[np.ndarray] = None,
                 sign: Optional[np.ndarray] = None, seed: int = 0,
                 sketch_prec: int = PREC_FP32, lift_prec: int = PREC_FP32):
        lib = load_library()
        self.n, self.m, self.k, self.p = int(n), int(m), int(k), int(p)
        self.ld = int(ld if ld is not None else n)
        self.dtype = dtype
        self.sketch_kind = sketch
        cfg = Config()
        cfg.n, cfg.m, cfg.ld, cfg.k, cfg.p = self.n, self.m, self.ld, self.k, self.p
        cfg.dtype, cfg.sketch, cfg.seed = dtype, sketch, seed
        cfg.sketch_prec, cfg.lift_prec = sketch_prec, lift_prec
        self._keep = []
        if idx is not None:
            idx = np.ascontiguousarray(idx, dtype=np.int32)
            cfg.nnz = idx.shape[1] if idx.ndim == 2 else 1
            cfg.sparse_idx = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            self._keep.append(idx)
        if sign is not None:
            sign = np.ascontiguousarray(sign, dtype=np.int8)
            cfg.sparse_sign = sign.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
            self._keep.append(sign)
        h = ctypes.c_void_p()
        _check(lib.cdmd_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._keep = []
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().cdmd_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- Algorithm 1
    def fit(self, video, stream=None):
        _check(load_library().cdmd_fit(self._h, _video_ptr(video, self.dtype, self.n, self.m, self.ld),
                                       _stream(stream)))
        return self

    def modes(self, video=None, phi=None, stream=None):
        """Returns dict(lam, b, sigma, phi_norm) (complex / float64 numpy); fills the
        device tensor ``phi`` ((k, n) complex64) with the full modes if given."""
        k = self.k
        lam, b = np.zeros(2 * k), np.zeros(2 * k)
        sig, pn = np.zeros(k), np.zeros(k)
        vptr = _video_ptr(video, self.dtype, self.n, self.m, self.ld) if video is not None else None
        pptr = None
        if phi is not None:
            import torch
            if phi.dtype != torch.complex64 or tuple(phi.shape) != (k, self.n) or not phi.is_contiguous():
                raise ValueError("phi must be a contiguous (k, n) complex64 device tensor")
            pptr = phi.data_ptr()
        _check(load_library().cdmd_modes(self._h, _dptr(lam), _dptr(b), _dptr(sig), _dptr(pn),
                                          vptr, pptr, _stream(stream) if pptr else None))
        return dict(lam=lam[0::2] + 1j * lam[1::2], b=b[0::2] + 1j * b[1::2], sigma=sig, phi_norm=pn)

    def select(self, selector: int = SEL_OMP, K: int = 10, omega_thr: float = 0.0,
               explicit: Optional[Sequence[int]] = None):
        k = self.k
        idx = np.zeros(k, dtype=np.int32)
        beta = np.zeros(2 * k)
        nsel = ctypes.c_int32(0)
        ex = None
        nex = 0
        if explicit is not None:
            ex_arr = np.ascontiguousarray(explicit, dtype=np.int32)
            ex = ex_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            nex = len(ex_arr)
        _check(load_library().cdmd_select(self._h, selector, K, omega_thr, ex, nex,
                                          idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          ctypes.byref(nsel), _dptr(beta)))
        ns = nsel.value
        return idx[:ns].copy(), (beta[0::2] + 1j * beta[1::2])[:ns].copy()

    def select_learned(self, params, confidence: float = 0.9, K_fallback: int = 10, stream=None):
        """Learned selection with the network parameters `params` (device float32 tensor
        of MLP_NPARAM).  Returns (S, beta, probabilities, used_fallback)."""
        k = self.k
        idx = np.zeros(k, dtype=np.int32)
        beta = np.zeros(2 * k)
        prob = np.zeros(k)
        nsel, fb = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(load_library().cdmd_select_learned(
            self._h, _tensor_ptr(params, MLP_NPARAM), confidence, K_fallback,
            idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(nsel), _dptr(beta),
            _dptr(prob), ctypes.byref(fb), _stream(stream)))
        ns = nsel.value
        return idx[:ns].copy(), (beta[0::2] + 1j * beta[1::2])[:ns].copy(), prob, bool(fb.value)

    def autotune(self, video, stream=None):
        """Pick the tile shapes of this model's size class by timing them on `video`."""
        _check(load_library().cdmd_autotune(self._h, _video_ptr(video, self.dtype, self.n, self.m, self.ld),
                                            _stream(stream)))

    def mode_features(self, out=None, stream=None):
        """Per-mode features (k x 6 float32 device tensor) of the last fit."""
        import torch
        out = torch.empty((self.k, 6), dtype=torch.float32, device="cuda") if out is None else out
        _check(load_library().cdmd_mode_features(self._h, _tensor_ptr(out, 6 * self.k), _stream(stream)))
        return out

    def background(self, video, L, t0: int = 0, t1: Optional[int] = None, static: bool = False,
                   stream=None):
        t1 = self.m if t1 is None else t1
        _check(load_library().cdmd_background(
            self._h, _video_ptr(video, self.dtype, self.n, self.m, self.ld), t0, t1, int(static),
            L.data_ptr(), L.stride(0) if L.dim() == 2 else self.n, _stream(stream)))

    def foreground(self, video, mask, tau: float, static: bool = False, bitpacked: bool = True,
                   counts: bool = False, stream=None):
        cnt = np.zeros(self.m, dtype=np.int64) if counts else None
        _check(load_library().cdmd_foreground(
            self._h, _video_ptr(video, self.dtype, self.n, self.m, self.ld), tau, int(static),
            int(bitpacked), mask.data_ptr(),
            cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if counts else None,
            _stream(stream)))
        return cnt

    def sketch(self, integer: bool = False):
        """The last fit's sketch Y^ (p x m): float64, complex128 for the SRFT sketch."""
        if self.sketch_kind == SKETCH_SRFT:
            Y = np.zeros(2 * self.m * self.p)
            _check(load_library().cdmd_get_sketch(self._h, _dptr(Y), None))
            return Y.view(np.complex128).reshape(self.m, self.p).T.copy()
        Y = np.zeros(self.m * self.p)
        Yi = np.zeros(self.m * self.p, dtype=np.int64) if integer else None
        _check(load_library().cdmd_get_sketch(
            self._h, _dptr(Y), Yi.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if integer else None))
        Y = Y.reshape(self.m, self.p).T.copy()
        return (Y, Yi.reshape(self.m, self.p).T.copy()) if integer else Y

    def force_valu_lift(self, on: bool = True):
        """Test hook: use the float32 vector-ALU lift instead of the MFMA lift."""
        _check(load_library().cdmd_dbg_force_valu_lift(self._h, int(on)))

    def force_gather_sketch(self, on: bool = True):
        """Test hook: gather form of the sparse sketch instead of the streaming form."""
        _check(load_library().cdmd_dbg_force_gather_sketch(self._h, int(on)))

    def sparse_form(self, form: int):
        """Test hook: the sparse-sketch form (-1 gather, or 10 F + V streaming)."""
        _check(load_library().cdmd_dbg_sparse_form(self._h, int(form)))

    def force_host_la(self, on: bool = True):
        """Test hook: float64 small linear algebra on the host instead of the device."""
        _check(load_library().cdmd_dbg_force_host_la(self._h, int(on)))

    def la_groups(self, groups: int):
        """Test hook: at most `groups` Lanczos row groups in the device solve (0: auto)."""
        _check(load_library().cdmd_dbg_la_groups(self._h, int(groups)))

    def la_phases(self) -> dict:
        """Phase times (ms) of the last device small-LA solve."""
        v = np.zeros(16)
        _check(load_library().cdmd_dbg_la_phases(self._h, _dptr(v)))
        return dict(zip(["lanczos", "checks", "atilde", "eigvals", "eigvecs", "G", "xchg_wait",
                         "matvec", "orth", "step_rest", "multisection", "tri_vectors", "ritz_QZ",
                         "xchg_read", "final_vectors"], v[:15]))

    def set_timing(self, enable: bool = True):
        _check(load_library().cdmd_set_timing(self._h, int(enable)))

    def store_measurement(self, on: bool = True, stream=None):
        """Keep the dense Gaussian C (BF16 / FP8 form) in device memory so that fits stream it
        instead of drawing it (cdmd_store_measurement)."""
        _check(load_library().cdmd_store_measurement(self._h, int(on), _stream(stream)))
        return self

    def set_amplitudes(self, space: int):
        """AMP_FULL (eq. (eq:b) on the full modes) or AMP_COMPRESSED (Remark 3: amplitudes and selection on the
        compressed modes; the next fit computes no lift)."""
        _check(load_library().cdmd_set_amplitudes(self._h, int(space)))

    def info(self) -> dict:
        inf = Info()
        _check(load_library().cdmd_info_get(self._h, ctypes.byref(inf)))
        return inf.as_dict()


class Batch:
    """Many models fitted by one graph launch (cdmd_batch_*).  Keeps the models alive."""

    def __init__(self, models):
        self.models = list(models)
        arr = (ctypes.c_void_p * len(self.models))(*[m._h.value for m in self.models])
        h = ctypes.c_void_p()
        _check(load_library().cdmd_batch_create(arr, len(self.models), ctypes.byref(h)))
        self._h = h

    def fit(self, videos, stream=None):
        """Fit models[i] on videos[i]; returns the per-model status list (raises when any
        model failed, after every model has been attempted)."""
        vp = (ctypes.c_void_p * len(self.models))(
            *[_video_ptr(v, m.dtype, m.n, m.m, m.ld) for v, m in zip(videos, self.models)])
        st = (ctypes.c_int32 * len(self.models))()
        rc = load_library().cdmd_batch_fit(self._h, vp, _stream(stream), st)
        if rc != OK:
            raise CdmdError(rc, load_library().cdmd_last_error().decode())
        return list(st)

    def statuses(self, videos, stream=None):
        """Like fit, but returns the statuses without raising."""
        vp = (ctypes.c_void_p * len(self.models))(
            *[_video_ptr(v, m.dtype, m.n, m.m, m.ld) for v, m in zip(videos, self.models)])
        st = (ctypes.c_int32 * len(self.models))()
        load_library().cdmd_batch_fit(self._h, vp, _stream(stream), st)
        return list(st)

    def foreground(self, videos, masks, tau: float, static_bg: bool = False, stream=None):
        """Bit-packed foreground masks of every (selected) model in one work-queue launch:
        masks[i] (int32 device tensor of m_i x mask_words(n_i)) as models[i].foreground."""
        vp = (ctypes.c_void_p * len(self.models))(
            *[_video_ptr(v, m.dtype, m.n, m.m, m.ld) for v, m in zip(videos, self.models)])
        mp = (ctypes.c_void_p * len(self.models))(
            *[_tensor_ptr(mk, m.m * mask_words(m.n)).value for mk, m in zip(masks, self.models)])
        _check(load_library().cdmd_batch_foreground(self._h, vp, float(tau), int(bool(static_bg)), mp,
                                                    _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            load_library().cdmd_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _tensor_ptr(t, numel: int):
    """Device pointer of a contiguous float32/int32 CUDA tensor of at least `numel` elements."""
    if not (t.is_cuda and t.is_contiguous() and t.numel() >= numel):
        raise ValueError("expected a contiguous device tensor with enough elements")
    return ctypes.c_void_p(t.data_ptr())


def mlp_grad(params, X, y, stream=None):
    """Mean loss and gradient of the selector network on (X, y) (device tensors)."""
    import torch
    n = X.shape[0]
    grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(load_library().cdmd_mlp_grad(_tensor_ptr(params, MLP_NPARAM), _tensor_ptr(X, 6 * n),
                                        _tensor_ptr(y, n), n, _tensor_ptr(grad, MLP_NPARAM),
                                        _tensor_ptr(loss, 1), _stream(stream)))
    return float(loss.item()), grad


def mlp_train(params, adam_m, adam_v, X, y, batch_idx, batch: int, lr: float = 1e-3, step0: int = 0,
              stream=None):
    """Adam steps over the batches in batch_idx (device int32, steps x batch); updates
    params / adam_m / adam_v in place and returns the per-step losses (device)."""
    import torch
    steps = batch_idx.numel() // batch
    losses = torch.empty(max(steps, 1), dtype=torch.float32, device="cuda")
    _check(load_library().cdmd_mlp_train(
        _tensor_ptr(params, MLP_NPARAM), _tensor_ptr(adam_m, MLP_NPARAM), _tensor_ptr(adam_v, MLP_NPARAM),
        _tensor_ptr(X, 6 * X.shape[0]), _tensor_ptr(y, X.shape[0]), X.shape[0],
        _tensor_ptr(batch_idx, steps * batch), batch, steps,
        lr, step0, _tensor_ptr(losses, max(steps, 1)), _stream(stream)))
    return losses[:steps]


def mlp_train_noalloc(params, adam_m, adam_v, X, y, batch_idx, batch: int, losses, lr: float = 1e-3,
                      step0: int = 0, stream=None):
    """mlp_train without any allocation (the library's static scratch; batch at most
    MLP_NOALLOC_MAX_BATCH): the per-step losses go to the caller's `losses` (device float32,
    at least steps entries); returns after enqueueing."""
    steps = batch_idx.numel() // batch
    _check(load_library().cdmd_mlp_train_noalloc(
        _tensor_ptr(params, MLP_NPARAM), _tensor_ptr(adam_m, MLP_NPARAM), _tensor_ptr(adam_v, MLP_NPARAM),
        _tensor_ptr(X, 6 * X.shape[0]), _tensor_ptr(y, X.shape[0]), X.shape[0],
        _tensor_ptr(batch_idx, steps * batch), batch, steps,
        lr, step0, _tensor_ptr(losses, max(steps, 1)), _stream(stream)))


MLP_NOALLOC_MAX_BATCH = 1024


def mlp_forward(params, X, bf16: bool = False, stream=None):
    import torch
    n = X.shape[0]
    z = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
    _check(load_library().cdmd_mlp_forward(_tensor_ptr(params, MLP_NPARAM), _tensor_ptr(X, 6 * n), n,
                                           int(bf16), _tensor_ptr(z, max(n, 1)), _stream(stream)))
    return z[:n]


def mask_median3(mask_in, mask_out, H: int, W: int, bitpacked: bool = True, stream=None):
    """3x3 median (majority, edges replicated) of every frame of a binary mask (cdmd_mask_median3):
    (m, ceil(HW/32)) int32/uint32 words or (m, HW) uint8 device tensors."""
    m = mask_in.shape[0]
    if mask_out.shape != mask_in.shape or mask_out.dtype != mask_in.dtype:
        raise ValueError("mask_out must match mask_in")
    _check(load_library().cdmd_mask_median3(mask_in.data_ptr(), mask_out.data_ptr(), int(H), int(W), int(m),
                                            int(bitpacked), _stream(stream)))


def mask_words(n: int) -> int:
    return (n + 31) // 32


def unpack_mask(words: np.ndarray, n: int) -> np.ndarray:
    """Bit-packed (m, ceil(n/32)) uint32 mask -> bool (m, n) (host helper)."""
    w = np.ascontiguousarray(words).view(np.uint8).reshape(words.shape[0], -1)
    bits = np.unpackbits(w, axis=1, bitorder="little")
    return bits[:, :n].astype(bool)
