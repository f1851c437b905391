"""The allocation-free training call (cdmd_mlp_train_noalloc) against the allocating one
(cdmd_mlp_train), through the C ABI: the same batches from the same start must give the
same parameters, Adam moments and losses, bit for bit (both run the same kernels on the
same partial layout), on two calls in a row, the second with a smaller batch so that it
reuses fewer partial slots of the shared scratch than the first left behind."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1512_04205_amd as P
import synthvideo as sv

pytestmark = pytest.mark.gpu


def _dev(a, dt=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _call(fn, th, am, av, X, y, bi, batch, steps, step0, losses):
    return fn(_ptr(th), _ptr(am), _ptr(av), _ptr(X), _ptr(y), X.shape[0], _ptr(bi), batch, steps,
              ctypes.c_float(1e-3), step0, _ptr(losses), None)


def test_noalloc_training_matches_allocating_call_twice():
    print("[gpu-case] mlp train no-alloc", flush=True)
    lib = P.load_library()
    rng = np.random.default_rng(404)
    n = 3000
    X = rng.normal(size=(n, 6)).astype(np.float32)
    y = (X[:, 0] + 0.5 * X[:, 3] > 0.2).astype(np.float32)
    theta0 = sv.mlp_init(405)
    Xd, yd = _dev(X), _dev(y)
    state = {}
    for name in ("alloc", "noalloc"):
        state[name] = [_dev(theta0), torch.zeros(P.MLP_NPARAM, device="cuda"),
                       torch.zeros(P.MLP_NPARAM, device="cuda")]
    calls = [(700, 4, 0), (90, 3, 4)]          # (batch, steps, step0): the second smaller
    for batch, steps, step0 in calls:
        bi = _dev(np.concatenate([rng.permutation(n)[:batch] for _ in range(steps)]), torch.int32)
        la = torch.zeros(steps, device="cuda")
        ln = torch.full((steps,), float("nan"), device="cuda")
        assert _call(lib.cdmd_mlp_train, *state["alloc"], Xd, yd, bi, batch, steps, step0, la) == 0
        assert _call(lib.cdmd_mlp_train_noalloc, *state["noalloc"], Xd, yd, bi, batch, steps, step0, ln) == 0
        torch.cuda.synchronize()
        assert torch.equal(la, ln), (la, ln)
        for a, b in zip(state["alloc"], state["noalloc"]):
            assert torch.equal(a, b)
    # a batch above the scratch's capacity is refused before any device work
    big = P.MLP_NOALLOC_MAX_BATCH + 1
    bi = torch.zeros(big, dtype=torch.int32, device="cuda")
    losses = torch.zeros(1, device="cuda")
    assert _call(lib.cdmd_mlp_train_noalloc, *state["noalloc"], Xd, yd, bi, big, 1, 0, losses) == P.E_INVALID_ARG
