"""Shared helpers of the GPU parity tests (comparison logic only)."""
import numpy as np
from scipy.optimize import linear_sum_assignment

# Relative gap between the oracle's OMP pick and the next candidate below which the
# pick counts as a near tie: the float32 form's correlations carry relative errors of
# order 1e-6, the bfloat16 form's of order 1e-3, so a pick closer than these may go
# either way; the GPU is then given the oracle's support (explicit selection).
NEAR_TIE_FP32 = 1e-4
NEAR_TIE_BF16 = 3e-2


def match_eigs(a, b):
    """Optimal matching of eigenvalue lists; returns (ia, ib, |a-b|)."""
    C = np.abs(np.asarray(a)[:, None] - np.asarray(b)[None, :])
    r, c = linear_sum_assignment(C)
    return r, c, C[r, c]


def eig_rel_err(gpu_lam, ref_lam):
    r, c, d = match_eigs(gpu_lam, ref_lam)
    rel = np.empty(len(gpu_lam))
    rel[r] = d / np.abs(np.asarray(ref_lam)[c])
    return rel, r, c


def mask_agreement(mask_gpu, mask_ref, x, L_ref, tau, band):
    """Fraction of identical mask entries, and whether every disagreement lies in the
    band ||x - L_ref| - tau| <= band."""
    diff = mask_gpu != mask_ref
    frac = 1.0 - diff.mean()
    if diff.any():
        margin = np.abs(np.abs(x - L_ref) - tau)[diff]
        inband = bool((margin <= band).all())
    else:
        inband = True
    return frac, inband, int(diff.sum())
