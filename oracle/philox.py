"""Counter-based Gaussian entries of the dense measurement matrix C (FP64 oracle side).

TEST INFRASTRUCTURE ONLY.  Used by tests/, __graft_entry__.smoke() and bench.py's CPU
baseline; the product path never imports anything under oracle/.

The paper draws C with i.i.d. Gaussian entries (Section "Measurement Matrices").  The
draw is made reproducible without storing C by defining every entry as a pure function
of (seed, row, pixel):

* Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and Shaw,
  "Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 128-bit counter is
  permuted by ten rounds keyed by a 64-bit key; each round multiplies two counter
  words by fixed odd constants, splits the 64-bit products into high and low words
  and mixes them with the other words and the round key; the key is advanced by
  two Weyl constants between rounds.
* Box-Muller (1958): two uniforms u1, u2 in (0, 1] give two independent standard
  normals sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2).

Entry layout: for row r and pixel j the counter is (j >> 2, r, 0, 0) and the key is
(seed mod 2^32, seed >> 32).  The four output words (w0, w1, w2, w3) become the
uniforms u = (w + 1) * 2^-32; (w0, w1) feed one Box-Muller pair, (w2, w3) the other,
giving normals z0..z3 for pixels 4*(j >> 2) + 0..3.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten-round Philox on arrays of 32-bit counter words; returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    ka, kb = k0 & 0xFFFFFFFF, k1 & 0xFFFFFFFF
    for rnd in range(10):
        if rnd:
            ka = (ka + W0) & 0xFFFFFFFF
            kb = (kb + W1) & 0xFFFFFFFF
        p0 = M0 * c0               # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(ka), lo1, hi0 ^ c3 ^ np.uint64(kb), lo0)
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def box_muller(wa, wb):
    """Two uint32 words -> two N(0,1) samples in float64."""
    u1 = (np.asarray(wa, dtype=np.float64) + 1.0) * 2.0 ** -32
    u2 = (np.asarray(wb, dtype=np.float64) + 1.0) * 2.0 ** -32
    r = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return r * np.cos(ang), r * np.sin(ang)


def gaussian_block(seed: int, r0: int, r1: int, j0: int, j1: int) -> np.ndarray:
    """Standard-normal entries z[r, j] for rows [r0, r1) and pixels [j0, j1), float64."""
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    jb0, jb1 = j0 >> 2, (j1 + 3) >> 2
    rows = np.arange(r0, r1, dtype=np.uint64)[:, None]
    blocks = np.arange(jb0, jb1, dtype=np.uint64)[None, :]
    w = philox4x32_10(blocks, rows, 0, 0, k0, k1)
    z0, z1 = box_muller(w[0], w[1])
    z2, z3 = box_muller(w[2], w[3])
    z = np.stack([z0, z1, z2, z3], axis=-1).reshape(r1 - r0, 4 * (jb1 - jb0))
    off = j0 - 4 * jb0
    return z[:, off:off + (j1 - j0)]


def srft_uniforms(seed: int, j0: int, j1: int) -> np.ndarray:
    """The uniforms u_j in [0, 1) of the SRFT's random diagonal (entry exp(2 pi i u_j),
    Section 3.3) for pixels j0 <= j < j1: word j mod 4 of Philox4x32-10 on the counter
    (j >> 2, 0, 0, 1) with the key (seed mod 2^32, seed >> 32), times 2^-32.  (The
    Gaussian entries use counters with last word 0, so the two never share a counter.)"""
    if j1 <= j0:
        return np.zeros(0)
    jb = np.arange(j0 >> 2, ((j1 - 1) >> 2) + 1, dtype=np.uint64)
    w = philox4x32_10(jb, 0, 0, 1, seed & 0xFFFFFFFF, seed >> 32)
    words = np.stack(w, axis=1).reshape(-1)
    s0 = j0 - 4 * (j0 >> 2)
    return words[s0:s0 + (j1 - j0)].astype(np.float64) * 2.0 ** -32

