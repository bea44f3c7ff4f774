"""Philox4x64-10 counter-based generator and the Box-Muller normal variates drawn from it.

Test infrastructure only (see ``oracle/__init__``).

The paper does not say how its normal variates W, W~ (Sec. II.A) are drawn.
The device path draws them from a counter-based generator so that a time step
is reproducible from (seed, step) alone; this module implements the same
published generator independently, to check the device stream.

Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11): state = four 64-bit words (the counter), key = two 64-bit
words.  One round replaces (x0, x1, x2, x3) by

    (hi(M1 x2) ^ x1 ^ k0,  lo(M1 x2),  hi(M0 x0) ^ x3 ^ k1,  lo(M0 x0))

with M0 = 0xD2E7470EE14C6C93, M1 = 0xCA5A826395121157 and hi/lo the upper and
lower halves of the 128-bit product; the key is bumped by the Weyl constants
(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B) after every round; ten rounds.

Noise layout used by the time step: key = (seed, stream) with stream 0 for W
and 1 for W~; counter = (block, step, 0, 0); block b yields normals
4b .. 4b+3 of the flat 3N vector.  Each 64-bit word x becomes a uniform
u = ((x >> 12) + 1/2) 2^-52 in (0, 1) (exact in FP64); pairs (u0, u1) and (u2, u3) become
normals by Box-Muller: sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b).

Pinned by (tests/test_oracle_philox.py): equality with numpy.random.Philox (an
independent implementation of Philox4x64-10) on many counters and keys, and
the published known-answer vector for zero counter and key
(tests/golden/philox4x64_10_kat.txt).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _M32, a >> _S32
    b_lo, b_hi = b & _M32, b >> _S32
    p_ll = a_lo * b_lo
    p_lh = a_lo * b_hi
    p_hl = a_hi * b_lo
    p_hh = a_hi * b_hi
    mid = (p_ll >> _S32) + (p_lh & _M32) + (p_hl & _M32)
    hi = p_hh + (p_lh >> _S32) + (p_hl >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64(counter, key, rounds=10):
    """Apply Philox4x64 to arrays of counters.

    ``counter``: array (..., 4) uint64; ``key``: array (..., 2) uint64 (broadcast).
    Returns an array (..., 4) uint64.
    """
    x = np.array(counter, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    x0, x1, x2, x3 = (x[..., i].copy() for i in range(4))
    k0 = np.broadcast_to(k[..., 0], x0.shape).copy()
    k1 = np.broadcast_to(k[..., 1], x0.shape).copy()
    with np.errstate(over="ignore"):
        for _ in range(rounds):
            hi0, lo0 = _mulhilo(M0, x0)
            hi1, lo1 = _mulhilo(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            k0 = k0 + W0
            k1 = k1 + W1
    return np.stack([x0, x1, x2, x3], axis=-1)


def uniforms(words):
    """Map 64-bit words to doubles in (0, 1): ((x >> 12) + 1/2) * 2^-52 (no rounding)."""
    w = np.asarray(words, dtype=np.uint64)
    return ((w >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52


def normals(count, seed, stream, step):
    """``count`` N(0,1) doubles of the noise stream (seed, stream) at time step ``step``."""
    nblocks = (count + 3) // 4
    ctr = np.zeros((nblocks, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(nblocks, dtype=np.uint64)
    ctr[:, 1] = np.uint64(step)
    key = np.array([seed, stream], dtype=np.uint64)
    u = uniforms(philox4x64(ctr, key))
    out = np.empty((nblocks, 4))
    for pa, pb in ((0, 1), (2, 3)):
        rad = np.sqrt(-2.0 * np.log(u[:, pa]))
        ang = 2.0 * np.pi * u[:, pb]
        out[:, pa] = rad * np.cos(ang)
        out[:, pb] = rad * np.sin(ang)
    return out.ravel()[:count]
