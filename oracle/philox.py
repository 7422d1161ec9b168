"""Philox4x64-10 counter-based generator (oracle side).

Written from the published definition: J. K. Salmon, M. A. Moraes, R. O. Dror,
D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 5 (the
Philox round: two 64x64->128 multiplies, a fixed permutation with key XOR,
and a Weyl key schedule), with the multipliers and Weyl constants of that
paper for N=4, W=64 and ten rounds.

Test infrastructure only (see the package docstring).  Vectorised over numpy
uint64 arrays; the 64x64->128 product is formed from 32-bit halves.

The sampler of the SRBE method (Sec. 3) draws its proposals from this stream
with the counter layout documented in ``oracle.sampler``.
"""

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mul128(a, b):
    """Return (hi, lo) of the 128-bit product of uint64 arrays a and b."""
    a_lo = a & _MASK32
    a_hi = a >> _S32
    b_lo = b & _MASK32
    b_hi = b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _MASK32) + (hl & _MASK32)
    lo = (ll & _MASK32) | ((mid & _MASK32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Apply ten Philox rounds.

    ctr: uint64 array of shape (..., 4); key: uint64 array of shape (..., 2).
    Returns a uint64 array of shape (..., 4).
    """
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., i].copy() for i in range(4))
    k0 = np.broadcast_to(key[..., 0], c0.shape).copy()
    k1 = np.broadcast_to(key[..., 1], c0.shape).copy()
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = _mul128(M0, c0)
            hi1, lo1 = _mul128(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1)


def u01_open(x):
    """Map uint64 words to doubles strictly inside (0, 1): ((x >> 12) + 1/2) * 2^-52 (exact in FP64)."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)
