"""Philox4x64-10 counter-based generator, written from its published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11. A Philox4x64 round maps the counter
(c0, c1, c2, c3) and key (k0, k1) to

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))

with the 64x64->128-bit products split into high and low words. Between
rounds the key is bumped by the Weyl constants (W0, W1). Ten rounds are used.

The method draws every random quantity from this generator (Sec. 3: each
iteration samples an independent copy S_k ~ D), so that a sketch is a pure
function of (seed, problem, iteration, coordinate).

Part of the oracle: test infrastructure only.
"""
import numpy as np

_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

# Published Philox4x64 constants (Salmon et al. 2011, Table 2 and Sec. 4.2).
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)  # golden ratio
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)  # sqrt(3) - 1


def _mulhilo(a, b):
    """Full 128-bit product of uint64 arrays, returned as (hi, lo) words."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _MASK32, a >> _S32
    b_lo, b_hi = b & _MASK32, b >> _S32
    p_ll = a_lo * b_lo
    p_lh = a_lo * b_hi
    p_hl = a_hi * b_lo
    p_hh = a_hi * b_hi
    mid = (p_ll >> _S32) + (p_lh & _MASK32) + (p_hl & _MASK32)
    hi = p_hh + (p_lh >> _S32) + (p_hl >> _S32) + (mid >> _S32)
    lo = a * b  # wraps modulo 2^64
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x64 rounds on (broadcastable) uint64 counter words.

    Returns the four output words (W0, W1, W2, W3) as uint64 arrays.
    """
    with np.errstate(over="ignore"):
        c0 = np.asarray(c0, dtype=np.uint64)
        c1 = np.asarray(c1, dtype=np.uint64)
        c2 = np.asarray(c2, dtype=np.uint64)
        c3 = np.asarray(c3, dtype=np.uint64)
        k0 = np.uint64(k0)
        k1 = np.uint64(k1)
        c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
        for rnd in range(10):
            if rnd > 0:
                k0 = k0 + PHILOX_W0
                k1 = k1 + PHILOX_W1
            hi0, lo0 = _mulhilo(PHILOX_M0, c0)
            hi1, lo1 = _mulhilo(PHILOX_M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3
