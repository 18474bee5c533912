"""Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11, Sec. 3.2 and Table 2).

The SRHT needs random signs, a random permutation and uniformly sampled row
sets (Sec. 2.1 of the SPCG paper); the paper does not name a generator, so
this implementation fixes the counter-based Philox4x64 with 10 rounds.  Test
infrastructure: see ``oracle/__init__.py``.

Two implementations are given:

* ``philox4x64_ref`` - one block with Python integers (exact big-int
  arithmetic, no wrap-around tricks), the readable definition;
* ``philox4x64``     - the same function vectorised over NumPy uint64 arrays
  (64x64 -> 128-bit products assembled from 32-bit halves).

Both are pinned against each other and against ``numpy.random.Philox``
(an independent library implementation of the same generator).
"""
import numpy as np

MASK64 = (1 << 64) - 1

# Multipliers and Weyl key increments of Philox4x64 (Salmon et al. 2011).
M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15  # golden ratio
W1 = 0xBB67AE8584CAA73B  # sqrt(3) - 1
ROUNDS = 10


def philox4x64_ref(counter, key, rounds=ROUNDS):
    """One Philox4x64 block with Python ints.

    counter: 4 ints in [0, 2^64); key: 2 ints.  Returns a tuple of 4 ints.
    Round: (hi0, lo0) = M0*c0, (hi1, lo1) = M1*c2,
           c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
    the key is bumped by (W0, W1) between rounds.
    """
    c0, c1, c2, c3 = (int(v) & MASK64 for v in counter)
    k0, k1 = (int(v) & MASK64 for v in key)
    for rnd in range(rounds):
        if rnd > 0:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """Full 128-bit product of uint64 arrays: returns (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & _M32, a >> _S32
    b0, b1 = b & _M32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Vectorised Philox4x64: every argument broadcasts as uint64 arrays.

    Returns four uint64 arrays (the output words 0..3).
    """
    with np.errstate(over="ignore"):
        c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(
            *(np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3, k0, k1)))
        c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
        k0, k1 = k0.copy(), k1.copy()
        m0 = np.uint64(M0)
        m1 = np.uint64(M1)
        for rnd in range(rounds):
            if rnd > 0:
                k0 = k0 + np.uint64(W0)
                k1 = k1 + np.uint64(W1)
            hi0, lo0 = _mulhilo(m0, c0)
            hi1, lo1 = _mulhilo(m1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3
