"""Nested CountSketch (test infrastructure): the SPCG-CS variant of Sec. 4.3.

Sec. 4.3 replaces the SRHT of the initialisation stage with CountSketch (a
sparse sketch, Sec. 2.1's list of classical operators; O(Nd) to apply, as
noted after Theorem 3.4).  A CountSketch with m rows sends row k of the
data to one bucket h(k) in [0, m) with a random sign s(k):

    (S M)[b] = sum over rows k with h(k) = b of s(k) M[k],

so every column of S holds a single +-1 and E[S^T S] = I (no scaling).

Readings where the paper is silent:

* buckets come from a keyed bijection q of the padded row range [0, N')
  (the Feistel network of ``feistel``, stream 5): h(k) = q(k) mod m.  Every
  bucket therefore receives floor(N'/m) or ceil(N'/m) of the N' (padded)
  rows, and rows k >= N are zero;
* the signs are the SRHT's D (Philox stream 1);
* nesting: the stage sizes m_1 | m_2 | ... | m_K (an integer growth factor),
  and S_i uses h_i(k) = q(k) mod m_i, so S_i M is S_{i+1} M with buckets b,
  b + m_i, b + 2 m_i, ... added together (folding);
* the preconditioner's sketch S-hat is independent: its own bijection
  (stream 6), its own signs (stream 7) and r buckets; H-hat = (S-hat X)^T
  (S-hat X) since E[S-hat^T S-hat] = I;
* stage problems use c^2 = 1 (the rows need no scaling).
"""
import numpy as np

from .feistel import feistel_forward
from .sketch import padded_bits, sign_vector, STREAM_SIGN

STREAM_CS = 5
STREAM_CS_HAT = 6
STREAM_CS_HAT_SIGN = 7


def slots(seed, L, hat=False):
    """q(k) for every padded row k < 2^L (the bucket map before the modulus)."""
    k = np.arange(1 << L, dtype=np.uint64)
    return feistel_forward(k, L, seed, STREAM_CS_HAT if hat else STREAM_CS).astype(np.int64)


def signs(seed, L, N, hat=False):
    """s(k) for rows k < N as float64 +-1."""
    return sign_vector(seed, L, rows=np.arange(N), stream=STREAM_CS_HAT_SIGN if hat else STREAM_SIGN)


def countsketch(M, seed, m, hat=False):
    """S M for the m-bucket CountSketch (S-hat's when ``hat``), FP64."""
    M = np.asarray(M, dtype=np.float64)
    N = M.shape[0]
    L, Np = padded_bits(N)
    if not 0 < m <= Np:
        raise ValueError("bucket count must lie in (0, N']")
    h = slots(seed, L, hat)[:N] % m
    s = signs(seed, L, N, hat).reshape((-1,) + (1,) * (M.ndim - 1))
    out = np.zeros((m,) + M.shape[1:], dtype=np.float64)
    np.add.at(out, h, s * M)
    return out


def fold(SM, m):
    """Buckets b, b + m, b + 2m, ... of a sketch with a multiple of m rows,
    added together: the m-bucket sketch of the same bucket map."""
    SM = np.asarray(SM, dtype=np.float64)
    if SM.shape[0] % m:
        raise ValueError("the finer sketch must have a multiple of m rows")
    return SM.reshape((SM.shape[0] // m, m) + SM.shape[1:]).sum(axis=0)


def nested_countsketch(X, Y, seed, sizes, r):
    """Stage sketches [(S_i X, S_i Y)] for the sizes m_i and S-hat X.

    Every size must divide the next (the nesting)."""
    sizes = [int(m) for m in sizes]
    for a, b in zip(sizes, sizes[1:]):
        if b % a:
            raise ValueError("nested CountSketch sizes must divide each other")
    stages = [(countsketch(X, seed, m), countsketch(Y, seed, m)) for m in sizes]
    return stages, countsketch(X, seed, r, hat=True)


__all__ = ["STREAM_CS", "STREAM_CS_HAT", "STREAM_CS_HAT_SIGN", "STREAM_SIGN", "slots", "signs",
           "countsketch", "fold", "nested_countsketch"]
