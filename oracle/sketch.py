"""Nested SRHT sketch (test infrastructure).

Follows Sec. 2.1 (SRHT S = sqrt(N/m) (HDP)_{I,:}) and Sec. 2.2 (nested
construction: (Z_X, Z_Y) = (HDPX, HDPY) computed once, nested row sets
I_1 c ... c I_K with doubling sizes, and an independent sketch S-hat of r
rows for the preconditioner).

Readings where the paper is silent:

* N is zero-padded to N' = 2^L, L = ceil(log2 N) (the SRHT is defined for
  powers of two only); padded rows of X and Y are zero.
* Randomness: Philox4x64-10 keyed by (seed, stream); D's sign for row k is
  bit (k mod 256) of the 256-bit block at counter (k div 256, 0, 0, 0),
  +1 for a 0 bit and -1 for a 1 bit; P, the nested order pi and the
  independent order pi-hat are Feistel bijections (``feistel``).
* W = D P X-tilde means W[k] = sign(k) * X-tilde[p(k)].
* S-hat shares the transform HDP with the S_i (one Hadamard transform, as
  the cost count of the proof of Theorem 3.4 assumes) and draws its r rows
  with an independent order pi-hat.

Outputs are the UNSCALED rows of Z = H_un W (H_un = sqrt(N') H):
B[t] = Z[pi(t)] for t < m_K and B_hat[t] = Z[pi_hat(t)] for t < r.
Then S_i X = B[:m_i] / sqrt(m_i) and S_hat X = B_hat / sqrt(r).
"""
import numpy as np

from .feistel import feistel_forward
from .fwht import fwht_rows
from .philox import philox4x64

STREAM_SIGN = 1
STREAM_P = 2
STREAM_PI = 3
STREAM_PIHAT = 4


def padded_bits(N):
    """L = ceil(log2 N) (at least 1) and N' = 2^L."""
    if N < 1:
        raise ValueError("N must be positive")
    L = max(1, (int(N) - 1).bit_length())
    return L, 1 << L


def sign_vector(seed, L, rows=None, stream=STREAM_SIGN):
    """+-1 entries of D for rows k (default: all 2^L rows), as float64.
    ``stream`` selects an independent sign sequence (the CountSketch of the
    preconditioner draws its own)."""
    k = np.arange(1 << L, dtype=np.uint64) if rows is None else np.asarray(rows, dtype=np.uint64)
    blk = k >> np.uint64(8)
    bit = k & np.uint64(255)
    w = philox4x64(blk, 0, 0, 0, np.uint64(seed), np.uint64(stream))
    words = np.stack(w)  # (4, n)
    word = words[(bit >> np.uint64(6)).astype(np.int64), np.arange(k.size)]
    b = (word >> (bit & np.uint64(63))) & np.uint64(1)
    return 1.0 - 2.0 * b.astype(np.float64)


def input_perm(seed, L, rows=None):
    """p(k) for rows k: W[k] = sign(k) * X-tilde[p(k)]."""
    k = np.arange(1 << L, dtype=np.uint64) if rows is None else np.asarray(rows, dtype=np.uint64)
    return feistel_forward(k, L, seed, STREAM_P).astype(np.int64)


def slot_rows(seed, L, m):
    """pi(t) for t < m: the rows of Z forming the nested set I (prefixes)."""
    t = np.arange(m, dtype=np.uint64)
    return feistel_forward(t, L, seed, STREAM_PI).astype(np.int64)


def hat_slot_rows(seed, L, r):
    """pi_hat(t) for t < r: the rows of Z forming S-hat's row set."""
    t = np.arange(r, dtype=np.uint64)
    return feistel_forward(t, L, seed, STREAM_PIHAT).astype(np.int64)


def transform(M, seed):
    """Z = H_un D P M-tilde for an N x c array M (returns N' x c, float64)."""
    M = np.asarray(M, dtype=np.float64)
    N = M.shape[0]
    L, Np = padded_bits(N)
    Mt = np.zeros((Np,) + M.shape[1:], dtype=np.float64)
    Mt[:N] = M
    p = input_perm(seed, L)
    sg = sign_vector(seed, L)
    W = Mt[p] * sg.reshape((-1,) + (1,) * (M.ndim - 1))
    return fwht_rows(W)


def nested_srht(X, Y, seed, m_K, r):
    """Unscaled nested sketch rows.

    Returns (B, BY, B_hat, info) with B = Z_X[pi(0..m_K)], BY = Z_Y[pi(0..m_K)],
    B_hat = Z_X[pi_hat(0..r)].
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    N = X.shape[0]
    L, Np = padded_bits(N)
    if not (0 < m_K <= Np and 0 < r <= Np):
        raise ValueError("sketch sizes must lie in (0, N']")
    ZX = transform(X, seed)
    ZY = transform(Y, seed)
    pi = slot_rows(seed, L, m_K)
    pih = hat_slot_rows(seed, L, r)
    info = {"L": L, "Np": Np, "pi": pi, "pi_hat": pih}
    return ZX[pi], ZY[pi], ZX[pih], info


class SrhtRowAccumulator:
    """Selected rows of Z = H_un D P X-tilde, accumulated over row blocks of X.

    Row i of Z is sum_k (-1)^{popcount(i & k)} sign(k) X-tilde[p(k)]
    (Sec. 2.1 with the unnormalised Sylvester H_un, H_un[i, k] =
    (-1)^{popcount(i & k)}).  Substituting n = p(k) lets X be read block by
    block in its own row order: row n contributes with k = p^{-1}(n).
    Padded rows are zero and contribute nothing."""

    def __init__(self, rows, seed, L):
        self.rows = np.asarray(rows, dtype=np.int64)
        self.seed, self.L = seed, L
        p = input_perm(seed, L)
        self.pinv = np.empty_like(p)
        self.pinv[p] = np.arange(p.size, dtype=np.int64)
        self.value = None

    def add(self, n0, Xb):
        """Adds the contribution of the float64 rows n0 .. n0 + len(Xb) - 1."""
        Xb = np.asarray(Xb, dtype=np.float64)
        k = self.pinv[n0:n0 + Xb.shape[0]]
        sg = sign_vector(self.seed, self.L, rows=k)
        par = np.bitwise_count(self.rows[:, None] & k[None, :]) & 1
        part = ((1.0 - 2.0 * par) * sg[None, :]) @ Xb
        self.value = part if self.value is None else self.value + part


def srht_rows_streamed(blocks, rows, seed, L):
    """Rows ``rows`` of Z = H_un D P X-tilde from the blocks (n0, Xb) of X
    (see SrhtRowAccumulator).  Returns len(rows) x c."""
    acc = SrhtRowAccumulator(rows, seed, L)
    for n0, Xb in blocks:
        acc.add(n0, Xb)
    return acc.value
