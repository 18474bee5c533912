"""Keyed Feistel bijections on L-bit integers (test infrastructure).

The SRHT of Sec. 2.1 needs a uniformly random permutation P of the N' rows
and a uniformly sampled row set I; the nested construction of Sec. 2.2 needs
I_1 c I_2 c ... c I_K.  Both come from one keyed bijection pi of [0, 2^L):
I_i = {pi(t) : t < m_i} is nested by construction and every prefix is a
set of distinct rows.  The paper does not fix how the permutation is drawn;
this implementation uses an alternating (unbalanced when L is odd) Feistel network of
``ROUNDS`` rounds whose round function is a Philox4x64-10 output word.

Definition used by both the oracle and the library (each writes its own
code for it):

* split x into a high part l of a = ceil(L/2) bits and a low part r of
  b = L - a bits; widths (wl, wr) = (a, b);
* round j: f = Philox(counter=(r, j, L, 0), key=(seed, stream)) word 0,
  masked to wl bits;  (l, r) <- (r, l XOR f) and the widths swap;
* after an even number of rounds the widths are (a, b) again and the
  output is (l << b) | r.

The inverse undoes the rounds in reverse order.
"""
import numpy as np

from .philox import philox4x64

ROUNDS = 6


def _split(L):
    a = (L + 1) // 2
    return a, L - a


def _round_fn(v, j, L, seed, stream):
    w0, _, _, _ = philox4x64(v, np.uint64(j), np.uint64(L), np.uint64(0),
                             np.uint64(seed), np.uint64(stream))
    return w0


def _mask(bits):
    return np.uint64((1 << bits) - 1)


def feistel_forward(x, L, seed, stream, rounds=ROUNDS):
    """pi(x) for an integer array x with 0 <= x < 2^L."""
    x = np.asarray(x, dtype=np.uint64)
    a, b = _split(L)
    wl, wr = a, b
    l = x >> np.uint64(b)
    r = x & _mask(b)
    for j in range(rounds):
        f = _round_fn(r, j, L, seed, stream) & _mask(wl)
        l, r = r, l ^ f
        wl, wr = wr, wl
    assert (wl, wr) == (a, b)
    return (l << np.uint64(b)) | r


def feistel_inverse(y, L, seed, stream, rounds=ROUNDS):
    """pi^{-1}(y): runs the rounds of ``feistel_forward`` backwards."""
    y = np.asarray(y, dtype=np.uint64)
    a, b = _split(L)
    l = y >> np.uint64(b)
    r = y & _mask(b)
    wl, wr = a, b  # widths of (l, r) after the last round
    for j in reversed(range(rounds)):
        # after round j: l = r_prev (width wr_prev), r = l_prev ^ f (width wl_prev)
        f = _round_fn(l, j, L, seed, stream) & _mask(wr)
        l, r = r ^ f, l
        wl, wr = wr, wl
    return (l << np.uint64(b)) | r
