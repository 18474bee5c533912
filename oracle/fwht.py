"""Unnormalised fast Walsh-Hadamard transform over rows (test infrastructure).

H in the SRHT of Sec. 2.1 is the normalised Walsh-Hadamard matrix of order
N' = 2^L; this module applies H_un = sqrt(N') H (the Sylvester matrix with
+-1 entries) to every column of an N' x d array.  Stage s (s = 0 first)
pairs rows k and k + 2^s whose bit s differs and maps (a, b) -> (a+b, a-b).
"""
import numpy as np


def fwht_rows(W):
    """Return H_un @ W for W of shape (2^L, ...), stages s = 0..L-1 in order."""
    Z = np.array(W, copy=True)
    n = Z.shape[0]
    L = n.bit_length() - 1
    if n != 1 << L:
        raise ValueError("row count must be a power of two")
    tail = Z.shape[1:]
    for s in range(L):
        h = 1 << s
        V = Z.reshape((n // (2 * h), 2, h) + tail)
        a = V[:, 0].copy()
        b = V[:, 1]
        V[:, 0] = a + b
        V[:, 1] = a - b
    return Z


def sylvester(L):
    """Dense Sylvester-Hadamard matrix of order 2^L (for tests)."""
    H = np.ones((1, 1))
    for _ in range(L):
        H = np.block([[H, H], [H, -H]])
    return H
