"""Pins for the oracle's Walsh-Hadamard transform and nested SRHT
(Sec. 2.1 definition S = sqrt(N/m) (HDP)_{I,:}; Sec. 2.2 nested sketches)."""
import numpy as np
import pytest

from oracle.fwht import fwht_rows, sylvester
from oracle.sketch import (input_perm, nested_srht, padded_bits, sign_vector, slot_rows,
                           transform)


@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 10])
def test_fwht_equals_dense_sylvester_exactly(L):
    rng = np.random.default_rng(L)
    W = rng.integers(-50, 50, size=(1 << L, 3)).astype(np.float64)
    assert np.array_equal(fwht_rows(W), sylvester(L) @ W)


def test_sylvester_entries_follow_bit_parity():
    # H[i, j] = (-1)^{popcount(i & j)} for the Sylvester construction
    L = 6
    H = sylvester(L)
    i, j = np.meshgrid(np.arange(1 << L), np.arange(1 << L), indexing="ij")
    par = np.vectorize(lambda v: bin(v).count("1") & 1)(i & j)
    assert np.array_equal(H, 1.0 - 2.0 * par)


def test_fwht_is_involution_up_to_scale():
    rng = np.random.default_rng(0)
    W = rng.integers(-9, 9, size=(1 << 12, 2)).astype(np.float64)
    assert np.array_equal(fwht_rows(fwht_rows(W)), (1 << 12) * W)


def test_transform_matches_dense_definition():
    # Z = H_un D P X-tilde written with dense matrices
    rng = np.random.default_rng(1)
    N, d, seed = 37, 4, 5
    L, Np = padded_bits(N)
    X = rng.standard_normal((N, d))
    Xt = np.zeros((Np, d))
    Xt[:N] = X
    P = np.zeros((Np, Np))
    P[np.arange(Np), input_perm(seed, L)] = 1.0
    D = np.diag(sign_vector(seed, L))
    Zd = sylvester(L) @ D @ P @ Xt
    np.testing.assert_allclose(transform(X, seed), Zd, rtol=0, atol=1e-12)


def test_full_sample_is_orthogonal():
    # with m = N' the SRHT is orthogonal: S^T S = I, so ||S X v|| = ||X v||
    rng = np.random.default_rng(2)
    N, d = 200, 5
    L, Np = padded_bits(N)
    X = rng.standard_normal((N, d))
    Y = rng.standard_normal(N)
    B, BY, _, _ = nested_srht(X, Y, 3, Np, 8)
    SX = B / np.sqrt(Np)
    np.testing.assert_allclose(SX.T @ SX, X.T @ X, rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose((BY / np.sqrt(Np)) @ (BY / np.sqrt(Np)), Y @ Y, rtol=1e-12)


def test_sketch_is_unbiased_in_expectation():
    # E[S^T S] = I_N (Monte Carlo over seeds, small N)
    N, m, reps = 16, 4, 3000
    L, Np = padded_bits(N)
    acc = np.zeros((N, N))
    I = np.eye(N)
    for s in range(reps):
        B, _, _, _ = nested_srht(I, np.zeros(N), 100 + s, m, 1)
        S = B / np.sqrt(m)
        acc += S.T @ S
    acc /= reps
    assert np.abs(acc - I).max() < 0.15


def test_distortion_shrinks_with_sketch_size():
    # Lemma 2.2 trend: the subspace-embedding distortion ||U^T S^T S U - I||
    # falls roughly like sqrt(d/m)
    rng = np.random.default_rng(4)
    N, d = 4096, 8
    U, _ = np.linalg.qr(rng.standard_normal((N, d)))
    B, _, _, _ = nested_srht(U, np.zeros(N), 9, 2048, 1)
    eps = []
    for m in (64, 256, 1024, 2048):
        SU = B[:m] / np.sqrt(m)
        eps.append(np.linalg.norm(SU.T @ SU - np.eye(d), 2))
    assert eps[0] > eps[1] > eps[2] > eps[3]
    assert eps[2] < 4 * np.sqrt(d / 1024)


def test_nested_prefix_views():
    rng = np.random.default_rng(6)
    N, d = 3000, 6
    X = rng.standard_normal((N, d))
    Y = rng.standard_normal(N)
    B, BY, Bh, info = nested_srht(X, Y, 21, 1024, 48)
    Z = transform(X, 21)
    L = info["L"]
    assert np.array_equal(B[:256], Z[slot_rows(21, L, 256)])
    assert np.array_equal(B, Z[info["pi"]])
    assert np.array_equal(Bh, Z[info["pi_hat"]])
    assert B.shape == (1024, d) and BY.shape == (1024,) and Bh.shape == (48, d)


def test_streamed_srht_rows_equal_the_dense_transform():
    # rows of Z = H_un D P X accumulated block by block in X's own row order
    # equal the same rows of the full transform, exactly on integer data
    # (ragged blocks, N not a power of two)
    from oracle.sketch import padded_bits, srht_rows_streamed, transform
    rng = np.random.default_rng(4)
    N, c, seed = 3000, 5, 11
    X = rng.integers(-8, 9, size=(N, c)).astype(np.float64)
    L, Np = padded_bits(N)
    Z = transform(X, seed)
    rows = rng.choice(Np, 40, replace=False)
    bounds = [0, 1, 700, 701, 2048, 2999, N]
    blocks = ((a, X[a:b]) for a, b in zip(bounds, bounds[1:]))
    got = srht_rows_streamed(blocks, rows, seed, L)
    assert np.array_equal(got, Z[rows])
