"""Pins for the oracle's nested CountSketch (SPCG-CS of Sec. 4.3; CountSketch
as a sparse sketching operator, Sec. 2.1).  Each property is fixed by the
definition of a CountSketch or by linear algebra, not by the code under test."""
import numpy as np
import pytest

from oracle.countsketch import countsketch, fold, nested_countsketch, signs, slots
from oracle.ols import ols_householder as ols
from oracle.sketch import padded_bits
from oracle.spcg import full_pcg, rel_pred_error, schedule, spcg


def test_matches_explicit_sparse_matrix():
    # S built column by column (one +-1 per column at its bucket), times X
    rng = np.random.default_rng(0)
    N, d, m, seed = 300, 4, 37, 11
    X = rng.integers(-20, 20, size=(N, d)).astype(np.float64)
    L, Np = padded_bits(N)
    h = slots(seed, L)[:N] % m
    s = signs(seed, L, N)
    S = np.zeros((m, N))
    for k in range(N):
        S[h[k], k] = s[k]
    assert np.array_equal(np.abs(S).sum(axis=0), np.ones(N))
    assert np.array_equal(countsketch(X, seed, m), S @ X)


@pytest.mark.parametrize("N,m", [(1000, 7), (1024, 256), (5000, 3000), (4097, 100)])
def test_buckets_are_balanced(N, m):
    # q is a bijection of [0, N'), so q mod m hits every bucket floor(N'/m)
    # or ceil(N'/m) times
    L, Np = padded_bits(N)
    q = slots(3, L)
    assert np.array_equal(np.sort(q), np.arange(Np))
    cnt = np.bincount(q % m, minlength=m)
    assert cnt.min() == Np // m and cnt.max() == -(-Np // m)


def test_full_width_sketch_is_orthogonal():
    # m = N': every bucket holds exactly one (padded) row, so S^T S = I and
    # the Gram is preserved exactly on integers
    rng = np.random.default_rng(1)
    N, d = 500, 6
    L, Np = padded_bits(N)
    X = rng.integers(-30, 30, size=(N, d)).astype(np.float64)
    SX = countsketch(X, 4, Np)
    assert np.array_equal(SX.T @ SX, X.T @ X)


def test_folding_gives_the_coarser_sketch():
    rng = np.random.default_rng(2)
    N, d = 3000, 5
    X = rng.integers(-40, 40, size=(N, d)).astype(np.float64)
    for m in (13, 52, 208):
        assert np.array_equal(fold(countsketch(X, 9, 4 * m), m), countsketch(X, 9, m))
    with pytest.raises(ValueError):
        fold(countsketch(X, 9, 50), 7)


def test_unbiased_gram_over_seeds():
    # E[S^T S] = I: the mean of (SX)^T(SX) over seeds approaches X^T X; with
    # a wrong sign rule (e.g. all +1) the cross terms of a non-centred X
    # would not cancel
    rng = np.random.default_rng(3)
    N, d, m, n = 400, 3, 20, 600
    X = rng.standard_normal((N, d)) + 1.0
    G = X.T @ X
    acc = np.zeros((d, d))
    for seed in range(n):
        SX = countsketch(X, seed, m)
        acc += SX.T @ SX
    acc /= n
    # each entry's spread over seeds is about sqrt(2/m) * |G|; 6 standard errors
    assert np.abs(acc - G).max() < 6 * np.sqrt(2.0 / m) * np.abs(G).max() / np.sqrt(n)


def test_signs_balanced_and_hat_independent():
    N = 1 << 14
    L, _ = padded_bits(N)
    s = signs(7, L, N)
    sh = signs(7, L, N, hat=True)
    assert abs(s.mean()) < 4 / np.sqrt(N) and abs(sh.mean()) < 4 / np.sqrt(N)
    assert abs((s * sh).mean()) < 4 / np.sqrt(N)          # independent streams
    q, qh = slots(7, L), slots(7, L, hat=True)
    assert np.mean(q % 97 == qh % 97) < 0.05              # independent bucket maps


def test_distortion_shrinks_with_sketch_size():
    rng = np.random.default_rng(4)
    N, d = 1 << 14, 8
    X = rng.standard_normal((N, d))
    Q, _ = np.linalg.qr(X)

    def eps(m):
        SQ = countsketch(Q, 5, m)
        sv = np.linalg.svd(SQ, compute_uv=False)
        return max(sv.max() ** 2 - 1, 1 - sv.min() ** 2)

    e = [eps(m) for m in (64, 512, 4096)]
    assert e[0] > e[1] > e[2] and e[2] < 0.2


def test_nested_sizes_must_divide():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((200, 3))
    Y = rng.standard_normal(200)
    with pytest.raises(ValueError):
        nested_countsketch(X, Y, 1, [10, 25], 12)
    stages, Bh = nested_countsketch(X, Y, 1, [10, 20, 40], 12)
    assert [A.shape[0] for A, _ in stages] == [10, 20, 40] and Bh.shape == (12, 3)
    assert np.allclose(fold(stages[2][0], 10), stages[0][0])


def test_spcg_cs_reaches_ols():
    # SPCG-CS (Sec. 4.3) converges to the OLS estimator like SPCG-SRHT
    rng = np.random.default_rng(6)
    N, d = 20000, 30
    X = rng.standard_normal((N, d)) * np.logspace(0, 3, d)
    beta = rng.standard_normal(d)
    Y = X @ beta + 0.1 * rng.standard_normal(N)
    bhat = ols(X, Y)
    b_cs, info = spcg(X, Y, 3, sketch="cs")
    assert rel_pred_error(X, b_cs, bhat) < 1e-6
    assert info["sizes"] == schedule(N, d)
    b_pcg, _ = full_pcg(X, Y, 3, sketch="cs")
    assert rel_pred_error(X, b_pcg, bhat) < 1e-6
