"""Pins for the oracle's Householder QR, triangular solves and OLS
(eq. (ols) of Sec. 1; preconditioner applied through a QR factorization, Sec. 4)."""
import numpy as np
import pytest

from oracle.fwht import sylvester
from oracle.linalg import householder_qr, precond_apply, solve_upper, solve_upper_transpose
from oracle.ols import ols_householder, ols_tsqr


@pytest.mark.parametrize("n,d", [(10, 10), (50, 7), (300, 40)])
def test_householder_matches_lapack_up_to_row_signs(n, d):
    rng = np.random.default_rng(n + d)
    A = rng.standard_normal((n, d)) * np.logspace(0, 3, d)
    R = householder_qr(A)
    Rl = np.linalg.qr(A, mode="r")          # LAPACK dgeqrf (independent code)
    Rl = np.sign(np.diag(Rl))[:, None] * Rl
    assert np.all(np.diag(R) > 0)
    assert np.allclose(np.tril(R, -1), 0.0)
    np.testing.assert_allclose(R, Rl, rtol=1e-10, atol=1e-10 * np.abs(Rl).max())
    np.testing.assert_allclose(R.T @ R, A.T @ A, rtol=1e-10, atol=1e-9 * np.abs(A.T @ A).max())


def test_triangular_solves_against_lapack():
    rng = np.random.default_rng(3)
    d = 30
    R = np.triu(rng.standard_normal((d, d))) + 5 * np.eye(d)
    b = rng.standard_normal(d)
    np.testing.assert_allclose(solve_upper(R, b), np.linalg.solve(R, b), rtol=1e-12)
    np.testing.assert_allclose(solve_upper_transpose(R, b), np.linalg.solve(R.T, b), rtol=1e-12)
    np.testing.assert_allclose(precond_apply(R, b), np.linalg.solve(R.T @ R, b), rtol=1e-10)


def test_ols_matches_lstsq_and_normal_equations():
    rng = np.random.default_rng(7)
    N, d = 2000, 12
    X = rng.standard_normal((N, d)) * np.logspace(0, 2, d)
    Y = X @ rng.standard_normal(d) + 0.1 * rng.standard_normal(N)
    b1 = ols_householder(X, Y)
    b2 = np.linalg.lstsq(X, Y, rcond=None)[0]            # LAPACK (independent)
    b3 = np.linalg.solve(X.T @ X, X.T @ Y)                # closed form of eq. (ols)
    np.testing.assert_allclose(b1, b2, rtol=1e-10)
    np.testing.assert_allclose(b1, b3, rtol=1e-8)


def test_tsqr_matches_householder():
    rng = np.random.default_rng(8)
    N, d = 5000, 9
    X = rng.standard_normal((N, d))
    Y = rng.standard_normal((N, 2))
    np.testing.assert_allclose(ols_tsqr(X, Y, block=700), ols_householder(X, Y), rtol=1e-10)


def test_ols_exact_on_hadamard_columns():
    # X = d columns of a Sylvester matrix: X^T X = N' I, so beta_hat = X^T Y / N'
    # exactly (dyadic rationals of small integers are exact in FP64)
    L, d = 9, 6
    H = sylvester(L)
    X = H[:, [1, 3, 4, 7, 10, 13]]
    rng = np.random.default_rng(9)
    Y = rng.integers(-100, 100, size=1 << L).astype(np.float64)
    exact = X.T @ Y / (1 << L)
    np.testing.assert_allclose(ols_householder(X, Y), exact, rtol=0, atol=1e-12)


def test_tsqr_concurrent_blocks_equal_sequential():
    # the block factorizations are independent: running them on threads
    # leaves the stacked order and so the R factor unchanged, and beta
    # agrees with LAPACK's least squares
    from oracle.ols import ols_tsqr, tsqr_r
    rng = np.random.default_rng(21)
    X = rng.standard_normal((9000, 12)) * np.logspace(0, 3, 12)
    Y = X @ rng.standard_normal(12) + 0.1 * rng.standard_normal(9000)
    A = np.concatenate([X, Y[:, None]], axis=1)
    blocks = [A[i:i + 1000] for i in range(0, 9000, 1000)]
    R1 = tsqr_r(iter(blocks), workers=1)
    R4 = tsqr_r(iter(blocks), workers=4)
    assert np.array_equal(R1, R4)
    b = ols_tsqr(X, Y, block=700, workers=3)
    ref = np.linalg.lstsq(X, Y, rcond=None)[0]
    assert np.linalg.norm(X @ (b - ref)) / np.linalg.norm(X @ ref) < 1e-12
