"""Householder QR and triangular solves in FP64 (test infrastructure).

The preconditioner of Sec. 2.2 is the fixed sketched Hessian
H_hat = (S_hat X)^T (S_hat X); the experiments of Sec. 4 apply it "through a
QR factorization": with S_hat X = Q R, H_hat = R^T R and
H_hat^{-1} g = R^{-1} (R^{-T} g).  Textbook Householder QR (Golub & Van Loan,
Matrix Computations, Alg. 5.2.1) written out column by column; the sign of
each row of R is fixed so that diag(R) > 0.
"""
import numpy as np


def householder_qr(A, extra=None):
    """R factor of A (n x d, n >= d) with diag(R) > 0.

    If ``extra`` (n x k) is given, Q^T extra is also returned (its first d
    rows pair with R; the remaining n - d rows are the part orthogonal to
    range(A)).  Returns R, or (R, QtE).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    n, d = A.shape
    if n < d:
        raise ValueError("householder_qr needs n >= d")
    E = None if extra is None else np.array(extra, dtype=np.float64, copy=True).reshape(n, -1)
    for j in range(d):
        x = A[j:, j]
        alpha = np.linalg.norm(x)
        if alpha == 0.0:
            continue
        # reflect x onto -sign(x0) * alpha * e1 (no cancellation in v0)
        s = 1.0 if x[0] >= 0 else -1.0
        v = x.copy()
        v[0] += s * alpha
        vnorm2 = v @ v
        A[j:, j:] -= np.outer(v, (2.0 / vnorm2) * (v @ A[j:, j:]))
        if E is not None:
            E[j:, :] -= np.outer(v, (2.0 / vnorm2) * (v @ E[j:, :]))
    R = np.triu(A[:d, :])
    # make diag(R) positive: R <- D R, Q <- Q D with D = sign(diag R)
    sg = np.where(np.diag(R) < 0, -1.0, 1.0)
    R = sg[:, None] * R
    if E is None:
        return R
    E[:d] = sg[:, None] * E[:d]
    return R, E


def solve_upper(R, b):
    """x with R x = b, R upper triangular (back substitution)."""
    R = np.asarray(R, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = R.shape[0]
    x = np.zeros_like(b, dtype=np.float64)
    for i in range(d - 1, -1, -1):
        x[i] = (b[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x


def solve_upper_transpose(R, b):
    """z with R^T z = b, R upper triangular (forward substitution)."""
    R = np.asarray(R, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = R.shape[0]
    z = np.zeros_like(b, dtype=np.float64)
    for i in range(d):
        z[i] = (b[i] - R[:i, i] @ z[:i]) / R[i, i]
    return z


def precond_apply(R, g):
    """H_hat^{-1} g = R^{-1} (R^{-T} g)."""
    return solve_upper(R, solve_upper_transpose(R, g))
