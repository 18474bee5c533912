"""The OLS estimator beta_hat = argmin 1/2 ||Y - X u||^2 (eq. (ols), Sec. 1).

Computed from a QR factorization of the augmented matrix [X | Y]:
[X | Y] = Q [[R, c], [0, rho]] gives beta_hat = R^{-1} c and
||Y - X beta_hat|| = |rho| (one column per right-hand side).  Test
infrastructure: see ``oracle/__init__.py``.

* ``ols_householder`` - the oracle's own Householder QR (``linalg``);
* ``ols_tsqr``        - tall-skinny QR for large N: the R factors of row
  blocks are stacked and factored again (Demmel et al., "Communication-
  optimal parallel and sequential QR and LU factorizations", 2012); the
  block factorizations call LAPACK through ``numpy.linalg.qr`` as a library
  primitive.  Blocks may be streamed so the full matrix never needs to be
  resident in FP64.
"""
import numpy as np

from .linalg import householder_qr, solve_upper


def ols_householder(X, Y):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    d = X.shape[1]
    R, QtY = householder_qr(X, extra=Y)
    c = QtY[:d]
    beta = np.stack([solve_upper(R, c[:, j]) for j in range(c.shape[1])], axis=1)
    return beta if Y.ndim == 2 else beta[:, 0]


def _block_r(blk):
    blk = np.asarray(blk, dtype=np.float64)
    return None if blk.shape[0] == 0 else np.linalg.qr(blk, mode="r")


def tsqr_r(blocks, workers=1):
    """R factor of the row-stacked blocks (each n_b x c, float64).

    The blocks are factored independently and their R factors stacked in
    block order and factored again.  With ``workers`` > 1 the block
    factorizations run concurrently on that many threads (one BLAS thread
    each); the stacked order, and so the result, is unchanged."""
    if workers <= 1:
        Rs = [_block_r(b) for b in blocks]
    else:
        from concurrent.futures import ThreadPoolExecutor
        from threadpoolctl import threadpool_limits
        Rs, pending = [], []
        with threadpool_limits(1), ThreadPoolExecutor(max_workers=workers) as ex:
            for b in blocks:
                pending.append(ex.submit(_block_r, b))
                if len(pending) >= 2 * workers:      # bound the blocks in flight
                    Rs.append(pending.pop(0).result())
            Rs.extend(f.result() for f in pending)
    Rs = [R for R in Rs if R is not None]
    R = np.linalg.qr(np.concatenate(Rs, axis=0), mode="r")
    return R


def ols_tsqr(X, Y, block=65536, workers=1):
    """OLS via TSQR of [X | Y] over row blocks of ``block`` rows."""
    X = np.asarray(X)
    Y = np.asarray(Y)
    d = X.shape[1]
    Y2 = Y.reshape(Y.shape[0], -1)

    def blocks():
        for i in range(0, X.shape[0], block):
            yield np.concatenate([np.asarray(X[i:i + block], dtype=np.float64),
                                  np.asarray(Y2[i:i + block], dtype=np.float64)], axis=1)

    Ra = tsqr_r(blocks(), workers)
    return ols_from_r(Ra, d, Y.ndim == 2)


def ols_from_r(Ra, d, multi=True):
    """beta_hat from the R factor of [X | Y]."""
    R = Ra[:d, :d]
    c = Ra[:d, d:]
    beta = np.stack([solve_upper(R, c[:, j]) for j in range(c.shape[1])], axis=1)
    return beta if multi else beta[:, 0]
