"""PCG on the normal equations of a least-squares problem (test infrastructure).

PCG(A, b, H_hat, beta_init, a) of Sec. 2.2: ``a`` iterations of
preconditioned conjugate gradients on c2 A^T A x = c2 A^T b started from
beta_init, preconditioned by H_hat = R^T R.  The recurrences are the
standard PCG ones (Nocedal & Wright, Numerical Optimization, Alg. 5.3) with
the residual kept in d-space:

    g = c2 A^T (b - A x);  z = H_hat^{-1} g;  p = z;  rho = g^T z
    repeat:  s = c2 A^T (A p);  alpha = rho / (p^T s)
             x += alpha p;  g -= alpha s;  z = H_hat^{-1} g
             rho' = g^T z;  p = z + (rho'/rho) p;  rho = rho'

One iteration costs 4md flops for the two products, 2d^2 for the two
triangular solves and ~10d for the vector work (the paper counts
(4m+13)d + 2d^2).  c2 = 1/m_i on the sketched problems makes
c2 (S_i X)^T S_i X comparable with X^T X; CG iterates are invariant under
that joint scaling.

Stopping test (used in Stage II only): sqrt(rho) estimates ||X(x - x*)||
within the factors of Lemma A.4, eq. (app-full-hessian); the run stops when
sqrt(rho) <= tol * ||A x|| (with ||A x|| from the latest product pass).
"""
import numpy as np

from .linalg import precond_apply


def pcg(A, b, c2, R, x0, iters, tol=None, history=False, g0=None):
    """Returns (x, info).

    iters: maximum number of iterations (the stage's a_i, or the remaining
    budget in Stage II).  tol: None -> run exactly ``iters`` iterations.
    g0: the starting gradient c2 A^T (b - A x0) when the caller already has
    it (nested-gradient reuse); computed here otherwise.
    info: {"iters": done, "rho": [...], "converged": bool, "xs": [...],
    "g": the final recurrence gradient}.
    A exact zero rho means the current x solves the system; no further
    iteration is taken (avoids 0/0).
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    if g0 is None:
        resid = b - A @ x
        g = c2 * (A.T @ resid)
    else:
        g = np.array(g0, dtype=np.float64, copy=True)
    ax_norm = np.linalg.norm(A @ x) * np.sqrt(c2) if tol is not None else None
    z = precond_apply(R, g)
    p = z.copy()
    rho = float(g @ z)
    info = {"rho": [rho], "xs": [x.copy()] if history else None, "converged": False}
    done = 0

    def _stop(rho_, axn):
        return tol is not None and np.sqrt(max(rho_, 0.0)) <= tol * axn

    if _stop(rho, ax_norm):
        info.update(iters=0, converged=True, g=g)
        return x, info
    while done < iters:
        if rho == 0.0:
            info["converged"] = True
            break
        Ap = A @ p
        s = c2 * (A.T @ Ap)
        pts = float(p @ s)
        if not (pts > 0.0) or not np.isfinite(pts):
            raise FloatingPointError("PCG breakdown: p^T s <= 0")
        if tol is not None:
            ax_norm = np.linalg.norm(A @ x) * np.sqrt(c2)
        alpha = rho / pts
        x = x + alpha * p
        g = g - alpha * s
        z = precond_apply(R, g)
        rho_new = float(g @ z)
        p = z + (rho_new / rho) * p
        rho = rho_new
        done += 1
        info["rho"].append(rho)
        if history:
            info["xs"].append(x.copy())
        if _stop(rho, ax_norm):
            info["converged"] = True
            break
    info["iters"] = done
    info["g"] = g
    return x, info
