"""Algorithm 1 (SPCG) and full-data PCG in FP64 (test infrastructure).

Stage I runs PCG for a_i iterations on each sketched problem
(S_i X, S_i Y), warm-started from the previous stage's output (Sec. 2.2 and
the warm-start relation at the start of Sec. 3); Stage II runs PCG on the
full problem (X, Y) from the Stage I result.  One preconditioner
H_hat = R^T R, from the QR factor of S_hat X, serves every solve.

Readings (where the paper leaves a choice open):

* schedule: m_i = m0 * growth^(i-1) while m_i < N (or <= m_max); the paper's
  experiments use m0 = 8d, growth 2 and m_K = N/2 (Sec. 4), which is this
  rule for N a power of two; the default here is m0 = 4d;
* r = 6d rows for S_hat, a_i = 3 (Sec. 4.1), beta_0 = 0, total budget T = 100;
* Stage II stops when sqrt(rho) <= tol * ||X x|| (see ``pcg``) or when the
  total iteration count reaches T; tol defaults to 5e-7 so that the relative
  prediction error ||X(x - beta_hat)|| / ||X beta_hat|| lands below 1e-6;
* ``sketch="cs"`` is SPCG-CS (Sec. 4.3): the nested CountSketch of
  ``countsketch`` replaces the SRHT for both the stage sketches and S-hat;
  its rows need no scaling (c^2 = 1, H-hat = (S-hat X)^T (S-hat X)).
"""
import time

import numpy as np

from .countsketch import countsketch, nested_countsketch
from .linalg import householder_qr
from .pcg import pcg
from .sketch import nested_srht, padded_bits
from .theory import theory_schedule


def schedule(N, d, m0=None, m_max=None, growth=2):
    """Sketch sizes m_1 < ... < m_K (Stage I); empty if m0 >= N."""
    m = 4 * d if m0 is None else int(m0)
    limit = N - 1 if m_max is None else min(int(m_max), N - 1)
    sizes = []
    while m <= limit:
        sizes.append(m)
        m *= growth
    return sizes


def precond_from_sketch(B_hat, scaled=True):
    """R with R^T R = B_hat^T B_hat / r (Householder QR of S_hat X); with
    ``scaled=False`` (CountSketch rows) R^T R = B_hat^T B_hat."""
    r = B_hat.shape[0]
    B_hat = np.asarray(B_hat, dtype=np.float64)
    return householder_qr(B_hat / np.sqrt(r) if scaled else B_hat)


def _stage_problems(X, Y, seed, sizes, r, sketch):
    """[(A_i, b_i (m_i x k), c2_i)] for the stages and R from S-hat."""
    Y2 = Y if Y.ndim == 2 else Y[:, None]
    if sketch == "cs":
        stages, B_hat = nested_countsketch(X, Y2, seed, sizes, r)
        t_sk = time.perf_counter()
        probs = [(A, b, 1.0) for A, b in stages]
        R = precond_from_sketch(B_hat, scaled=False)
        L, Np = padded_bits(X.shape[0])
        return probs, R, {"L": L, "Np": Np}, t_sk
    if sketch != "srht":
        raise ValueError("sketch must be 'srht' or 'cs'")
    mK = sizes[-1] if sizes else 1
    B, BY, B_hat, sk = nested_srht(X, Y2, seed, mK, r)
    t_sk = time.perf_counter()
    probs = [(B[:m], BY[:m], 1.0 / m) for m in sizes]
    return probs, precond_from_sketch(B_hat), sk, t_sk


def spcg(X, Y, seed, m0=None, m_max=None, r=None, a=3, tol=5e-7, T=100,
         growth=2, history=False, sketch="srht", sizes=None, nested_gradient=False,
         timings=None):
    """Algorithm 1.  Returns (beta_T, info) for Y of shape (N,) or (N, k).
    ``sizes`` gives the stage sizes explicitly (e.g. the tuned schedule of
    Sec. 4.3); ``a`` may be a number, a per-stage list, or ("theory", omega)
    for the counts of Theorems 3.3 / 3.4 (``theory.theory_schedule``).

    ``nested_gradient`` (SRHT only): the sketches are nested prefixes
    (Sec. 2.2), so with c2_i = 1/m_i the stage-(i+1) starting gradient is
    (m_i/m_{i+1}) g_i(x) + c2_{i+1} dA^T (db - dA x) over the new rows
    dA = rows m_i..m_{i+1} only, g_i the previous stage's final gradient.

    ``timings`` (a dict, optional) receives the wall-clock seconds of the
    sketch, the preconditioner, Stage I and Stage II (instrumentation only)."""
    clock = time.perf_counter
    t0 = clock()
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    N, d = X.shape
    r = 6 * d if r is None else int(r)
    sizes = schedule(N, d, m0, m_max, growth) if sizes is None else [int(m) for m in sizes]
    if isinstance(a, tuple) and a and a[0] == "theory":
        a_list = theory_schedule(sizes, d, a[1])
    else:
        a_list = [a] * len(sizes) if np.isscalar(a) else list(a)
    probs, R, sk, t_sketch = _stage_problems(X, Y, seed, sizes, r, sketch)
    t1 = t_pc = clock()
    multi = Y.ndim == 2
    Ys = Y if multi else Y[:, None]
    betas, infos = [], []
    for c in range(Ys.shape[1]):
        x = np.zeros(d)
        stage_x = []
        t = 0
        g_prev, m_prev = None, 0
        for (A, b, c2), ai in zip(probs, a_list):
            g0 = None
            if nested_gradient and g_prev is not None:
                if sketch != "srht":
                    raise ValueError("nested-gradient reuse needs nested prefixes (the SRHT)")
                dA, db = A[m_prev:], b[m_prev:, c]
                g0 = (m_prev / A.shape[0]) * g_prev + c2 * (dA.T @ (db - dA @ x))
            x, inf1 = pcg(A, b[:, c], c2, R, x, ai, g0=g0)
            g_prev, m_prev = inf1["g"], A.shape[0]
            t += ai
            stage_x.append(x.copy())
        t_s1 = clock()
        x, inf2 = pcg(X, Ys[:, c], 1.0, R, x, max(T - t, 0), tol=tol, history=history)
        t_s2 = clock()
        if timings is not None:
            timings["stage1"] = timings.get("stage1", 0.0) + (t_s1 - t1)
            timings["stage2"] = timings.get("stage2", 0.0) + (t_s2 - t_s1)
            t1 = t_s2
        betas.append(x)
        infos.append({"stage_x": stage_x, "stage2": inf2, "T_stage1": t,
                      "T": t + inf2["iters"], "a_list": a_list})
    beta = np.stack(betas, axis=1) if multi else betas[0]
    info = {"sizes": sizes, "R": R, "per_rhs": infos, "L": sk["L"], "Np": sk["Np"]}
    if timings is not None:
        timings["sketch"] = t_sketch - t0
        timings["precond"] = t_pc - t_sketch
    return beta, info


def full_pcg(X, Y, seed, r=None, tol=5e-7, T=100, sketch="srht"):
    """Full-data PCG from beta_0 = 0 with the same S_hat preconditioner."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    N, d = X.shape
    r = 6 * d if r is None else int(r)
    if sketch == "cs":
        R = precond_from_sketch(countsketch(X, seed, r, hat=True), scaled=False)
    else:
        _, _, B_hat, _ = nested_srht(X, Y, seed, 1, r)
        R = precond_from_sketch(B_hat)
    multi = Y.ndim == 2
    Ys = Y if multi else Y[:, None]
    betas, infos = [], []
    for c in range(Ys.shape[1]):
        x, inf = pcg(X, Ys[:, c], 1.0, R, np.zeros(d), T, tol=tol)
        betas.append(x)
        infos.append(inf)
    beta = np.stack(betas, axis=1) if multi else betas[0]
    return beta, {"R": R, "per_rhs": infos}


def rel_pred_error(X, beta, beta_ref):
    """||X (beta - beta_ref)|| / ||X beta_ref|| (columnwise max for k > 1)."""
    X = np.asarray(X, dtype=np.float64)
    D = X @ (np.asarray(beta, dtype=np.float64) - np.asarray(beta_ref, dtype=np.float64))
    Rf = X @ np.asarray(beta_ref, dtype=np.float64)
    num = np.linalg.norm(D, axis=0)
    den = np.linalg.norm(Rf, axis=0)
    return float(np.max(num / den))


__all__ = ["schedule", "precond_from_sketch", "spcg", "full_pcg",
           "rel_pred_error", "padded_bits"]
