"""Pins for the oracle's PCG (Sec. 2.2) and Algorithm 1 (Stage I / II)."""
import numpy as np
import pytest

from oracle.linalg import householder_qr
from oracle.ols import ols_householder
from oracle.pcg import pcg
from oracle.sketch import nested_srht
from oracle.spcg import full_pcg, precond_from_sketch, rel_pred_error, schedule, spcg
from oracle.theory import cg_bound_factor, stage_contraction


def _problem(N=3000, d=10, cond=1e3, sigma=0.1, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, d)) * np.logspace(0, np.log10(cond), d)
    beta = rng.standard_normal(d)
    Y = X @ beta + sigma * rng.standard_normal(N)
    return X, Y, beta


def test_exact_preconditioner_converges_in_one_step():
    X, Y, _ = _problem()
    R = householder_qr(X)
    x, info = pcg(X, Y, 1.0, R, np.zeros(X.shape[1]), 1)
    np.testing.assert_allclose(x, np.linalg.lstsq(X, Y, rcond=None)[0], rtol=1e-9)


def test_cg_terminates_in_at_most_d_steps():
    X, Y, _ = _problem(N=400, d=6, cond=10)
    x, _ = pcg(X, Y, 1.0, np.eye(6), np.zeros(6), 6)
    np.testing.assert_allclose(x, ols_householder(X, Y), rtol=1e-8)


def test_cg_error_monotone_and_within_lemma_a2():
    # ||A(x_j - x*)|| is non-increasing and obeys Lemma A.2 with the measured
    # condition number of the preconditioned normal matrix
    X, Y, _ = _problem(N=2000, d=20, cond=1e4, seed=2)
    xs = ols_householder(X, Y)
    _, _, Bh, _ = nested_srht(X, Y, 4, 1, 120)
    R = precond_from_sketch(Bh)
    Ri = np.linalg.inv(R)
    ev = np.linalg.eigvalsh(Ri.T @ X.T @ X @ Ri)
    kappa = ev[-1] / ev[0]
    x0 = np.zeros(20)
    _, info = pcg(X, Y, 1.0, R, x0, 15, history=True)
    e = [np.linalg.norm(X @ (x - xs)) for x in info["xs"]]
    e0 = e[0]
    for j, ej in enumerate(e):
        assert ej <= cg_bound_factor(kappa, j) * e0 * (1 + 1e-9) + 1e-12
        if j:
            assert ej <= e[j - 1] * (1 + 1e-9)


def test_zero_rhs_returns_immediately():
    X, _, _ = _problem(N=100, d=4)
    x, info = pcg(X, np.zeros(100), 1.0, np.eye(4), np.zeros(4), 5, tol=1e-6)
    assert info["iters"] == 0 and np.all(x == 0)
    x, info = pcg(X, np.zeros(100), 1.0, np.eye(4), np.zeros(4), 5)
    assert np.all(x == 0)


def test_breakdown_is_reported():
    X, Y, _ = _problem(N=100, d=4)
    Y = Y.copy()
    Y[3] = np.nan
    with pytest.raises(FloatingPointError):
        pcg(X, Y, 1.0, np.eye(4), np.zeros(4), 3)


def test_stage_contraction_inequality_with_measured_distortion():
    # Proof of Theorem 3.1, eq. (app-stage-intermediate):
    # ||X(beta_a - beta_tilde)|| <= 2 sqrt((1+e)/(1-e)) e^a ||X(beta_0 - beta_tilde)||
    # with e the largest measured distortion of S_i and S_hat on range(X); for
    # e < 1/9 the theta = 1/4 form of eq. (app-stage-exact) follows.
    rng = np.random.default_rng(11)
    N, d = 1 << 14, 4
    X = rng.standard_normal((N, d)) * np.array([1.0, 3.0, 10.0, 30.0])
    Y = X @ rng.standard_normal(d) + rng.standard_normal(N)
    U, _ = np.linalg.qr(X)
    m, r = 4096, 4096
    B, BY, Bh, _ = nested_srht(X, Y, 13, m, r)
    Bu, _, Bhu, _ = nested_srht(U, np.zeros(N), 13, m, r)
    eps_i = np.linalg.norm((Bu / np.sqrt(m)).T @ (Bu / np.sqrt(m)) - np.eye(d), 2)
    eps_h = np.linalg.norm((Bhu / np.sqrt(r)).T @ (Bhu / np.sqrt(r)) - np.eye(d), 2)
    eps = max(eps_i, eps_h)
    assert eps < 1.0 / 9.0
    R = precond_from_sketch(Bh)
    bt = ols_householder(B, BY)                    # exact sketched estimator
    x0 = rng.standard_normal(d) * 5
    for a in (1, 2, 3):
        xa, _ = pcg(B, BY, 1.0 / m, R, x0, a)
        lhs = np.linalg.norm(X @ (xa - bt))
        rhs0 = np.linalg.norm(X @ (x0 - bt))
        assert lhs <= stage_contraction(eps, a) * rhs0 * (1 + 1e-8) + 1e-9
        assert lhs <= 0.25 ** a * rhs0 * (1 + 1e-8) + 1e-9


def test_spcg_reaches_ols_and_full_pcg_agrees():
    X, Y, _ = _problem(N=20000, d=20, cond=1e3, sigma=0.1, seed=5)
    bh = ols_householder(X, Y)
    b_spcg, info = spcg(X, Y, seed=1)
    b_pcg, _ = full_pcg(X, Y, seed=1)
    assert rel_pred_error(X, b_spcg, bh) <= 1e-6
    assert rel_pred_error(X, b_pcg, bh) <= 1e-6
    # warm start: each stage starts where the previous one stopped, and the
    # schedule is the doubling one
    assert info["sizes"] == schedule(20000, 20)
    assert info["per_rhs"][0]["T_stage1"] == 3 * len(info["sizes"])


def test_spcg_multi_rhs_equals_column_runs():
    X, Y, _ = _problem(N=5000, d=8, seed=6)
    Y2 = np.stack([Y, 2 * Y + 1], axis=1)
    b2, _ = spcg(X, Y2, seed=3)
    b0, _ = spcg(X, Y2[:, 0], seed=3)
    b1, _ = spcg(X, Y2[:, 1], seed=3)
    np.testing.assert_array_equal(b2[:, 0], b0)
    np.testing.assert_array_equal(b2[:, 1], b1)


def test_spcg_prediction_error_reaches_ols_level():
    # Sec. 4.2: SPCG reaches the OLS error level; Delta_T vs Delta_OLS over seeds
    ratios = []
    for s in range(4):
        X, Y, beta = _problem(N=1 << 14, d=16, cond=1e4, sigma=1e-4, seed=20 + s)
        bh = ols_householder(X, Y)
        bT, _ = spcg(X, Y, seed=s + 1, m0=8 * 16, tol=1e-12)
        ratios.append(np.linalg.norm(X @ (bT - beta)) ** 2 / np.linalg.norm(X @ (bh - beta)) ** 2)
    assert max(ratios) < 1.01


def test_nested_gradient_reuse_equals_direct_gradient():
    # Nested prefixes (Sec. 2.2): with c2 = 1/m the stage-start gradient of
    # the larger prefix is the rescaled gradient of the smaller one plus the
    # new rows' term, for any x
    from oracle.pcg import pcg
    from oracle.spcg import precond_from_sketch, spcg, rel_pred_error
    from oracle.sketch import nested_srht
    from oracle.ols import ols_householder
    rng = np.random.default_rng(11)
    N, d = 4096, 12
    X = rng.standard_normal((N, d)) * np.logspace(0, 2, d)
    Y = X @ rng.standard_normal(d) + 0.1 * rng.standard_normal(N)
    B, BY, Bh, _ = nested_srht(X, Y, 3, 1024, 72)
    R = precond_from_sketch(Bh)
    x = rng.standard_normal(d)
    m1, m2 = 256, 512
    g1 = (B[:m1].T @ (BY[:m1] - B[:m1] @ x)) / m1
    direct = (B[:m2].T @ (BY[:m2] - B[:m2] @ x)) / m2
    nested = (m1 / m2) * g1 + (B[m1:m2].T @ (BY[m1:m2] - B[m1:m2] @ x)) / m2
    np.testing.assert_allclose(nested, direct, rtol=1e-12, atol=1e-12 * np.abs(direct).max())
    # the PCG's final recurrence gradient equals the true gradient at its iterate
    xe, info = pcg(B[:m1], BY[:m1], 1.0 / m1, R, np.zeros(d), 3)
    true_g = (B[:m1].T @ (BY[:m1] - B[:m1] @ xe)) / m1
    np.testing.assert_allclose(info["g"], true_g, rtol=1e-9, atol=1e-9 * np.abs(true_g).max())
    # and SPCG with reuse reaches the OLS estimator with the same stage counts
    b1, i1 = spcg(X, Y, 3, nested_gradient=True)
    b0, i0 = spcg(X, Y, 3)
    bh = ols_householder(X, Y)
    assert rel_pred_error(X, b1, bh) < 1e-6
    assert i1["per_rhs"][0]["T_stage1"] == i0["per_rhs"][0]["T_stage1"]
    assert abs(i1["per_rhs"][0]["stage2"]["iters"] - i0["per_rhs"][0]["stage2"]["iters"]) <= 1
