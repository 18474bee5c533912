"""Pins for the FP64 schedule-network reference: the analytic gradient
equals central finite differences of the loss (with both masks), the loss
reduces to log-sum-exp closed forms when the hidden layers are silent, the
first Adam step moves every parameter by lr * sign(g), the features take
known values on constructed inputs, and the per-stage Theorem 3.3 feature
equals the bound computed by hand."""
import numpy as np

from oracle import mlp


def _batch(rng, n):
    X = rng.standard_normal((n, mlp.F))
    a = rng.integers(0, mlp.NA, n)
    g = rng.integers(0, 2, n)
    s = rng.integers(0, 20, n)
    wa = rng.integers(0, 2, n).astype(float)
    ws = 1.0 - wa
    ws[0] = 1.0
    wa[1] = 1.0
    return X, a, g, s, wa, ws


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = mlp.init(1) + 0.05 * rng.standard_normal(mlp.n_params())
    args = _batch(rng, 9)
    _, grad = mlp.loss_and_grad(theta, *args)
    h = 1e-6
    # every bias plus a random subset of weights
    nb = [(mlp.H * mlp.F) + i for i in range(mlp.H)] + list(range(mlp.n_params() - mlp.O, mlp.n_params()))
    idx = np.concatenate([rng.choice(mlp.n_params(), 80, replace=False), nb])
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss_and_grad(tp, *args)[0] - mlp.loss_and_grad(tm, *args)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_loss_closed_form_silent_hidden_layers():
    # zero weights: every output equals its bias, for every sample
    theta = np.zeros(mlp.n_params())
    b3 = np.array([1.0, 2.0, 0.5, -1.0, 0.75, 0.25, -0.5, 0.3])
    theta[-mlp.O:] = b3
    X = np.ones((3, mlp.F))
    a = np.array([1, 1, 4])
    g = np.array([0, 1, 1])
    s = np.array([3.0, 5.0, 3.0])
    wa = np.array([1.0, 0.0, 1.0])
    ws = np.array([0.0, 1.0, 1.0])
    lse_a = np.log(np.exp(b3[:5]).sum())
    lse_g = np.log(np.exp(b3[5:7]).sum())
    ce = lambda ai, gi: (lse_a - b3[ai]) + (lse_g - b3[5 + gi])
    expect = (ce(1, 0) + mlp.LAMBDA * (0.3 - 0.5) ** 2 + ce(4, 1)) / 3.0
    loss, grad = mlp.loss_and_grad(theta, X, a, g, s, wa, ws)
    assert abs(loss - expect) < 1e-12
    pa = np.exp(b3[:5]) / np.exp(b3[:5]).sum()
    # d loss / d b3[0:5] = mean over masked samples of softmax - one-hot
    want = (2 * pa - np.array([0, 1, 0, 0, 1.0])) / 3.0
    assert np.allclose(grad[-mlp.O:-3], want, atol=1e-14)
    pg = np.exp(b3[5:7]) / np.exp(b3[5:7]).sum()
    # masked samples 0 and 2 carry stop labels 0 and 1
    assert np.allclose(grad[-3:-1], (2 * pg - np.array([1.0, 1.0])) / 3.0, atol=1e-14)
    want7 = (2 * mlp.LAMBDA * (0.3 - 0.5) + 2 * mlp.LAMBDA * (0.3 - 0.3)) / 3.0
    assert abs(grad[-1] - want7) < 1e-14


def test_first_adam_step_is_signed_lr():
    rng = np.random.default_rng(3)
    theta = rng.standard_normal(50)
    grad = rng.standard_normal(50)
    new, m, v = mlp.adam_step(theta, grad, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=0.0)
    assert np.allclose(new - theta, -1e-3 * np.sign(grad), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * grad) and np.allclose(v, 0.001 * grad ** 2)


def test_policy_and_unchecked_iterations():
    assert mlp.policy_stage([0, 0, 0, 5, 0, 1, 2, 0]) == (3, 1)
    assert mlp.policy_stage([1, 1, 1, 1, 1, 0, 0, 0]) == (0, 0)  # ties: first index
    assert mlp.policy_stage([0, 0, 0, 0, 7, 3, 1, 0]) == (4, 0)
    assert mlp.unchecked_iters(0.74, 1, 100) == 6
    assert mlp.unchecked_iters(0.75, 1, 100) == 7
    assert mlp.unchecked_iters(-0.3, 1, 100) == 0
    assert mlp.unchecked_iters(9.0, 0, 40) == 40


def test_features_on_constructed_inputs():
    N, d = 1 << 12, 16
    rows = mlp.sample_rows(N)
    assert len(rows) == 256 and rows[0] == 8 and rows[-1] == N - 8
    assert len(np.unique(rows)) == 256
    assert list(mlp.sample_rows(5)) == [0, 1, 2, 3, 4]
    Xr = np.ones((256, d))
    Xr[7] *= 10.0  # one row with 100x the squared norm
    R = np.array([2.0] * 15 + [2000.0])
    f = mlp.features_pre(Xr, N, d, R)
    q = np.full(256, float(d)); q[7] = 100.0 * d
    assert np.isclose(f[0], np.log10(N) - 5) and np.isclose(f[1], np.log10(16) - 2)
    assert np.isclose(f[2], 8 / 8 - 1)
    assert np.isclose(f[3], 3 / 3 - 1)
    assert np.isclose(f[4], np.log10(q.max() / q.mean()) / 2)
    assert np.all(f[5:] == 0)
    fi = mlp.features_ii(f, rho=1e-10, ax2=1e2, resid2=1e-4, tol=1e-6)
    assert np.allclose(fi[:5], f[:5])
    assert np.isclose(fi[5], np.log10(1e-5 / (1e-6 * 10)) / 3)
    assert np.isclose(fi[6], -1.0) and fi[7] == 1.0
    assert mlp.features_ii(f, 0.0, 1.0, 0.0, 1e-6)[5] == -3.0
    assert mlp.features_ii(f, 1e30, 1.0, 1e30, 1e-6)[5] == 3.0


def test_stage_features_and_theorem_3_3_bound():
    # doubling from m_0 = 4 d: r_{i-1,i}^2 = 2 + d / (m_{i-1} - d) (Sec. 3,
    # after Theorem 3.3); at omega = 1/2 the bound is
    # ln((1.5 r + 1) / 0.5) / ln 4, here evaluated by hand
    d = 100
    sizes = [400, 800, 1600, 3200]
    r2 = 2 + d / (800 - d)                      # stage 2: (m_1, m_2)
    assert np.isclose((1600 - d) / (800 - d), r2)
    b2 = np.log((1.5 * np.sqrt(r2) + 1) / 0.5) / np.log(4)
    assert np.isclose(mlp.thm33_bound(800, 1600, d), b2)
    # by hand: r = sqrt(15/7) = 1.463850, (1.5 r + 1) / 0.5 = 6.391550, ln 6.391550 / ln 4 = 1.854980 / 1.386294
    assert abs(b2 - 1.338083) < 1e-6
    f_pre = np.array([0.1, -0.2, 0.3, 0.4, 0.5, 0, 0, 0])
    f = mlp.features_stage(f_pre, sizes, 2, d, resid2=1e-2, ax2=1e4)
    assert np.allclose(f[[0, 1, 3, 4]], f_pre[[0, 1, 3, 4]])
    assert np.isclose(f[2], np.log2(16) / 8 - 1)
    assert np.isclose(f[5], b2 / 4)
    assert np.isclose(f[6], -1.0) and np.isclose(f[7], 0.5)
    # stage 0 takes the pair (m_0, m_1); one stage: r = 1
    f0 = mlp.features_stage(f_pre, sizes, 0, d, resid2=1.0, ax2=0.0)
    assert np.isclose(f0[5], mlp.thm33_bound(400, 800, d) / 4) and f0[6] == 2.0 and f0[7] == 0.0
    f1 = mlp.features_stage(f_pre, [400], 0, d, resid2=0.0, ax2=1.0)
    assert np.isclose(f1[5], np.log(5.0) / np.log(4.0) / 4) and f1[6] == -2.0
