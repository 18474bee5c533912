"""FP64 reference of the schedule network and its features (test infrastructure).

Only tests, the smoke check and the CPU leg of the benchmark use this module.

The learned schedule is this project's answer to the open question of
choosing the schedule automatically (Sec. 4.3 fixes a_i = 3 and a doubling
schedule and leaves automatic selection open).  At the start of every
sketched stage i (Algorithm 1, Stage I) the network sees that stage's
features and predicts
  * the stage's iteration count a_i in {0, 1, 2, 3, 4} (0: the stage only
    refreshes its starting gradient, its PCG iterations are skipped),
  * whether Stage I stops after this stage (stop in {0, 1}: the larger
    sketches are not visited and Stage II starts next);
at the start of Stage II, from the Stage II features, it predicts
  * the number of Stage II iterations s_II the plain stopping test takes.

Network: three dense layers F -> H -> H -> O with ReLU after the first two.
Outputs 0..4 are logits for a_i, 5..6 logits for stop, output 7 regresses
s_II / S_SCALE.  Per-sample loss with masks w_a, w_s:
    w_a * [CE(out[0:5], a) + CE(out[5:7], g)] + w_s * LAMBDA * (out[7] - s / S_SCALE)^2
averaged over the n samples.  Parameters form one flat vector in the order
W1 (H x F, row-major), b1 (H), W2 (H x H), b2 (H), W3 (O x H), b3 (O).

Features (8 values, all scale-free), see `features_pre`, `features_stage`
and `features_ii`.
"""
import numpy as np

F, H, O = 8, 64, 8
NA = 5                    # a_i in 0..NA-1
LAMBDA = 0.5
S_SCALE = 10.0
N_SAMPLE_ROWS = 256


def sizes():
    return [(H, F), (H,), (H, H), (H,), (O, H), (O,)]


def n_params():
    return sum(int(np.prod(s)) for s in sizes())


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for s in sizes():
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def forward(theta, X):
    """Returns (outputs (n x O), cache)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ W3.T + b3
    return out, (X, z1, h1, z2, h2)


def _softmax(z):
    m = z.max(axis=1, keepdims=True)
    e = np.exp(z - m)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grad(theta, X, a_label, g_label, s_label, w_a, w_s):
    """Mean loss and its gradient w.r.t. the flat parameter vector.

    a_label in {0..4} (a_i), g_label in {0, 1} (stop), s_label the Stage II
    count; w_a, w_s per-sample weights of the two parts."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    out, (Xc, z1, h1, z2, h2) = forward(theta, X)
    n = Xc.shape[0]
    idx = np.arange(n)
    a = np.asarray(a_label, dtype=np.int64)
    g = np.asarray(g_label, dtype=np.int64)
    t = np.asarray(s_label, dtype=np.float64) / S_SCALE
    wa = np.asarray(w_a, dtype=np.float64)
    ws = np.asarray(w_s, dtype=np.float64)
    pa = _softmax(out[:, 0:NA])
    pg = _softmax(out[:, NA:NA + 2])
    ce = -np.log(pa[idx, a]) - np.log(pg[idx, g])
    sq = (out[:, NA + 2] - t) ** 2
    loss = float(np.mean(wa * ce + ws * LAMBDA * sq))
    d_out = np.zeros_like(out)
    d_out[:, 0:NA] = pa
    d_out[idx, a] -= 1.0
    d_out[:, NA:NA + 2] = pg
    d_out[idx, NA + g] -= 1.0
    d_out[:, 0:NA + 2] *= wa[:, None]
    d_out[:, NA + 2] = ws * 2.0 * LAMBDA * (out[:, NA + 2] - t)
    d_out /= n
    gW3 = d_out.T @ h2
    gb3 = d_out.sum(axis=0)
    d2 = (d_out @ W3) * (z2 > 0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (z1 > 0)
    gW1 = d1.T @ Xc
    gb1 = d1.sum(axis=0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, grad


def adam_step(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1); t counts from 1.
    Returns the new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def policy_stage(out_row):
    """(a_i, stop) from the network outputs of one stage's features:
    arg-max of each logit group, first index on ties."""
    out_row = np.asarray(out_row)
    return int(np.argmax(out_row[0:NA])), int(np.argmax(out_row[NA:NA + 2]))


def unchecked_iters(out7, margin, t_left):
    """Stage II iterations run before the first stopping test:
    clamp(round-half-away(out7 * S_SCALE) - margin, 0, t_left)."""
    s = float(out7) * S_SCALE
    r = np.floor(abs(s) + 0.5) * np.sign(s)
    return int(min(max(r - margin, 0), t_left))


def init(seed=0):
    """He-style initialisation (zero biases)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in sizes():
        if len(s) == 2:
            parts.append(rng.standard_normal(s).ravel() * np.sqrt(2.0 / s[1]))
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


# ----------------------------------------------------------------- features

def sample_rows(N):
    """Rows whose norms give the leverage proxy: floor((2t+1) N / 512) for
    t < 256 when N >= 256, else every row."""
    if N < N_SAMPLE_ROWS:
        return np.arange(N)
    t = np.arange(N_SAMPLE_ROWS, dtype=np.int64)
    return ((2 * t + 1) * N) // (2 * N_SAMPLE_ROWS)


def features_pre(X_rows, N, d, R_diag):
    """Features known before Stage I.

    X_rows: the sampled rows (stored values, upcast, column scales applied);
    R_diag: diagonal of the preconditioner factor R.
      f0 = log10 N - 5            f1 = log10 d - 2
      f2 = log2(N / d) / 8 - 1    f3 = log10(max|R_jj| / min|R_jj|) / 3 - 1  (3 if min = 0)
      f4 = log10(max_j q_j / mean_j q_j) / 2, q_j = ||x_j||^2 over sampled rows (0 if all zero)
      f5 = f6 = f7 = 0"""
    f = np.zeros(F)
    f[0] = np.log10(N) - 5.0
    f[1] = np.log10(d) - 2.0
    f[2] = np.log2(N / d) / 8.0 - 1.0
    rd = np.abs(np.asarray(R_diag, dtype=np.float64))
    f[3] = 3.0 if rd.min() <= 0 else np.log10(rd.max() / rd.min()) / 3.0 - 1.0
    q = (np.asarray(X_rows, dtype=np.float64) ** 2).sum(axis=1)
    f[4] = 0.0 if q.sum() <= 0 else np.log10(q.max() / q.mean()) / 2.0
    return f


def thm33_bound(m_prev, m, d, omega=0.5):
    """The iteration lower bound of Theorem 3.3 for a stage of size m after
    one of size m_prev: ln{[(1 + omega) r + 1] / omega} / ln 4 with
    r = sqrt((m - d) / (m_prev - d))."""
    r = np.sqrt((m - d) / (m_prev - d))
    return np.log(((1.0 + omega) * r + 1.0) / omega) / np.log(4.0)


def features_stage(f_pre, sizes, s, d, resid2, ax2):
    """Features at the start of sketched stage s of the planned sizes
    m_0 < ... < m_{K-1} (every prefix of the sketch):
      f0, f1, f3, f4 as in features_pre;
      f2 = log2(m_s / d) / 8 - 1;
      f5 = B_s / 4, B_s the Theorem 3.3 bound for (m_{s-1}, m_s) with
           omega = 1/2 (stage 0: the pair (m_0, m_1); 1 when K = 1 -- r = 1);
      f6 = clamp(log10(resid2 / ax2) / 6, -2, 2) from the stage-start pass
           (-2 if resid2 <= 0, 2 if ax2 <= 0);
      f7 = s / K."""
    K = len(sizes)
    f = np.array(f_pre, dtype=np.float64).copy()
    m = float(sizes[s])
    f[2] = np.log2(m / d) / 8.0 - 1.0
    if K == 1:
        b = thm33_bound(1.0 + d, 1.0 + d, d)
    elif s == 0:
        b = thm33_bound(float(sizes[0]), float(sizes[1]), d)
    else:
        b = thm33_bound(float(sizes[s - 1]), m, d)
    f[5] = b / 4.0
    if resid2 <= 0:
        f6 = -2.0
    elif ax2 <= 0:
        f6 = 2.0
    else:
        f6 = np.log10(resid2 / ax2) / 6.0
    f[6] = min(max(f6, -2.0), 2.0)
    f[7] = s / K
    return f


def features_ii(f_pre, rho, ax2, resid2, tol):
    """Features at the start of Stage II: f0..f4 as before, then
      f5 = clamp(log10(sqrt(rho) / (tol sqrt(ax2))) / 3, -3, 3)   (-3 if rho <= 0, 3 if ax2 <= 0)
      f6 = clamp(log10(resid2 / ax2) / 6, -2, 2)                  (-2 if resid2 <= 0, 2 if ax2 <= 0)
      f7 = 1"""
    f = np.array(f_pre, dtype=np.float64).copy()
    if rho <= 0:
        f5 = -3.0
    elif ax2 <= 0:
        f5 = 3.0
    else:
        f5 = np.log10(np.sqrt(rho) / (tol * np.sqrt(ax2))) / 3.0
    if resid2 <= 0:
        f6 = -2.0
    elif ax2 <= 0:
        f6 = 2.0
    else:
        f6 = np.log10(resid2 / ax2) / 6.0
    f[5] = min(max(f5, -3.0), 3.0)
    f[6] = min(max(f6, -2.0), 2.0)
    f[7] = 1.0
    return f
