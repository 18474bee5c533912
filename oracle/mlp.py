"""FP64 reference of the schedule network and its features (test infrastructure).

Only tests, the smoke check and the CPU leg of the benchmark use this module.

The learned schedule is this project's answer to the open question of
choosing the schedule automatically (Sec. 4.3 fixes a_i = 3 and a doubling
schedule and leaves automatic selection open).  From features of a problem
the network predicts
  * the per-stage iteration count a in {1, 2, 3, 4} of Stage I,
  * the prefix stride in {1, 2} (sketch sizes grow by 2 or by 4 per stage),
  * the number of Stage II iterations s_II the plain stopping test takes.

Network: three dense layers F -> H -> H -> O with ReLU after the first two.
Outputs 0..3 are logits for a - 1, 4..5 logits for stride - 1, output 6
regresses s_II / S_SCALE.  Per-sample loss with masks w_a, w_s:
    w_a * [CE(out[0:4], a) + CE(out[4:6], g)] + w_s * LAMBDA * (out[6] - s / S_SCALE)^2
averaged over the n samples.  Parameters form one flat vector in the order
W1 (H x F, row-major), b1 (H), W2 (H x H), b2 (H), W3 (O x H), b3 (O).

Features (8 values, all scale-free), see `features_pre` / `features_ii`.
"""
import numpy as np

F, H, O = 8, 64, 7
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

    a_label in {0..3} (a - 1), g_label in {0, 1} (stride - 1), s_label the
    Stage II count; w_a, w_s per-sample weights of the two parts."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    out, (Xc, z1, h1, z2, h2) = forward(theta, X)
    n = Xc.shape[0]
    idx = np.arange(n)
    a = np.asarray(a_label, dtype=np.int64)
    g = np.asarray(g_label, dtype=np.int64)
    t = np.asarray(s_label, dtype=np.float64) / S_SCALE
    wa = np.asarray(w_a, dtype=np.float64)
    ws = np.asarray(w_s, dtype=np.float64)
    pa = _softmax(out[:, 0:4])
    pg = _softmax(out[:, 4:6])
    ce = -np.log(pa[idx, a]) - np.log(pg[idx, g])
    sq = (out[:, 6] - t) ** 2
    loss = float(np.mean(wa * ce + ws * LAMBDA * sq))
    d_out = np.zeros_like(out)
    d_out[:, 0:4] = pa
    d_out[idx, a] -= 1.0
    d_out[:, 4:6] = pg
    d_out[idx, 4 + g] -= 1.0
    d_out[:, 0:6] *= wa[:, None]
    d_out[:, 6] = ws * 2.0 * LAMBDA * (out[:, 6] - t)
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


def policy(out_row):
    """(a, stride) from the network outputs of the pre-Stage-I features:
    arg-max of each logit group, first index on ties."""
    out_row = np.asarray(out_row)
    return int(np.argmax(out_row[0:4])) + 1, int(np.argmax(out_row[4:6])) + 1


def unchecked_iters(out6, margin, t_left):
    """Stage II iterations run before the first stopping test:
    clamp(round-half-away(out6 * S_SCALE) - margin, 0, t_left)."""
    s = float(out6) * S_SCALE
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
