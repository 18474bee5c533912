"""Seeded synthetic least-squares workloads (Y = X beta + zeta).

Input generators shared by the tests, the benchmark and the smoke check.
This package holds none of the method's arithmetic: it only draws X, beta
and the noise, and stores X in the requested precision.  Every generator
is seeded and device-agnostic (torch generators on the target device), so
a GPU run draws its inputs on the GPU and a test can copy the very same
tensors to the host for the oracle.

Shapes follow the experiments of Sec. 4 of the SPCG paper (X = G D with G
Gaussian and D a diagonal of column scales chosen for a target condition
number, beta ~ N(0, I), zeta ~ N(0, sigma^2 I)) and extended workloads
(Haar-SVD, Student-t rows with a correlation factor, batched problems,
high-leverage rows).

Stored precisions: float64, float32, bfloat16 (torch's round-to-nearest-
even cast) and float8_e4m3fn with a per-column power-of-two scale
2^ceil(log2(amax_j / 448)), so that stored * scale is exact in FP32/FP64.
Y is always float64 and computed from the unquantized FP64/FP32 X.
"""
import math
from dataclasses import dataclass, field
from typing import Optional

import torch

BASE_SEED = 20261203
FP8_MAX = 448.0


@dataclass
class Problem:
    name: str
    X: torch.Tensor                 # stored matrix, N x d (row-major, contiguous)
    Y: torch.Tensor                 # float64, N x k
    beta: torch.Tensor              # float64, d x k (true coefficients)
    sigma: float
    col_scale: Optional[torch.Tensor] = None  # float32 d (FP8 storage only)
    meta: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.X.shape[0]

    @property
    def d(self):
        return self.X.shape[1]

    @property
    def k(self):
        return self.Y.shape[1]

    def x_f64(self, rows=None):
        """Stored values upcast exactly to float64 (optionally a row slice)."""
        Xs = self.X if rows is None else self.X[rows]
        Xd = Xs.to(torch.float64)
        if self.col_scale is not None:
            Xd = Xd * self.col_scale.to(torch.float64)
        return Xd


def generator(device, seed):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def log_spaced(lo, hi, n, device="cpu"):
    if n == 1:
        return torch.tensor([float(lo)], dtype=torch.float64, device=device)
    return torch.logspace(math.log10(lo), math.log10(hi), n, dtype=torch.float64, device=device)


def haar_orthonormal(n, d, g, device):
    """n x d with Haar-distributed orthonormal columns (QR of a Gaussian,
    signs fixed by diag(R) > 0)."""
    G = torch.randn(n, d, generator=g, device=device, dtype=torch.float64)
    Q, R = torch.linalg.qr(G)
    return Q * torch.sign(torch.diagonal(R)).unsqueeze(0)


def store(X, storage):
    """Cast X to the stored precision; returns (X_stored, col_scale or None)."""
    if storage in ("f64", torch.float64):
        return X.to(torch.float64).contiguous(), None
    if storage in ("f32", torch.float32):
        return X.to(torch.float32).contiguous(), None
    if storage in ("bf16", torch.bfloat16):
        return X.to(torch.bfloat16).contiguous(), None
    if storage in ("fp8", torch.float8_e4m3fn):
        Xf = X.to(torch.float32)
        amax = Xf.abs().amax(dim=0).clamp_min(torch.finfo(torch.float32).tiny)
        scale = torch.exp2(torch.ceil(torch.log2(amax / FP8_MAX)))
        q = (Xf / scale).to(torch.float8_e4m3fn)
        return q.contiguous(), scale.to(torch.float32).contiguous()
    raise ValueError(f"unknown storage {storage!r}")


def _responses(Xf, beta, sigma, g, device, chunk=1 << 18):
    """Y = X beta + sigma * zeta in float64, row chunk by row chunk."""
    N = Xf.shape[0]
    k = beta.shape[1]
    Y = torch.empty(N, k, dtype=torch.float64, device=device)
    for i in range(0, N, chunk):
        xb = Xf[i:i + chunk].to(torch.float64)
        Y[i:i + chunk] = xb @ beta
    Y += sigma * torch.randn(N, k, generator=g, device=device, dtype=torch.float64)
    return Y


def gauss_colscale(N, d, cond, sigma, storage="f32", k=1, seed=BASE_SEED + 1,
                   device="cpu", leverage_frac=0.0, leverage_scale=100.0, name=None):
    """X = G diag(s), G Gaussian, s log-spaced 1..cond (the generator of
    Sec. 4 with D chosen for the condition number); optional high-leverage
    rows: a seeded random fraction of rows multiplied by ``leverage_scale``."""
    g = generator(device, seed)
    s = log_spaced(1.0, cond, d, device).to(torch.float32)
    X = torch.randn(N, d, generator=g, device=device, dtype=torch.float32)
    X.mul_(s.unsqueeze(0))
    if leverage_frac > 0:
        nlev = max(1, int(round(leverage_frac * N)))
        rows = torch.randperm(N, generator=g, device=device)[:nlev]
        X[rows] *= leverage_scale
    beta = torch.randn(d, k, generator=g, device=device, dtype=torch.float64)
    if storage in ("f64", torch.float64):
        X = X.to(torch.float64)
    Y = _responses(X, beta, sigma, g, device)
    Xs, sc = store(X, storage)
    return Problem(name or "gauss_colscale", Xs, Y, beta, sigma, sc,
                   {"cond": cond, "storage": str(storage), "seed": seed})


def haar_svd(N=20000, d=50, cond=1e3, sigma=0.1, k=1, seed=BASE_SEED + 0, device="cpu",
             storage="f64"):
    """X = U diag(s) V^T with Haar U (N x d), V (d x d), s log-spaced 1..cond."""
    g = generator(device, seed)
    U = haar_orthonormal(N, d, g, device)
    V = haar_orthonormal(d, d, g, device)
    s = log_spaced(1.0, cond, d, device)
    X = (U * s.unsqueeze(0)) @ V.T
    beta = torch.randn(d, k, generator=g, device=device, dtype=torch.float64)
    Y = _responses(X, beta, sigma, g, device)
    Xs, sc = store(X, storage)
    return Problem("haar_svd", Xs, Y, beta, sigma, sc, {"cond": cond, "seed": seed})


def t3_corr(N=4_000_000, d=1000, cond=1e5, sigma=0.5, storage="bf16", k=1,
            seed=BASE_SEED + 2, device="cpu", chunk=1 << 18):
    """X = T C with T i.i.d. Student-t (3 d.o.f.) rows and a correlation
    factor C = Q1 diag(s) Q2^T (Haar Q1, Q2; s log-spaced 1..cond)."""
    g = generator(device, seed)
    Q1 = haar_orthonormal(d, d, g, device)
    Q2 = haar_orthonormal(d, d, g, device)
    s = log_spaced(1.0, cond, d, device)
    C = ((Q1 * s.unsqueeze(0)) @ Q2.T).to(torch.float32)
    beta = torch.randn(d, k, generator=g, device=device, dtype=torch.float64)
    X32 = torch.empty(N, d, dtype=torch.float32, device=device)
    for i in range(0, N, chunk):
        n = min(chunk, N - i)
        z = torch.randn(n, d, generator=g, device=device, dtype=torch.float32)
        chi = torch.randn(n, d, 3, generator=g, device=device, dtype=torch.float32).pow_(2).sum(-1)
        T = z / torch.sqrt(chi / 3.0)
        X32[i:i + n] = T @ C
    Y = _responses(X32, beta, sigma, g, device)
    Xs, sc = store(X32, storage)
    del X32
    return Problem("t3_corr", Xs, Y, beta, sigma, sc, {"cond": cond, "storage": str(storage),
                                                       "seed": seed})


def paper_table1(N, kappa, d=64, sigma2=1e-8, seed=BASE_SEED + 10, device="cpu", storage="f64"):
    """Sec. 4 setting: X = G D, d = 64, noise variance 1e-8, FP64."""
    return gauss_colscale(N, d, kappa, math.sqrt(sigma2), storage=storage, seed=seed,
                          device=device, name="paper_table1")


def batched(n_prob=256, N_range=(50_000, 500_000), d_range=(32, 512), cond_range=(1e2, 1e5),
            k_range=(1, 16), seed=BASE_SEED + 3, device="cpu", storage="f32", sigma=1.0):
    """Independent problems of uneven N, d, condition and RHS count."""
    g = generator("cpu", seed)
    probs = []
    for i in range(n_prob):
        u = torch.rand(4, generator=g, dtype=torch.float64)
        N = int(N_range[0] + u[0].item() * (N_range[1] - N_range[0]))
        d = int(d_range[0] + u[1].item() * (d_range[1] - d_range[0]))
        lc = math.log(cond_range[0]) + u[2].item() * (math.log(cond_range[1]) - math.log(cond_range[0]))
        k = int(k_range[0] + math.floor(u[3].item() * (k_range[1] - k_range[0] + 1)))
        k = min(k, k_range[1])
        probs.append(gauss_colscale(N, d, math.exp(lc), sigma, storage=storage, k=k,
                                    seed=seed * 1000 + i, device=device, name=f"batched_{i}"))
    return probs


def schedule_training_problem(i, device="cpu", seed=BASE_SEED + 4, storage="f32"):
    """Problem ``i`` of the schedule network's training distribution:
    N log-uniform in [1e4, 2e6] (at least 32 d), d log-uniform in [16, 1024], condition
    log-uniform in [1e1, 1e6], noise sigma log-uniform in [1e-3, 1], rows
    Gaussian with column scales or Student-t (3 d.o.f.) times a correlation
    factor, with equal probability.  storage="mix" stores X as FP32, BF16 or
    FP8 e4m3 with probabilities 0.6, 0.2, 0.2."""
    g = generator("cpu", seed * 100003 + i)
    u = torch.rand(6, generator=g, dtype=torch.float64).tolist()
    if storage == "mix":
        storage = "f32" if u[5] < 0.6 else ("bf16" if u[5] < 0.8 else "fp8")
    d = int(round(2 ** (4 + 6 * u[1])))
    N = max(int(round(10 ** (4 + math.log10(200.0) * u[0]))), 32 * d)
    cond = 10 ** (1 + 5 * u[2])
    sigma = 10 ** (-3 + 3 * u[4])
    pseed = seed * 1000 + i
    if u[3] < 0.5:
        p = gauss_colscale(N, d, cond, sigma, storage=storage, seed=pseed, device=device,
                           name=f"train_{i}")
    else:
        p = t3_corr(N, d, cond, sigma, storage=storage, seed=pseed, device=device)
        p.name = f"train_{i}"
    p.meta.update({"rows": "gauss" if u[3] < 0.5 else "t3", "sigma": sigma, "index": i, "storage": storage})
    return p


CONFIGS = {
    0: dict(kind="haar_svd", N=20000, d=50, cond=1e3, sigma=0.1, storage="f64"),
    1: dict(kind="gauss_colscale", N=1_000_000, d=500, cond=1e4, sigma=1.0, storage="f32"),
    2: dict(kind="t3_corr", N=4_000_000, d=1000, cond=1e5, sigma=0.5, storage="bf16"),
    4: dict(kind="leverage", N=2_000_000, d=256, cond=1e4, sigma=1.0, storage="f32"),
}


def make_config(cfg, device="cpu", N=None, d=None, storage=None, k=1, seed=None):
    """Workload ``cfg`` (0, 1, 2 or 4) with optional size/storage overrides."""
    c = dict(CONFIGS[cfg])
    N = c["N"] if N is None else int(N)
    d = c["d"] if d is None else int(d)
    storage = c["storage"] if storage is None else storage
    seed = BASE_SEED + cfg if seed is None else seed
    if c["kind"] == "haar_svd":
        return haar_svd(N, d, c["cond"], c["sigma"], k=k, seed=seed, device=device, storage=storage)
    if c["kind"] == "gauss_colscale":
        return gauss_colscale(N, d, c["cond"], c["sigma"], storage=storage, k=k, seed=seed,
                              device=device, name=f"cfg{cfg}")
    if c["kind"] == "t3_corr":
        return t3_corr(N, d, c["cond"], c["sigma"], storage=storage, k=k, seed=seed, device=device)
    if c["kind"] == "leverage":
        return gauss_colscale(N, d, c["cond"], c["sigma"], storage=storage, k=k, seed=seed,
                              device=device, leverage_frac=0.01, leverage_scale=100.0,
                              name="leverage")
    raise ValueError(cfg)
