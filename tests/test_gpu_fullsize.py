"""The headline workload at full size (N = 4e6, d = 1000, X = T C with
Student-t(3) rows and a correlation factor of condition 1e5, sigma = 0.5)
against the oracle, in the launch configuration the benchmark times.

For each storage type (FP32, which is the unquantized data; BF16; FP8-e4m3
with per-column power-of-two scales) one streamed pass over the stored
values, upcast exactly to FP64, feeds
* the oracle's TSQR of [X | Y] (eq. (ols) by Householder QR of row blocks),
  so that rel = ||X (beta - beta_hat)|| / ||X beta_hat|| = ||R (beta -
  beta_hat)|| / ||R beta_hat|| with the oracle's R; the bar is 1e-6;
* 32 sampled rows of the last stage sketch S_K X and 32 rows of S_hat X,
  each the oracle's row of H_un D P X (Sec. 2.1, Sec. 2.2) summed over all
  4e6 rows.
The error of every reduced-precision solve against the OLS estimator of the
unquantized data is computed from the unquantized TSQR and printed: it is
stated, not bounded (it measures the quantization, not the solver).
"""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle.ols import ols_from_r, tsqr_r
from oracle.sketch import SrhtRowAccumulator, hat_slot_rows, padded_bits, slot_rows

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1500)]

DEV = "cuda:0"
BLOCK = 1 << 16
WORKERS = 16


@pytest.fixture(scope="module")
def S():
    import paper_2607_25272_amd as spcg_mod
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    return spcg_mod


@pytest.fixture(scope="module")
def ctx(S):
    c = S.Context(0)
    yield c
    c.close()


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def data():
    _log("full size cfg2: generate (FP32 = unquantized)")
    p = workloads.make_config(2, device=DEV, storage="f32")
    torch.cuda.synchronize()
    return {"p": p, "cache": {}}


def _stored(data, storage):
    p = data["p"]
    if storage == "f32":
        return p.X, None
    if storage not in data["cache"]:
        data["cache"][storage] = workloads.store(p.X, storage)
    return data["cache"][storage]


def _oracle_pass(Xs, scale, Y, rows, seed, L):
    """One streamed pass over the stored rows: the TSQR R factor of [X | Y],
    the sampled rows of H_un D P X, and the per-column max |X|."""
    N, d = Xs.shape
    acc = SrhtRowAccumulator(rows, seed, L)
    amax = np.zeros(d)
    Yh = Y.cpu().numpy()
    sc = None if scale is None else scale.cpu().to(torch.float64)

    def blocks():
        for n0 in range(0, N, BLOCK):
            xb = Xs[n0:n0 + BLOCK].cpu().to(torch.float64)
            if sc is not None:
                xb = xb * sc
            xb = xb.numpy()
            acc.add(n0, xb)
            np.maximum(amax, np.abs(xb).max(axis=0), out=amax)
            if (n0 // BLOCK) % 8 == 0:
                _log(f"  oracle pass: rows {n0} of {N}")
            yield np.concatenate([xb, Yh[n0:n0 + BLOCK]], axis=1)

    R = tsqr_r(blocks(), workers=WORKERS)
    return R, acc.value, amax


def _run(S, ctx, data, storage):
    p = data["p"]
    Xs, scale = _stored(data, storage)
    N, d = Xs.shape
    L, Np = padded_bits(N)
    _log(f"full size cfg2 {storage}: solve")
    beta, st = S.spcg_solve(ctx, Xs, p.Y, col_scale=scale, seed=1)
    torch.cuda.synchronize()
    assert st["converged"] and st["K"] == 10
    _log(f"full size cfg2 {storage}: K={st['K']} T1={st['T_stage1']} T2={st['T_stage2']}")
    _log(f"full size cfg2 {storage}: sketch rows")
    sk = S.spcg_sketch(ctx, Xs, p.Y, seed=1, col_scale=scale)
    mK, r = sk.sizes[-1], sk.info.r
    rng = np.random.default_rng(2)
    t = np.sort(rng.choice(mK, 32, replace=False))
    th = np.sort(rng.choice(r, 32, replace=False))
    A_last, _, _ = sk.view_tensor(len(sk.sizes) - 1)
    got = A_last[torch.from_numpy(t).to(DEV)].double().cpu().numpy()
    del A_last
    Bh, _, _ = sk.view_tensor(-1)
    got_h = Bh[torch.from_numpy(th).to(DEV)].double().cpu().numpy()
    sk_dtype = sk.info.sketch_dtype
    sk.free()
    torch.cuda.empty_cache()
    rows = np.concatenate([slot_rows(1, L, mK)[t], hat_slot_rows(1, L, r)[th]])
    _log(f"full size cfg2 {storage}: oracle TSQR + sampled rows ({WORKERS} threads)")
    R, Z, amax = _oracle_pass(Xs, scale, p.Y, rows, 1, L)
    # sampled sketch rows: the transform runs in FP32 (relative rounding per
    # butterfly stage, L stages, values up to sqrt(N') max|X_j| in a column);
    # BF16 stage rows add one rounding of at most 2^-8 of the value
    tol_t = 2e-6 * L * math.sqrt(Np) * amax
    bf16_rows = sk_dtype == S.SPCG_BF16
    err = np.abs(got - Z[:32])
    bound = tol_t + (2.0 ** -8 * np.abs(Z[:32]) if bf16_rows else 0.0)
    assert np.all(err <= bound), float(np.max(err / bound))
    assert np.all(np.abs(got_h - Z[32:]) <= tol_t), float(np.max(np.abs(got_h - Z[32:]) / tol_t))
    # the solve against the OLS estimator of the stored data
    bh = ols_from_r(R, d, multi=False)
    Rd = R[:d, :d]
    b = beta.cpu().numpy()
    rel = np.linalg.norm(Rd @ (b - bh)) / np.linalg.norm(Rd @ bh)
    _log(f"full size cfg2 {storage}: rel vs OLS of the stored data = {rel:.3e}")
    assert rel <= 1e-6
    return b, R


def _unquantized(S, ctx, data):
    if "ref" not in data:
        b, R = _run(S, ctx, data, "f32")
        d = data["p"].d
        data["ref"] = (ols_from_r(R, d, multi=False), R[:d, :d])
    return data["ref"]


def test_full_size_config2_fp32_against_ols(S, ctx, data):
    _unquantized(S, ctx, data)


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
def test_full_size_config2_reduced_precision_against_ols(S, ctx, data, storage):
    bh64, R64 = _unquantized(S, ctx, data)
    b, _ = _run(S, ctx, data, storage)
    q = np.linalg.norm(R64 @ (b - bh64)) / np.linalg.norm(R64 @ bh64)
    _log(f"full size cfg2 {storage}: rel vs OLS of the unquantized FP64 data = {q:.3e} (stated)")
    assert np.isfinite(q)
