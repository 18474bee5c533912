"""Parity of the one-pass PCG products for every storage type and load width.

The products (s = c2 A^T A p; g = c2 A^T (b - A x) with ||b - A x||^2; both
fused in one pass when the gradient is refreshed) are checked through PCG
steps with the identity preconditioner, where the oracle's FP64 PCG
(Sec. 2.2 PCG) on the same stored values gives the expected iterate:
from x = 0, g0 = c2 A^T b = p0, s = c2 A^T A p0, alpha = g0.g0 / p0.s,
x1 = alpha p0, and so on.  The shapes cover the register kernel (rows of at
most 32 load vectors) and the LDS-staged kernel with 16- and 4-byte loads
and 1, 2 or 4 vectors per lane, ragged row counts (not a multiple of the
8-row tile or of the 256 blocks) and padded leading dimensions.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle.pcg import pcg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (storage, m, d, lda): comments name the kernel path the shape selects
CASES = [
    ("f64", 3001, 30, 30),       # register kernel
    ("f64", 5003, 100, 100),     # staged, 16-byte loads, 1 vector per lane
    ("f64", 4099, 250, 256),     # staged, 16-byte loads, 2 vectors per lane, padded ld
    ("f32", 9001, 132, 132),     # staged, 16-byte, 1 vector
    ("f32", 9001, 129, 129),     # staged, 16-byte loads of rows only 4-byte aligned (last row shifted)
    ("f32", 20011, 500, 500),    # staged, 16-byte, 2 vectors
    ("f32", 7013, 1000, 1024),   # staged, 16-byte, 4 vectors, padded ld
    ("f32", 5000, 250, 251),     # staged, 4-byte loads, odd ld
    ("bf16", 3001, 200, 200),    # register kernel
    ("bf16", 12007, 1000, 1000), # staged, 16-byte, 2 vectors
    ("bf16", 6001, 300, 302),    # staged, 4-byte loads, padded ld
    ("fp8", 4003, 1024, 1024),   # staged, 16-byte, 1 vector of 16
    ("fp8", 8009, 1000, 1000),   # staged, 16-byte loads of rows only 4-byte aligned (last row shifted)
    ("fp8", 1001, 1000, 1000),   # the same with one row per block-tile tail (last block of 9 rows)
    ("fp8", 3001, 700, 704),     # staged, 4-byte loads (16-byte vectors would pass d)
    ("fp8", 2003, 64, 64),       # register kernel
]


@pytest.fixture(scope="module")
def S():
    import paper_2607_25272_amd as spcg_mod
    return spcg_mod


@pytest.fixture(scope="module")
def ctx(S):
    c = S.Context(0)
    yield c
    c.close()


def _stored(storage, m, d, lda, seed):
    """A (m x d view with leading dimension lda, stored type), its exact FP64
    values, b and the FP8 column scales."""
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    full = torch.randn(m, lda, generator=g, device=DEV, dtype=torch.float64)
    full *= torch.logspace(0, 2, lda, device=DEV, dtype=torch.float64)
    Xs, sc = workloads.store(full, storage)
    A = Xs[:, :d]
    Ad = Xs.to(torch.float64)
    if sc is not None:
        Ad = Ad * sc.to(torch.float64)
        sc = sc[:d].contiguous()
    Ad = Ad[:, :d].cpu().numpy()
    b = torch.randn(m, 1, generator=g, device=DEV, dtype=torch.float64)
    return A, Ad, b, sc


@pytest.mark.parametrize("refresh", [False, True])
@pytest.mark.parametrize("storage,m,d,lda", CASES)
def test_products_through_pcg_steps(S, ctx, storage, m, d, lda, refresh):
    print(f"products {storage} m={m} d={d} lda={lda} refresh={refresh}", flush=True)
    A, Ad, b, sc = _stored(storage, m, d, lda, seed=m + d + lda)
    assert A.stride(0) == lda and A.shape == (m, d)
    c2 = 1.0 / m
    pc = S.spcg_precond_from_r(ctx, torch.eye(d, dtype=torch.float64))
    bh = b.cpu().numpy()[:, 0]
    g0 = c2 * (Ad.T @ bh)
    for iters in (1, 3):
        beta = torch.zeros(d, dtype=torch.float64, device=DEV)
        st = S.spcg_pcg_stage(ctx, A, b, c2, pc, beta, iters, refresh=refresh, col_scale=sc)
        x_ref, _ = pcg(Ad, bh, c2, np.eye(d), np.zeros(d), iters)
        x = beta.cpu().numpy()
        # stage start (G pass): g0^T g0 and c2 ||b||^2 accumulate in FP64
        assert abs(st["rho0"] - g0 @ g0) <= 1e-10 * (g0 @ g0)
        assert abs(st["resid_norm2"] - c2 * (bh @ bh)) <= 1e-10 * c2 * (bh @ bh)
        tol = 1e-11 if storage == "f64" else 2e-5 * iters
        err = np.linalg.norm(Ad @ (x - x_ref)) / np.linalg.norm(Ad @ x_ref)
        assert err <= tol, (iters, err)
    pc.free()


def test_products_repeat_bit_for_bit(S, ctx):
    # fixed reduction order: the same stage twice gives identical bits
    A, Ad, b, sc = _stored("bf16", 12007, 1000, 1000, seed=3)
    pc = S.spcg_precond_from_r(ctx, torch.eye(1000, dtype=torch.float64))
    out = []
    for _ in range(2):
        beta = torch.zeros(1000, dtype=torch.float64, device=DEV)
        S.spcg_pcg_stage(ctx, A, b, 1.0 / 12007, pc, beta, 3, refresh=True)
        out.append(beta.clone())
    assert torch.equal(out[0], out[1])
    pc.free()
