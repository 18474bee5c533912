"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Sketch randomness and FP64 sketch rows are compared bit for bit; FP32
sketch rows, the QR factor, PCG stages and whole solves within stated
tolerances; whole solves must reach the OLS estimator of the stored data to
a relative prediction error of 1e-6 (Sec. 1 eq. (ols); Algorithm 1).
"""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle.linalg import householder_qr
from oracle.ols import ols_householder, ols_tsqr
from oracle.pcg import pcg
from oracle.sketch import (hat_slot_rows, input_perm, nested_srht, padded_bits, sign_vector,
                           slot_rows)
from oracle.spcg import precond_from_sketch, rel_pred_error, schedule, spcg

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


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


def _problem(N, d, cond=1e3, sigma=0.1, storage="f64", seed=5, k=1):
    p = workloads.gauss_colscale(N, d, cond, sigma, storage=storage, k=k, seed=seed, device=DEV)
    return p


# ------------------------------------------------------------ randomness

@pytest.mark.parametrize("N,d,seed", [(20000, 50, 1), (3000, 10, 77)])
def test_device_randomness_bit_exact(S, ctx, N, d, seed):
    _log(f"randomness N={N} d={d} seed={seed}")
    p = _problem(N, d, seed=seed)
    sk = S.spcg_sketch(ctx, p.X, p.Y, seed=seed)
    ex = sk.export()
    L = sk.info.L
    mK = sk.sizes[-1]
    assert np.array_equal(ex["slot_rows"], slot_rows(seed, L, mK))
    assert np.array_equal(ex["hat_rows"], hat_slot_rows(seed, L, sk.info.r))
    assert np.array_equal(ex["input_perm"], input_perm(seed, L))
    bits = np.unpackbits(ex["sign_bits"], bitorder="little")[: 1 << L]
    assert np.array_equal(1.0 - 2.0 * bits, sign_vector(seed, L))


def test_device_randomness_large_sampled(S, ctx):
    # N' = 2^22 (the 4e6-row workload): every exported slot and sign is
    # compared at 20000 sampled positions
    N, d, seed = 4_000_000, 4, 3
    _log("randomness N'=2^22 sampled")
    X = torch.zeros(N, d, dtype=torch.float32, device=DEV)
    X[:, 0] = 1.0
    Y = torch.zeros(N, 1, dtype=torch.float64, device=DEV)
    sk = S.spcg_sketch(ctx, X, Y, seed=seed, m0=1 << 20)
    ex = sk.export()
    L = sk.info.L
    assert L == 22
    rng = np.random.default_rng(0)
    t = rng.integers(0, sk.sizes[-1], 20000)
    from oracle.feistel import feistel_forward
    from oracle.sketch import STREAM_P, STREAM_PI
    assert np.array_equal(ex["slot_rows"][t], feistel_forward(t.astype(np.uint64), L, seed, STREAM_PI).astype(np.int64))
    k = rng.integers(0, 1 << L, 20000)
    assert np.array_equal(ex["input_perm"][k], feistel_forward(k.astype(np.uint64), L, seed, STREAM_P).astype(np.int64))
    bits = np.unpackbits(ex["sign_bits"], bitorder="little")
    assert np.array_equal(1.0 - 2.0 * bits[k], sign_vector(seed, L, k))


# ---------------------------------------------------------------- sketch

@pytest.mark.parametrize("N,d", [(20000, 50), (2500, 7), (4096, 64), (70000, 24)])
def test_sketch_rows_f64_bit_exact(S, ctx, N, d):
    # FP64 path: same butterflies in the same stage order -> identical bits
    _log(f"sketch f64 N={N} d={d}")
    p = _problem(N, d, seed=N + d)
    sk = S.spcg_sketch(ctx, p.X, p.Y, seed=11)
    B, BY, Bh, _ = nested_srht(p.x_f64().cpu().numpy(), p.Y.cpu().numpy(), 11, sk.sizes[-1], sk.info.r)
    Ag, bg, _ = sk.view_tensor(len(sk.sizes) - 1)
    Hg, _, _ = sk.view_tensor(-1)
    assert np.array_equal(Ag.cpu().numpy(), B)
    assert np.array_equal(bg.cpu().numpy(), BY)
    assert np.array_equal(Hg.cpu().numpy(), Bh)
    # prefix views: stage i = first m_i rows
    A0, b0, c2 = sk.view_tensor(0)
    assert A0.shape[0] == sk.sizes[0] and c2 == 1.0 / sk.sizes[0]
    assert np.array_equal(A0.cpu().numpy(), B[: sk.sizes[0]])


def test_sketch_rows_f64_eleven_bit_passes(S, ctx):
    # N' = 2^22: two 11-bit passes with 128-byte row segments; still bit-exact
    N, d = (1 << 21) + 5, 3
    _log("sketch f64 N'=2^22")
    p = _problem(N, d, seed=99)
    sk = S.spcg_sketch(ctx, p.X, p.Y, seed=7, m0=1 << 16, m_max=1 << 17, r=64)
    B, BY, Bh, _ = nested_srht(p.x_f64().cpu().numpy(), p.Y.cpu().numpy(), 7, sk.sizes[-1], 64)
    Ag, bg, _ = sk.view_tensor(len(sk.sizes) - 1)
    Hg, _, _ = sk.view_tensor(-1)
    assert sk.info.L == 22
    assert np.array_equal(Ag.cpu().numpy(), B)
    assert np.array_equal(bg.cpu().numpy(), BY)
    assert np.array_equal(Hg.cpu().numpy(), Bh)


@pytest.mark.parametrize("N,k", [(150_001, 3), (150_001, 8), (70_000, 9), (70_000, 16), (40_000, 17),
                                 ((1 << 21) + 5, 5)])
def test_sketch_multi_rhs_rows_match_oracle(S, ctx, N, k):
    # FP64 responses of 2..8, 9..16 and more columns are transformed in rows
    # of 8, 16 and 32-multiple columns (two passes: 9 + 9, 9 + 8, 8 + 8 and
    # 11 + 11 bits): same butterflies in the same order -> identical bits
    _log(f"sketch multi-rhs N={N} k={k}")
    p = _problem(N, 5, seed=N % 97 + k, k=k)
    big = dict(m0=1 << 12, m_max=1 << 13, r=64) if N > (1 << 20) else {}
    sk = S.spcg_sketch(ctx, p.X, p.Y, seed=12, **big)
    B, BY, Bh, _ = nested_srht(p.x_f64().cpu().numpy(), p.Y.cpu().numpy(), 12, sk.sizes[-1], sk.info.r)
    _, bg, _ = sk.view_tensor(len(sk.sizes) - 1)
    assert bg.shape == (sk.sizes[-1], k)
    assert np.array_equal(bg.cpu().numpy(), BY)


def test_sketch_tiny_and_multi_rhs(S, ctx):
    # N' = 8 (one 3-bit pass) and a three-column response
    X = torch.arange(10, dtype=torch.float64, device=DEV).reshape(5, 2) - 3.0
    Y = torch.arange(15, dtype=torch.float64, device=DEV).reshape(5, 3) * 0.5
    sk = S.spcg_sketch(ctx, X, Y, seed=2, m0=3, r=4)
    B, BY, Bh, _ = nested_srht(X.cpu().numpy(), Y.cpu().numpy(), 2, sk.sizes[-1], 4)
    Ag, bg, _ = sk.view_tensor(len(sk.sizes) - 1)
    Hg, _, _ = sk.view_tensor(-1)
    assert sk.info.L == 3
    assert np.array_equal(Ag.cpu().numpy(), B)
    assert np.array_equal(bg.cpu().numpy(), BY)
    assert np.array_equal(Hg.cpu().numpy(), Bh)


@pytest.mark.parametrize("storage,N,d,stage_dtype", [("f32", 9000, 37, 0), ("bf16", 6000, 40, 0),
                                                     ("fp8", 5000, 48, 0), ("bf16", 6000, 40, 1),
                                                     ("f32", 7000, 40, 2)])
def test_sketch_rows_reduced_precision(S, ctx, storage, N, d, stage_dtype):
    # FP32 transform of exactly-widened stored values vs the FP64 oracle on
    # the same stored values; error bounded by L * u32 * row-norm scale, plus
    # the 2^-9 relative rounding of BF16 stage rows (the default for BF16 and
    # FP8 input; stage_dtype 1 forces FP32 rows, 2 forces BF16)
    _log(f"sketch {storage} N={N} d={d} stage_dtype={stage_dtype}")
    tol = 2e-6
    p = _problem(N, d, storage=storage, seed=3)
    sk = S.spcg_sketch(ctx, p.X, p.Y, seed=5, col_scale=p.col_scale, stage_dtype=stage_dtype)
    bf16_rows = stage_dtype == S.SPCG_BF16 or (stage_dtype == 0 and storage != "f32")
    assert sk.info.sketch_dtype == (S.SPCG_BF16 if bf16_rows else S.SPCG_F32)
    Xd = p.x_f64().cpu().numpy()
    B, BY, Bh, info = nested_srht(Xd, p.Y.cpu().numpy(), 5, sk.sizes[-1], sk.info.r)
    Ag, bg, _ = sk.view_tensor(len(sk.sizes) - 1)
    Hg, _, _ = sk.view_tensor(-1)
    assert Ag.dtype == (torch.bfloat16 if bf16_rows else torch.float32) and Hg.dtype == torch.float32
    scale = np.sqrt(info["Np"]) * np.abs(Xd).max(axis=0)   # |Z| <= sqrt(N') * column max
    Af = Ag.float().cpu().numpy().astype(np.float64)
    err = np.abs(Af - B) / scale
    assert err.max() < tol * info["L"] + (2.0 ** -8 if bf16_rows else 0.0)
    if bf16_rows:
        # rounding is to nearest: within half a BF16 ulp of the exact row plus the transform error
        rel = np.abs(Af - B) / np.maximum(np.abs(B), 1e-300)
        big = np.abs(B) > 0.05 * scale
        assert rel[big].max() < 2.0 ** -8 + 1e-3
    errh = np.abs(Hg.cpu().numpy().astype(np.float64) - Bh) / scale
    assert errh.max() < tol * info["L"]
    assert np.array_equal(bg.cpu().numpy(), BY)   # Y is always FP64


def _raw_rows(sk, stage):
    A, _, _ = sk.view_tensor(stage)
    A = A.contiguous()
    return A.view(torch.int16 if A.dtype == torch.bfloat16 else torch.int32).cpu().numpy()


@pytest.mark.parametrize("storage,N,d", [("f32", 600_001, 40), ("f32", 600_001, 37),
                                         ("bf16", 700_000, 24), ("fp8", 700_000, 48),
                                         ("bf16", 700_000, 26), ("fp8", 700_000, 44),
                                         ("f32", 1_100_000, 12)])
def test_sketch_streaming_transform_matches_tiled(S, ctx, storage, N, d):
    # N' = 2^20 (two 10-bit passes): the default transform streams tiles
    # through LDS in persistent blocks; transform_segment = 256 forces one
    # tile per block.  Same butterflies in the same order -> identical bits
    # (d = 37, 26 (BF16), 44 (FP8): rows of X only 4-byte aligned, staged
    # with 16-byte loads that may reach into the next row and row N - 1 from
    # its padded copy, Z row-major;
    # N' = 2^21: an 11-bit first pass, half-tile staged by default, with
    # chunk-major Z in both runs)
    _log(f"sketch streaming {storage} N={N} d={d}")
    p = _problem(N, d, storage=storage, seed=N % 89)
    rows = []
    for seg in (0, 256):
        sk = S.spcg_sketch(ctx, p.X, p.Y, seed=5, col_scale=p.col_scale, transform_segment=seg)
        rows.append((_raw_rows(sk, len(sk.sizes) - 1), _raw_rows(sk, -1), sk.info.L))
    assert rows[0][2] == (20 if N < (1 << 20) else 21)
    assert np.array_equal(rows[0][0], rows[1][0])
    assert np.array_equal(rows[0][1], rows[1][1])


@pytest.mark.parametrize("storage,N,d,L", [("f32", 200_001, 40, 18), ("f32", 300_001, 37, 19),
                                           ("bf16", 150_000, 24, 18), ("fp8", 250_001, 48, 18),
                                           ("f32", 200_001, 37, 18), ("bf16", 150_000, 26, 18),
                                           ("fp8", 250_001, 44, 18), ("f32", 100_001, 70, 17)])
def test_sketch_streaming_nine_bit_passes_match_tiled(S, ctx, storage, N, d, L):
    # 9-bit passes stream 512-row x 256-byte tiles: N' = 2^18 (9 + 9 bits,
    # chunk-major Z), 2^19 (10 + 9: two tile widths, Z row-major) and 2^17
    # (9 + 8: the 8-bit pass stays tiled); d = 37, 26 (BF16), 44 (FP8): rows
    # of X only 4-byte aligned (16-byte loads, row N - 1 from its padded
    # copy).  Same butterflies in the same order -> identical bits to one
    # tile per block.
    _log(f"sketch streaming 9-bit {storage} N={N} d={d}")
    p = _problem(N, d, storage=storage, seed=N % 83)
    rows = []
    for seg in (0, 256):
        sk = S.spcg_sketch(ctx, p.X, p.Y, seed=6, col_scale=p.col_scale, transform_segment=seg)
        rows.append((_raw_rows(sk, len(sk.sizes) - 1), _raw_rows(sk, -1), sk.info.L))
    assert rows[0][2] == L
    assert np.array_equal(rows[0][0], rows[1][0])
    assert np.array_equal(rows[0][1], rows[1][1])


@pytest.mark.parametrize("storage,N,d", [("f32", 2_200_001, 40), ("f32", 2_500_000, 37),
                                         ("bf16", 2_300_000, 24), ("fp8", 2_150_000, 48),
                                         ("fp8", 2_150_000, 44), ("fp8", 1_500_000, 44),
                                         ("bf16", 1_200_000, 64)])
def test_sketch_split_eleven_bit_passes_match_tiled(S, ctx, storage, N, d):
    # 11-bit passes stage half-tiles of 2048 rows x 128 bytes: N' = 2^22
    # (11 + 11 bits, both passes) and N' = 2^21 (the 11-bit first pass, then
    # a streamed 10-bit pass).  Rows of X only 4-byte aligned (d = 37 FP32,
    # FP8 rows of 44 bytes) are staged with 16-byte loads that may reach
    # into the next row, row N - 1 from its padded copy.
    # transform_segment = 256 runs one tile per block, -64
    # half-tile staging (the default and -32: the quarter-tile ring).  Same
    # butterflies in the same order -> identical bits.
    _log(f"sketch split 11-bit {storage} N={N} d={d}")
    p = _problem(N, d, storage=storage, seed=N % 79)
    rows = []
    for seg in (0, 256, -32, -64):
        sk = S.spcg_sketch(ctx, p.X, p.Y, seed=7, col_scale=p.col_scale, transform_segment=seg)
        rows.append((_raw_rows(sk, len(sk.sizes) - 1), _raw_rows(sk, -1), sk.info.L))
        del sk
    assert rows[0][2] == (N - 1).bit_length()
    for r in rows[1:]:
        assert np.array_equal(rows[0][0], r[0])
        assert np.array_equal(rows[0][1], r[1])


def test_sketch_streaming_transform_against_oracle(S, ctx):
    # the streaming path at N' = 2^20 against the FP64 oracle on the same
    # stored values (tolerance as for the tiled FP32 transform)
    N, d = 600_001, 16
    _log("sketch streaming vs oracle N'=2^20")
    p = _problem(N, d, storage="f32", seed=21)
    sk = S.spcg_sketch(ctx, p.X, p.Y, seed=9, m0=1 << 14, m_max=1 << 16, r=256)
    Xd = p.x_f64().cpu().numpy()
    B, BY, Bh, info = nested_srht(Xd, p.Y.cpu().numpy(), 9, sk.sizes[-1], 256)
    assert info["L"] == 20
    Ag, bg, _ = sk.view_tensor(len(sk.sizes) - 1)
    Hg, _, _ = sk.view_tensor(-1)
    scale = np.sqrt(info["Np"]) * np.abs(Xd).max(axis=0)
    assert (np.abs(Ag.cpu().numpy().astype(np.float64) - B) / scale).max() < 2e-6 * info["L"]
    assert (np.abs(Hg.cpu().numpy().astype(np.float64) - Bh) / scale).max() < 2e-6 * info["L"]
    assert np.array_equal(bg.cpu().numpy(), BY)


# ------------------------------------------------------- preconditioner

@pytest.mark.parametrize("passes", [0, 1, 2, 3])
def test_precond_qr_matches_householder(S, ctx, passes):
    N, d, cond = 30000, 60, 1e4
    _log(f"precond passes={passes}")
    p = _problem(N, d, cond=cond, seed=8)
    sk = S.spcg_sketch(ctx, p.X, p.Y, seed=2)
    _, _, Bh, _ = nested_srht(p.x_f64().cpu().numpy(), p.Y.cpu().numpy(), 2, sk.sizes[-1], sk.info.r)
    R_or = precond_from_sketch(Bh)
    pc = S.spcg_precond_build(ctx, sk, qr_passes=passes)
    R, used = pc.export()
    assert used == (1 if passes in (0, 1) else passes)
    assert np.all(np.diag(R) > 0) and np.allclose(np.tril(R, -1), 0)
    kappa = np.linalg.cond(R_or)
    u = 2.0 ** -53
    bound = 50 * d * (kappa ** 2 if used == 1 else kappa) * u
    rel = np.linalg.norm(R - R_or) / np.linalg.norm(R_or)
    assert rel < bound, (rel, bound)


@pytest.mark.parametrize("d", [64, 65, 130, 200])
def test_precond_blocked_cholesky_panels(S, ctx, d):
    # one fused launch per 64-row panel: d = 64 (the first block only), 65
    # (one step, 1-wide trailing tile), 130 and 200 (several steps, partial
    # last tiles) against Householder R of the same sketch rows
    N, cond = 30000, 1e3
    _log(f"precond blocked Cholesky d={d}")
    p = _problem(N, d, cond=cond, seed=d)
    sk = S.spcg_sketch(ctx, p.X, p.Y, seed=3)
    _, _, Bh, _ = nested_srht(p.x_f64().cpu().numpy(), p.Y.cpu().numpy(), 3, sk.sizes[-1], sk.info.r)
    R_or = precond_from_sketch(Bh)
    pc = S.spcg_precond_build(ctx, sk, qr_passes=1)
    R, used = pc.export()
    assert used == 1
    assert np.all(np.diag(R) > 0) and np.array_equal(np.tril(R, -1), np.zeros_like(R))
    kappa = np.linalg.cond(R_or)
    bound = 50 * d * kappa ** 2 * 2.0 ** -53
    rel = np.linalg.norm(R - R_or) / np.linalg.norm(R_or)
    assert rel < bound, (rel, bound)


def test_precond_ill_conditioned_falls_back_to_three_passes(S, ctx):
    N, d = 1 << 14, 16
    _log("precond kappa=1e8")
    p = _problem(N, d, cond=1e8, storage="f64", seed=9)
    sk = S.spcg_sketch(ctx, p.X, p.Y, seed=4)
    pc = S.spcg_precond_build(ctx, sk, qr_passes=0)
    R, used = pc.export()
    assert used == 3
    _, _, Bh, _ = nested_srht(p.x_f64().cpu().numpy(), p.Y.cpu().numpy(), 4, sk.sizes[-1], sk.info.r)
    R_or = precond_from_sketch(Bh)
    # the factor is accurate column-relative (it preconditions to kappa ~ 1)
    Mi = np.linalg.solve(R.T, (Bh / np.sqrt(sk.info.r)).T).T
    sv = np.linalg.svd(Mi, compute_uv=False)
    assert sv.max() / sv.min() < 1.01
    assert np.linalg.norm(R - R_or) / np.linalg.norm(R_or) < 1e-6


def test_precond_rank_deficient_is_reported(S, ctx):
    p = _problem(5000, 12, seed=10, storage="f64")
    X = p.X.clone()
    X[:, 5] = X[:, 3]
    sk = S.spcg_sketch(ctx, X, p.Y, seed=1)
    with pytest.raises(S.SpcgError) as e:
        S.spcg_precond_build(ctx, sk, qr_passes=3)
    assert e.value.code == S.SPCG_E_RANK



def test_solve_after_failed_solve_on_same_context(S, ctx):
    # A solve that fails in the preconditioner leaves the response transform
    # of its sketch (run beside the preconditioner on the side stream) in
    # flight.  The next solve on the context (a larger problem, so the
    # transform scratch grows) waits for it first and gives the same bits as
    # the same solve on a fresh context.
    _log("solve after a failed solve")
    bad = _problem(50_000, 12, seed=10, storage="f64")
    Xb = bad.X.clone()
    Xb[:, 5] = Xb[:, 3]
    with pytest.raises(S.SpcgError) as e:
        S.spcg_solve(ctx, Xb, bad.Y, seed=2, qr_passes=3)
    assert e.value.code == S.SPCG_E_RANK
    good = _problem(300_000, 40, cond=1e3, sigma=1.0, storage="f32", seed=11)
    b1, st1 = S.spcg_solve(ctx, good.X, good.Y, seed=2)
    c2 = S.Context(0)
    try:
        b2, _ = S.spcg_solve(c2, good.X, good.Y, seed=2)
    finally:
        c2.close()
    assert st1["converged"]
    assert torch.equal(b1, b2)
    Xd = good.x_f64().cpu().numpy()
    bh = ols_tsqr(Xd, good.Y.cpu().numpy()[:, 0])
    assert rel_pred_error(Xd, b1.cpu().numpy(), bh) <= 1e-6

# ------------------------------------------------------------ PCG stage

@pytest.mark.parametrize("storage,rtol", [("f64", 1e-9), ("f32", 2e-3)])
def test_pcg_stage_matches_oracle(S, ctx, storage, rtol):
    # isolate the stage: the oracle's sketch rows and R are fed to both sides
    N, d, a = 20000, 50, 3
    _log(f"stage {storage}")
    p = workloads.make_config(0, device=DEV, storage=storage)
    Xd = p.x_f64().cpu().numpy()
    Yd = p.Y.cpu().numpy()[:, 0]
    sizes = schedule(N, d)
    B, BY, Bh, _ = nested_srht(Xd, Yd, 1, sizes[-1], 6 * d)
    R = precond_from_sketch(Bh)
    pc = S.spcg_precond_from_r(ctx, torch.from_numpy(R))
    x_or = np.zeros(d)
    beta = torch.zeros(d, dtype=torch.float64, device=DEV)
    tdt = torch.float64 if storage == "f64" else torch.float32
    for i, m in enumerate(sizes):
        A = torch.from_numpy(B[:m]).to(DEV, tdt)
        b = torch.from_numpy(BY[:m]).to(DEV).unsqueeze(1)
        x_or, _ = pcg(A.double().cpu().numpy(), BY[:m], 1.0 / m, R, x_or, a)
        st = S.spcg_pcg_stage(ctx, A, b, 1.0 / m, pc, beta, a)
        assert st["iters"] == a
        xg = beta.cpu().numpy()
        err = np.linalg.norm(Xd @ (xg - x_or)) / np.linalg.norm(Xd @ x_or)
        assert err < rtol, (i, err)
    # Stage II with the stopping test on the full data
    st = S.spcg_pcg_stage(ctx, p.X, p.Y, 1.0, pc, beta, 80, tol=5e-7)
    assert st["converged"]
    bh = ols_householder(Xd, Yd)
    assert rel_pred_error(Xd, beta.cpu().numpy(), bh) < 1e-6


@pytest.mark.parametrize("d", [20, 64, 65, 130, 200, 321, 450])
def test_pcg_stage_exact_preconditioner_one_step(S, ctx, d):
    # M = R^{-1} R^{-T} from the exact R: one PCG step reaches the OLS
    # solution.  d = 65, 130, 200 exercise partial 64-column blocks in the
    # recursive-doubling inverse (two and three levels); the pairs of a
    # level share one batched launch, whose last pair is narrower at
    # d = 200 (8 columns at s = 64), 321 (1 column) and 450 (2 and 66
    # columns at s = 64 and 128)
    N = 5000
    _log(f"exact preconditioner d={d}")
    p = _problem(N, d, seed=12)
    Xd = p.x_f64().cpu().numpy()
    R = householder_qr(Xd)
    pc = S.spcg_precond_from_r(ctx, torch.from_numpy(R))
    beta = torch.zeros(d, dtype=torch.float64, device=DEV)
    S.spcg_pcg_stage(ctx, p.X, p.Y, 1.0, pc, beta, 1)
    bh = ols_householder(Xd, p.Y.cpu().numpy()[:, 0])
    assert rel_pred_error(Xd, beta.cpu().numpy(), bh) < 1e-12


def test_pcg_stage_zero_rhs_and_breakdown(S, ctx):
    N, d = 3000, 8
    p = _problem(N, d, seed=13)
    R = householder_qr(p.x_f64().cpu().numpy())
    pc = S.spcg_precond_from_r(ctx, torch.from_numpy(R))
    beta = torch.zeros(d, dtype=torch.float64, device=DEV)
    st = S.spcg_pcg_stage(ctx, p.X, torch.zeros_like(p.Y), 1.0, pc, beta, 5, tol=1e-6)
    assert st["converged"] and st["iters"] == 0 and torch.all(beta == 0)
    Ybad = p.Y.clone()
    Ybad[17] = float("nan")
    with pytest.raises(S.SpcgError) as e:
        S.spcg_pcg_stage(ctx, p.X, Ybad, 1.0, pc, beta, 3)
    assert e.value.code == S.SPCG_E_BREAKDOWN


# -------------------------------------------------------------- solves

@pytest.mark.parametrize("method", ["spcg", "pcg"])
def test_solve_config0_matches_ols(S, ctx, method):
    _log(f"solve cfg0 {method}")
    p = workloads.make_config(0, device=DEV)
    Xd = p.x_f64().cpu().numpy()
    Yd = p.Y.cpu().numpy()[:, 0]
    beta, st = S.spcg_solve(ctx, p.X, p.Y, method=method, seed=1)
    assert st["rc"] == 0 and st["converged"]
    bh = ols_householder(Xd, Yd)
    assert rel_pred_error(Xd, beta.cpu().numpy(), bh) <= 1e-6
    if method == "spcg":
        assert st["K"] == 7 and st["T_stage1"] == 21
        b_or, info = spcg(Xd, Yd, seed=1)
        # same algorithm on both sides: the Stage II iteration counts agree
        assert abs(st["T_stage2"] - info["per_rhs"][0]["stage2"]["iters"]) <= 1


@pytest.mark.parametrize("storage,N,d", [("f32", 1 << 17, 100), ("f32", 100_003, 33),
                                         ("bf16", 1 << 17, 128), ("fp8", 1 << 16, 64)])
def test_solve_reduced_precision_storage(S, ctx, storage, N, d):
    _log(f"solve {storage} N={N} d={d}")
    p = _problem(N, d, cond=1e4, sigma=1.0, storage=storage, seed=21)
    beta, st = S.spcg_solve(ctx, p.X, p.Y, col_scale=p.col_scale, seed=3)
    assert st["converged"]
    Xd = p.x_f64().cpu().numpy()
    bh = ols_tsqr(Xd, p.Y.cpu().numpy()[:, 0])
    assert rel_pred_error(Xd, beta.cpu().numpy(), bh) <= 1e-6


def test_solve_argument_errors(S, ctx):
    p = _problem(100, 8, seed=1)
    with pytest.raises(S.SpcgError) as e:
        S.spcg_solve(ctx, p.X[:8], p.Y[:8])
    assert e.value.code == S.SPCG_E_SHAPE
    with pytest.raises(S.SpcgError) as e:
        S.spcg_solve(ctx, p.X, p.Y[:50])
    assert e.value.code == S.SPCG_E_SHAPE
    with pytest.raises(S.SpcgError) as e:
        S.spcg_solve(ctx, p.X, p.Y.float())
    assert e.value.code == S.SPCG_E_DTYPE


# ------------------------------------------------ full-size workload

def test_full_size_config1_against_ols(S, ctx):
    """The benchmark workload (N = 1e6, d = 500, FP32, kappa 1e4) in the
    benchmark's launch configuration: the solve must reach the OLS of the
    stored data (oracle TSQR) to 1e-6, and 32 sampled sketch rows must equal
    the oracle's H_un D P X rows computed one by one."""
    _log("full size cfg1: generate")
    p = workloads.make_config(1, device=DEV)
    N, d = p.N, p.d
    _log("full size cfg1: solve")
    beta, st = S.spcg_solve(ctx, p.X, p.Y, seed=1)
    assert st["converged"] and st["K"] == 9
    _log("full size cfg1: oracle TSQR")
    Xh = p.X.cpu().numpy()
    Yh = p.Y.cpu().numpy()[:, 0]
    bh = ols_tsqr(Xh, Yh, block=1 << 16)
    Xb = beta.cpu().numpy()
    num = np.linalg.norm(Xh.astype(np.float64) @ (Xb - bh))
    den = np.linalg.norm(Xh.astype(np.float64) @ bh)
    assert num / den <= 1e-6
    _log("full size cfg1: sampled sketch rows")
    sk = S.spcg_sketch(ctx, p.X, p.Y, seed=1)
    A_last, _, _ = sk.view_tensor(len(sk.sizes) - 1)
    L, Np = padded_bits(N)
    rng = np.random.default_rng(1)
    t = rng.choice(sk.sizes[-1], 32, replace=False)
    rows = slot_rows(1, L, sk.sizes[-1])[t]
    perm = input_perm(1, L)
    sg = sign_vector(1, L)
    valid = perm < N
    k = np.arange(Np)
    # Z[i] = sum_k (-1)^{popcount(i & k)} sign(k) X[p(k)]
    W_idx = k[valid]
    Xp = Xh[perm[valid]].astype(np.float64) * sg[valid, None]
    for i, row in enumerate(rows):
        par = np.zeros(W_idx.size, dtype=np.int64)
        v = W_idx & row
        while np.any(v):
            par ^= v & 1
            v >>= 1
        z = (1.0 - 2.0 * par) @ Xp
        got = A_last[t[i]].cpu().numpy().astype(np.float64)
        scale = math.sqrt(Np) * np.abs(Xh).max(axis=0)
        assert np.max(np.abs(got - z) / scale) < 2e-6 * L
