"""GPU parity of the multi-RHS and batched forms (k independent PCGs per
problem sharing the products; many problems per launch) against the FP64
oracle: every column of every problem must reach its OLS estimator to a
relative prediction error of 1e-6."""
import numpy as np
import pytest
import torch

import workloads
from oracle.ols import ols_tsqr
from oracle.spcg import rel_pred_error

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def S():
    import paper_2607_25272_amd as spcg_mod
    return spcg_mod


@pytest.fixture(scope="module")
def ctx(S):
    c = S.Context(0)
    yield c
    c.close()


def _check(p, beta):
    Xd = p.x_f64().cpu().numpy()
    bh = ols_tsqr(Xd, p.Y.cpu().numpy())
    B = beta.cpu().numpy().reshape(p.d, -1)
    for c in range(bh.shape[1]):
        assert rel_pred_error(Xd, B[:, c], bh[:, c]) <= 1e-6, c


@pytest.mark.parametrize("N,d,k,storage", [(1 << 16, 100, 5, "f32"), (50_000, 512, 16, "f32"),
                                           (40_000, 37, 3, "bf16"), (30_000, 16, 16, "f32")])
def test_multi_rhs_solve(S, ctx, N, d, k, storage):
    print(f"multi-rhs N={N} d={d} k={k} {storage}", flush=True)
    p = workloads.gauss_colscale(N, d, 1e3, 1.0, storage=storage, k=k, seed=N + d + k, device=DEV)
    beta, st = S.spcg_solve(ctx, p.X, p.Y, seed=1)
    assert st["converged"] and beta.shape == (d, k)
    _check(p, beta)


def test_multi_rhs_columns_match_single_rhs_solves(S, ctx):
    # each column of a k-RHS solve is its own PCG: it agrees with the solve
    # of that column alone (both within 1e-6 of the same OLS estimator)
    p = workloads.gauss_colscale(1 << 15, 40, 1e2, 1.0, storage="f32", k=4, seed=3, device=DEV)
    beta, _ = S.spcg_solve(ctx, p.X, p.Y, seed=2)
    Xd = p.x_f64().cpu().numpy()
    for c in range(4):
        b1, _ = S.spcg_solve(ctx, p.X, p.Y[:, c:c + 1].contiguous(), seed=2)
        assert rel_pred_error(Xd, beta[:, c].cpu().numpy(), b1.cpu().numpy()) < 2e-6


def test_multi_rhs_tolerance_below_fp32_floor_does_not_diverge(S, ctx):
    # Iterating past the accuracy floor of the FP32 products must neither
    # freeze the refreshed gradient nor drift away from the solution.
    p = workloads.gauss_colscale(1 << 15, 40, 1e2, 1.0, storage="f32", k=4, seed=3, device=DEV)
    Xd = p.x_f64().cpu().numpy()
    bh = ols_tsqr(Xd, p.Y.cpu().numpy())
    for T in (60, 100):
        beta, st = S.spcg_solve(ctx, p.X, p.Y, seed=2, tol=1e-13, T=T)
        B = beta.cpu().numpy()
        errs = [rel_pred_error(Xd, B[:, c], bh[:, c]) for c in range(4)]
        print("T", T, "rc", st["rc"], "T2", st["T_stage2"], ["%.1e" % e for e in errs], flush=True)
        assert max(errs) <= 1e-6


def test_batched_uneven_problems(S, ctx):
    probs = workloads.batched(n_prob=12, N_range=(20_000, 120_000), d_range=(32, 512),
                              cond_range=(1e2, 1e5), k_range=(1, 16), device=DEV)
    print("batched shapes", [(q.N, q.d, q.k) for q in probs], flush=True)
    betas, stats = S.spcg_solve_batched(ctx, [q.X for q in probs], [q.Y for q in probs], seed=1)
    for q, b, st in zip(probs, betas, stats):
        assert st["converged"], (q.N, q.d, q.k, st)
        _check(q, b)


def test_batched_preconditioner_fallback_per_problem(S, ctx):
    # the one-pass factors of a batch are queued on several lanes and their
    # pivot statuses checked together; a badly scaled factor (column scales
    # spanning 1e6 > 1e5) is rebuilt with shifted CholeskyQR3 for that
    # problem alone, the others keep one pass
    probs = [workloads.gauss_colscale(N, d, cond, 1.0, storage="f32", k=k, seed=N + d, device=DEV)
             for N, d, cond, k in ((30_000, 48, 1e2, 2), (40_000, 64, 1e6, 1), (25_000, 96, 1e3, 3),
                                   (35_000, 40, 1e2, 1), (20_000, 80, 1e3, 2), (28_000, 56, 1e2, 1),
                                   (33_000, 72, 1e3, 1), (22_000, 24, 1e2, 2), (26_000, 32, 1e6, 2))]
    betas, stats = S.spcg_solve_batched(ctx, [q.X for q in probs], [q.Y for q in probs], seed=3)
    for q, b, st in zip(probs, betas, stats):
        print("problem", q.N, q.d, "qr_passes", st["qr_passes"], flush=True)
        assert st["qr_passes"] == (3 if q.N in (40_000, 26_000) else 1)
        assert st["converged"], st
        _check(q, b)


def test_batched_full_pcg_and_bf16(S, ctx):
    probs = [workloads.gauss_colscale(N, d, 1e3, 1.0, storage="bf16", k=k, seed=N, device=DEV)
             for N, d, k in ((30_000, 64, 2), (45_000, 128, 1), (25_000, 200, 7))]
    for method in ("spcg", "pcg"):
        betas, stats = S.spcg_solve_batched(ctx, [q.X for q in probs], [q.Y for q in probs],
                                            method=method, seed=5)
        for q, b, st in zip(probs, betas, stats):
            assert st["converged"]
            _check(q, b)


def test_batched_argument_errors(S, ctx):
    p = workloads.gauss_colscale(2000, 8, 10, 1.0, storage="f64", k=2, seed=1, device=DEV)
    with pytest.raises(S.SpcgError) as e:
        S.spcg_solve_batched(ctx, [p.X], [p.Y])
    assert e.value.code == S.SPCG_E_DTYPE
    q = workloads.gauss_colscale(2000, 600, 10, 1.0, storage="f32", k=1, seed=1, device=DEV)
    with pytest.raises(S.SpcgError) as e:
        S.spcg_solve_batched(ctx, [q.X], [q.Y])
    assert e.value.code == S.SPCG_E_SHAPE


def _uneven(n=10, seed=11):
    return workloads.batched(n_prob=n, N_range=(20_000, 90_000), d_range=(32, 512),
                             cond_range=(1e2, 1e5), k_range=(1, 16), seed=seed, device=DEV)


def test_batched_graphs_replay_matches_direct_launches(S, ctx):
    # The captured graphs hold exactly the direct launches: with the same
    # task granularity, one Stage I graph per stage and the Stage II product
    # and d-space graphs (replayed once per iteration, with the host's
    # stopping test and copies between replays) give identical bits, solve
    # after solve.
    probs = _uneven()
    Xs, Ys = [q.X for q in probs], [q.Y for q in probs]
    ref, st_d = S.spcg_solve_batched(ctx, Xs, Ys, seed=3, batch_direct=True, batch_tasks_per_cu=4)
    assert st_d[0]["batch_graphs"] == 0
    for rep in range(2):
        got, st_g = S.spcg_solve_batched(ctx, Xs, Ys, seed=3, batch_tasks_per_cu=4)
        assert st_g[0]["batch_graphs"] > 0 and st_g[0]["batch_tasks_per_cu"] == 4
        for q, a, b, s1, s2 in zip(probs, ref, got, st_d, st_g):
            assert s1["T_stage2"] == s2["T_stage2"]
            assert torch.equal(a, b), (rep, q.N, q.d, q.k)
    for q, b, st in zip(probs, got, st_g):
        assert st["converged"]
        _check(q, b)


def test_batched_autotuned_granularity(S, ctx):
    # The tuner picks 2, 4 or 8 tasks per CU once per context and storage
    # type; its timing passes leave the iterates untouched, so the tuned
    # solve equals a solve run with that granularity fixed.
    probs = _uneven(n=6, seed=12)
    Xs, Ys = [q.X for q in probs], [q.Y for q in probs]
    c2 = S.Context(0)
    try:
        got, st = S.spcg_solve_batched(c2, Xs, Ys, seed=4)
        tpc = st[0]["batch_tasks_per_cu"]
        assert tpc in (2, 4, 8)
        fixed, st_f = S.spcg_solve_batched(c2, Xs, Ys, seed=4, batch_tasks_per_cu=tpc)
        again, st_a = S.spcg_solve_batched(c2, Xs, Ys, seed=4)
        assert st_a[0]["batch_tasks_per_cu"] == tpc
        for a, b, c in zip(got, fixed, again):
            assert torch.equal(a, b) and torch.equal(a, c)
        for q, b, s in zip(probs, got, st):
            assert s["converged"]
            _check(q, b)
    finally:
        c2.close()


def test_batched_tile_shapes_are_bit_identical(S, ctx):
    # The three tile shapes of the product launches (three barriers per
    # tile; the two-tile pipeline with 3 and with 4 LDS slots) run the same
    # MFMA chains and reductions in the same order per task, so with the
    # same granularity they give identical bits; the autotuned shapes are
    # reported per launch bucket (class * 2 + (k > 8)).
    probs = _uneven(n=8, seed=13)
    Xs, Ys = [q.X for q in probs], [q.Y for q in probs]
    ref, st_r = S.spcg_solve_batched(ctx, Xs, Ys, seed=5, batch_tasks_per_cu=4, batch_shape=1)
    assert all(v in (0, 1) for v in st_r[0]["batch_shapes"])
    for shape in (2, 3):
        got, st = S.spcg_solve_batched(ctx, Xs, Ys, seed=5, batch_tasks_per_cu=4, batch_shape=shape)
        used = [v for v in st[0]["batch_shapes"] if v]
        assert used and all(v == shape for v in used), (shape, used)
        for q, a, b, s1, s2 in zip(probs, ref, got, st_r, st):
            assert s1["T_stage2"] == s2["T_stage2"]
            assert torch.equal(a, b), (shape, q.N, q.d, q.k)
    for q, b, s in zip(probs, ref, st_r):
        assert s["converged"]
        _check(q, b)
    # a fresh context tunes the shapes (timing passes only, iterates
    # untouched): its tuned solve equals its fixed-shape solve
    c2 = S.Context(0)
    try:
        tuned, st_t = S.spcg_solve_batched(c2, Xs, Ys, seed=5, batch_tasks_per_cu=4)
        assert any(v > 0 for v in st_t[0]["batch_tune_ms"])
        assert all(v in (0, 1, 2, 3) for v in st_t[0]["batch_shapes"])
        fixed, _ = S.spcg_solve_batched(c2, Xs, Ys, seed=5, batch_tasks_per_cu=4, batch_shape=1)
    finally:
        c2.close()
    for q, a, b in zip(probs, tuned, fixed):
        assert torch.equal(a, b), (q.N, q.d, q.k)


def test_batched_one_launch_per_pass(S, ctx):
    # every task of a pass in one launch of the widest row-width class (the
    # comparison point for per-bucket launches): tasks are split over one
    # launch instead of one per bucket, so the sums round differently, and
    # every column still reaches its OLS estimator
    probs = _uneven(n=6, seed=14)
    Xs, Ys = [q.X for q in probs], [q.Y for q in probs]
    got, st = S.spcg_solve_batched(ctx, Xs, Ys, seed=6, batch_one_launch=True, batch_tasks_per_cu=4)
    used = [b for b, v in enumerate(st[0]["batch_shapes"]) if v]
    assert used == [10], used   # class 4x8 (5), k bucket 0
    for q, b, s in zip(probs, got, st):
        assert s["converged"]
        _check(q, b)



def test_batched_nested_gradient_start(S, ctx):
    # Stage I stages after the first start from the previous stage's
    # gradient plus a G pass over the new prefix rows (nested SRHT sketches,
    # Sec. 2.2): the same stage structure as the direct start, Stage II
    # counts within one, every column at its OLS estimator
    probs = _uneven(n=6, seed=15)
    Xs, Ys = [q.X for q in probs], [q.Y for q in probs]
    nest, st_n = S.spcg_solve_batched(ctx, Xs, Ys, seed=7, batch_tasks_per_cu=4)
    direct, st_d = S.spcg_solve_batched(ctx, Xs, Ys, seed=7, batch_tasks_per_cu=4, nested_gradient=False)
    for q, b1, b2, s1, s2 in zip(probs, nest, direct, st_n, st_d):
        assert s1["converged"] and s2["converged"]
        assert s1["K"] == s2["K"] and s1["T_stage1"] == s2["T_stage1"]
        assert abs(s1["T_stage2"] - s2["T_stage2"]) <= 1, (s1["T_stage2"], s2["T_stage2"])
        _check(q, b1)
        _check(q, b2)


@pytest.mark.parametrize("storage,d,k,m", [("f32", 37, 3, 1000), ("f32", 50, 4, 777), ("f32", 6, 2, 300),
                                           ("f32", 241, 2, 500), ("f32", 254, 16, 1003), ("f32", 301, 5, 600),
                                           ("f32", 510, 9, 999), ("bf16", 38, 4, 700), ("f32", 37, 2, 40)])
def test_unaligned_rows_match_padded_rows(S, ctx, storage, d, k, m):
    # Dense rows whose byte length is a multiple of 4 but not of 16 are read
    # with 16-byte loads from 4-byte aligned addresses (a row's last vector
    # reaches into the next row; the matrix's last row is loaded a few bytes
    # early, into the previous row); the same values in padded rows whose
    # stride is not a multiple of 16 bytes take 4-byte loads.  The tiles and
    # the MFMA order are the same, so the iterates agree bit for bit, with
    # and without the refreshed gradient (S and SG passes).
    print(f"unaligned rows {storage} d={d} k={k} m={m}", flush=True)
    g = torch.Generator().manual_seed(7 * d + k)
    dt = torch.float32 if storage == "f32" else torch.bfloat16
    A = (torch.randn(m, d, generator=g, dtype=torch.float64) *
         torch.logspace(0, 2, d, dtype=torch.float64)).to(dt).to(DEV)
    dp = (d + 7) // 8 * 8 + (1 if storage == "f32" else 2)
    Ap = torch.zeros(m, dp, dtype=dt, device=DEV)
    Ap[:, :d] = A
    Av = Ap[:, :d]
    assert Av.stride(0) == dp and (dp * Av.element_size()) % 16 != 0
    b = torch.randn(m, k, generator=g, dtype=torch.float64).to(DEV)
    R = np.linalg.qr(A.double().cpu().numpy(), mode="r")
    pc = S.spcg_precond_from_r(ctx, torch.from_numpy(R))
    for refresh in (False, True):
        outs = []
        for X in (A, Av):
            beta = torch.zeros(d, k, dtype=torch.float64, device=DEV)
            st = S.spcg_pcg_stage(ctx, X, b, 1.0 / m, pc, beta, 4, refresh=refresh)
            assert st["iters"] == 4
            outs.append(beta.clone())
        assert torch.equal(outs[0], outs[1]), refresh
    # and it is the PCG of this system: 4 steps with the exact preconditioner
    # of A reach its least-squares solution
    Ad = A.double().cpu().numpy()
    xs = np.linalg.lstsq(Ad, b.cpu().numpy(), rcond=None)[0]
    err = np.abs(Ad @ (outs[0].cpu().numpy() - xs)).max() / np.abs(Ad @ xs).max()
    assert err < 1e-4, err
