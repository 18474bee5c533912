"""GPU checks of the schedule options: explicit stage
sizes (the tuned schedule of Sec. 4.3: 2^10 ... 2^16, then one larger
transition stage, a_i = 4) and the theory-driven stage counts of Theorems
3.3 / 3.4.  Both must keep the stated stage structure and still reach the
OLS estimator to 1e-6; the oracle's FP64 SPCG on the same schedule gives the
reference Stage II count."""
import numpy as np
import pytest
import torch

import workloads
from oracle.ols import ols_householder
from oracle.spcg import rel_pred_error, spcg
from oracle.theory import theory_schedule

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TUNED = [2 ** k for k in range(10, 15)] + [2 ** 16]


@pytest.fixture(scope="module")
def S():
    import paper_2607_25272_amd as spcg_mod
    return spcg_mod


@pytest.fixture(scope="module")
def ctx(S):
    c = S.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def prob():
    return workloads.gauss_colscale(1 << 17, 64, 1e4, 1e-4, storage="f64", seed=31, device=DEV)


@pytest.mark.parametrize("sketch", ["srht", "cs"])
def test_tuned_size_list(S, ctx, prob, sketch):
    print(f"tuned sizes {sketch}", flush=True)
    beta, st = S.spcg_solve(ctx, prob.X, prob.Y, seed=2, m_list=TUNED, a=4, sketch=sketch)
    assert st["converged"] and st["K"] == len(TUNED) and st["T_stage1"] == 4 * len(TUNED)
    Xd = prob.x_f64().cpu().numpy()
    Yd = prob.Y.cpu().numpy()[:, 0]
    assert rel_pred_error(Xd, beta.cpu().numpy(), ols_householder(Xd, Yd)) <= 1e-6
    _, info = spcg(Xd, Yd, 2, sizes=TUNED, a=4, sketch=sketch)
    assert abs(st["T_stage2"] - info["per_rhs"][0]["stage2"]["iters"]) <= 1


@pytest.mark.parametrize("omega", [0.5, 0.1])
def test_theory_stage_counts(S, ctx, prob, omega):
    print(f"theory counts omega={omega}", flush=True)
    beta, st = S.spcg_solve(ctx, prob.X, prob.Y, seed=2, a_rule="theory", omega=omega)
    sizes = [st_m for st_m in S.spcg_sketch(ctx, prob.X, prob.Y, seed=2).sizes]
    expect = theory_schedule(sizes, prob.d, omega)
    assert st["converged"] and st["T_stage1"] == sum(expect) and st["policy_a"] == expect[-1]
    Xd = prob.x_f64().cpu().numpy()
    Yd = prob.Y.cpu().numpy()[:, 0]
    assert rel_pred_error(Xd, beta.cpu().numpy(), ols_householder(Xd, Yd)) <= 1e-6
    _, info = spcg(Xd, Yd, 2, a=("theory", omega))
    assert info["per_rhs"][0]["a_list"] == expect
    assert abs(st["T_stage2"] - info["per_rhs"][0]["stage2"]["iters"]) <= 1


def test_schedule_option_errors(S, ctx, prob):
    with pytest.raises(S.SpcgError) as e:
        S.spcg_solve(ctx, prob.X, prob.Y, m_list=[2048, 1024])
    assert e.value.code == S.SPCG_E_SHAPE
    with pytest.raises(S.SpcgError) as e:
        S.spcg_solve(ctx, prob.X, prob.Y, m_list=[1024, 1 << 17])
    assert e.value.code == S.SPCG_E_SHAPE
    with pytest.raises(S.SpcgError) as e:   # CountSketch nesting needs dividing sizes
        S.spcg_solve(ctx, prob.X, prob.Y, m_list=[1000, 2500], sketch="cs")
    assert e.value.code == S.SPCG_E_SHAPE
    with pytest.raises(S.SpcgError) as e:
        S.spcg_solve(ctx, prob.X, prob.Y, a_rule="theory", omega=1.5)
    assert e.value.code == S.SPCG_E_INVALID_ARG
    q = workloads.gauss_colscale(20000, 16, 1e2, 1.0, storage="f32", k=2, seed=3, device=DEV)
    with pytest.raises(S.SpcgError) as e:   # multi-RHS runs the batched form: fixed a only
        S.spcg_solve(ctx, q.X, q.Y, a_rule="theory")
    assert e.value.code == S.SPCG_E_INVALID_ARG


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_nested_gradient_reuse(S, ctx, storage):
    # Nested-gradient reuse: stage starts from the previous stage's gradient plus a
    # G pass over the new prefix rows; same stage structure, same accuracy
    print(f"nested gradient {storage}", flush=True)
    p = workloads.gauss_colscale(1 << 17, 96, 1e4, 1.0, storage=storage, seed=41, device=DEV)
    Xd = p.x_f64().cpu().numpy()
    Yd = p.Y.cpu().numpy()[:, 0]
    bh = ols_householder(Xd, Yd)
    b0, s0 = S.spcg_solve(ctx, p.X, p.Y, seed=5, nested_gradient=False)
    b1, s1 = S.spcg_solve(ctx, p.X, p.Y, seed=5, nested_gradient=True)
    assert s1["converged"] and s1["K"] == s0["K"] and s1["T_stage1"] == s0["T_stage1"]
    assert abs(s1["T_stage2"] - s0["T_stage2"]) <= 1
    assert rel_pred_error(Xd, b1.cpu().numpy(), bh) <= 1e-6
    if storage == "f64":
        _, info = spcg(Xd, Yd, 5, nested_gradient=True)
        assert abs(s1["T_stage2"] - info["per_rhs"][0]["stage2"]["iters"]) <= 1
    # a CountSketch ignores the option (its stages are folds, not prefixes)
    c0, _ = S.spcg_solve(ctx, p.X, p.Y, seed=5, sketch="cs")
    c1, _ = S.spcg_solve(ctx, p.X, p.Y, seed=5, sketch="cs", nested_gradient=True)
    assert torch.equal(c0, c1)
