"""Pins for the schedule reading and the closed forms of Sec. 3."""
import math
import os

import numpy as np
import pytest

from oracle.spcg import schedule
from oracle.theory import (alpha_bound, complexity_terms, doubling_ratio_sq,
                           iteration_lower_bound, pcg_flops, prediction_efficiency,
                           stage_ratio)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_spcg_iterations.txt")


def _table1():
    rows = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            lg, kap, it = line.split()
            rows.append((int(lg), float(kap), int(it)))
    return rows


def test_paper_schedule_reproduces_table1_iteration_pattern():
    # Sec. 4: m_1 = 8d, m_K = N/2, a_i = 3; Table 1's SPCG iteration counts
    # sit within -1..+2 of 3K (Stage I) for every setting
    for lg, _, it in _table1():
        N = 1 << lg
        sizes = schedule(N, 64, m0=8 * 64)
        assert sizes[0] == 512 and sizes[-1] == N // 2
        K = len(sizes)
        assert K == lg - 9
        assert -1 <= it - 3 * K <= 2


def test_baseline_schedules():
    assert len(schedule(20000, 50)) == 7
    assert schedule(20000, 50)[-1] == 12800
    assert len(schedule(1_000_000, 500)) == 9
    assert len(schedule(4_000_000, 1000)) == 10
    assert len(schedule(2_000_000, 256)) == 11
    assert schedule(100, 30) == []


def test_iteration_bound_figure1_claims():
    # Sec. 4.1 / Fig. 1(a), N = 2^20, d = 64, m_1 = 512: the unrounded bounds
    # for a_2 and a_K stay below three, decrease in omega and nearly coincide
    N, d = 1 << 20, 64
    sizes = schedule(N, d, m0=512)
    omegas = [2.0 ** -4, 2.0 ** -3, 2.0 ** -2, 2.0 ** -1, 1.0]
    a2 = [iteration_lower_bound(sizes[0], sizes[1], d, w) for w in omegas]
    aK = [iteration_lower_bound(sizes[-2], sizes[-1], d, w) for w in omegas]
    assert max(a2) < 3 and max(aK) < 3
    assert all(x > y for x, y in zip(a2, a2[1:]))
    assert all(x > y for x, y in zip(aK, aK[1:]))
    assert max(abs(x - y) for x, y in zip(a2, aK)) < 0.05
    assert all(x >= y for x, y in zip(a2, aK))


def test_iteration_bound_special_values():
    # r = 1 (m_i = m_{i-1}) and omega = 1: ln(3)/ln(4)
    assert iteration_lower_bound(100, 100, 10, 1.0) == pytest.approx(math.log(3) / math.log(4))
    # definition: theta^a [(1+omega) r + 1] = omega at the bound (theta = 1/4)
    a = iteration_lower_bound(512, 1024, 64, 0.25)
    r = stage_ratio(512, 1024, 64)
    assert 0.25 ** a * (1.25 * r + 1) == pytest.approx(0.25)


def test_doubling_identity():
    d = 64
    for m in (512, 1024, 4096):
        assert stage_ratio(m, 2 * m, d) ** 2 == pytest.approx(doubling_ratio_sq(m, d))
    assert doubling_ratio_sq(10 ** 9, 1) == pytest.approx(2.0)


def test_complexity_and_flops():
    # first-stage bound uses alpha = bound at r_bar = r_{1,2}
    N, d, w = 1 << 20, 64, 0.5
    a = alpha_bound(512, 1024, d, w)
    assert a == pytest.approx(iteration_lower_bound(512, 1024, d, w))
    t = complexity_terms(N, d, w, 1e-4, 11, 512, 1024)
    assert t["init"] == N * d * 20
    assert t["stage1"] == pytest.approx(4 * a * N * d)
    assert pcg_flops(1000, 10) == (4 * 1000 + 13) * 10 + 200
    assert prediction_efficiency(1000, 10, 505) == pytest.approx(2.0)


def test_theory_schedule_follows_theorems_3_3_and_3_4():
    # doubling from m_1 = 4d: r_{1,2}^2 = 2 + d/(m_1 - d) (remark after
    # Theorem 3.3), the bounds decrease with i, and a_1 = ceil(alpha)
    from oracle.theory import alpha_bound, theory_schedule
    d, omega = 50, 0.5
    sizes = [4 * d * 2 ** i for i in range(7)]
    a = theory_schedule(sizes, d, omega)
    r12 = math.sqrt(2 + d / (sizes[0] - d))
    assert a[0] == math.ceil(math.log((1 + (1 + omega) * r12) / omega) / math.log(4))
    assert a[0] == math.ceil(alpha_bound(sizes[0], sizes[1], d, omega))
    for i in range(1, 7):
        r = math.sqrt((sizes[i] - d) / (sizes[i - 1] - d))
        assert a[i] == math.ceil(math.log(((1 + omega) * r + 1) / omega) / math.log(4))
    assert all(x >= y for x, y in zip(a, a[1:]))
    # omega -> smaller demands more iterations; a single stage uses r = 1
    assert sum(theory_schedule(sizes, d, 0.05)) > sum(a)
    assert theory_schedule([1000], d, 0.5) == [math.ceil(math.log(2.5 / 0.5) / math.log(4))]
    # the tuned sizes of Sec. 4.3: the jump 2^16 -> 2^20 (r ~ 4) asks for more
    # iterations than a doubling step before rounding, and never fewer after
    tuned = [2 ** k for k in range(10, 17)] + [2 ** 20]
    at = theory_schedule(tuned, 64, 0.5)
    assert iteration_lower_bound(tuned[-2], tuned[-1], 64, 0.5) > iteration_lower_bound(tuned[-3], tuned[-2], 64, 0.5)
    assert at[-1] >= at[-2]


def test_oracle_spcg_with_size_list_and_theory_counts():
    from oracle.spcg import spcg, rel_pred_error
    from oracle.ols import ols_householder
    from oracle.theory import theory_schedule
    rng = np.random.default_rng(9)
    N, d = 1 << 14, 16
    X = rng.standard_normal((N, d)) * np.logspace(0, 2, d)
    Y = X @ rng.standard_normal(d) + 0.01 * rng.standard_normal(N)
    sizes = [2 ** k for k in range(7, 12)] + [2 ** 13]
    b, info = spcg(X, Y, 1, sizes=sizes, a=("theory", 0.5))
    assert info["sizes"] == sizes
    assert info["per_rhs"][0]["a_list"] == theory_schedule(sizes, d, 0.5)
    assert info["per_rhs"][0]["T_stage1"] == sum(theory_schedule(sizes, d, 0.5))
    assert rel_pred_error(X, b, ols_householder(X, Y)) < 1e-6


def _theorem32_recursion(e0, a_list, deltas, s, delta_ols, theta=0.25):
    """The error recursion behind Theorem 3.2, run step by step: the stage
    bound e_i <= theta^{a_i} e_{i-1} + (1 + theta^{a_i}) delta_i (Theorem 3.1
    with the warm start), then the full-data stage
    e_T <= theta^s e_{T_dagger} + (1 + theta^s) delta_OLS (second-stage lemma
    plus the triangle inequality), each taken with equality."""
    e = e0
    for a, dl in zip(a_list, deltas):
        e = theta ** a * e + (1.0 + theta ** a) * dl
    return theta ** s * e + (1.0 + theta ** s) * delta_ols


def test_global_bound_ols_hand_values():
    # theta = 1/4, T = 3, e0 = 8, s = 1, C = 3, delta_OLS = 2:
    # 8/64 + [1 + (1/4)(1 + 5)] 2 = 0.125 + 5 = 5.125
    from oracle.theory import global_bound_ols
    assert global_bound_ols(0.25, 3, 8.0, 1, 3.0, 2.0) == pytest.approx(5.125, rel=1e-15)
    # s = 0: [2 + 5C/3] delta_OLS;  C = 0 recovers (1 + theta^s) delta_OLS
    assert global_bound_ols(0.25, 0, 0.0, 0, 3.0, 1.0) == pytest.approx(7.0, rel=1e-15)
    assert global_bound_ols(0.25, 5, 0.0, 2, 0.0, 1.0) == pytest.approx(1.0625, rel=1e-15)


def test_global_bound_ols_dominates_the_recursion():
    # Theorem 3.2: with a_i >= 1 and delta_i <= C delta_OLS the recursion is
    # bounded by eq. (global-ols) for any e0, schedule and s
    from oracle.theory import global_bound_ols
    rng = np.random.default_rng(32)
    for _ in range(2000):
        K = int(rng.integers(1, 14))
        a = [int(x) for x in rng.integers(1, 6, K)]
        s = int(rng.integers(0, 8))
        C = float(rng.uniform(0.1, 20))
        dols = float(rng.uniform(0.01, 3))
        deltas = list(rng.uniform(0, C * dols, K))
        e0 = float(rng.uniform(0, 1e3))
        T = sum(a) + s
        lhs = _theorem32_recursion(e0, a, deltas, s, dols)
        assert lhs <= global_bound_ols(0.25, T, e0, s, C, dols) * (1 + 1e-12)


def test_global_bound_ols_is_tight_for_unit_stages():
    # a_i = 1 and delta_i = C delta_OLS make every step of the proof an
    # equality except the geometric tail: the gap to eq. (global-ols) is
    # C delta_OLS theta^s (1 + theta) theta^K / (1 - theta) and vanishes as K grows
    from oracle.theory import global_bound_ols
    C, dols, e0 = 2.0, 1.5, 10.0
    for s in (0, 1, 3):
        for K in (1, 4, 30):
            T = K + s
            lhs = _theorem32_recursion(e0, [1] * K, [C * dols] * K, s, dols)
            gap = C * dols * 0.25 ** s * 1.25 * 0.25 ** K / 0.75
            assert global_bound_ols(0.25, T, e0, s, C, dols) - lhs == pytest.approx(gap, rel=1e-9, abs=1e-13)


def test_first_stage_iterations_hand_values():
    # proof of Theorem 3.4: a_1 = ln(q_1 / omega) / ln 4 solves theta^{a_1} q_1 = omega
    from oracle.theory import first_stage_iterations
    assert first_stage_iterations(2.0, 0.5) == pytest.approx(1.0, rel=1e-15)
    assert first_stage_iterations(8.0, 0.5) == pytest.approx(2.0, rel=1e-15)
    assert first_stage_iterations(1.0, 1.0 / 64) == pytest.approx(3.0, rel=1e-15)
    for q1, w in ((1.7, 0.3), (5.0, 0.05), (1.01, 0.9)):
        a1 = first_stage_iterations(q1, w)
        assert 0.25 ** a1 * q1 == pytest.approx(w, rel=1e-13)


def test_first_stage_iterations_bracketed_as_theorem_3_4_states():
    # 1 < q_1 < 1 + (1 + omega) r_bar implies ln(1/omega)/ln 4 < a_1 < alpha
    from oracle.theory import alpha_bound, first_stage_iterations, stage_ratio
    d = 64
    for m1 in (512, 1024, 4096):
        rbar = stage_ratio(m1, 2 * m1, d)
        for w in (0.0625, 0.25, 0.5, 0.9):
            lo = math.log(1.0 / w) / math.log(4.0)
            hi = alpha_bound(m1, 2 * m1, d, w)
            for q1 in np.linspace(1.0, 1.0 + (1.0 + w) * rbar, 12)[1:-1]:
                a1 = first_stage_iterations(q1, w)
                assert lo < a1 < hi


def test_complexity_second_stage_term():
    # proof of Theorem 3.4: T = ln(1/sigma)/ln 4 total iterations minus
    # K ln(1/omega)/ln 4 in Stage I leaves ln(omega^K/sigma)/ln 4 full-data
    # iterations of 4 N d FLOPs each.  omega = 1/2, sigma = 4^-10, K = 4:
    # ln(2^16)/ln 4 = 8 iterations, i.e. 32 N d
    N, d = 1 << 16, 8
    t = complexity_terms(N, d, 0.5, 4.0 ** -10, 4, 128, 256)
    assert t["stage2"] == pytest.approx(32 * N * d, rel=1e-12)
    for K, w, sg in ((3, 0.3, 1e-6), (8, 0.7, 1e-9)):
        t = complexity_terms(N, d, w, sg, K, 128, 256)
        T = math.log(1 / sg) / math.log(4)
        assert t["stage2"] / (4 * N * d) == pytest.approx(T - K * math.log(1 / w) / math.log(4), rel=1e-12)
    # positive exactly when omega > sigma^(1/K)
    sg, K = 1e-4, 4
    assert complexity_terms(N, d, sg ** (1 / K) * 1.01, sg, K, 128, 256)["stage2"] > 0
    assert complexity_terms(N, d, sg ** (1 / K) * 0.99, sg, K, 128, 256)["stage2"] < 0
