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
