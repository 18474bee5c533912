"""Closed forms from the convergence analysis (Sec. 3 and Appendix A).

Test infrastructure: see ``oracle/__init__.py``.  Every function states the
result it writes out.
"""
import math

THETA = 0.25  # contraction factor of Theorem 3.1


def stage_ratio(m_prev, m_cur, d):
    """r_{i-1,i} = sqrt((m_i - d) / (m_{i-1} - d))   (Theorem 3.3)."""
    return math.sqrt((m_cur - d) / (m_prev - d))


def iteration_lower_bound(m_prev, m_cur, d, omega):
    """Unrounded lower bound of Theorem 3.3:
    a_i >= ln{[(1 + omega) r_{i-1,i} + 1] / omega} / ln 4."""
    r = stage_ratio(m_prev, m_cur, d)
    return math.log(((1.0 + omega) * r + 1.0) / omega) / math.log(4.0)


def doubling_ratio_sq(m_prev, d):
    """Under m_i = 2 m_{i-1}: r_{i-1,i}^2 = 2 + d / (m_{i-1} - d)
    (remark after Theorem 3.3 and proof of Theorem 3.4)."""
    return 2.0 + d / (m_prev - d)


def alpha_bound(m1, m2, d, omega):
    """alpha = ln{[1 + (1 + omega) r_bar] / omega} / ln 4 with r_bar = r_{1,2}
    (Theorem 3.4)."""
    rbar = stage_ratio(m1, m2, d)
    return math.log((1.0 + (1.0 + omega) * rbar) / omega) / math.log(4.0)


def theory_schedule(sizes, d, omega=0.5):
    """Stage iteration counts from Theorems 3.3 and 3.4 (the theory-driven
    schedule): a_i = ceil of the Theorem 3.3 bound for i >= 2, and a_1 =
    ceil(alpha), the bound Theorem 3.4 gives for every stage (with r = 1 when
    there is one stage)."""
    sizes = list(sizes)
    out = []
    for i in range(len(sizes)):
        if len(sizes) < 2:
            val = math.log((2.0 + omega) / omega) / math.log(4.0)
        elif i == 0:
            val = alpha_bound(sizes[0], sizes[1], d, omega)
        else:
            val = iteration_lower_bound(sizes[i - 1], sizes[i], d, omega)
        out.append(max(1, math.ceil(val - 1e-12)))
    return out


def first_stage_iterations(q1, omega):
    """Smallest unrounded a_1 with theta^{a_1} q_1 <= omega:
    a_1 = ln(q_1 / omega) / ln 4   (proof of Theorem 3.4)."""
    return math.log(q1 / omega) / math.log(4.0)


def complexity_terms(N, d, omega, sigma, K, m1, m2):
    """Dominant costs of Theorem 3.4: initialization N d log2 N, first stage
    4 alpha N d, second stage 4 [ln(omega^K / sigma) / ln 4] N d."""
    a = alpha_bound(m1, m2, d, omega)
    return {
        "init": N * d * math.log2(N),
        "stage1": 4.0 * a * N * d,
        "stage2": 4.0 * (math.log(omega ** K / sigma) / math.log(4.0)) * N * d,
    }


def pcg_flops(m, d):
    """FLOPs of one PCG iteration on an m x d system: (4m + 13) d + 2 d^2
    (Sec. 2.2)."""
    return (4 * m + 13) * d + 2 * d * d


def cg_bound_factor(kappa, j):
    """Lemma A.2: ||B(x_j - x*)|| <= 2 ((sqrt k - 1)/(sqrt k + 1))^j ||B(x_0 - x*)||."""
    sk = math.sqrt(kappa)
    return 2.0 * ((sk - 1.0) / (sk + 1.0)) ** j


def stage_contraction(eps, a):
    """Deterministic per-stage factor of the proof of Theorem 3.1,
    eq. (app-stage-intermediate): 2 sqrt((1+eps)/(1-eps)) eps^a."""
    return 2.0 * math.sqrt((1.0 + eps) / (1.0 - eps)) * eps ** a


def prediction_efficiency(N, d, m):
    """Finite-sample proxy of Lemma A.7: PE(i) <= (N - d) / (m_i - d)."""
    return (N - d) / (m - d)


def global_bound_ols(theta, T, e0, s, C, delta_ols):
    """Right side of eq. (global-ols), Theorem 3.2:
    theta^T e0 + [1 + theta^s (1 + 5C/3)] delta_OLS."""
    return theta ** T * e0 + (1.0 + theta ** s * (1.0 + 5.0 * C / 3.0)) * delta_ols
