"""Pins of the oracle's MLMC estimators (Section 2) and of Algorithm 1."""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy.stats import binom

from oracle import mlmc

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_sample_variance_population_form():
    y = np.array([1.0, 2.0, 4.0, 7.0])
    assert abs(mlmc.sample_variance(y) - np.var(y)) < 1e-15
    assert mlmc.mc_estimate(y) == 3.5


def test_optimal_samples_meet_constraint_and_minimise_cost():
    V = np.array([4.0, 0.5, 0.09, 0.01])
    C = np.array([1.0, 4.5, 19.0, 81.0])
    e_s = 0.01
    N = mlmc.optimal_samples(V, C, e_s)
    assert abs(mlmc.sampling_error_sq(V, N) - e_s ** 2) < 1e-14
    assert abs(mlmc.mlmc_cost(N, C) - mlmc.optimal_cost(V, C, e_s)) < 1e-9 * mlmc.mlmc_cost(N, C)
    # brute force: any other allocation on the constraint surface costs more
    rng = np.random.default_rng(0)
    for _ in range(200):
        scale = np.exp(0.3 * rng.standard_normal(4))
        N2 = N * scale
        N2 *= mlmc.sampling_error_sq(V, N2) / e_s ** 2        # back onto sum V/N = e_s^2
        assert abs(mlmc.sampling_error_sq(V, N2) - e_s ** 2) < 1e-12
        assert mlmc.mlmc_cost(N2, C) >= mlmc.mlmc_cost(N, C) * (1 - 1e-12)


def test_error_split_and_bias_estimate():
    e_s, e_b = mlmc.error_split(0.2, 0.5)
    assert abs(e_s ** 2 + e_b ** 2 - 0.04) < 1e-15 and abs(e_s - e_b) < 1e-15
    assert abs(mlmc.bias_estimate(-0.3, 1.0, 4) - 0.1) < 1e-15


def test_complexity_exponents_reproduce_paper():
    t1, t2 = GOLD["test1_rates"], GOLD["test2_rates"]
    # Test II numbers are reproduced to the printed precision
    assert abs(mlmc.mlmc_complexity_exponent(t2["alpha"], t2["beta"], t2["gamma"]) - t2["mlmc_exponent_printed"]) < 0.01
    assert abs(mlmc.mc_complexity_exponent(t2["alpha"], t2["gamma"]) - t2["mc_exponent_printed"]) < 0.01
    assert abs(mlmc.sr_cost_exponent(t2["alpha"], t2["gamma"]) - t2["sr_cost_exponent_printed"]) < 1e-12
    # Test I: the paper prints 2.68 / 3.64 for alpha=0.786, beta=0.740, gamma=1.3;
    # the formula gives 2.71 / 3.65 (the printed rates are rounded)
    assert abs(mlmc.mlmc_complexity_exponent(t1["alpha"], t1["beta"], t1["gamma"]) - t1["mlmc_exponent_printed"]) < 0.04
    assert abs(mlmc.mc_complexity_exponent(t1["alpha"], t1["gamma"]) - t1["mc_exponent_printed"]) < 0.02
    # three regimes of Eq. mlmcComplexity
    assert mlmc.mlmc_complexity_exponent(1.0, 2.0, 1.0) == 2.0
    assert mlmc.mlmc_complexity_exponent(1.0, 1.0, 1.0) == 2.0


def test_paper_tables_savings():
    for row in GOLD["table1"]["rows"][1:]:
        assert abs(row["mc"] / row["mlmc"] - row["saving"]) < 0.01
    for row in GOLD["table_test2"]["rows"]:
        assert abs(row["mlmc"] / row["mlmc_sr"] - row["saving_mlmc"]) < 0.04
    lay = GOLD["test2_layup"]
    assert abs(lay["tolerance_deg"] / lay["z"] - lay["sigma_deg"]) < 0.04


def test_biased_estimator_relative_variance_exact():
    # enumerate the binomial distribution of x+ exactly
    for N, p, k in [(50, 0.01, 1), (200, 0.003, 2), (1000, 0.02, 1)]:
        x = np.arange(N + 1)
        pmf = binom.pmf(x, N, p)
        pt = (x + k) / (N + k)
        m = np.sum(pmf * pt)
        v = np.sum(pmf * (pt - m) ** 2)
        assert abs(v / m ** 2 - mlmc.biased_relative_variance(N, p, k)) < 1e-10
        assert mlmc.biased_relative_variance(N, p, k) < 1
    assert mlmc.biased_p(3, 100, 1) == 4 / 101


def test_trinomial_moments_brute_force():
    for pp, pm in [(0.01, 0.0), (0.02, 0.005), (0.3, 0.1)]:
        vals = np.array([1.0, -1.0, 0.0])
        prob = np.array([pp, pm, 1 - pp - pm])
        mean = np.sum(prob * vals)
        var = np.sum(prob * (vals - mean) ** 2)
        m, v = mlmc.trinomial_moments(pp, pm)
        assert abs(m - mean) < 1e-15 and abs(v - var) < 1e-15


def test_fit_rate():
    M = np.array([100.0, 400.0, 1600.0, 6400.0])
    assert abs(mlmc.fit_rate(M, 3.0 * M ** -0.786) - 0.786) < 1e-12


def test_telescoping_sum_fixed_sample():
    # Eq. MLMC_expectation for one fixed sample: Q_0 + sum_l (Q_l - Q_{l-1}) = Q_L
    q = np.array([66.77589107, 66.26174098, 66.26631043, 66.26966832])
    ys = [np.array([q[0]])] + [np.array([q[l] - q[l - 1]]) for l in range(1, 4)]
    assert abs(mlmc.mlmc_estimate(ys) - q[-1]) < 1e-13


def _synthetic_sampler(mu0=10.0, c_mean=0.4, c_var=0.5, alpha=1.0, beta=1.5, v0=4.0, seed=7):
    """Y_l ~ N(mean_l, V_l) with mean_l = c 4^-alpha l, V_l = c 4^-beta l (l >= 1)."""
    def sampler(level, start, n):
        idx = np.arange(start, start + n)
        out = np.empty(n)
        for i, j in enumerate(idx):
            g = np.random.default_rng([seed, level, int(j)])
            if level == 0:
                out[i] = mu0 + math.sqrt(v0) * g.standard_normal()
            else:
                out[i] = c_mean * 4.0 ** (-alpha * level) + math.sqrt(c_var * 4.0 ** (-beta * level)) * g.standard_normal()
        return out
    return sampler


def test_algorithm1_synthetic():
    sampler = _synthetic_sampler()
    cost = lambda l: 4.0 ** l
    res = mlmc.algorithm1(sampler, cost, e=0.05, theta=0.5, n_star=100, m=4, L_max=8)
    assert res.converged
    e_s, e_b = mlmc.error_split(0.05, 0.5)
    assert res.bias < e_b
    # the final sampling error is at most e_s^2 (N_l rounded up from the optimum)
    assert mlmc.sampling_error_sq(res.V, res.N) <= e_s ** 2 * 1.0001
    # every level holds at least N* samples and the estimate is within 4 RMSE of the truth
    assert min(res.N) >= 100
    true = 10.0 + sum(0.4 * 4.0 ** (-l) for l in range(1, res.L + 1))
    assert abs(res.estimate - true) < 4 * 0.05
    # deterministic: same sampler, same decisions
    res2 = mlmc.algorithm1(sampler, cost, e=0.05, theta=0.5, n_star=100, m=4, L_max=8)
    assert res2.N == res.N and res2.estimate == res.estimate


def test_algorithm1_stops_at_top_level_uncertified():
    sampler = _synthetic_sampler(alpha=0.2)
    res = mlmc.algorithm1(sampler, lambda l: 4.0 ** l, e=0.01, theta=0.5, n_star=50, m=4, L_max=2,
                          max_new=5000)
    assert res.L == 2 and not res.converged


def test_indicator_variance_is_the_sample_variance_when_events_are_common():
    # with the biased rates switched off (below = 0) the estimate is the plain
    # population variance of the 0/1 or -1/0/+1 samples (Eq. varianceestim)
    rng = np.random.default_rng(3)
    q = (rng.random(500) < 0.3).astype(float)
    assert abs(mlmc.indicator_variance(int(q.sum()), 0, 500, below=0, two_sided=False) - np.var(q)) < 1e-15
    y = rng.choice([-1.0, 0.0, 1.0], size=400, p=[0.1, 0.7, 0.2])
    v = mlmc.indicator_variance(int(np.sum(y == 1)), int(np.sum(y == -1)), 400, below=0)
    assert abs(v - np.var(y)) < 1e-15
    # the default threshold (10 events) leaves common events at their frequency
    assert mlmc.indicator_variance(int(np.sum(y == 1)), int(np.sum(y == -1)), 400) == v


def test_bernoulli_level_uses_the_biased_rate_of_its_failures_only():
    # Q in {0, 1} has no -1 outcome: V = p~ (1 - p~) with p~ = (x + k)/(N + k)
    for x, N, k in [(0, 100, 1), (3, 1000, 1), (7, 150, 2)]:
        pt = (x + k) / (N + k)
        assert mlmc.indicator_variance(x, 0, N, k=k, two_sided=False) == pytest.approx(pt * (1 - pt), rel=1e-15)
    # the two-sided form adds a biased p- as well, so it is strictly larger
    assert mlmc.indicator_variance(0, 0, 100) > mlmc.indicator_variance(0, 0, 100, two_sided=False)


def test_two_level_estimate_telescopes_on_shared_chains():
    # base and difference taken on the same samples: Qhat_j + mean(Q_L - Q_j) = mean(Q_L)
    rng = np.random.default_rng(11)
    qj = (rng.random(300) < 0.05).astype(float)
    qL = qj.copy()
    flip = rng.random(300) < 0.02
    qL[flip] = 1.0 - qL[flip]
    r = mlmc.two_level_rare_event(qj, qL - qj)
    assert abs(r["estimate"] - qL.mean()) < 1e-15
    assert r["n_plus"] == int(np.sum((qL - qj) == 1)) and r["n_minus"] == int(np.sum((qL - qj) == -1))


def test_two_level_variance_against_exact_enumeration():
    # exact distribution of Qhat_0 + Yhat: X0 ~ Bin(N0, p0) independent of
    # (X+, X-) ~ Multinomial(N1; p+, p-).  With the biased rates off the
    # estimator's variance is p0 (1 - p0)/N0 + (p+ + p- - (p+ - p-)^2)/N1, and
    # the expected plug-in estimate is (N-1)/N of it for each term; with the
    # biased rates on, rare-event variances are bounded from above
    from scipy.stats import multinomial
    N0, N1 = 12, 9
    for p0, pp, pm in [(0.05, 0.03, 0.01), (0.2, 0.1, 0.0), (0.01, 0.004, 0.002)]:
        est_m = est_v = 0.0
        mean_mse_plain = mean_mse_biased = 0.0
        probs = []
        for x0 in range(N0 + 1):
            w0 = binom.pmf(x0, N0, p0)
            for xp in range(N1 + 1):
                for xm in range(N1 + 1 - xp):
                    w = w0 * multinomial.pmf([xp, xm, N1 - xp - xm], N1, [pp, pm, 1 - pp - pm])
                    q = np.r_[np.ones(x0), np.zeros(N0 - x0)]
                    y = np.r_[np.ones(xp), -np.ones(xm), np.zeros(N1 - xp - xm)]
                    r = mlmc.two_level_rare_event(q, y)
                    rp = mlmc.two_level_rare_event(q, y, below=0)
                    probs.append(w)
                    est_m += w * r["estimate"]
                    est_v += w * r["estimate"] ** 2
                    mean_mse_plain += w * rp["rmse"] ** 2
                    mean_mse_biased += w * r["rmse"] ** 2
        assert abs(sum(probs) - 1.0) < 1e-12
        var_true = p0 * (1 - p0) / N0 + (pp + pm - (pp - pm) ** 2) / N1
        assert abs(est_m - (p0 + pp - pm)) < 1e-14
        assert abs(est_v - est_m ** 2 - var_true) < 1e-14
        plain = p0 * (1 - p0) * (N0 - 1) / N0 ** 2 + (pp + pm - (pp - pm) ** 2) * (N1 - 1) / N1 ** 2
        assert abs(mean_mse_plain - plain) < 1e-14
        assert mean_mse_biased > var_true
