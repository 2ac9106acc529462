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
