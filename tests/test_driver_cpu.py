"""Host logic of the product's Algorithm 1 against the oracle's Algorithm 1.

Both run on the same synthetic sampler (no GPU): the product keeps FP64
level sums, the oracle keeps the samples; their decisions (levels added,
sample numbers, stopping) and estimates must agree."""
import math

import numpy as np
import pytest

from oracle import mlmc as omlmc
from paper_1907_10271_amd.driver import LevelSums, adaptive_mlmc


def synthetic(level, start, n, mu0=10.0, c_mean=0.4, c_var=0.5, alpha=1.0, beta=1.5, v0=4.0, seed=7):
    out = np.empty(n)
    for i, j in enumerate(range(start, start + n)):
        g = np.random.default_rng([seed, level, int(j)])
        if level == 0:
            out[i] = mu0 + math.sqrt(v0) * g.standard_normal()
        else:
            out[i] = c_mean * 4.0 ** (-alpha * level) + math.sqrt(c_var * 4.0 ** (-beta * level)) * g.standard_normal()
    return out


class SumSampler:
    def __init__(self, gen, cost):
        self.gen, self._cost, self.s = gen, cost, {}

    def sample(self, level, n):
        ls = self.s.setdefault(level, LevelSums())
        y = self.gen(level, ls.n, n)
        ls.n += n
        ls.sum_y += float(np.sum(y))
        ls.sum_y2 += float(np.sum(y * y))

    def acc(self, level):
        return self.s[level]

    def cost(self, level):
        return self._cost(level)


@pytest.mark.parametrize("kw", [dict(), dict(alpha=0.6, beta=1.0), dict(v0=0.5, c_mean=1.0)])
@pytest.mark.parametrize("eps", [0.05, 0.02])
def test_algorithm1_matches_oracle(kw, eps):
    gen = lambda l, s, n: synthetic(l, s, n, **kw)
    cost = lambda l: 4.0 ** l
    ref = omlmc.algorithm1(gen, cost, e=eps, theta=0.5, n_star=100, m=4, L_max=6)
    res = adaptive_mlmc(SumSampler(gen, cost), L_max=6, eps_abs=eps, theta=0.5, n_star=100, m=4)
    assert res.L == ref.L and res.converged == ref.converged
    assert [lv["N"] for lv in res.levels] == ref.N
    assert abs(res.estimate - ref.estimate) <= 1e-12 * abs(ref.estimate)
    for lv, v in zip(res.levels, ref.V):
        assert abs(lv["var"] - v) <= 1e-9 * abs(v)


def test_relative_tolerance_and_alpha_fit_match_oracle():
    gen = lambda l, s, n: synthetic(l, s, n, alpha=0.8)
    cost = lambda l: 4.0 ** (1.2 * l)
    M = [100.0 * 4 ** l for l in range(7)]
    ref = omlmc.algorithm1(gen, cost, e=None, eps_rel=3e-3, theta=0.5, n_star=50, m=4, L_max=6, M=M)
    res = adaptive_mlmc(SumSampler(gen, cost), L_max=6, eps_rel=3e-3, theta=0.5, n_star=50, m=4, dofs=M)
    assert res.L == ref.L and [lv["N"] for lv in res.levels] == ref.N
    assert abs(res.alpha - ref.alpha) < 1e-9
    assert abs(res.e_abs - ref.e_abs) <= 1e-12 * ref.e_abs


def test_population_variance():
    s = LevelSums(4, 14.0, 70.0)
    assert s.mean == 3.5 and s.var == np.var([1.0, 2.0, 4.0, 7.0])


def test_sr_exit_levels_match_oracle_chain():
    from oracle.sr import sr_chain, sr_pair
    from paper_1907_10271_amd.driver import sr_exit_levels
    rng = np.random.default_rng(9)
    for trial in range(300):
        ell = int(rng.integers(1, 5))
        base = 0.88 + 0.05 * rng.standard_normal()
        lam = base + 0.02 * 4.0 ** -np.arange(ell + 1) * rng.uniform(0.5, 2.0)
        lam_star = 0.88 + 0.01 * rng.standard_normal()
        ex = sr_exit_levels(lam[None, :], lam_star, 4.0, 1.0, 1)[0]
        val, j, _ = sr_chain(lambda k: lam[k], ell, lam_star, 4.0, 1.0, 1)
        assert j == ex and val == lam[ex]
        # Y from the same chain, truncated at ell - 1
        qf, qc, y, _ = sr_pair(lambda k: lam[k], ell, lam_star, 4.0, 1.0, 1)
        lam_c = lam[min(ex, ell - 1)]
        assert qf == int(lam[ex] < lam_star) and qc == int(lam_c < lam_star)


def test_indicator_sums_biased_variance():
    from oracle import mlmc as omlmc
    from paper_1907_10271_amd.driver import IndicatorSums
    a = IndicatorSums(n=1000, n_plus=3, n_minus=0, k=1)
    pp, pm = omlmc.biased_p(3, 1000, 1), omlmc.biased_p(0, 1000, 1)
    assert abs(a.var - omlmc.trinomial_moments(pp, pm)[1]) < 1e-15
    b = IndicatorSums(n=1000, n_plus=40, n_minus=12)
    assert abs(b.var - omlmc.trinomial_moments(0.04, 0.012)[1]) < 1e-15


def test_level_zero_indicator_variance_has_no_minus_term():
    # Y_0 = Q_0 in {0, 1}: the variance is p~ (1 - p~) with the biased p+ only,
    # as the oracle's Bernoulli form gives, and never the trinomial one
    from paper_1907_10271_amd.driver import IndicatorSums
    for n, x in [(100, 0), (100, 1), (5000, 7), (300, 40)]:
        a = IndicatorSums(n=n, n_plus=x, two_sided=False)
        ref = omlmc.indicator_variance(x, 0, n, two_sided=False)
        assert abs(a.var - ref) < 1e-15
        p = omlmc.indicator_rate(x, n)
        assert abs(a.var - p * (1 - p)) < 1e-15
        b = IndicatorSums(n=n, n_plus=x, n_minus=0)
        assert abs(b.var - omlmc.indicator_variance(x, 0, n)) < 1e-15


def test_two_level_counts_and_variance_follow_the_oracle():
    # the driver's two-level bookkeeping (counts from chains, variances from
    # IndicatorSums) on synthetic chains, against the oracle's estimator
    from oracle.sr import sr_pair
    from paper_1907_10271_amd.driver import IndicatorSums, sr_exit_levels
    rng = np.random.default_rng(21)
    lam_star, L, j = 0.875, 3, 0
    n0, n1 = 700, 300
    lam0 = 0.89 + 0.01 * rng.standard_normal(n0)
    base = lam0 < lam_star
    lam = 0.89 + 0.01 * rng.standard_normal((n1, 1)) - 0.004 * (1 - 4.0 ** -np.arange(L + 1)) \
        + 0.0005 * rng.standard_normal((n1, L + 1))
    ex = sr_exit_levels(lam, lam_star, 4.0, 1.0, 1)
    qL = lam[np.arange(n1), ex] < lam_star
    qj = lam[np.arange(n1), np.minimum(ex, j)] < lam_star
    y_ref = []
    for r in lam:
        qf, _, _, _ = sr_pair(lambda k: r[k], L, lam_star, 4.0, 1.0, 1)
        y_ref.append(qf - int(r[0] < lam_star))
    assert np.array_equal(qL.astype(int) - qj.astype(int), np.array(y_ref))
    b = IndicatorSums(n=n0, n_plus=int(base.sum()), two_sided=False)
    d = IndicatorSums(n=n1, n_plus=int(np.sum(qL & ~qj)), n_minus=int(np.sum(qj & ~qL)))
    ref = omlmc.two_level_rare_event(base.astype(float), np.array(y_ref, float))
    assert d.n_plus == ref["n_plus"] and d.n_minus == ref["n_minus"] and b.n_plus == ref["n_base_plus"]
    assert abs(b.mean + d.mean - ref["estimate"]) < 1e-15
    assert abs(math.sqrt(b.var / n0 + d.var / n1) - ref["rmse"]) < 1e-15
    assert d.n_plus > 0
