"""Monte Carlo and multilevel Monte Carlo estimators (Section 2 of the paper).

Every function states the equation it writes out.  Readings where the
paper is ambiguous:

* bias estimate: the absolute value ``|Y_L| / (m^alpha - 1)`` is used
  (Eq. bias_estimate omits it);
* Algorithm 1 starts with ``L = -1`` and never increments it; the level is
  incremented at the top of every pass, and the loop also stops at the
  configured top level (the bias is then reported as uncertified);
* the bias estimate (Eq. bias_estimate) is derived for level differences
  ``Y_l, l >= 1``; at ``L = 0`` (where ``Y_0 = Q_0``) the test is not
  applied and the loop always continues;
* trinomial moments: ``E[Y] = p+ - p-`` and
  ``V[Y] = p+ + p- - (p+ - p-)^2`` (the printed signs are inconsistent
  with ``Y`` taking the values +1 and -1);
* sample variance uses the population form ``1/N`` as printed
  (Eq. varianceestim).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


def mc_estimate(q) -> float:
    """Standard MC estimator, Eq. MC_estimator: the sample mean."""
    q = np.asarray(q, dtype=np.float64)
    return float(math.fsum(q) / len(q))


def error_split(e: float, theta: float):
    """Eq. tausplit: ``e_s^2 = theta e^2`` and ``e_b^2 = (1 - theta) e^2``; returns ``(e_s, e_b)``."""
    return math.sqrt(theta) * e, math.sqrt(1.0 - theta) * e


def sample_variance(y) -> float:
    """Eq. varianceestim: ``(1/N) sum Y^2 - Yhat^2``."""
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    m = math.fsum(y) / n
    return float(math.fsum(y * y) / n - m * m)


def optimal_samples(V, C, e_s: float) -> np.ndarray:
    """Eq. optimal_Nl: ``N_l = e_s^-2 (sum_k sqrt(V_k C_k)) sqrt(V_l / C_l)`` (real valued)."""
    V = np.asarray(V, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    return (np.sum(np.sqrt(V * C)) / e_s ** 2) * np.sqrt(V / C)


def mlmc_cost(N, C) -> float:
    """Eq. MLMC_cost: ``sum_l N_l C_l``."""
    return float(np.dot(np.asarray(N, float), np.asarray(C, float)))


def optimal_cost(V, C, e_s: float) -> float:
    """Cost at the optimal real-valued ``N_l`` (the equality in Eq. mlmcComplexity with ``e_s``)."""
    V = np.asarray(V, float)
    C = np.asarray(C, float)
    return float(np.sum(np.sqrt(V * C)) ** 2 / e_s ** 2)


def sampling_error_sq(V, N) -> float:
    """Sampling part of the MLMC mean square error: ``sum_l V_l / N_l``."""
    return float(np.sum(np.asarray(V, float) / np.asarray(N, float)))


def bias_estimate(y_hat_L: float, alpha: float, m: float = 4.0) -> float:
    """Eq. bias_estimate: ``|Y_L| / (m^alpha - 1)``."""
    return abs(y_hat_L) / (m ** alpha - 1.0)


def mlmc_complexity_exponent(alpha: float, beta: float, gamma: float) -> float:
    """Exponent ``2 + max(0, (gamma - beta)/alpha)`` of Eq. mlmcComplexity."""
    return 2.0 + max(0.0, (gamma - beta) / alpha)


def mc_complexity_exponent(alpha: float, gamma: float) -> float:
    """Exponent ``2 + gamma/alpha`` of the standard MC cost bound (Section 2.1)."""
    return 2.0 + gamma / alpha


def sr_cost_exponent(alpha: float, gamma: float) -> float:
    """Eq. costpersample: per-sample cost of selective refinement grows like ``M^(gamma - alpha)``."""
    return gamma - alpha


def fit_rate(M, v) -> float:
    """Least-squares rate ``r`` with ``|v| ~ M^-r`` (the log-log fits of Sections 3.2 and 4.2)."""
    x = np.log(np.asarray(M, float))
    y = np.log(np.abs(np.asarray(v, float)))
    A = np.stack([x, np.ones_like(x)], axis=1)
    slope = np.linalg.lstsq(A, y, rcond=None)[0][0]
    return float(-slope)


def mlmc_estimate(level_samples: List[np.ndarray]) -> float:
    """Eq. MLMC_defn: ``Q_hat = sum_l mean(Y_l)`` with ``Y_0 = Q_0``."""
    return float(math.fsum(mc_estimate(y) for y in level_samples))


def biased_p(x: int, N: int, k: int = 1) -> float:
    """Eq. biased_estimator: ``(x + k) / (N + k)``."""
    return (x + k) / (N + k)


def biased_relative_variance(N: int, p: float, k: int) -> float:
    """Relative variance of the biased estimator, ``N p (1 - p) / (N p + k)^2``."""
    return N * p * (1.0 - p) / (N * p + k) ** 2


def indicator_rate(x: int, N: int, k: int = 1, below: int = 10) -> float:
    """Rate of an event seen ``x`` times in ``N`` samples: the frequency
    ``x / N``, or, while fewer than ``below`` events have been seen, the biased
    ``p~ = (x + k) / (N + k)`` of Eq. biased_estimator, which bounds a rare
    rate from above (Section 2.4; reading: ``k = 1``, switched on below 10
    events)."""
    if x < below:
        return biased_p(x, N, k)
    return x / N


def indicator_variance(n_plus: int, n_minus: int, N: int, k: int = 1, below: int = 10,
                       two_sided: bool = True) -> float:
    """Variance estimate of an indicator level from its event counts.

    ``two_sided``: a difference ``Y = Q_f - Q_c`` in {-1, 0, +1}, with the
    trinomial variance ``p+ + p- - (p+ - p-)^2`` (the printed moments read with
    consistent signs); otherwise an indicator ``Q`` in {0, 1} with no coarse
    term, where ``p- = 0`` and the variance is ``p (1 - p)``.  Each rate comes
    from ``indicator_rate``."""
    pp = indicator_rate(n_plus, N, k, below)
    pm = indicator_rate(n_minus, N, k, below) if two_sided else 0.0
    return pp + pm - (pp - pm) ** 2


def two_level_rare_event(q_base, y, k: int = 1, below: int = 10) -> dict:
    """Two-level estimate ``E[Q] ~ Qhat_j + Yhat_{L,j}``, ``Y_{L,j} = Q_L - Q_j``
    (Section 4.3).  ``q_base``: indicators of the base level ``j`` on their own
    samples; ``y``: differences ``Q_L - Q_j`` on an independent set of samples,
    both terms of one sample from the same selective-refinement chain.  The
    estimate is the sum of the two sample means (Eq. MLMC_defn with two
    terms); its mean square sampling error is ``V_j / N_j + V_Y / N_Y`` with
    each variance from ``indicator_variance`` (Bernoulli for the base,
    trinomial for the difference)."""
    q = np.asarray(q_base, dtype=np.float64)
    d = np.asarray(y, dtype=np.float64)
    n0, n1 = len(q), len(d)
    x0 = int(np.sum(q == 1.0))
    xp, xm = int(np.sum(d == 1.0)), int(np.sum(d == -1.0))
    assert x0 == int(np.sum(q != 0.0)) and xp + xm == int(np.sum(d != 0.0)), "indicators must be 0/1 and -1/0/1"
    v0 = indicator_variance(x0, 0, n0, k, below, two_sided=False)
    vy = indicator_variance(xp, xm, n1, k, below, two_sided=True)
    est = x0 / n0 + (xp - xm) / n1
    mse = v0 / n0 + vy / n1
    return {"estimate": est, "rmse": math.sqrt(mse), "var_base": v0, "var_y": vy, "n0": n0, "n1": n1,
            "n_base_plus": x0, "n_plus": xp, "n_minus": xm}


def trinomial_moments(p_plus: float, p_minus: float):
    """Mean and variance of ``Y`` in {-1, 0, +1} with ``P(+1) = p+``, ``P(-1) = p-``."""
    mean = p_plus - p_minus
    return mean, p_plus + p_minus - mean * mean


@dataclass
class Alg1Result:
    estimate: float
    N: List[int]
    V: List[float]
    Yhat: List[float]
    C: List[float]
    L: int
    bias: float
    e_abs: float
    converged: bool
    passes: int
    alpha: float
    samples: List[np.ndarray] = field(default_factory=list)


def algorithm1(sampler: Callable[[int, int, int], np.ndarray], cost: Callable[[int], float],
               e: Optional[float], theta: float, n_star: int, m: float, L_max: int,
               alpha_default: float = 1.0, eps_rel: Optional[float] = None,
               M: Optional[List[float]] = None, max_new: int = 10 ** 9) -> Alg1Result:
    """Algorithm 1 (adaptive MLMC).

    ``sampler(level, start, n)`` returns ``n`` samples of ``Y_level`` with
    indices ``start..start+n-1`` of that level's stream; ``cost(level)`` is
    the cost ``C_l`` of one sample.  The tolerance is ``e`` (absolute) or, if
    ``eps_rel`` is given, ``eps_rel * |Q_hat|`` re-evaluated every pass.
    ``alpha`` is fitted on ``|Yhat_l|, l >= 1`` against ``M`` once two such
    levels exist, otherwise ``alpha_default``.
    """
    samples: List[np.ndarray] = []
    L = -1
    passes = 0
    converged = False
    alpha = alpha_default
    bias = math.inf
    e_abs = e if e is not None else math.inf
    while not converged:
        L += 1
        passes += 1
        samples.append(np.asarray(sampler(L, 0, n_star), dtype=np.float64))
        V = [sample_variance(y) for y in samples]
        Cs = [cost(l) for l in range(L + 1)]
        if eps_rel is not None:
            e_abs = eps_rel * abs(mlmc_estimate(samples))
        e_s, e_b = error_split(e_abs, theta)
        Nhat = np.ceil(optimal_samples(V, Cs, e_s))
        for l in range(L + 1):
            n_have = len(samples[l])
            if n_have < Nhat[l]:
                extra = int(min(Nhat[l] - n_have, max_new))
                samples[l] = np.concatenate([samples[l], sampler(l, n_have, extra)])
        Yhat = [mc_estimate(y) for y in samples]
        if M is not None and L >= 2:
            alpha = fit_rate(M[1:L + 1], Yhat[1:L + 1])
        bias = bias_estimate(Yhat[L], alpha, m) if L >= 1 else math.inf
        if bias < e_b:
            converged = True
        elif L >= L_max:
            break
    V = [sample_variance(y) for y in samples]
    return Alg1Result(mlmc_estimate(samples), [len(y) for y in samples], V,
                      [mc_estimate(y) for y in samples], [cost(l) for l in range(L + 1)],
                      L, bias, e_abs, converged, passes, alpha, samples)
