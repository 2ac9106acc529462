"""Selective refinement for failure probabilities (Section 2.4, Algorithm 2).

For one sample, the eigenvalue is computed on levels ``j = 0, 1, ...``; from
level ``j_min`` on, the chain stops as soon as the level-``j`` value is
further from the threshold than its estimated discretisation error
(Eqs. sampleBias and testFailure):
``|lam_j - lam*| >= |lam_j - lam_{j-1}| / (m^alpha - 1)``.
The quantity of interest is the indicator ``Q = 1(lam < lam*)`` of the last
value computed.  Readings: the printed test starts at ``j > 1`` while the
rare-event table has most samples stopping after level 1, so the first
level at which the test is applied is a parameter ``j_min`` (default 1);
the printed indicator ``1(lam - lam*)`` is read as ``1(lam < lam*)``.

For a multilevel difference ``Y_l = Q_l - Q_{l-1}`` both terms come from
the same chain, the second truncated at level ``l - 1``.
"""
from __future__ import annotations

from typing import Callable, List, Tuple


def sr_chain(lam_at: Callable[[int], float], ell: int, lam_star: float, m: float, alpha: float,
             j_min: int = 1) -> Tuple[float, int, List[float]]:
    """Algorithm 2 for one sample up to level ``ell``.

    Returns ``(lambda_used, exit_level, lambdas_computed)``.
    """
    lams: List[float] = []
    fac = 1.0 / (m ** alpha - 1.0)
    for j in range(ell + 1):
        lam_j = lam_at(j)
        lams.append(lam_j)
        if j >= max(j_min, 1):
            if abs(lam_j - lam_star) >= abs(lam_j - lams[j - 1]) * fac:
                return lam_j, j, lams
    return lams[-1], ell, lams


def indicator(lam: float, lam_star: float) -> int:
    """``Q = 1(lam < lam*)``."""
    return 1 if lam < lam_star else 0


def sr_pair(lam_at: Callable[[int], float], ell: int, lam_star: float, m: float, alpha: float,
            j_min: int = 1):
    """``(Q_ell, Q_{ell-1}, Y_ell, levels_solved)`` from one chain (``Q_{-1} = 0``)."""
    lam_f, exit_f, lams = sr_chain(lam_at, ell, lam_star, m, alpha, j_min)
    q_f = indicator(lam_f, lam_star)
    if ell == 0:
        return q_f, 0, q_f, len(lams)
    cached = lams.copy()
    lam_c, _, _ = sr_chain(lambda j: cached[j], ell - 1, lam_star, m, alpha, j_min)
    q_c = indicator(lam_c, lam_star)
    return q_f, q_c, q_f - q_c, len(lams)
