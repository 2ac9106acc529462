"""MLMC drivers over the HIP sample-solve library (Section 2 of the paper).

* :func:`adaptive_mlmc` is Algorithm 1 (adaptive MLMC) written over per-level
  FP64 accumulators (``N_l``, ``sum Y``, ``sum Y^2``): sample means,
  Eq. varianceestim for ``V_l``, Eq. optimal_Nl for the sample numbers,
  Eq. bias_estimate for the stopping test and Eq. tausplit for the split of
  the tolerance.  Readings where the paper is ambiguous: the level counter
  is incremented at the top of every pass (the printed loop never does it);
  the bias estimate uses ``|Yhat_L|`` and, being derived for level
  differences, is not applied at ``L = 0``; ``alpha`` is fitted on the levels
  ``l >= 1`` once two exist (otherwise a default); the run stops at the top
  configured level with ``converged = False`` if the bias test never passes.
* :class:`StripSampler` draws strip samples (seeded parameter rows), solves
  coupled fine/coarse pairs on the GPU and accumulates the level sums on the
  GPU; the cost ``C_l`` of a sample is the measured wall time per sample.

The sampler interface is ``sample(level, n) -> None`` (adds ``n`` samples to
the level's accumulator) plus ``acc[level]`` and ``cost(level)``, so the same
algorithm drives any sampler (tests use synthetic ones).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from ._lib import FP64, LevelAcc


@dataclass
class LevelSums:
    """FP64 level accumulator (host side): N, sum Y, sum Y^2 and the cost spent."""
    n: int = 0
    sum_y: float = 0.0
    sum_y2: float = 0.0
    seconds: float = 0.0

    @property
    def mean(self) -> float:
        return self.sum_y / self.n

    @property
    def var(self) -> float:
        """Population variance (1/N), Eq. varianceestim."""
        m = self.mean
        return self.sum_y2 / self.n - m * m

    @property
    def var_unbiased(self) -> float:
        return self.var * self.n / (self.n - 1) if self.n > 1 else float("nan")

    @staticmethod
    def from_acc(acc: LevelAcc, seconds: float) -> "LevelSums":
        return LevelSums(int(acc.n), acc.sum_y + acc.comp_y, acc.sum_y2 + acc.comp_y2, seconds)


@dataclass
class MLMCResult:
    estimate: float
    levels: List[Dict]
    L: int
    converged: bool
    e_abs: float
    bias: float
    sampling_err2: float
    alpha: float
    passes: int
    seconds: float
    history: List[Dict] = field(default_factory=list)

    def as_dict(self) -> Dict:
        return {"estimate": self.estimate, "L": self.L, "converged": self.converged, "e_abs": self.e_abs,
                "bias_estimate": self.bias, "sampling_err2": self.sampling_err2, "alpha": self.alpha,
                "passes": self.passes, "seconds": self.seconds, "levels": self.levels}


def _alpha_fit(M: List[float], yhat: List[float]) -> float:
    x = np.log(np.asarray(M, float))
    y = np.log(np.abs(np.asarray(yhat, float)))
    slope = np.polyfit(x, y, 1)[0]
    return float(-slope)


def adaptive_mlmc(sampler, L_max: int, eps_abs: Optional[float] = None, eps_rel: Optional[float] = None,
                  theta: float = 0.5, n_star: int = 100, m: float = 4.0, alpha_default: float = 1.0,
                  dofs: Optional[List[float]] = None, max_new: int = 10 ** 9,
                  log: Optional[Callable[[Dict], None]] = None, eps_floor: float = 0.0) -> MLMCResult:
    """Algorithm 1.  The tolerance is ``eps_abs`` or ``eps_rel * max(|estimate|,
    eps_floor)`` (re-evaluated after every pass; the floor gives a relative
    tolerance a scale while the estimate is still zero, e.g. a failure
    probability before the first failure).  ``dofs[l]`` (M_l) enables the fit
    of alpha."""
    if (eps_abs is None) == (eps_rel is None):
        raise ValueError("give exactly one of eps_abs, eps_rel")
    t0 = time.perf_counter()
    L = -1
    passes = 0
    alpha = alpha_default
    converged = False
    hist: List[Dict] = []
    e_abs = eps_abs
    bias = math.inf
    while True:
        L += 1
        passes += 1
        sampler.sample(L, n_star)
        est = sum(sampler.acc(l).mean for l in range(L + 1))
        if eps_rel is not None:
            e_abs = eps_rel * max(abs(est), eps_floor)
        if not e_abs > 0.0:
            raise ValueError("tolerance is zero: give eps_abs or a positive eps_floor")
        e_s2 = theta * e_abs * e_abs
        e_b = math.sqrt(1.0 - theta) * e_abs
        V = [max(sampler.acc(l).var, 0.0) for l in range(L + 1)]
        C = [sampler.cost(l) for l in range(L + 1)]
        s = sum(math.sqrt(v * c) for v, c in zip(V, C))
        for l in range(L + 1):
            n_opt = math.ceil(s * math.sqrt(V[l] / C[l]) / e_s2) if C[l] > 0 else 0
            have = sampler.acc(l).n
            if have < n_opt:
                sampler.sample(l, int(min(n_opt - have, max_new)))
        yhat = [sampler.acc(l).mean for l in range(L + 1)]
        if dofs is not None and L >= 2:
            alpha = _alpha_fit(dofs[1:L + 1], yhat[1:L + 1])
        bias = abs(yhat[L]) / (m ** alpha - 1.0) if L >= 1 else math.inf
        rec = {"pass": passes, "L": L, "N": [sampler.acc(l).n for l in range(L + 1)], "yhat": yhat,
               "V": [sampler.acc(l).var for l in range(L + 1)], "C": C, "e_abs": e_abs, "bias": bias,
               "e_b": e_b, "alpha": alpha, "t": time.perf_counter() - t0}
        hist.append(rec)
        if log:
            log(rec)
        if bias < e_b:
            converged = True
            break
        if L >= L_max:
            break
    levels = []
    for l in range(L + 1):
        a = sampler.acc(l)
        levels.append({"level": l, "N": a.n, "mean": a.mean, "var": a.var, "var_unbiased": a.var_unbiased,
                       "cost_per_sample_s": sampler.cost(l)})
    est = sum(lv["mean"] for lv in levels)
    samp = sum(lv["var"] / lv["N"] for lv in levels)
    return MLMCResult(est, levels, L, converged, e_abs, bias, samp, alpha, passes,
                      time.perf_counter() - t0, hist)


class StripSampler:
    """Coupled strip samples on the GPU: Y_0 = Q_0, Y_l = Q_l - Q_{l-1} (same row)."""

    def __init__(self, ctx, cfg: Dict, precision: int = FP64, rtol: float = 0.0, max_batch: int = 4096,
                 cost_model: Optional[Callable[[int], float]] = None, log: Optional[Callable] = None):
        import torch
        import mlmc_inputs as mi
        self.torch = torch
        self.mi = mi
        self.ctx = ctx
        self.cfg = cfg
        self.precision = precision
        self.rtol = rtol
        self.max_batch = max_batch
        self.cost_model = cost_model
        self.next_row = {}
        self._acc: Dict[int, LevelAcc] = {}
        self._sec: Dict[int, float] = {}
        self.failures = 0
        self.solves = {}
        self.log = log

    def acc(self, level: int) -> LevelSums:
        return LevelSums.from_acc(self._acc[level], self._sec.get(level, 0.0))

    def cost(self, level: int) -> float:
        if self.cost_model is not None:
            return self.cost_model(level)
        a = self._acc[level]
        return self._sec[level] / max(a.n, 1)

    def sample(self, level: int, n: int) -> None:
        torch = self.torch
        done = 0
        while done < n:
            k = min(self.max_batch, n - done)
            start = self.next_row.get(level, 0)
            rows = self.mi.strip_xi(self.cfg, level, start, k)
            xi = torch.from_numpy(rows).to("cuda")
            req = [(j, level, level > 0) for j in range(k)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            qf, qc, info = self.ctx.solve_batch(req, xi, precision=self.precision, rtol=self.rtol)
            acc = self._acc.setdefault(level, LevelAcc())
            self.ctx.level_stats(level, qf, qc if level > 0 else None, acc=acc)
            dt = time.perf_counter() - t0
            bad = int(np.sum(info["status_f"] != 0) + (np.sum(info["status_c"] != 0) if level > 0 else 0))
            if bad:
                self.failures += bad
                raise RuntimeError(f"level {level}: {bad} solves did not converge (rows {start}..{start + k})")
            self._sec[level] = self._sec.get(level, 0.0) + dt
            self.next_row[level] = start + k
            self.solves[level] = self.solves.get(level, 0) + k * (2 if level > 0 else 1)
            done += k
            if self.log:
                self.log({"level": level, "batch": k, "done": done, "of": n, "seconds": round(dt, 3)})


def run_strip_mlmc(ctx, cfg: Dict, precision: int = FP64, eps_rel: Optional[float] = None,
                   eps_abs: Optional[float] = None, L_max: Optional[int] = None, log=None,
                   cost_model=None) -> MLMCResult:
    """Algorithm 1 on the strip workload ``cfg`` with the GPU sampler."""
    ml = cfg.get("mlmc", {})
    if eps_rel is None and eps_abs is None:
        eps_rel = ml.get("eps_rel", 1e-3)
    L_max = cfg["n_levels"] - 1 if L_max is None else L_max
    sampler = StripSampler(ctx, cfg, precision=precision, cost_model=cost_model, log=log)
    dofs = [ctx.level_info(l)["n_dofs"] for l in range(cfg["n_levels"])]
    res = adaptive_mlmc(sampler, L_max, eps_abs=eps_abs, eps_rel=eps_rel, theta=ml.get("theta", 0.5),
                        n_star=ml.get("n_star", 100), m=ml.get("m", 4), alpha_default=ml.get("alpha_default", 1.0),
                        dofs=dofs, log=log)
    res.history.append({"solves_per_level": dict(sampler.solves)})
    return res


# ---------------------------------------------------------------------- plate
def sr_exit_levels(lam: np.ndarray, lam_star: float, m: float, alpha: float, j_min: int = 1) -> np.ndarray:
    """Exit level of the selective-refinement chain (Algorithm 2) for each row of
    ``lam`` (``[n, ell + 1]``, NaN where not computed): the first ``j >= j_min``
    with ``|lam_j - lam*| >= |lam_j - lam_{j-1}| / (m^alpha - 1)`` (Eqs.
    sampleBias, testFailure), else the last level."""
    n, L1 = lam.shape
    fac = 1.0 / (m ** alpha - 1.0)
    out = np.full(n, L1 - 1, dtype=np.int64)
    alive = np.ones(n, dtype=bool)
    for j in range(max(j_min, 1), L1):
        stop = alive & (np.abs(lam[:, j] - lam_star) >= np.abs(lam[:, j] - lam[:, j - 1]) * fac)
        out[stop] = j
        alive &= ~stop
    return out


@dataclass
class IndicatorSums:
    """Level accumulator of a failure indicator: a difference Y in {-1, 0, 1}
    (``two_sided``, levels above 0) or, with no coarse term (level 0), an
    indicator Q in {0, 1}."""
    n: int = 0
    n_plus: int = 0
    n_minus: int = 0
    k: int = 1
    seconds: float = 0.0
    use_biased_below: int = 10
    two_sided: bool = True

    @property
    def mean(self) -> float:
        return (self.n_plus - self.n_minus) / self.n

    def rate(self, x: int) -> float:
        """Rate of an event seen ``x`` times: the frequency, or, when fewer than
        ``use_biased_below`` events were seen, the biased p~ = (x + k)/(N + k)
        of Eq. biased_estimator (an upper bound for rare events)."""
        return (x + self.k) / (self.n + self.k) if x < self.use_biased_below else x / self.n

    @property
    def var(self) -> float:
        """Variance of Y, V = p+ + p- - (p+ - p-)^2 with each rate from
        ``rate``; without a coarse term Y = Q cannot be -1, so p- = 0 and
        V = p (1 - p)."""
        pp = self.rate(self.n_plus)
        pm = self.rate(self.n_minus) if self.two_sided else 0.0
        return pp + pm - (pp - pm) ** 2

    @property
    def var_unbiased(self) -> float:
        m = self.mean
        return (self.n_plus + self.n_minus - self.n * m * m) / max(self.n - 1, 1)


class PlateSRSampler:
    """Samples of Y_l = 1(lam_l < lam*) - 1(lam_{l-1} < lam*) with selective
    refinement (Algorithm 2): the chain of each sample is solved level by level
    on the GPU (the surviving samples of a level form one batch), and both terms
    come from the same chain, the second truncated at l - 1.  Batches are
    large (``max_batch`` rows; the library splits each level's solves into
    launches that fit its workspace), so that the few survivors that reach the
    fine levels, whose solves take a work-group each for about a second, are
    solved together rather than a handful per launch."""

    def __init__(self, ctx, cfg: Dict, lam_star: float, precision: int = FP64, j_min: Optional[int] = None,
                 alpha: Optional[float] = None, m: Optional[float] = None, max_batch: int = 65536, k_biased: int = 1,
                 stream_offset: int = 0, log=None):
        import torch
        import mlmc_inputs as mi
        self.torch, self.mi, self.ctx, self.cfg = torch, mi, ctx, cfg
        sr = cfg.get("sr", {})
        self.lam_star = lam_star
        self.j_min = sr.get("j_min", 1) if j_min is None else j_min
        self.alpha = sr.get("alpha", 1.0) if alpha is None else alpha
        self.m = sr.get("m", 4) if m is None else m
        self.precision = precision
        self.max_batch = max_batch
        self.k_biased = k_biased
        self.stream_offset = stream_offset
        self.next_row: Dict[int, int] = {}
        self._acc: Dict[int, IndicatorSums] = {}
        self.solves = np.zeros(cfg["n_levels"], dtype=np.int64)
        self.failures = 0
        self.log = log

    def acc(self, level: int) -> IndicatorSums:
        return self._acc[level]

    def cost(self, level: int) -> float:
        a = self._acc[level]
        return a.seconds / max(a.n, 1)

    def chains(self, level: int, offsets: np.ndarray):
        """Solve the chains of ``offsets`` rows up to ``level``; returns
        ``(lam [n, level + 1], exit_level [n])``."""
        torch = self.torch
        n = len(offsets)
        lam = np.full((n, level + 1), np.nan)
        off_d = torch.from_numpy(np.ascontiguousarray(offsets)).to("cuda")
        alive = np.arange(n)
        exit_lv = np.full(n, level, dtype=np.int64)
        fac = 1.0 / (self.m ** self.alpha - 1.0)
        for j in range(level + 1):
            if len(alive) == 0:
                break
            lf, _, info = self.ctx.buckle_batch([(int(i), j, False) for i in alive], off_d,
                                                precision=self.precision)
            vals = lf.cpu().numpy()
            bad = np.sum(info["status_f"] != 0)
            if bad:
                self.failures += int(bad)
                raise RuntimeError(f"level {j}: {bad} eigen-solves failed")
            lam[alive, j] = vals
            self.solves[j] += len(alive)
            if j >= max(self.j_min, 1) and j < level:
                stop = np.abs(vals - self.lam_star) >= np.abs(vals - lam[alive, j - 1]) * fac
                exit_lv[alive[stop]] = j
                alive = alive[~stop]
        return lam, exit_lv

    def sample(self, level: int, n: int) -> None:
        torch = self.torch
        done = 0
        while done < n:
            k = min(self.max_batch, n - done)
            start = self.next_row.get(level, 0)
            rows = self.mi.plate_offsets(self.cfg, level, start, k, stream=level + self.stream_offset)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam, ex = self.chains(level, rows)
            idx = np.arange(k)
            lam_f = lam[idx, ex]
            acc = self._acc.setdefault(level, IndicatorSums(k=self.k_biased, two_sided=level > 0))
            if level > 0:
                lam_c = lam[idx, np.minimum(ex, level - 1)]
                qd = torch.from_numpy(np.stack([lam_f, lam_c])).to("cuda")
                la = self.ctx.level_stats(level, qd[0], qd[1], lambda_star=self.lam_star)
            else:
                qd = torch.from_numpy(lam_f).to("cuda")
                la = self.ctx.level_stats(level, qd, None, lambda_star=self.lam_star)
            dt = time.perf_counter() - t0
            acc.n += int(la.n)
            acc.n_plus += int(la.n_plus)
            acc.n_minus += int(la.n_minus)
            acc.seconds += dt
            self.next_row[level] = start + k
            done += k
            if self.log:
                self.log({"level": level, "batch": k, "done": done, "of": n, "seconds": round(dt, 3),
                          "solves": self.solves.tolist()})


def run_plate_mlmc_sr(ctx, cfg: Dict, lam_star: Optional[float] = None, tau_rel: Optional[float] = None,
                      precision: int = FP64, L_max: Optional[int] = None, n_star: Optional[int] = None,
                      log=None) -> MLMCResult:
    """MLMC with selective refinement for P(lambda < lambda*) (Sections 2.3-2.4):
    Algorithm 1 over the SR sampler, tolerance ``tau_rel * p_hat``."""
    ml = cfg.get("mlmc", {})
    lam_star = cfg["lambda_crit"] if lam_star is None else lam_star
    tau_rel = ml.get("tau_rel", 0.043) if tau_rel is None else tau_rel
    L_max = cfg["n_levels"] - 1 if L_max is None else L_max
    sampler = PlateSRSampler(ctx, cfg, lam_star, precision=precision, log=log)
    dofs = [ctx.level_info(l)["n_dofs"] for l in range(cfg["n_levels"])]
    res = adaptive_mlmc(sampler, L_max, eps_rel=tau_rel, theta=ml.get("theta", 0.5),
                        n_star=ml.get("n_star", 100) if n_star is None else n_star, m=cfg.get("sr", {}).get("m", 4),
                        alpha_default=cfg.get("sr", {}).get("alpha", 1.0), dofs=None, log=log,
                        eps_floor=cfg.get("p_target", 0.0))
    res.history.append({"solves_per_level": sampler.solves.tolist()})
    return res


def two_level_rare_event(ctx, cfg: Dict, L: int, n0: int, n1: int, lam_star: Optional[float] = None,
                         precision: int = FP64, j: int = 0, k_biased: int = 1) -> Dict:
    """The two-level estimator E[Q] ~ Qhat_j + Yhat_{L,j}, Y_{L,j} = Q_L - Q_j
    (Section 4.3).  The base term takes ``n0`` samples of level ``j`` (rows of
    stream 100), each a selective-refinement chain truncated at ``j``; the
    difference takes ``n1`` chains up to ``L`` (rows of stream 101), with Q_L
    from the whole chain and Q_j from the same chain truncated at ``j``.
    Variances use the biased rates of Eq. biased_estimator below 10 events
    (Bernoulli for the base term, trinomial for the difference); the RMSE is
    the sampling error ``sqrt(V_j / n0 + V_Y / n1)``.  ``rows`` holds the
    per-sample loads and exit levels behind the counts."""
    if not 0 <= j < L:
        raise ValueError(f"need 0 <= j < L, got j={j}, L={L}")
    lam_star = cfg["lambda_crit"] if lam_star is None else lam_star
    s = PlateSRSampler(ctx, cfg, lam_star, precision=precision, stream_offset=100)
    t0 = time.perf_counter()
    rows0 = s.mi.plate_offsets(cfg, j, 0, n0, stream=100)
    lam0, ex0 = s.chains(j, rows0)
    q0 = lam0[np.arange(n0), ex0] < lam_star
    rows1 = s.mi.plate_offsets(cfg, L, 0, n1, stream=101)
    lam1, ex1 = s.chains(L, rows1)
    i1 = np.arange(n1)
    qL = lam1[i1, ex1] < lam_star
    qj = lam1[i1, np.minimum(ex1, j)] < lam_star
    base = IndicatorSums(n=n0, n_plus=int(q0.sum()), k=k_biased, two_sided=False)
    diff = IndicatorSums(n=n1, n_plus=int(np.sum(qL & ~qj)), n_minus=int(np.sum(qj & ~qL)), k=k_biased)
    est = base.mean + diff.mean
    mse = base.var / n0 + diff.var / n1
    return {"estimate": est, "rmse": math.sqrt(mse), "n0": n0, "n1": n1, "L": L, "j": j,
            "n_base_plus": base.n_plus, "n_plus": diff.n_plus, "n_minus": diff.n_minus,
            "var_base": base.var, "var_y": diff.var, "solves": s.solves.tolist(),
            "seconds": time.perf_counter() - t0, "p_base": base.mean, "yhat": diff.mean,
            "rows": {"lam_base": lam0, "exit_base": ex0, "lam": lam1, "exit": ex1}}
