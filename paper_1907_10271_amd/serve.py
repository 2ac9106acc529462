"""Serving loop: continuous micro-batching of sample-solve requests.

A request is one MLMC sample of a given kind and level (a coupled fine and
coarse pair above level 0): a waviness strip solve or a panel buckling solve.
Requests enter per-(kind, level) FIFO queues as they arrive.  A pool of
workers, each with its own library contexts and its own HIP stream, shares
the device memory budget: at start-up every worker reserves, for every level
of both models, as many request slots as its share of the budget holds
(``mlmc_footprint`` bytes per request, ``mlmc_reserve``), so that serving
itself allocates nothing.  A free worker takes the queue whose head has
waited longest and admits as many of its requests as it has slots for that
level.  Classes whose solves take long (fine strip levels, large panels:
``long_from`` gives the first long level per model) go only to the last
``long_workers`` workers, which also take short work when no long work
waits; a multi-second panel batch therefore never holds up a short request.
Batches of different workers overlap on the GPU, and requests that arrive
meanwhile join the next batch of their queue, so the GPU never waits for a
batch to fill.  Mode tables, level geometry and the solver pools stay
resident in the contexts; only a request's parameter row travels to the
device, where its field is synthesised.

A sample's result does not depend on the batch it rides in (every reduction
has a fixed order per sample), so a request gives the same answer alone and
in the mix.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from ._lib import FP64, Context

STRIP, PLATE = 0, 1
KIND_NAME = {STRIP: "strip", PLATE: "plate"}


@dataclass
class Request:
    rid: int
    kind: int
    level: int
    sample: int           # row index in the (kind, level) parameter stream
    t_arrive: float = 0.0
    t_start: float = 0.0
    t_done: float = 0.0
    q_fine: float = float("nan")
    q_coarse: float = float("nan")
    status: int = -1
    batch: int = -1
    worker: int = -1


@dataclass
class ServeStats:
    rate: float
    requests: int
    seconds: float
    throughput: float
    p50_ms: float
    p99_ms: float
    mean_batch: float
    max_inflight_bytes: int
    failed: int
    per_class: Dict[str, dict] = field(default_factory=dict)


class Server:
    """Worker pool over one GPU; see the module docstring for the policy."""

    def __init__(self, strip_cfg: dict, plate_cfg: dict, precision: int = FP64, workers: int = 4,
                 max_batch: int = 512, mem_budget_bytes: int = 64 << 30,
                 n_levels: Optional[Dict[int, int]] = None, long_from: Optional[Dict[int, int]] = None,
                 long_workers: int = 0):
        import torch
        import mlmc_inputs
        self.torch, self.inputs = torch, mlmc_inputs
        if not torch.cuda.is_available():
            raise RuntimeError("the serving loop needs a GPU")
        self.cfg = {STRIP: strip_cfg, PLATE: plate_cfg}
        self.precision = precision
        self.max_batch = max_batch
        self.budget = mem_budget_bytes
        self.inflight = 0
        self.max_inflight = 0
        self.cv = threading.Condition()
        self.queues: Dict[Tuple[int, int], deque] = {}
        self.n_done = 0
        self.n_batches = 0
        self.stop = False
        self.errors: List[BaseException] = []
        self.long_from = dict(long_from or {})
        self.n_long_workers = min(max(long_workers, 0), workers - 1) if self.long_from else 0
        self.workers = workers
        # the budget is split evenly over workers, the two models and their
        # levels; every pool is allocated now, so serving allocates nothing
        per_ctx = mem_budget_bytes // max(workers, 1) // 2
        self.ctx = [{STRIP: Context(strip_cfg, per_ctx), PLATE: Context(plate_cfg, per_ctx)}
                    for _ in range(workers)]
        self.streams = [torch.cuda.Stream() for _ in range(workers)]
        self.footprint, self.cap = {}, {}
        self.n_levels = {}
        for k in (STRIP, PLATE):
            nlev = self.ctx[0][k].n_levels
            if n_levels and k in n_levels:
                nlev = min(nlev, n_levels[k])     # serve only the coarsest nlev levels
            self.n_levels[k] = nlev
            for l in range(nlev):
                fp = self.ctx[0][k].footprint(k, l, precision)
                self.footprint[(k, l)] = fp
                self.cap[(k, l)] = int(max(1, min(max_batch, int(0.85 * per_ctx / nlev) // max(fp, 1))))
        for c in self.ctx:
            for (k, l), n in self.cap.items():
                c[k].reserve(l, n, precision)
        self.threads = [threading.Thread(target=self._work, args=(w,), daemon=True) for w in range(workers)]
        for t in self.threads:
            t.start()

    # ------------------------------------------------------------ queueing
    def submit(self, reqs: List[Request]) -> None:
        with self.cv:
            for r in reqs:
                if r.kind not in (STRIP, PLATE) or not 0 <= r.level < self.n_levels[r.kind]:
                    raise ValueError(f"bad request kind/level {r.kind}/{r.level}")
                self.queues.setdefault((r.kind, r.level), deque()).append(r)
            self.cv.notify_all()

    def is_long(self, key: Tuple[int, int]) -> bool:
        first = self.long_from.get(key[0])
        return first is not None and key[1] >= first

    def _take(self, w: int) -> Optional[List[Request]]:
        """For worker w: the queue whose head waited longest among the classes
        the worker serves (long-class workers prefer long classes); as many of
        its requests as the worker's reserved slots of that level hold."""
        long_worker = w >= self.workers - self.n_long_workers
        best, t_best = None, None
        for want_long in ((True, False) if long_worker else (False,)):
            for key, q in self.queues.items():
                if not q or (self.n_long_workers and self.is_long(key) != want_long):
                    continue
                if t_best is None or q[0].t_arrive < t_best:
                    best, t_best = key, q[0].t_arrive
            if best is not None:
                break
        if best is None:
            return None
        q = self.queues[best]
        per = max(self.footprint[best], 1)
        n = min(len(q), self.cap[best])
        batch = [q.popleft() for _ in range(n)]
        self.inflight += n * per
        self.max_inflight = max(self.max_inflight, self.inflight)
        self.n_batches += 1
        for r in batch:
            r.batch = self.n_batches
        return batch

    def _work(self, w: int) -> None:
        self.torch.cuda.set_device(0)
        while True:
            with self.cv:
                batch = self._take(w)
                while batch is None and not self.stop:
                    self.cv.wait()
                    batch = self._take(w)
                if batch is None:
                    return
            key = (batch[0].kind, batch[0].level)
            try:
                self._run(w, batch)
            except BaseException as e:   # surfaced by wait()
                self.errors.append(e)
                for r in batch:
                    r.status = -2
            finally:
                with self.cv:
                    self.inflight -= len(batch) * max(self.footprint[key], 1)
                    self.n_done += len(batch)
                    self.cv.notify_all()

    def _rows(self, kind: int, level: int, batch: List[Request]) -> np.ndarray:
        cfg, gen = self.cfg[kind], (self.inputs.strip_xi if kind == STRIP else self.inputs.plate_offsets)
        s = np.array([r.sample for r in batch])
        if np.all(np.diff(s) == 1):
            return gen(cfg, level, int(s[0]), len(s))
        return np.concatenate([gen(cfg, level, int(x), 1) for x in s])

    def _run(self, w: int, batch: List[Request]) -> None:
        torch = self.torch
        kind, level = batch[0].kind, batch[0].level
        t0 = time.perf_counter()
        rows = self._rows(kind, level, batch)
        ctx = self.ctx[w][kind]
        with torch.cuda.stream(self.streams[w]):
            x = torch.from_numpy(rows).to("cuda")
            reqs = [(k, level, level > 0) for k in range(len(batch))]
            if kind == STRIP:
                qf, qc, info = ctx.solve_batch(reqs, x, precision=self.precision)
            else:
                qf, qc, info = ctx.buckle_batch(reqs, x, precision=self.precision)
            qf, qc = qf.cpu().numpy(), qc.cpu().numpy()
        t1 = time.perf_counter()
        for k, r in enumerate(batch):
            r.q_fine, r.q_coarse = float(qf[k]), float(qc[k])
            st = int(info[k]["status_f"])
            r.status = st if (st != 0 or level == 0) else int(info[k]["status_c"])
            r.t_start, r.t_done, r.worker = t0, t1, w

    def wait(self, n_total: int) -> None:
        with self.cv:
            while self.n_done < n_total:
                self.cv.wait(0.05)
        if self.errors:
            raise self.errors[0]

    def close(self) -> None:
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()
        for c in self.ctx:
            for x in c.values():
                x.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------ streams
    def run_stream(self, arrivals: np.ndarray, classes: np.ndarray, first_sample: Optional[Dict] = None,
                   warmup_s: float = 0.0) -> Tuple[ServeStats, List[Request]]:
        """Replay an arrival stream in real time: ``arrivals`` (s from now, sorted),
        ``classes[i] = (kind, level)``.  Sample indices run on per class from
        ``first_sample`` (default 0).  Latency is completion minus arrival;
        requests that arrive before ``warmup_s`` are served but not counted."""
        counters = dict(first_sample or {})
        reqs = []
        for i, (k, l) in enumerate(classes):
            key = (int(k), int(l))
            reqs.append(Request(i, key[0], key[1], counters.get(key, 0)))
            counters[key] = counters.get(key, 0) + 1
        with self.cv:
            base = self.n_done
            self.max_inflight = self.inflight
        t0 = time.perf_counter()
        i, n = 0, len(reqs)
        while i < n:
            now = time.perf_counter() - t0
            j = i
            while j < n and arrivals[j] <= now:
                reqs[j].t_arrive = t0 + float(arrivals[j])
                j += 1
            if j > i:
                self.submit(reqs[i:j])
                i = j
            else:
                time.sleep(min(float(arrivals[i]) - now, 0.002))
        self.wait(base + n)
        rate = n / float(arrivals[-1]) if n and arrivals[-1] > 0 else float("inf")
        return summarize(reqs, t0, warmup_s, self.max_inflight, rate), reqs


def summarize(reqs: List[Request], t0: float, warmup_s: float, max_inflight: int, rate: float) -> ServeStats:
    sel = [r for r in reqs if r.t_arrive - t0 >= warmup_s]
    lat = np.array([r.t_done - r.t_arrive for r in sel]) * 1e3
    if sel:
        span = max(r.t_done for r in sel) - min(r.t_arrive for r in sel)
    else:
        span = float("nan")
    per: Dict[str, dict] = {}
    for key in sorted({(r.kind, r.level) for r in sel}):
        l = np.array([r.t_done - r.t_arrive for r in sel if (r.kind, r.level) == key]) * 1e3
        per[f"{KIND_NAME[key[0]]}{key[1]}"] = {"n": int(len(l)), "p50_ms": float(np.percentile(l, 50)),
                                               "p99_ms": float(np.percentile(l, 99))}
    nb = len({r.batch for r in reqs})
    return ServeStats(rate, len(sel), span, len(sel) / span if span and span > 0 else float("nan"),
                      float(np.percentile(lat, 50)) if len(lat) else float("nan"),
                      float(np.percentile(lat, 99)) if len(lat) else float("nan"),
                      len(reqs) / max(nb, 1), int(max_inflight),
                      sum(1 for r in reqs if r.status != 0), per)


def serve_sweep(serve_cfg: dict, precision: int = FP64, rates=None, duration_s: Optional[float] = None,
                max_requests: int = 40000, log=None) -> List[ServeStats]:
    """The request stream of a serving configuration at each arrival rate: Poisson
    arrivals, kinds and levels drawn from the configured mix."""
    import mlmc_inputs as mi
    strip_cfg = dict(mi.load_config(serve_cfg["strip_config"]), **serve_cfg.get("strip_overrides", {}))
    plate_cfg = dict(mi.load_config(serve_cfg["plate_config"]), **serve_cfg.get("plate_overrides", {}))
    rates = rates or serve_cfg["rates"]
    dur = duration_s or serve_cfg["duration_s"]
    out = []
    long_from = {STRIP: serve_cfg["long_from"]["strip"], PLATE: serve_cfg["long_from"]["plate"]} \
        if "long_from" in serve_cfg else None
    with Server(strip_cfg, plate_cfg, precision, serve_cfg["workers"], serve_cfg["max_batch"],
                int(serve_cfg["mem_budget_gib"] * (1 << 30)), long_from=long_from,
                long_workers=serve_cfg.get("long_workers", 0)) as srv:
        first: Dict[Tuple[int, int], int] = {}
        # warm every class once so the pools are allocated outside the measurement
        warm_cls = np.array([(k, l) for k in (STRIP, PLATE) for l in range(srv.n_levels[k])])
        srv.run_stream(np.zeros(len(warm_cls)), warm_cls, first)
        for key in map(tuple, warm_cls):
            first[key] = first.get(key, 0) + 1
        for i, rate in enumerate(rates):
            d = min(dur, max_requests / rate)
            t = mi.poisson_arrivals(rate, d, seed=i)
            cls = mi.request_mix(len(t), i, serve_cfg["strip_share"], serve_cfg["strip_level_weights"],
                                 serve_cfg["plate_level_weights"])
            st, reqs = srv.run_stream(t, cls, first, warmup_s=min(serve_cfg["warmup_s"], 0.2 * d))
            for r in reqs:
                first[(r.kind, r.level)] = max(first.get((r.kind, r.level), 0), r.sample + 1)
            if log:
                log(f"rate {rate:g}/s: {st.requests} req in {st.seconds:.2f} s -> {st.throughput:.0f}/s, "
                    f"p50 {st.p50_ms:.1f} ms p99 {st.p99_ms:.1f} ms, mean batch {st.mean_batch:.1f}, "
                    f"failed {st.failed}")
            out.append(st)
    return out
