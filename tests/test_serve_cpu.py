"""Host side of the serving loop: request stream generators and the latency summary."""
import numpy as np

import mlmc_inputs as mi
from paper_1907_10271_amd.serve import PLATE, STRIP, Request, summarize


def test_poisson_arrivals_rate_and_gaps():
    t = mi.poisson_arrivals(1000.0, 20.0, seed=3)
    assert np.all(np.diff(t) > 0) and t[-1] < 20.0
    assert abs(len(t) / 20.0 - 1000.0) < 4 * np.sqrt(1000.0 / 20.0) * 1.0 + 30
    gaps = np.diff(t)
    # exponential gaps: mean = sd = 1/rate
    assert abs(gaps.mean() - 1e-3) < 5e-5 and abs(gaps.std() - 1e-3) < 5e-5


def test_request_mix_shares():
    cfg = mi.load_config("serve_c5")
    cls = mi.request_mix(200000, 0, cfg["strip_share"], cfg["strip_level_weights"], cfg["plate_level_weights"])
    strip = cls[:, 0] == STRIP
    assert abs(strip.mean() - 0.7) < 0.005
    w = np.asarray(cfg["strip_level_weights"], float)
    got = np.bincount(cls[strip, 1], minlength=len(w)) / strip.sum()
    assert np.allclose(got, w / w.sum(), atol=0.005)
    w = np.asarray(cfg["plate_level_weights"], float)
    got = np.bincount(cls[~strip, 1], minlength=len(w)) / (~strip).sum()
    assert np.allclose(got, w / w.sum(), atol=0.005)
    assert cls[~strip, 1].max() < len(w)


def test_summarize_percentiles():
    reqs = []
    for i in range(100):
        r = Request(i, STRIP if i % 2 else PLATE, 0, i, t_arrive=10.0 + 0.01 * i)
        r.t_done = r.t_arrive + (i + 1) * 1e-3
        r.status, r.batch = 0, i // 10
        reqs.append(r)
    st = summarize(reqs, 10.0, 0.0, 123, rate=100.0)
    lat = np.arange(1, 101, dtype=float)
    assert st.requests == 100 and st.failed == 0 and st.max_inflight_bytes == 123
    assert abs(st.p50_ms - np.percentile(lat, 50)) < 1e-9
    assert abs(st.p99_ms - np.percentile(lat, 99)) < 1e-9
    assert st.mean_batch == 10.0
    assert set(st.per_class) == {"strip0", "plate0"}
    # warm-up exclusion
    st2 = summarize(reqs, 10.0, 0.5, 0, rate=100.0)
    assert st2.requests == 50


def _policy_server(workers=4, long_workers=1):
    """A server object with only the queueing state (no contexts), to test the policy."""
    import threading
    from collections import deque
    from paper_1907_10271_amd.serve import Server
    s = Server.__new__(Server)
    s.queues, s.cv = {}, threading.Condition()
    s.inflight = s.max_inflight = s.n_batches = 0
    s.long_from = {STRIP: 4, PLATE: 2}
    s.workers, s.n_long_workers = workers, long_workers
    s.footprint = {(k, l): 1 for k in (STRIP, PLATE) for l in range(5)}
    s.cap = {(k, l): 3 for k in (STRIP, PLATE) for l in range(5)}
    s.queues = {}
    for key, times in {(STRIP, 0): [2.0, 3.0, 4.0, 5.0], (PLATE, 3): [1.0], (STRIP, 4): [1.5]}.items():
        s.queues[key] = deque(Request(i, key[0], key[1], i, t_arrive=t) for i, t in enumerate(times))
    return s


def test_short_workers_never_take_long_classes():
    s = _policy_server()
    b = s._take(0)                                   # a short worker: oldest short queue, capped at 3
    assert [(r.kind, r.level) for r in b] == [(STRIP, 0)] * 3
    b = s._take(1)
    assert [(r.kind, r.level) for r in b] == [(STRIP, 0)]
    assert s._take(2) is None                        # only long work is left
    b = s._take(3)                                   # the long worker: oldest long queue first
    assert [(r.kind, r.level) for r in b] == [(PLATE, 3)]
    b = s._take(3)
    assert [(r.kind, r.level) for r in b] == [(STRIP, 4)]
    assert s._take(3) is None


def test_long_worker_takes_short_work_when_no_long_work_waits():
    s = _policy_server()
    s.queues[(PLATE, 3)].clear()
    s.queues[(STRIP, 4)].clear()
    b = s._take(3)
    assert [(r.kind, r.level) for r in b] == [(STRIP, 0)] * 3
    # without long workers every worker takes the oldest queue of any class
    s = _policy_server(long_workers=0)
    s.n_long_workers = 0
    b = s._take(0)
    assert [(r.kind, r.level) for r in b] == [(PLATE, 3)]
