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
