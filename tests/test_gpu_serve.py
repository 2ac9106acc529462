"""Serving loop on the GPU: every request's result is the same alone and in
the mix (the library is batch-invariant, so the comparison is exact), batches
respect the reserved slots, and batches of different workers overlap."""
import numpy as np
import pytest

import mlmc_inputs as mi

pytestmark = pytest.mark.gpu


def _alone(ctxs, cfgs, r, precision):
    from paper_1907_10271_amd.serve import STRIP
    import torch
    gen = mi.strip_xi if r.kind == STRIP else mi.plate_offsets
    x = torch.from_numpy(gen(cfgs[r.kind], r.level, r.sample, 1)).to("cuda:0")
    req = [(0, r.level, r.level > 0)]
    if r.kind == STRIP:
        qf, qc, info = ctxs[r.kind].solve_batch(req, x, precision=precision)
    else:
        qf, qc, info = ctxs[r.kind].buckle_batch(req, x, precision=precision)
    return float(qf.cpu()[0]), float(qc.cpu()[0])


@pytest.mark.parametrize("precision", [0, 1])
def test_serve_same_alone_and_in_mix(precision):
    import paper_1907_10271_amd as pk
    from paper_1907_10271_amd.serve import PLATE, STRIP, Server
    strip_cfg, plate_cfg = mi.load_config("strip_c1"), mi.load_config("plate_c4")
    cfgs = {STRIP: strip_cfg, PLATE: plate_cfg}
    n = 160
    g = np.random.default_rng(5)
    kinds = (g.random(n) < 0.3).astype(int)
    levels = np.where(kinds == STRIP, g.integers(0, 2, n), g.integers(0, 2, n))
    classes = np.stack([kinds, levels], axis=1)
    arrivals = np.sort(g.uniform(0.0, 0.25, n))
    with Server(strip_cfg, plate_cfg, precision=precision, workers=3, max_batch=32,
                mem_budget_bytes=6 << 30, n_levels={PLATE: 2}) as srv:
        cap = dict(srv.cap)
        stats, reqs = srv.run_stream(arrivals, classes)
    print(f"precision {precision}: {stats.requests} requests, mean batch {stats.mean_batch:.1f}, "
          f"p50 {stats.p50_ms:.1f} ms p99 {stats.p99_ms:.1f} ms", flush=True)
    assert stats.failed == 0
    assert all(r.status == 0 for r in reqs)
    # admission: no batch holds more requests of a class than a worker reserved
    sizes = {}
    for r in reqs:
        sizes.setdefault(r.batch, []).append((r.kind, r.level))
    for b, members in sizes.items():
        assert len(set(members)) == 1
        assert len(members) <= cap[members[0]]
    assert max(len(m) for m in sizes.values()) > 1
    # batches of different workers were in flight at the same time
    spans = {}
    for r in reqs:
        spans[r.batch] = (r.worker, r.t_start, r.t_done)
    sp = sorted(spans.values(), key=lambda v: v[1])
    overlap = any(a[0] != b[0] and b[1] < a[2] for i, a in enumerate(sp) for b in sp[i + 1:])
    assert overlap
    # same answers alone
    ctxs = {STRIP: pk.Context(strip_cfg), PLATE: pk.Context(plate_cfg)}
    for r in reqs:
        qf, qc = _alone(ctxs, cfgs, r, precision)
        assert qf == r.q_fine, (r, qf)
        if r.level > 0:
            assert qc == r.q_coarse, (r, qc)
    for c in ctxs.values():
        c.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_serve_long_classes_same_alone_and_in_mix(precision):
    """The serving workload's own classes, long ones included (strip levels
    0..4 up to 1024x256 on the five-level waviness strip, panels 16² .. 64²),
    with the serving configuration's long-class worker: every result is
    bit-identical alone and in the mix."""
    import paper_1907_10271_amd as pk
    from paper_1907_10271_amd.serve import PLATE, STRIP, Server
    scfg = mi.load_config("serve_c5")
    strip_cfg, plate_cfg = mi.load_config(scfg["strip_config"]), mi.load_config(scfg["plate_config"])
    cfgs = {STRIP: strip_cfg, PLATE: plate_cfg}
    g = np.random.default_rng(17)
    # every class at least once (the long ones exactly twice), short ones filling up the stream
    classes = [(STRIP, l) for l in range(5)] + [(PLATE, l) for l in range(3)] + [(STRIP, 4), (PLATE, 2)]
    classes += [(STRIP, int(l)) for l in g.integers(0, 3, 30)] + [(PLATE, int(l)) for l in g.integers(0, 2, 12)]
    classes = np.array(classes)[g.permutation(len(classes))]
    arrivals = np.sort(g.uniform(0.0, 0.4, len(classes)))
    long_from = {STRIP: scfg["long_from"]["strip"], PLATE: scfg["long_from"]["plate"]}
    with Server(strip_cfg, plate_cfg, precision=precision, workers=3, max_batch=64, mem_budget_bytes=24 << 30,
                n_levels={PLATE: 3}, long_from=long_from, long_workers=scfg["long_workers"]) as srv:
        stats, reqs = srv.run_stream(arrivals, classes)
    print(f"precision {precision}: {stats.requests} requests, mean batch {stats.mean_batch:.1f}, "
          f"p50 {stats.p50_ms:.1f} ms p99 {stats.p99_ms:.1f} ms", flush=True)
    assert stats.failed == 0 and all(r.status == 0 for r in reqs)
    assert {(r.kind, r.level) for r in reqs} == {tuple(c) for c in classes}
    # long classes ran on the long-class worker only
    long_workers = {r.worker for r in reqs if (r.kind, r.level) in {(STRIP, 4), (PLATE, 2)}}
    assert len(long_workers) == 1
    ctxs = {STRIP: pk.Context(strip_cfg), PLATE: pk.Context(plate_cfg)}
    for r in reqs:
        qf, qc = _alone(ctxs, cfgs, r, precision)
        assert qf == r.q_fine, (r.kind, r.level, r.sample, qf, r.q_fine)
        if r.level > 0:
            assert qc == r.q_coarse, (r.kind, r.level, r.sample, qc, r.q_coarse)
    for c in ctxs.values():
        c.close()
