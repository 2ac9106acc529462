#!/usr/bin/env python3
"""At-scale check of the buckling solver against the oracle (not a pytest
module: it needs a GPU and minutes of oracle time).

Draws ``--n`` ply-offset rows of one level of a panel workload, solves them
on the GPU through the C ABI (default start and lowest-mode check) and with
the oracle's shift-invert eigensolver (``oracle.plate.PlateModel``, one
process per worker), and prints one JSON line: the largest relative
difference of lambda, how many samples differ by more than ``--rtol``, and
the GPU's status counts (``MLMC_S_NOTLOWEST`` = 5 marks a sample whose
eigen-solve stopped at a higher mode).  Exit status 1 if any sample fails.

    python tests/check_plate_at_scale.py --config plate_t2 --level 0 --n 2000 --workers 16
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import mlmc_inputs as mi  # noqa: E402


def _oracle_loads(args):
    name, level, start, n = args
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle.plate import PlateModel
    cfg = mi.load_config(name)
    model = PlateModel(cfg, level)
    return [float(model.buckling_load(r)) for r in mi.plate_offsets(cfg, level, start, n)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="plate_t2")
    ap.add_argument("--level", type=int, default=0)
    ap.add_argument("--n", type=int, default=2000)
    ap.add_argument("--start", type=int, default=0, help="first row of the level's stream")
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--precision", type=int, default=0)
    a = ap.parse_args()

    import torch
    import paper_1907_10271_amd as pk
    cfg = mi.load_config(a.config)
    ctx = pk.Context(mi.config_text(a.config))
    off = torch.from_numpy(mi.plate_offsets(cfg, a.level, a.start, a.n)).to("cuda")
    t0 = time.perf_counter()
    lam, _, info = ctx.buckle_batch([(k, a.level, False) for k in range(a.n)], off, precision=a.precision)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    lam = lam.cpu().numpy()
    print(f"gpu: {a.n} solves in {t_gpu:.2f} s", file=sys.stderr, flush=True)

    chunk = max(1, a.n // (4 * a.workers))
    jobs = [(a.config, a.level, a.start + s, min(chunk, a.n - s)) for s in range(0, a.n, chunk)]
    ref = []
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=a.workers) as ex:
        for k, part in enumerate(ex.map(_oracle_loads, jobs)):
            ref.extend(part)
            if k % 8 == 7:
                print(f"oracle: {len(ref)}/{a.n}", file=sys.stderr, flush=True)
    t_cpu = time.perf_counter() - t0
    ref = np.array(ref)
    rel = np.abs(lam - ref) / ref
    status = info["status_f"]
    bad = np.nonzero((rel > a.rtol) | (status != 0))[0]
    out = {"config": a.config, "level": a.level, "n": a.n, "start": a.start, "precision": a.precision,
           "max_rel_diff": float(rel.max()), "n_above_rtol": int(np.sum(rel > a.rtol)), "rtol": a.rtol,
           "status_counts": np.bincount(status, minlength=6).tolist(), "failing_rows": (a.start + bad).tolist()[:50],
           "gpu_s": round(t_gpu, 2), "oracle_s": round(t_cpu, 1), "workers": a.workers}
    print(json.dumps(out))
    return 1 if len(bad) else 0


if __name__ == "__main__":
    sys.exit(main())
