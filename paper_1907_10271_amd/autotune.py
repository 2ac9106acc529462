"""Autotuner of the strip solver's per-level choices.

For every mesh of the given strip workloads it times, on the current GPU, each
combination of

* engine: ``small`` (one work-group solves a whole sample, PCG state on chip;
  only where it fits) or ``lockstep`` (all samples of a batch iterate together
  through the column-sweep operator pass and the vector pass), and
* angle storage: ``theta`` (angle codes tan theta, cos/sin 2theta formed
  every iteration) or ``cs`` (stored cos/sin 2theta pairs, twice the bytes),

on a batch of uncoupled samples sized to fill the GPU, and keeps the fastest;
for lock-step meshes it then times the operator pass's tile height (4, 8, 12
or 16 node rows against the library's per-launch choice, which follows the
number of waves in flight) on that batch and on one twice as large, and fixes
a height only where one beats the per-launch choice by more than 1% on both.
The result, keyed by mesh (``"NXxNY"``), is written as JSON; contexts created
through the Python binding apply it as ``level_options`` unless the workload
definition has its own.  Every choice is fixed per mesh, never per batch, so a
sample's result does not depend on the batch it rides in; the angle storage
does not change results at all, the engine changes them at rounding level.

Usage: ``python -m paper_1907_10271_amd.autotune [--out FILE] [strip workload ...]``
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "mi355x.json")


def batch_size(nnode: int) -> int:
    """Samples per timed batch: about two million nodes, within 32..4096."""
    return int(min(4096, max(32, round(2.0e6 / nnode))))


def tune(workloads, reps: int = 2, log=print) -> dict:
    import torch

    import mlmc_inputs as mi
    from ._lib import Context
    out = {}
    for name in workloads:
        cfg = mi.load_config(name)
        for level in range(cfg["n_levels"]):
            nx, ny = cfg["nx0"] << level, cfg["ny0"] << level
            key = f"{nx}x{ny}"
            if key in out:
                continue
            nnode = (nx + 1) * (ny + 1)
            n = batch_size(nnode)
            xi = torch.from_numpy(mi.strip_xi(cfg, level, 0, n)).to("cuda")
            reqs = [(k, level, False) for k in range(n)]
            times = {}
            for engine in ("small", "lockstep"):
                for angles in ("theta", "cs"):
                    opts = {key: {"engine": engine, "angles": angles}}
                    ctx = Context(dict(cfg, level_options=opts))
                    if engine == "small" and ctx.level_info(level)["n_nodes"] and not _uses_small(ctx, level, xi):
                        ctx.close()
                        continue
                    ctx.solve_batch(reqs, xi)          # warm-up and pool allocation
                    torch.cuda.synchronize()
                    best = float("inf")
                    for _ in range(reps):
                        t0 = time.perf_counter()
                        ctx.solve_batch(reqs, xi)
                        torch.cuda.synchronize()
                        best = min(best, time.perf_counter() - t0)
                    ctx.close()
                    times[f"{engine}/{angles}"] = round(best * 1e3, 3)
                    log(f"{key}: {engine}/{angles} {n} samples {best * 1e3:.2f} ms")
            pick = min(times, key=times.get)
            engine, angles = pick.split("/")
            rows, rows_ms = 0, {}
            if engine == "lockstep":
                # two batch sizes: a height is fixed for the mesh only if it beats
                # the per-launch choice (which follows the batch) at both
                xi2 = torch.from_numpy(mi.strip_xi(cfg, level, 0, 2 * n)).to("cuda")
                for nb, x in ((n, xi), (2 * n, xi2)):
                    r2 = [(k, level, False) for k in range(nb)]
                    for ty in (0, 4, 8, 12, 16):
                        ctx = Context(dict(cfg, level_options={key: {"engine": engine, "angles": angles,
                                                                     "sweep_rows": ty}}))
                        ctx.solve_batch(r2, x)
                        torch.cuda.synchronize()
                        best = float("inf")
                        for _ in range(reps):
                            t0 = time.perf_counter()
                            ctx.solve_batch(r2, x)
                            torch.cuda.synchronize()
                            best = min(best, time.perf_counter() - t0)
                        ctx.close()
                        rows_ms.setdefault(ty, []).append(round(best * 1e3, 3))
                        log(f"{key}: {nb} samples, tile height {ty or 'per launch'} {best * 1e3:.2f} ms")
                wins = [t for t in rows_ms if t and all(a < 0.99 * b for a, b in zip(rows_ms[t], rows_ms[0]))]
                if wins:
                    rows = min(wins, key=lambda t: sum(rows_ms[t]))
            out[key] = {"engine": engine, "angles": angles, "batch": n, "ms": times, "sweep_rows": rows,
                        "sweep_rows_ms": {str(t): v for t, v in rows_ms.items()}}
            log(f"{key}: chose {pick}, tile height {rows or 'per launch'}")
    return out


def _uses_small(ctx, level, xi) -> bool:
    """Whether the context solves this level with the whole-solve kernel (no
    lock-step operator-pass launches)."""
    import torch
    ctx.profile(True)
    ctx.solve_batch([(0, level, False)], xi[:1])
    torch.cuda.synchronize()
    used = ctx.profile_read(0)["launches"] == 0
    ctx.profile(False)
    return used


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("workloads", nargs="*", default=["strip_c1", "strip_c3"])
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--reps", type=int, default=2)
    a = ap.parse_args(argv)
    res = tune(a.workloads, a.reps, log=lambda m: print(m, file=sys.stderr, flush=True))
    doc = {"device": _device_name(), "choices": res}
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    print(json.dumps(doc))
    return 0


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0)


if __name__ == "__main__":
    sys.exit(main())
