"""Pilot that fixes the failure threshold lambda* of the panel workload.

The panel workload asks for a threshold with failure probability about
1/150 (the rare-event regime of Section 4.3).  This script takes the
empirical quantile of the level-0 buckling load over a fixed-seed pilot
sample (the oracle's sparse eigen-solve, one process per core) and scales
it by the ratio of the pristine loads on the finest and the coarsest level,
so the threshold refers to the finest discretisation.  The result is written
to ``tests/golden/lambda_crit.json`` (``lambda_crit_<workload>.json`` for a
panel workload other than the 500 mm one) and to the workload definition.

Run: ``python -m oracle.pilot_lambda_crit [n_samples] [workload]`` (oracle only).
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import mlmc_inputs as mi  # noqa: E402
from oracle.plate import PlateModel  # noqa: E402

PILOT_STREAM = 7  # stream index of the pilot draws (levels use 0..n_levels-1)
_M = None


def _solve(row):
    return _M.buckling_load(row)


def main(n: int = 6000, name: str = "plate_c4") -> dict:
    global _M
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    cfg = mi.load_config(name)
    _M = PlateModel(cfg, 0)
    rows = mi.plate_offsets(cfg, 0, 0, n, stream=PILOT_STREAM)
    t0 = time.time()
    with mp.get_context("fork").Pool(min(len(os.sched_getaffinity(0)), 16)) as pool:
        lam0 = np.array(pool.map(_solve, list(rows), chunksize=16))
    q = float(np.quantile(lam0, cfg["p_target"]))
    top = cfg["n_levels"] - 1
    pristine = [PlateModel(cfg, l).buckling_load(np.zeros(len(cfg["layup_deg"]))) for l in (0, top)]
    lam_crit = q * pristine[1] / pristine[0]
    out = {"lambda_crit": lam_crit, "level0_quantile": q, "p_target": cfg["p_target"], "n_pilot": n,
           "pristine_level0": pristine[0], "pristine_top": pristine[1], "pilot_stream": PILOT_STREAM,
           "level0_mean": float(lam0.mean()), "level0_std": float(lam0.std()), "seconds": time.time() - t0,
           "source": "oracle/pilot_lambda_crit.py"}
    gold = "lambda_crit.json" if name == "plate_c4" else f"lambda_crit_{name}.json"
    out["workload"] = name
    with open(os.path.join(ROOT, "tests", "golden", gold), "w") as f:
        json.dump(out, f, indent=1)
    path = mi.config_path(name)
    c = json.load(open(path))
    c["lambda_crit"] = lam_crit
    c["lambda_crit_source"] = "oracle/pilot_lambda_crit.py (level-0 quantile x pristine top/level-0 ratio)"
    with open(path, "w") as f:
        json.dump(c, f, indent=2)
        f.write("\n")
    return out


if __name__ == "__main__":
    print(json.dumps(main(int(sys.argv[1]) if len(sys.argv) > 1 else 6000,
                          sys.argv[2] if len(sys.argv) > 2 else "plate_c4"), indent=1))
