#!/usr/bin/env python3
"""Write ``rare_event_plate_c4.json``: the oracle's buckling loads behind the
two-level rare-event test (Section 4.3, estimator ``Qhat_j + Yhat_{L,j}``).

Rows: the first ``N0`` ply-offset rows of stream 100 (base term) at levels 0
and 1, and the first ``N1`` rows of stream 101 (difference term) at levels
0 .. L, all of the 500 mm panel workload.  Only ``oracle/`` and the seeded
input module are used; the loads come from the oracle's shift-invert
eigensolver.  Run from the repository root:
``python tests/golden/make_rare_event_lambdas.py`` (about a minute on 8 cores).
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mlmc_inputs as mi  # noqa: E402
from oracle.plate import PlateModel  # noqa: E402

CONFIG, N0, N1, L = "plate_c4", 256, 64, 2
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rare_event_plate_c4.json")


def loads(args):
    stream, row, levels = args
    cfg = mi.load_config(CONFIG)
    off = mi.plate_offsets(cfg, 0, row, 1, stream=stream)[0]
    return [float(PlateModel(cfg, l).buckling_load(off)) for l in levels]


def main():
    jobs = [(100, r, [0, 1]) for r in range(N0)] + [(101, r, list(range(L + 1))) for r in range(N1)]
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        res = list(ex.map(loads, jobs, chunksize=4))
    doc = {"config": CONFIG, "L": L, "n0": N0, "n1": N1,
           "source": "oracle.plate.PlateModel.buckling_load (scipy eigsh, shift-invert with a sparse LU of K)",
           "base_stream": 100, "chain_stream": 101,
           "lam_base": res[:N0], "lam_chain": res[N0:]}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
