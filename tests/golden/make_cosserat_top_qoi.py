#!/usr/bin/env python3
"""Write ``cosserat_top_qoi.json``: the oracle's strength QoI (Eq.
failureCriterion) of rows 0 and 1 of level 5 of the Cosserat workload
(256 x 256 elements, 198k unknowns, 300 KL terms: the paper's finest Test I
mesh), from the oracle's sparse direct solve.  Only ``oracle/`` and the
seeded input module are used.  Run from the repository root:
``python tests/golden/make_cosserat_top_qoi.py`` (a few minutes).
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mlmc_inputs as mi  # noqa: E402
from oracle.cosserat import CosseratModel  # noqa: E402

LEVEL, ROWS = 5, [0, 1]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cosserat_top_qoi.json")


def main():
    cfg = mi.load_config("cosserat_t1")
    model = CosseratModel(cfg, LEVEL)
    xi = mi.strip_xi(cfg, LEVEL, 0, max(ROWS) + 1)
    q = []
    for r in ROWS:
        s = model.solve(xi[r], method="direct")
        print(f"row {r}: q = {s.q!r} (true relative residual {s.true_relres:.2e})", flush=True)
        q.append(s.q)
    doc = {"config": "cosserat_t1", "level": LEVEL, "rows": ROWS, "q": q,
           "source": "oracle.cosserat.CosseratModel.solve(method='direct') (scipy splu)"}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
