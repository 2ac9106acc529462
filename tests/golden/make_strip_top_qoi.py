"""Writes ``strip_c3_level4_qoi.json``: the oracle's quantity of interest for
two samples of the five-level strip workload's top level (1024x256 elements,
about 526k unknowns), by sparse direct solve of the assembled system, so the
GPU path can be compared with the oracle at that size without the minutes of
oracle set-up inside a test.  Calls only the oracle and the seeded input
generators.  Run: ``python tests/golden/make_strip_top_qoi.py`` (about 3 min).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import mlmc_inputs as mi  # noqa: E402
from oracle.kl import KL  # noqa: E402
from oracle.strip import StripModel  # noqa: E402

NAME, LEVEL, ROWS = "strip_c3", 4, (0, 5)


def main():
    cfg = mi.load_config(NAME)
    t0 = time.time()
    model = StripModel(cfg, LEVEL, KL(cfg))
    xi = mi.strip_xi(cfg, LEVEL, 0, max(ROWS) + 1)
    q = {str(r): model.solve(xi[r], method="direct").q for r in ROWS}
    out = {"workload": NAME, "level": LEVEL, "mesh": f"{cfg['nx0'] << LEVEL}x{cfg['ny0'] << LEVEL}",
           "rows": list(ROWS), "q": q, "method": "oracle sparse direct solve",
           "seconds": round(time.time() - t0, 1), "source": "tests/golden/make_strip_top_qoi.py"}
    with open(os.path.join(ROOT, "tests", "golden", "strip_c3_level4_qoi.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
