"""Writes c1_reference.json: the FP64 oracle's SNMPBB run on the planted dense workload
n=8192, r=64 (seed 1001) for 2000 outer iterations from the seeded W0.  The residual
after the last iteration defines the time-to-target goal (1 + 1e-4) * res_ref of the
benchmark.  Calls only the CPU reference and the seeded input generators.

    python tests/golden/make_c1_reference.py [outer]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2606_02887_amd import gen  # noqa: E402


def main(outer=2000):
    prob = gen.config(1)
    A, W0 = prob["A"], prob["W0"]
    lam = O.default_lambda(A)
    t0 = time.time()
    _, _, hist = O.snmpbb(A, W0, O.Params(lam=lam), outer, monitor_every=10)
    out = {"workload": "planted dense n=8192 r=64 seed 1001 (noise 0.01)", "outer": outer,
           "lambda": lam, "res_ref": hist[-1]["res_WH"], "pg_ref": hist[-1]["pg"],
           "seconds": time.time() - t0,
           "history": [{k: h[k] for k in ("outer", "res_WH", "pg", "sym_gap")} for h in hist]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_reference.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["res_ref"], out["seconds"])


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2000)
