"""Writes c0_ensemble.json: the FP64 oracle's SNMPBB runs of the planted dense workload
n=500, r=10 (seed 1000) for 500 outer iterations, from the seeded W0 and from 31
rounding-level changes of it (every entry times 1 + 2^-24 u, u = +-1 drawn from
default_rng(seed), seeds 1..31: the size of change an FP32 copy of W0 makes).  Their
spread at the end is how far the iteration itself carries such differences, the
envelope a GPU solve of the same workload must land in.  Calls only the CPU reference
and the seeded input generators.

    python tests/golden/make_c0_ensemble.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2606_02887_amd import gen  # noqa: E402

OUTER = 500


def main():
    prob = gen.config(0)
    A, W0 = prob["A"], prob["W0"]
    lam = O.default_lambda(A)
    runs = []
    for seed in range(32):
        if seed == 0:
            W = W0
        else:
            u = np.random.default_rng(seed).choice([-1.0, 1.0], size=W0.shape)
            W = W0 * (1.0 + 2.0 ** -24 * u)
        _, _, hist = O.snmpbb(A, W, O.Params(lam=lam), OUTER)
        h = hist[-1]
        runs.append({"seed": seed, **{k: h[k] for k in ("res_WH", "res_WWt", "pg", "sym_gap",
                                                        "objective")}})
        print(runs[-1])
    out = {"workload": "planted dense n=500 r=10 seed 1000 (noise 0.01)", "outer": OUTER,
           "lambda": lam, "perturbation": "W0 * (1 + 2^-24 u), u = +-1 from default_rng(seed); "
                                           "seed 0 is W0 itself", "runs": runs}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c0_ensemble.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
