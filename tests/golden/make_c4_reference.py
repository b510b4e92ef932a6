"""Writes c4_reference.json: the FP64 oracle's solve of every instance of the batched
workload (256 SBM graphs, n ~ U[500, 5000], k = r in {8, 16, 32}, 8 random starts each,
seed 1004 + g) for 20 outer iterations.  For each instance: whether the iteration broke
down (a factor collapsed to zero, so rho = ||P^T P||_2 = 0 for the next half-step), the
number of completed outer iterations, and the monitor record after the last of them; and
the same twice more with rounding-size changes of both factors after every outer
iteration: every entry of X in {W, Ht} plus eps max|X| u, u standard normal from
default_rng(7919 g + s), projected to >= 0, with eps = 2^-52 ("perturbed", the absolute
size of FP64 rounding in a sum) and eps = 2^-24 ("perturbed32", FP32).  These measure how
far each instance's own iteration carries rounding differences within 20 outer
iterations.  The change is additive on purpose: at the saddle points that these
instances approach (graphs below the detection threshold), whole columns of W and Ht are
exactly zero and their gradient columns vanish, so a relative change (x (1 + eps u))
leaves them dead, while a rounding-size entry revives them and the iteration leaves the
saddle, a thousandfold per outer iteration.  Calls only the CPU reference and the seeded
input generators.

    python tests/golden/make_c4_reference.py [workers]
"""
import json
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

OUTER = 20
_GRAPHS = None


def _run(A, W0, lam, rng=None, eps=0.0):
    import oracle as O
    prm = O.Params(lam=lam)
    W = np.array(W0, dtype=np.float64)
    Ht = W.copy()
    rec, done, broke = None, 0, False
    for _ in range(OUTER):
        try:
            W = O.half_step(A, W, Ht, prm)
            Ht = O.half_step(A, Ht, W, prm)
        except FloatingPointError:
            broke = True
            break
        done += 1
        rec = O.monitor(A, W, Ht, prm)
        if rng is not None:
            W = np.maximum(W + eps * np.abs(W).max() * rng.standard_normal(W.shape), 0.0)
            Ht = np.maximum(Ht + eps * np.abs(Ht).max() * rng.standard_normal(Ht.shape), 0.0)
    out = {"breakdown": broke, "outer": done}
    if rec is not None:
        out.update({k: rec[k] for k in ("res_WH", "res_WWt", "pg", "sym_gap", "objective")})
    return out


def _solve(job):
    g, s = job
    gr = _GRAPHS[g]
    A = gr["A"]
    lam = 0.01 * float(np.sqrt(np.sum(np.asarray(A.data, dtype=np.float64) ** 2)))
    W0 = np.asarray(gr["W0"][s], dtype=np.float64)
    out = {"g": g, "s": s, "n": int(gr["n"]), "r": int(gr["r"])}
    out.update(_run(A, W0, lam))
    out["perturbed"] = _run(A, W0, lam, np.random.default_rng(7919 * g + s), 2.0 ** -52)
    out["perturbed32"] = _run(A, W0, lam, np.random.default_rng(7919 * g + s), 2.0 ** -24)
    return out


def _init():
    global _GRAPHS
    from paper_2606_02887_amd import gen
    _GRAPHS = gen.config(4)


def main(workers=4):
    from paper_2606_02887_amd import gen
    graphs = gen.config(4)
    S = len(graphs[0]["W0"])
    jobs = [(g, s) for g in range(len(graphs)) for s in range(S)]
    with mp.Pool(workers, initializer=_init) as pool:
        res = pool.map(_solve, jobs, chunksize=8)
    out = {"workload": "256 SBM graphs, n ~ U[500,5000], k = r in {8,16,32}, 8 starts, seed 1004",
           "outer": OUTER, "lambda": "0.01 ||A_g||_F per graph", "instances": res}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_reference.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(path, sum(r["breakdown"] for r in res), "breakdowns")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 4)
