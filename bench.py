"""SNMPBB benchmark on one MI355X: outer iterations per second and time to target on the
planted dense workload n=8192, r=64 (A = W* W*^T + E, FP32), plain FP32 form vs the
split-BF16 form.

A "step" is one outer iteration of the method: a W-step and an H-step, each = Gram,
rho, the A-pass A P, the gradient, and 5 inner NMPBB iterations.  The timed region runs
exactly --steps outer iterations through the C ABI with A already resident in HBM.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, R = 8192, 64
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--target-outer", type=int, default=2000,
                    help="outer iterations that define the batch targets (and cap those runs)")
    ap.add_argument("--target-cap", type=int, default=4000,
                    help="iteration cap of the dense time-to-target runs (their target is the "
                         "FP64 reference after 2000 outer iterations, which the FP32 forms "
                         "reach a few dozen iterations later)")
    ap.add_argument("--no-target", action="store_true")
    ap.add_argument("--fuse-inner", type=int, choices=(0, 1), default=1,
                    help="single and NMF solves: one kernel per inner iteration (1) or two (0)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-outer", type=int, default=0,
                    help="outer iterations of the CPU-reference sample (0: pick ~15 s)")
    ap.add_argument("--workload", choices=("c1", "c2", "c3", "c4", "c4ws", "scale", "nmf"), default="c1",
                    help="c1: dense n=8192, r=64 (the headline line); c4: 256 SBM graphs, "
                         "8 restarts each, in one batched solve; c4ws: the learned warm start "
                         "(trained here) against random starts and the frame alone on c4; c2: "
                         "Graph-SNMPBB on an SBM graph n=20000, r=20 with its kNN Laplacian; "
                         "c3: LAI-SNMPBB on a rank-64 surrogate of a power-law graph n=200000, "
                         "r=32; scale: the sparse and low-rank A-pass kernels at n=2e6 (past "
                         "the caches) against the HBM roofline, beside a device copy; nmf: "
                         "NMPBB for rectangular NMF on a dense and a sparse V")
    ap.add_argument("--tuning-cache", default=None,
                    help="c4: JSON cache of the batch autotuner (default: the user cache)")
    ap.add_argument("--train-graphs", type=int, default=2048)
    ap.add_argument("--train-outer", type=int, default=300)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch-apass-only", action="store_true",
                    help="only the stacked split-BF16 A-pass of 8 batched restarts, 20 times "
                         "(for hardware counters)")
    ap.add_argument("--apass-only", action="store_true",
                    help="only a 256 MiB device copy (the counter scale reference) and 20 "
                         "A-pass launches of each form; for hardware-counter runs")
    return ap.parse_args()


def _cpu_baseline(A64, W0, lam, outer):
    """The FP64 CPU reference, timed on a bounded sample of the same workload."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    O.snmpbb(A64, W0, O.Params(lam=lam), 1)
    one = time.perf_counter() - t0
    if outer <= 0:
        outer = max(2, min(60, int(15.0 / max(one, 1e-3))))
    t0 = time.perf_counter()
    O.snmpbb(A64, W0, O.Params(lam=lam), outer)
    dt = time.perf_counter() - t0
    out = {"value": outer / dt, "unit": "outer iterations/s", "cores": int(threads),
           "kind": "oracle",
           "sample": f"{outer} outer iterations of the FP64 numpy reference on the same "
                     f"n={N}, r={R} workload ({dt:.1f} s)"}
    # the same reference on one thread (BLAS limited to one), one outer iteration
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            O.snmpbb(A64, W0, O.Params(lam=lam), 1)
            d1 = time.perf_counter() - t0
        out["single_thread"] = {"value": 1.0 / d1, "unit": "outer iterations/s", "cores": 1,
                                "sample": f"1 outer iteration on one thread ({d1:.1f} s)"}
    except Exception as e:  # pragma: no cover
        out["single_thread"] = {"error": str(e)}
    return out


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()
                        if i.get("user_api") == "blas"] or [1]))
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def _cpu_sample(run, unit_per_call, what, budget_s=10.0, cap=50):
    """The oracle timed on a bounded sample: run(k) performs k units of work (outer
    iterations, or instance outer iterations); one unit first sizes k to about budget_s."""
    t0 = time.perf_counter()
    run(1)
    one = time.perf_counter() - t0
    k = max(1, min(cap, int(budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    run(k)
    dt = time.perf_counter() - t0
    return {"value": k * unit_per_call / dt, "unit": "outer iterations/s" if unit_per_call == 1
            else "instance outer iterations/s", "cores": _blas_threads(), "kind": "oracle",
            "sample": f"{k} x {what} of the FP64 numpy reference ({dt:.1f} s)"}


COPY_BYTES = 256 << 20


def _apass_only(torch, S, A, W0, lam):
    """A plain copy of COPY_BYTES (its FETCH_SIZE / WRITE_SIZE calibrate the counters) and
    20 launches of each A-pass form, nothing else."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=A.device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    for prec in (S.F32, S.BF16X3):
        with S.Plan(S.dense(A), R, S.params(lam=lam, prec=prec, max_outer=1)) as pl:
            B = torch.empty_like(W0)
            for _ in range(20):
                pl.apass(W0, B)
            torch.cuda.synchronize()
    print(json.dumps({"apass_only": True, "copy_bytes": COPY_BYTES}))


def _batch_apass_only(torch, np, S, gen, A, A64):
    """A plain copy of COPY_BYTES (the counter calibration) and 21 launches of the stacked
    split-BF16 A-pass of 8 restarts (one untimed), nothing else."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=A.device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    rng = np.random.default_rng(1101)
    W0b = torch.from_numpy(np.stack([gen.start_factor(rng, N, R, float(A64.mean()))
                                     for _ in range(8)])).to(A.device, torch.float32)
    with S.Batch([S.dense(A)], [R], S.params(prec=S.BF16X3, max_outer=1), 8) as bt:
        ms = bt.time_apass(W0b.reshape(-1), 20)
    torch.cuda.synchronize()
    print(json.dumps({"batch_apass_only": True, "copy_bytes": COPY_BYTES,
                      "ms_split_and_product": ms}))


def _traffic(kernel_src, name):
    """HBM bytes per launch of `name` from the committed hardware-counter summary, or None
    if that summary is missing or was taken on a different kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "apass_c1_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    try:
        blob = json.loads(txt.split("```json")[1].split("```")[0])
    except (IndexError, ValueError):
        return None
    src = os.path.join(ROOT, "paper_2606_02887_amd", "csrc", kernel_src)
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if blob.get("source_sha256") != sha or name not in blob.get("kernels", {}):
        return None
    return blob["kernels"][name]["bytes_per_launch"]


def _bench_c4(a, torch, np, S, gen):
    """256 SBM graphs (n ~ U[500, 5000], r in {8, 16, 32}), 8 random starts each, solved
    together by the batching form in FP32.  value: instance outer iterations per second."""
    dev = torch.device("cuda:0")
    graphs = gen.config(4)
    restarts = len(graphs[0]["W0"])
    As = [S.csr_from_scipy(g["A"], torch.float32) for g in graphs]
    rs = [g["r"] for g in graphs]
    lams = [0.01 * float(np.sqrt(np.sum(g["A"].data.astype(np.float32).astype(np.float64) ** 2)))
            for g in graphs]
    W0s = [torch.from_numpy(np.stack(g["W0"])).to(dev, torch.float32).contiguous() for g in graphs]
    torch.cuda.synchronize()
    # launch shape of this batch from the autotuner (timed here unless cached)
    from paper_2606_02887_amd import autotune
    t0 = time.perf_counter()
    tune_log = []
    tuning, cached = autotune.tune(S, torch, As, rs, restarts, W0s, S.F32, lam=lams,
                                   cache_path=a.tuning_cache, log=tune_log)
    t_tune = time.perf_counter() - t0
    steps = a.steps
    with S.Batch(As, rs, S.params(prec=S.F32, max_outer=steps, check_every=1 << 30,
                                  tuning=tuning), restarts, lam=lams) as b:
        b.solve(W0s)                                   # graph capture + warm clocks
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, infos, _ = b.solve(W0s)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ninst = b.ninst
        elements = b.elements
    out = {"metric": "batched SNMPBB instance outer iterations/s (256 SBM graphs x 8 restarts)",
           "value": ninst * steps / el, "unit": "instance outer iterations/s", "n_gpus": 1,
           "steps": steps, "warmup": steps, "ms_per_step": 1e3 * el / steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "256 SBM graphs, n ~ U[500,5000], r in {8,16,32}, seed 1004",
                      "instances": ninst, "restarts": restarts,
                      "sum_n": int(sum(g["n"] for g in graphs)),
                      "sum_nnz": int(sum(g["A"].nnz for g in graphs)),
                      "elements_per_buffer": int(elements), "parallelism": "single GPU"},
           "tuning": {"config": tuning, "from_cache": cached, "seconds": t_tune,
                      "candidates": tune_log}}
    if not a.no_target:
        # tau_g = (1 + 1e-4) x best final residual over the graph's restarts after
        # target_outer iterations; time to target = when its best restart first meets it
        T = a.target_outer
        with S.Batch(As, rs, S.params(prec=S.F32, max_outer=T, check_every=1 << 30,
                                      tuning=tuning), restarts, lam=lams) as b:
            _, _, infos, tr = b.solve(W0s, trace=True)
        hz = S.clock_rate_hz()
        tts, its, frac, broken, no_valid = [], [], [], 0, 0
        for g in range(len(graphs)):
            valid = []
            for s_ in range(restarts):
                i = g * restarts + s_
                if infos[i]["status"] != 0 or infos[i]["outer"] < 1:
                    broken += 1
                    continue
                k = infos[i]["outer"]
                valid.append((tr[i, :k, 0], tr[i, :k, 5]))
            if not valid:
                no_valid += 1
                continue
            tau = (1 + 1e-4) * min(r_[-1] for r_, _ in valid)
            firsts = []
            for r_, t_ in valid:
                hit = np.nonzero(r_ <= tau)[0]
                firsts.append((int(hit[0]), t_[hit[0]]) if hit.size else None)
            ok = [f for f in firsts if f is not None]
            frac.append(len(ok) / restarts)
            best = min(ok)
            its.append(best[0] + 1)
            tts.append(best[1] / hz)
        out["time_to_target"] = {
            "rule": f"tau_g = (1 + 1e-4) x best restart residual after {T} outer iterations",
            "median_seconds": float(np.median(tts)), "max_seconds": float(np.max(tts)),
            "median_outer": float(np.median(its)),
            "fraction_of_restarts_reaching": float(np.mean(frac)),
            "restarts_broken_down": broken, "graphs_without_a_valid_restart": no_valid}
    out["instances_broken_down"] = int(sum(i["status"] != 0 for i in infos))
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = _c4_cpu(np, graphs, lams)
    print(json.dumps(out))


def _c4_cpu(np, graphs, lams, count=16):
    """The oracle on a sample of the batch: the first start of the first `count` graphs,
    solved one after another (instance outer iterations per second)."""
    import oracle as O
    As = [g["A"].astype(np.float32).astype(np.float64) for g in graphs[:count]]
    W0 = [np.asarray(g["W0"][0], dtype=np.float64) for g in graphs[:count]]

    def run(k):
        for A, w, lam in zip(As, W0, lams[:count]):
            O.snmpbb(A, w, O.Params(lam=lam), k)
    return _cpu_sample(run, count, f"outer iterations of {count} instances (the first start of "
                       f"the first {count} graphs)")


def _arm_stats(np, graphs, restarts, infos, tr, hz, taus, extra_s=0.0):
    its, secs, reached, frac = [], [], 0, []
    for g in range(len(graphs)):
        best, nhit = None, 0
        for s_ in range(restarts):
            i = g * restarts + s_
            if infos[i]["status"] != 0 or infos[i]["outer"] < 1:
                continue
            k = infos[i]["outer"]
            hit = np.nonzero(tr[i, :k, 0] <= taus[g])[0]
            if hit.size:
                nhit += 1
                cand = (int(hit[0]), tr[i, hit[0], 5] / hz)
                best = cand if best is None or cand < best else best
        frac.append(nhit / restarts)
        if best is not None:
            reached += 1
            its.append(best[0] + 1)
            secs.append(best[1] + extra_s)
    return {"graphs_reaching": reached, "median_outer": float(np.median(its)) if its else None,
            "mean_outer": float(np.mean(its)) if its else None,
            "median_seconds": float(np.median(secs)) if secs else None,
            "fraction_of_starts_reaching": float(np.mean(frac))}


def _bench_c4ws(a, torch, np, S, gen):
    """Learned warm start on the 256-graph workload: train the per-rank networks on
    separately seeded graphs, then time-to-target of random, frame-only and learned starts
    (8 starts per graph each).  tau_g = (1 + 1e-4) x best random-start residual."""
    from paper_2606_02887_amd import train_ws
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    train_graphs = gen.batched_sbm(num_graphs=a.train_graphs, restarts=1, seed=20000)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    pools = train_ws.training_pools(S, torch, train_graphs, outer=a.train_outer)
    torch.cuda.synchronize()
    t_pool = time.perf_counter() - t0
    log = []
    t0 = time.perf_counter()
    models = train_ws.train(S, torch, pools, epochs=a.epochs, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    graphs = gen.config(4)
    restarts = len(graphs[0]["W0"])
    As = [S.csr_from_scipy(g["A"], torch.float32) for g in graphs]
    rs = [g["r"] for g in graphs]
    lams = train_ws.lambdas(graphs)
    W0r = torch.from_numpy(np.concatenate([np.stack(g["W0"]).ravel() for g in graphs])).to(
        dev, torch.float32)
    T = a.target_outer
    hz = S.clock_rate_hz()
    out_arms = {}
    with S.Batch(As, rs, S.params(prec=S.F32, max_outer=T, check_every=1 << 30), restarts,
                 lam=lams) as b:
        Om = train_ws._sketch_buffer(torch, graphs, restarts, 9000, dev, torch.float32)
        b.warmstart([], Om)                                  # warm up (lazy scratch)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        W0s = b.warmstart([], Om)
        torch.cuda.synchronize()
        t_spa = time.perf_counter() - t1
        mlist = [models[r] for r in sorted(models)]
        t1 = time.perf_counter()
        W0l = b.warmstart(mlist, Om)
        torch.cuda.synchronize()
        t_ml = time.perf_counter() - t1
        runs = {}
        for arm, W in (("random", W0r), ("frame_only", W0s), ("learned", W0l)):
            _, _, infos, tr = b.solve(b.split(W), trace=True)
            runs[arm] = (infos, tr)
    infos, tr = runs["random"]
    taus = []
    for g in range(len(graphs)):
        fin = [tr[g * restarts + s_, infos[g * restarts + s_]["outer"] - 1, 0]
               for s_ in range(restarts)
               if infos[g * restarts + s_]["status"] == 0 and infos[g * restarts + s_]["outer"] > 0]
        taus.append((1 + 1e-4) * min(fin) if fin else -1.0)
    for arm, (inf, trr) in runs.items():
        extra = {"random": 0.0, "frame_only": t_spa, "learned": t_ml}[arm]
        out_arms[arm] = _arm_stats(np, graphs, restarts, inf, trr, hz, taus, extra)
        out_arms[arm]["start_seconds"] = extra
        out_arms[arm]["median_final_res"] = float(np.median(
            [i["res_WH"] for i in inf if i["status"] == 0]))
    out = {"metric": "median outer iterations to tau_g, learned warm start vs random starts "
                     "(256 SBM graphs x 8 starts)",
           "value": out_arms["learned"]["median_outer"], "unit": "outer iterations",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "vs_baseline": None,
           "config": {"workload": "256 SBM graphs, n ~ U[500,5000], r in {8,16,32}, seed 1004",
                      "train_graphs": a.train_graphs, "train_seed": 20000,
                      "train_outer": a.train_outer, "epochs": a.epochs,
                      "target_outer": T, "parallelism": "single GPU"},
           "tau_rule": f"(1 + 1e-4) x best random-start residual after {T} outer iterations",
           "arms": out_arms,
           "training": {"generate_s": t_gen, "solve_frame_targets_s": t_pool,
                        "train_s": t_train, "log": log,
                        "target_solves_ok": {str(r): v[4] for r, v in pools.items()},
                        "pool_rows": {str(r): int(v[0].shape[0]) for r, v in pools.items()},
                        "held_rows": {str(r): int(v[2].shape[0]) for r, v in pools.items()}}}
    print(json.dumps(out))


def _timed_solve(torch, plan, W0, steps):
    plan.solve(W0, trace=False)                          # graph capture, warm clocks
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, Ht, info = plan.solve(W0, trace=True)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, Ht, info


def _bench_c2(a, torch, np, S, gen):
    """Graph-SNMPBB (eq. (2.3)) on the SBM workload: A = D^-1/2 Adj D^-1/2 (CSR), the
    normalised 10-NN Laplacian of the node features (built on the device by the graph
    preprocessing, timed on its own), r = 20, gamma = 0.2."""
    from scipy.optimize import linear_sum_assignment
    dev = torch.device("cuda:0")
    p = gen.config(2)
    A, W0n, labels = p["A"], p["W0"], p["labels"]
    n, r = A.shape[0], W0n.shape[1]
    lam = 0.01 * float(np.sqrt(np.sum(A.data.astype(np.float32).astype(np.float64) ** 2)))
    Xf = torch.from_numpy(p["X"]).to(dev, torch.float32)
    S.knn_graph(Xf, p["knn"])                                  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Lg = S.knn_graph(Xf, p["knn"])
    torch.cuda.synchronize()
    lap_s = time.perf_counter() - t0
    L_nnz = int(Lg.keep[2].numel())
    Ag = S.csr_from_scipy(A, torch.float32)
    W0 = torch.from_numpy(W0n).to(dev, torch.float32)
    prm = S.params(lam=lam, gamma=0.2, prec=S.F32, max_outer=a.steps, check_every=1 << 30,
                   fuse_inner=a.fuse_inner)
    with S.Plan(Ag, r, prm, Lg) as pl:
        el, Ht, info = _timed_solve(torch, pl, W0, a.steps)
        ms = pl.time_apass(W0, 100)
    byts = 8.0 * (n + 1) + 8.0 * A.nnz + 2 * 4.0 * n * r    # CSR + X once + Y
    ach = byts / (ms * 1e-3) / 1e9
    pred = Ht.float().cpu().numpy().argmax(axis=1)
    k = int(labels.max()) + 1
    conf = np.zeros((k, r))
    np.add.at(conf, (labels, pred), 1)
    ri, ci = linear_sum_assignment(-conf)
    acc = conf[ri, ci].sum() / n
    try:
        from sklearn.metrics import adjusted_rand_score
        ari = float(adjusted_rand_score(labels, pred))
    except Exception:  # pragma: no cover
        ari = None
    print(json.dumps({
        "metric": "Graph-SNMPBB outer iterations/s (SBM n=20000, r=20, CSR + Laplacian)",
        "value": a.steps / el, "unit": "outer iterations/s", "n_gpus": 1, "steps": a.steps,
        "ms_per_step": 1e3 * el / a.steps, "higher_is_better": True, "dtype": "f32",
        "data": "synthetic", "vs_baseline": None,
        "config": {"workload": "SBM n=20000, 20 clusters, p_in 0.02, p_out 0.0005, seed 1002",
                   "nnz_A": int(A.nnz), "nnz_L": L_nnz, "r": r, "gamma": 0.2,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_spmm (A-pass B = A P, CSR)", "ms_per_launch": ms,
                     "algorithmic_per_launch": f"{byts:.4g} B (CSR + P + B)"},
        "res_WH": info["res_WH"], "pg_norm": info["pg_norm"],
        "laplacian_seconds": lap_s,
        "laplacian": "device: brute-force 10-NN over 16-dim features (FP64 distances), union "
                     "pattern, normalised Laplacian",
        "clustering": {"accuracy": float(acc), "ari": ari},
        **({} if a.no_cpu_baseline else {"cpu_baseline": _c2_cpu(np, p, lam, r, W0n)})}))


def _c2_cpu(np, p, lam, r, W0n):
    """The oracle's Graph-SNMPBB on the same workload (its Laplacian built by the oracle's
    own preprocessing beforehand, outside the timed sample)."""
    import oracle as O
    A64 = p["A"].astype(np.float32).astype(np.float64)
    L = O.knn_laplacian(p["X"].astype(np.float32).astype(np.float64), p["knn"])
    prm = O.Params(lam=lam, gamma=0.2)
    return _cpu_sample(lambda k: O.snmpbb(A64, W0n, prm, k, L=L), 1,
                       "outer iterations on the n=20000, r=20 graph workload")


def _bench_c3(a, torch, np, S, gen):
    """LAI-SNMPBB (Section 2.3) on the rank-64 surrogate U diag(lam) U^T of a power-law
    graph, n = 200000, r = 32; the surrogate is built on the device by the range finder
    (snmf_lai_sketch: 64 + 10 columns, two power iterations), timed on its own."""
    dev = torch.device("cuda:0")
    q = gen.config(3)
    W0n = q["W0"]
    Ag = S.csr_from_scipy(q["A"], torch.float32)
    Om = torch.from_numpy(q["Omega"]).to(dev, torch.float32)
    S.lai_sketch(Ag, q["rank"], q["power_iters"], Om)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ug, lg = S.lai_sketch(Ag, q["rank"], q["power_iters"], Om)
    torch.cuda.synchronize()
    sketch_s = time.perf_counter() - t0
    lamv = lg.cpu().numpy()
    n, ell = Ug.shape
    r = W0n.shape[1]
    lam = 0.01 * float(np.sqrt(np.sum(lamv ** 2)))
    W0 = torch.from_numpy(W0n).to(dev, torch.float32)
    prm = S.params(lam=lam, prec=S.F32, max_outer=a.steps, check_every=1 << 30,
                   fuse_inner=a.fuse_inner)
    with S.Plan(S.lowrank(Ug, lg), r, prm) as pl:
        el, Ht, info = _timed_solve(torch, pl, W0, a.steps)
        ms = pl.time_apass(W0, 100)
    byts = 2 * 4.0 * n * ell + 2 * 4.0 * n * r          # U twice + P + B
    ach = byts / (ms * 1e-3) / 1e9
    print(json.dumps({
        "metric": "LAI-SNMPBB outer iterations/s (n=200000, ell=64, r=32)",
        "value": a.steps / el, "unit": "outer iterations/s", "n_gpus": 1, "steps": a.steps,
        "ms_per_step": 1e3 * el / a.steps, "higher_is_better": True, "dtype": "f32",
        "data": "synthetic", "vs_baseline": None,
        "config": {"workload": "power-law CSR n=200000 (exponent 2.1, mean degree 10), "
                               "range finder ell=64, seed 1003", "r": r, "ell": ell,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_lai_utp + k_lai_reduce + k_lai_ut (B = U (lam (U^T P)))",
                     "ms_per_launch": ms,
                     "algorithmic_per_launch": f"{byts:.4g} B (U twice + P + B)"},
        "res_WH_surrogate": info["res_WH"], "pg_norm": info["pg_norm"],
        "range_finder_seconds": sketch_s,
        "range_finder": "device: A Omega (CSR, 74 columns), 2 power iterations (4 more "
                        "products), 5 shifted/plain Cholesky QR rounds, Q^T A Q, Jacobi",
        **({} if a.no_cpu_baseline else {"cpu_baseline": _c3_cpu(np, Ug, lg, lam, W0n)})}))


def _c3_cpu(np, Ug, lg, lam, W0n):
    """The oracle's LAI-SNMPBB on the same surrogate (U, lam from the device sketch)."""
    import oracle as O
    lr = O.LowRank(Ug.double().cpu().numpy(), lg.cpu().numpy())
    prm = O.Params(lam=lam)
    return _cpu_sample(lambda k: O.snmpbb(lr, W0n, prm, k), 1,
                       "outer iterations on the n=200000, ell=64, r=32 surrogate")


def _bench_nmf(a, torch, np, S, gen):
    """NMPBB for rectangular NMF (eq. (1.1)): a planted dense V (m = 8192, n = 4096,
    r = 64, FP32, read in place) and a sparse V (m = 100000, n = 20000, 0.1% of the
    entries, r = 32, FP32, transposed once on the device).  value: dense outer iterations/s
    (W-step and H-step of 5 inner iterations each)."""
    dev = torch.device("cuda:0")
    out = {"metric": "NMF outer iterations/s (dense V 8192 x 4096, r = 64, FP32)",
           "unit": "outer iterations/s", "n_gpus": 1, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    cases = {}
    for name, prob, r, ncols in (("dense", gen.planted_rect(8192, 4096, 64, 1031), 64, 4096),
                                 ("csr", gen.random_rect_csr(100000, 20000, 0.001, 32, 1032), 32,
                                  20000)):
        if name == "dense":
            Vt = torch.from_numpy(prob["V"]).to(dev, torch.float32)
            M = S.dense(Vt)
        else:
            M = S.csr_from_scipy(prob["V"], torch.float32)
        W0 = torch.from_numpy(prob["W0"]).to(dev, torch.float32)
        H0 = torch.from_numpy(prob["Ht0"]).to(dev, torch.float32)
        S.nmf_solve(M, ncols, W0, H0, S.params(prec=S.F32, lam=0.0, max_outer=a.warmup,
                                               fuse_inner=a.fuse_inner))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, info = S.nmf_solve(M, ncols, W0, H0, S.params(prec=S.F32, lam=0.0,
                                                           max_outer=a.steps,
                                                           check_every=1 << 30,
                                                           fuse_inner=a.fuse_inner))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        cases[name] = {"outer_per_s": a.steps / el, "ms_per_outer": 1e3 * el / a.steps,
                       "res_WH": info["res_WH"], "m": int(M.n), "n": int(ncols), "r": r,
                       "nnz": int(prob["V"].nnz) if name == "csr" else None}
    out.update({"value": cases["dense"]["outer_per_s"], "steps": a.steps, "warmup": a.warmup,
                "ms_per_step": cases["dense"]["ms_per_outer"],
                "config": {"workload": "planted dense V = max(W* H*^T + E, 0) 8192 x 4096, "
                                       "seed 1031; sparse V 100000 x 20000, seed 1032",
                           "parallelism": "single GPU"},
                "cases": cases})
    print(json.dumps(out))


def _bench_scale(a, torch, np, S, gen):
    """The HBM-bound A-pass kernels at a size past the L2 and the 256 MB last-level cache:
    the CSR SpMM (random symmetric graph, n = 2e6, mean degree 30, r = 20 and 32; the SBM
    graph workload at 100 times its size, clusters contiguous and permuted, r = 20) and the
    LAI products (n = 2e6, ell = 64, r = 32), each against 8 TB/s and against a measured
    device-to-device copy."""
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = 2_000_000
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)        # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    rows = []
    a_host = gen.random_symmetric_csr(n, 30.0, gen.SEED_BASE + 20)
    A = S.csr_from_scipy(a_host, torch.float32)
    nnz = a_host.nnz
    for r in (20, 32):
        P = torch.rand((n, r), device=dev, dtype=torch.float32)
        with S.Plan(A, r, S.params(lam=0.0, prec=S.F32, max_outer=1)) as pl:
            ms = pl.time_apass(P, 50)
        byts = 8.0 * (n + 1) + 8.0 * nnz + 2 * 4.0 * n * r        # CSR + P once + B
        rows.append({"kernel": "k_spmm (CSR A-pass)", "n": n, "nnz": nnz, "r": r, "ms": ms,
                     "algorithmic_bytes": byts, "gbs": byts / (ms * 1e-3) / 1e9})
    del A, a_host
    # the graph workload's kind at 100 times its size: SBM n = 2e6, 20 clusters of 1e5
    # contiguous node ids, the degrees of the n = 20000 workload (p_in 2e-4, p_out 5e-6),
    # A = D^-1/2 Adj D^-1/2; and the same graph with its node ids randomly permuted (no
    # locality left in the gathers)
    adj, _ = gen.sbm_adjacency(n, 20, 2e-4, 5e-6, np.random.default_rng(gen.SEED_BASE + 22))
    a_sbm = gen.normalized_adjacency(adj)
    del adj
    perm = np.random.default_rng(gen.SEED_BASE + 23).permutation(n)
    for name, a_host in (("SBM, clusters contiguous", a_sbm),
                         ("SBM, node ids permuted", a_sbm[perm][:, perm].tocsr())):
        a_host.sort_indices()
        A = S.csr_from_scipy(a_host, torch.float32)
        nnz = a_host.nnz
        P = torch.rand((n, 20), device=dev, dtype=torch.float32)
        with S.Plan(A, 20, S.params(lam=0.0, prec=S.F32, max_outer=1)) as pl:
            ms = pl.time_apass(P, 50)
        byts = 8.0 * (n + 1) + 8.0 * nnz + 2 * 4.0 * n * 20
        rows.append({"kernel": f"k_spmm (CSR A-pass), {name}", "n": n, "nnz": nnz, "r": 20,
                     "ms": ms, "algorithmic_bytes": byts, "gbs": byts / (ms * 1e-3) / 1e9})
        del A
    del a_sbm
    ell, r = 64, 32
    U, lamv = gen.random_lowrank(n, ell, gen.SEED_BASE + 21)
    Ug = torch.from_numpy(U).to(dev)
    lg = torch.from_numpy(lamv).to(dev, torch.float64)
    P = torch.rand((n, r), device=dev, dtype=torch.float32)
    with S.Plan(S.lowrank(Ug, lg), r, S.params(lam=0.0, prec=S.F32, max_outer=1)) as pl:
        ms = pl.time_apass(P, 50)
    byts = 2 * 4.0 * n * ell + 2 * 4.0 * n * r                     # U twice + P + B
    rows.append({"kernel": "k_lai_utp32 + k_lai_reduce32 + k_lai_ut32 (LAI A-pass)", "n": n,
                 "ell": ell, "r": r, "ms": ms, "algorithmic_bytes": byts,
                 "gbs": byts / (ms * 1e-3) / 1e9})
    for row in rows:
        row["frac_of_peak"] = row["gbs"] / HBM_PEAK_GBS
        row["frac_of_copy"] = row["gbs"] / copy_gbs
    print(json.dumps({
        "metric": "HBM-bound A-pass kernels at n = 2e6 (GB/s of algorithmic bytes)",
        "value": min(row["frac_of_peak"] for row in rows), "unit": "fraction of 8 TB/s (worst kernel)",
        "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "vs_baseline": None,
        "config": {"workload": "random symmetric CSR n=2e6 mean degree 30 (seed 1020); SBM "
                               "n=2e6, 20 clusters, p_in 2e-4, p_out 5e-6 (seed 1022), ordered "
                               "and permuted (seed 1023); Gaussian U n=2e6 x 64 (seed 1021)",
                   "parallelism": "single GPU"},
        "copy_gbs": copy_gbs, "peak_gbs": HBM_PEAK_GBS, "kernels": rows}))


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(the multi-GPU row sharding is a design, not part of this build).")
        sys.exit(2)
    import numpy as np
    import torch
    if a.workload != "c1":
        from paper_2606_02887_amd import gen
        from paper_2606_02887_amd import snmf as S
        {"c2": _bench_c2, "c3": _bench_c3, "c4": _bench_c4, "c4ws": _bench_c4ws,
         "scale": _bench_scale, "nmf": _bench_nmf}[a.workload](
            a, torch, np, S, gen)
        return

    from paper_2606_02887_amd import gen
    from paper_2606_02887_amd import snmf as S

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = gen.config(1)                                  # planted dense n=8192, r=64
    A64, W064 = prob["A"], prob["W0"]
    lam = 0.01 * float(np.sqrt(np.sum(A64 * A64)))        # lambda = 0.01 ||A||_F
    A = torch.from_numpy(A64.astype(np.float32)).to(dev)
    W0 = torch.from_numpy(W064.astype(np.float32)).to(dev)
    torch.cuda.synchronize()

    if a.apass_only:
        _apass_only(torch, S, A, W0, lam)
        return
    if a.batch_apass_only:
        _batch_apass_only(torch, np, S, gen, A, A64)
        return

    forms = {}
    plans = {}
    for name, prec in (("fp32", S.F32), ("bf16x3", S.BF16X3)):
        pl = S.Plan(S.dense(A), R, S.params(lam=lam, prec=prec, max_outer=a.steps,
                                            check_every=1 << 30, fuse_inner=a.fuse_inner))
        plans[name] = pl
        wp = S.Plan(S.dense(A), R, S.params(lam=lam, prec=prec, max_outer=max(1, a.warmup),
                                            fuse_inner=a.fuse_inner))
        wp.solve(W0, trace=False)                        # warmup (graph capture, clocks)
        wp.close()
        pl.solve(W0, trace=False)                        # first call captures its graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, info = pl.solve(W0, trace=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        forms[name] = {"outer_per_s": a.steps / el, "ms_per_outer": 1e3 * el / a.steps,
                       "device_ms_per_outer": 1e3 * info["seconds"] / max(info["outer"], 1),
                       "res_WH": info["res_WH"], "pg_norm": info["pg_norm"],
                       "outer": info["outer"]}

    # ---------------------------------------------------------------- batched restarts
    # the batching form on the same problem: 8 random starts solved together
    rng = np.random.default_rng(1101)
    W0b = torch.from_numpy(np.stack([gen.start_factor(rng, N, R, float(A64.mean()))
                                     for _ in range(8)])).to(dev, torch.float32).contiguous()
    # (FP32: one A-pass per restart; BF16X3: one stacked product of all 8 restarts' factors,
    # 8192 x 8192 times 8192 x 512, A_hi and A_lo read once)
    for name, prec in (("batched8_fp32", S.F32), ("batched8_bf16x3", S.BF16X3)):
        with S.Batch([S.dense(A)], [R], S.params(lam=lam, prec=prec, max_outer=a.steps,
                                                 check_every=1 << 30), 8) as bt:
            bt.solve([W0b])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, binf, _ = bt.solve([W0b])
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            ms_ap = bt.time_apass(W0b.reshape(-1), 20)
        forms[name] = {"restart_outer_per_s": 8 * a.steps / el,
                       "ms_per_outer": 1e3 * el / a.steps,
                       "res_WH_best": min(i["res_WH"] for i in binf),
                       "apass_ms_all_8": ms_ap,
                       "apass_tflops": (3 if prec == S.BF16X3 else 1) * 2.0 * N * N * 8 * R
                       / (ms_ap * 1e-3) / 1e12}

    # ---------------------------------------------------------------- roofline (A-pass)
    P = W0.clone()
    ms32 = plans["fp32"].time_apass(P, 50)
    flops = 2.0 * N * N * R
    ach32 = flops / (ms32 * 1e-3) / 1e12
    msbf = plans["bf16x3"].time_apass(P, 50)
    bytes_bf = 2.0 * 2 * N * N + 2.0 * 2 * N * R + 4.0 * N * R   # A_hi, A_lo, P_hi/lo, B
    achbf = bytes_bf / (msbf * 1e-3) / 1e9
    roof = {"bound": "mfma", "achieved": ach32, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach32 / FP32_PEAK_TFLOPS,
            "traffic": _traffic("k_apass_dense.hip", "k_apass_f32w"),
            "kernel": "k_apass_f32w (B = A P, FP32 MFMA)", "ms_per_launch": ms32,
            "algorithmic_per_launch": f"{flops:.4g} flop (2 n^2 r)"}
    forms["bf16x3"]["apass"] = {"bound": "hbm", "achieved": achbf, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": achbf / HBM_PEAK_GBS,
                                "traffic": _traffic("k_apass_dense.hip", "k_apass_bf16x3"),
                                "ms_per_launch": msbf,
                                "tflops": 3 * flops / (msbf * 1e-3) / 1e12}

    # ---------------------------------------------------------------- time to target
    ref_path = os.path.join(ROOT, "tests", "golden", "c1_reference.json")
    target = None
    if not a.no_target and os.path.exists(ref_path):
        ref = json.load(open(ref_path))
        target = (1 + 1e-4) * ref["res_ref"]
        for name, prec in (("fp32", S.F32), ("bf16x3", S.BF16X3)):
            with S.Plan(S.dense(A), R, S.params(lam=lam, prec=prec, max_outer=a.target_cap,
                                                target_res=target, check_every=16,
                                                fuse_inner=a.fuse_inner)) as tp:
                _, _, info = tp.solve(W0, trace=True)
            forms[name]["time_to_target_s"] = info["seconds_to_target"] if info["converged_at"] else None
            forms[name]["outer_to_target"] = info["converged_at"] or None
            forms[name]["final_res_after_cap"] = info["res_WH"]
            forms[name]["gap_to_target"] = info["res_WH"] / target - 1.0
        # the 8 stacked restarts with the same target: the batch's wall time until its
        # first restart meets it (the restarts reach different local minima, so not every
        # one does)
        for name, prec in (("batched8_fp32", S.F32), ("batched8_bf16x3", S.BF16X3)):
            with S.Batch([S.dense(A)], [R], S.params(lam=lam, prec=prec,
                                                     max_outer=a.target_cap, target_res=target,
                                                     check_every=16), 8) as bt:
                _, _, binf, _ = bt.solve([W0b])
            hits = [i for i in binf if i["converged_at"]]
            forms[name]["time_to_target_s"] = (min(i["seconds_to_target"] for i in hits)
                                               if hits else None)
            forms[name]["outer_to_target"] = (min(i["converged_at"] for i in hits)
                                              if hits else None)
            forms[name]["restarts_reaching_target"] = len(hits)
        forms["target"] = {"res": target, "rule": "(1 + 1e-4) x FP64 reference residual after "
                           f"{ref['outer']} outer iterations", "res_ref": ref["res_ref"]}

    for pl in plans.values():
        pl.close()

    cpu = None
    if not a.no_cpu_baseline:
        cpu = _cpu_baseline(A64, W064, lam, a.cpu_outer)

    f32 = forms["fp32"]
    out = {"metric": "SNMPBB outer iterations/s (n=8192, r=64, plain FP32)",
           "value": f32["outer_per_s"], "unit": "outer iterations/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": f32["ms_per_outer"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": "planted dense A = W* W*^T + E, seed 1001",
                                           "n": N, "r": R, "inner_iters": 5,
                                           "parallelism": "single GPU"},
           "roofline": roof, "cpu_baseline": cpu, "forms": forms}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
