"""Autotuner of the batched solve's launch shape (snmf_batch_tuning).

Two shapes decide how the batching form's launches fill the GPU, and the best values
depend on the batch: the row tiles per workgroup of the inner kernels, one value per rank
class (r <= 8, 16, 32, 64), and the rows per workgroup of the batched SpMM.  The tuner
times short batched solves of the caller's own problems (a few outer iterations from the
caller's starts) over a small candidate set, one coordinate at a time from the library's
defaults, and keeps a candidate only if it is at least 1% faster.  Choices are cached in
a JSON file keyed by the device, the precision, the format and a coarse summary of the
batch (per rank class: instance count, median n and total rows, each rounded to a power
of two), so that batches of the same kind reuse them.

Host-side sequencing only: every timed step runs in the library's kernels.
"""
from __future__ import annotations

import json
import math
import os
import time

TILES = (1, 2, 4, 8, 16)
SPMM_ROWS = (4, 8, 16, 32, 64)
DEFAULT = {"tiles_per_wg": [4, 4, 4, 4], "spmm_rows_per_wg": 16}


def default_cache_path() -> str:
    return os.environ.get("SNMF_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache",
                                       "paper_2606_02887_amd", "batch_tuning.json"))


def rank_class(r: int) -> int:
    """0..3 for ranks up to 8, 16, 32, 64 (the library's rank padding classes)."""
    rp = 4
    while rp < r:
        rp *= 2
    return 0 if rp <= 8 else 1 if rp <= 16 else 2 if rp <= 32 else 3


def _p2(x: float) -> int:
    return int(round(math.log2(max(x, 1.0))))


def workload_key(ns, rs, restarts: int, prec: int, fmt: str, device: str) -> str:
    """Cache key: device, precision, format, restarts and, per rank class, log2 of the
    instance count, of the median n and of the total rows (rounded)."""
    classes: dict[int, list[int]] = {}
    for n, r in zip(ns, rs):
        classes.setdefault(rank_class(int(r)), []).append(int(n))
    parts = [device, f"prec{prec}", fmt, f"S{restarts}"]
    for q in sorted(classes):
        v = sorted(classes[q])
        parts.append(f"q{q}:count2^{_p2(len(v) * restarts)}:median_n2^{_p2(v[len(v) // 2])}"
                     f":rows2^{_p2(sum(v) * restarts)}")
    return "|".join(parts)


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path: str, data: dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _valid(cfg) -> bool:
    try:
        return (len(cfg["tiles_per_wg"]) == 4 and all(1 <= int(t) <= 64 for t in cfg["tiles_per_wg"])
                and 1 <= int(cfg["spmm_rows_per_wg"]) <= 4096)
    except (KeyError, TypeError, ValueError):
        return False


def tune(S, torch, As, rs, restarts: int, W0s, prec: int, lam=None, outer: int = 8,
         reps: int = 3, cache_path: str | None = None, refresh: bool = False, log=None):
    """The launch shape for this batch: from the cache, or timed and then cached.

    As, rs, restarts, lam, W0s: the batch as snmf.Batch takes it (W0s: per-problem
    (restarts, n, r) device tensors).  Returns (config dict, from_cache)."""
    fmt = "dense" if As[0].desc.fmt == S.DENSE else "csr"
    device = torch.cuda.get_device_name(torch.cuda.current_device())
    key = workload_key([a.n for a in As], rs, restarts, prec, fmt, device)
    path = cache_path or default_cache_path()
    cache = load_cache(path)
    if not refresh and key in cache and _valid(cache[key]):
        return cache[key], True

    def measure(cfg):
        prm = S.params(prec=prec, max_outer=outer, check_every=1 << 30, tuning=cfg)
        with S.Batch(As, rs, prm, restarts, lam=lam) as b:
            b.solve(W0s)                                  # lazy scratch, graph capture, clocks
            torch.cuda.synchronize()
            best = math.inf
            for _ in range(reps):
                t0 = time.perf_counter()
                b.solve(W0s)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
        if log is not None:
            log.append({"config": json.loads(json.dumps(cfg)), "seconds": best})
        return best

    best = json.loads(json.dumps(DEFAULT))
    t_best = measure(best)
    for q in sorted({rank_class(int(r)) for r in rs}):
        for c in TILES:
            if c == best["tiles_per_wg"][q]:
                continue
            cfg = json.loads(json.dumps(best))
            cfg["tiles_per_wg"][q] = c
            t = measure(cfg)
            if t < 0.99 * t_best:
                best, t_best = cfg, t
    if fmt == "csr":
        for c in SPMM_ROWS:
            if c == best["spmm_rows_per_wg"]:
                continue
            cfg = json.loads(json.dumps(best))
            cfg["spmm_rows_per_wg"] = c
            t = measure(cfg)
            if t < 0.99 * t_best:
                best, t_best = cfg, t
    cache = load_cache(path)                              # re-read: another process may have
    cache[key] = best                                     # written other keys meanwhile
    save_cache(path, cache)
    return best, False
