"""Training of the warm-start networks (one per rank) on the GPU through the C ABI.

1. Solve every training graph with the batching form (one random start each).
2. Frame every graph from a seeded Gaussian sketch (sketch, SPA anchors, coordinates C).
3. Targets: the converged Ht with its columns matched to the anchor order, divided by s.
4. Adam on minibatches of rows drawn from a seeded permutation of the row pool.
Every numerical step runs in the library's kernels; this module only sequences the calls.
"""
from __future__ import annotations

import numpy as np


def _sketch_buffer(torch, graphs, restarts, seed, device, dtype):
    from . import gen
    parts = []
    for g, gr in enumerate(graphs):
        for s in range(restarts):
            parts.append(gen.sketch_matrix(gr["n"], gr["r"], seed + 1000 * g + s).ravel())
    return torch.from_numpy(np.concatenate(parts)).to(device, dtype)


def lambdas(graphs):
    """lambda = 0.01 ||A||_F of every graph (values as stored in FP32)."""
    return [0.01 * float(np.sqrt(np.sum(g["A"].data.astype(np.float32).astype(np.float64) ** 2)))
            for g in graphs]


def training_pools(S, torch, graphs, outer=300, sketch_seed=7000, device="cuda"):
    """Row pools {r: (C, T)} (float32 device tensors, rows x r) from solved graphs."""
    pools = {}
    for r in sorted({g["r"] for g in graphs}):
        sub = [g for g in graphs if g["r"] == r]
        As = [S.csr_from_scipy(g["A"], torch.float32) for g in sub]
        W0s = [torch.from_numpy(np.asarray(g["W0"][0])[None]).to(device, torch.float32).contiguous()
               for g in sub]
        with S.Batch(As, [r] * len(sub), S.params(prec=S.F32, max_outer=outer,
                                                   check_every=1 << 30), 1,
                     lam=lambdas(sub)) as b:
            _, Hs, infos, _ = b.solve(W0s)
            Ht = torch.cat([h.reshape(-1) for h in Hs])
            Om = _sketch_buffer(torch, sub, 1, sketch_seed + r, device, torch.float32)
            _, C, _ = b.frame(Om)
            T, _ = b.targets(C, Ht)
        ok = [i["status"] == 0 for i in infos]
        pools[r] = (C.view(-1, r), T.view(-1, r), float(np.mean(ok)))
    return pools


def train(S, torch, pools, epochs=4, batch=4096, lr=2e-3, mu=1.0, seed=11, device="cuda",
          log=None):
    """One network per rank, trained with Adam on its row pool; returns {r: Mlp}."""
    from . import gen
    models = {}
    for r, (C, T, _) in pools.items():
        m = S.Mlp(gen.mlp_init(r, 128, seed + r), device=device)
        N = C.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed + r)
        for ep in range(epochs):
            perm = torch.randperm(N, generator=g).to(device=device, dtype=torch.int32)
            last = None
            for at in range(0, N - batch + 1, batch):
                want = at + 2 * batch > N
                last = m.train_step(C, T, perm[at: at + batch], mu, lr, want_loss=want)
            if log is not None:
                log.append({"r": r, "epoch": ep + 1, "loss": last})
        models[r] = m
    return models
