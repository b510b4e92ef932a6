"""Training of the warm-start networks (one per rank) on the GPU through the C ABI.

1. Solve every training graph with the batching form (one random start each).
2. Frame every graph from a seeded Gaussian sketch (sketch, SPA anchors, coordinates C
   scaled to rms(relu(C)) = 1).
3. Targets: the converged Ht with its columns matched to the anchor order, divided by its
   entry RMS.  Graphs whose solve broke down are left out; every tenth graph is held out
   for validation.
4. Adam on minibatches of rows drawn from a seeded permutation of the row pool, with a
   cosine learning-rate decay.
Every step of the method runs in the library's kernels; this module only sequences the
calls.  The validation losses it logs (the network's and that of the frame's own start
relu(C) on the same held-out targets) are computed with torch from the network's outputs:
diagnostics, not part of the warm start.
"""
from __future__ import annotations

import math

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


def training_pools(S, torch, graphs, outer=300, sketch_seed=7000, device="cuda", hold_every=10):
    """Row pools {r: (C, T, C_held, T_held, ok_fraction)} (float32 device tensors,
    rows x r): graphs g with g % hold_every == hold_every - 1 form the held-out pool."""
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
            offs = b.offsets()
        C, T = C.view(-1, r), T.view(-1, r)
        rows = {True: [], False: []}
        for g, (gr, info) in enumerate(zip(sub, infos)):
            if info["status"] != 0:
                continue
            o = offs[g] // r
            rows[g % hold_every == hold_every - 1].append(torch.arange(o, o + gr["n"]))
        pick = {k: (torch.cat(v).to(device) if v else torch.zeros(0, dtype=torch.int64,
                                                                   device=device))
                for k, v in rows.items()}
        pools[r] = (C[pick[False]].contiguous(), T[pick[False]].contiguous(),
                    C[pick[True]].contiguous(), T[pick[True]].contiguous(),
                    float(np.mean([i["status"] == 0 for i in infos])))
    return pools


def _mse(torch, y, t):
    return float(torch.mean((y.double() - t.double()) ** 2)) if y.numel() else float("nan")


def train(S, torch, pools, epochs=8, batch=4096, lr=2e-3, mu=1.0, seed=11, device="cuda",
          log=None):
    """One network per rank, trained with Adam on its row pool (cosine decay of the
    learning rate to zero over all steps); returns {r: Mlp}.  log (a list) receives, per
    rank and epoch, the mean minibatch loss and the held-out losses of the network and of
    the frame's own start."""
    from . import gen
    models = {}
    for r, pool in pools.items():
        C, T, Ch, Th = pool[:4]
        m = S.Mlp(gen.mlp_init(r, 128, seed + r), device=device)
        N = C.shape[0]
        steps = max(1, epochs * (N // batch))
        g = torch.Generator(device="cpu").manual_seed(seed + r)
        frame_held = _mse(torch, torch.clamp(Ch, min=0.0), Th)
        if log is not None:
            log.append({"r": r, "epoch": 0, "rows": int(N), "held_rows": int(Ch.shape[0]),
                        "held_loss": _mse(torch, m.forward(Ch), Th) if Ch.numel() else None,
                        "frame_held_loss": frame_held})
        t = 0
        for ep in range(epochs):
            perm = torch.randperm(N, generator=g).to(device=device, dtype=torch.int32)
            losses = []
            for at in range(0, N - batch + 1, batch):
                lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * t / steps))
                want = (at // batch) % 8 == 0
                loss = m.train_step(C, T, perm[at: at + batch], mu, lr_t, want_loss=want)
                if want:
                    losses.append(loss)
                t += 1
            if log is not None:
                log.append({"r": r, "epoch": ep + 1,
                            "train_loss": float(np.mean(losses)) if losses else None,
                            "held_loss": _mse(torch, m.forward(Ch), Th) if Ch.numel() else None,
                            "frame_held_loss": frame_held})
        models[r] = m
    return models
