"""GPU parity of the learned warm start against the oracle (oracle/warmstart.py).

Frame (sketch, SPA anchors, coordinates), column matching of the targets, the network's
forward pass, one training step (the gradient is read back from Adam's first moment,
m = (1 - beta1) g after step 1) and the batched warm start end to end.  Where a
floating-point comparison decides an integer (the SPA argmax, the assignment), the oracle
is run on the device's own floating-point inputs and must take the same decisions.
"""
import numpy as np
import pytest

import oracle as O
from oracle import warmstart as WS
from paper_2606_02887_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
DT = {"f64": torch.float64, "f32": torch.float32}


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_02887_amd import snmf
    return snmf


def nrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (d if d > 0 else 1.0)


SHAPES = [(140, 3), (261, 8), (300, 16), (90, 5)]


def _setup(S, dt, shapes=SHAPES, restarts=2, seed=31):
    graphs, As, a_in = [], [], []
    for g, (n, r) in enumerate(shapes):
        rng = np.random.default_rng(seed + g)
        adj, _ = gen.sbm_adjacency(n, r, 0.3, 0.02, rng)
        a = gen.normalized_adjacency(adj)
        As.append(S.csr_from_scipy(a, dt))
        b = a.copy()
        b.data = torch.from_numpy(a.data).to(dt).double().numpy()
        a_in.append(b)
        graphs.append((n, r))
    om = []
    for g, (n, r) in enumerate(shapes):
        for s in range(restarts):
            om.append(gen.sketch_matrix(n, r, 500 + 10 * g + s).ravel())
    Omega = torch.from_numpy(np.concatenate(om)).to(DEV, dt)
    return graphs, As, a_in, Omega


def _blocks(buf, graphs, restarts):
    out, at = [], 0
    for n, r in graphs:
        for _ in range(restarts):
            out.append(buf[at: at + n * r].reshape(n, r))
            at += n * r
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_frame_matches_oracle(S, prec):
    dt = DT[prec]
    graphs, As, a_in, Omega = _setup(S, dt)
    p = S.F64 if prec == "f64" else S.F32
    with S.Batch(As, [r for _, r in graphs], S.params(prec=p), restarts=2) as b:
        Y, C, anc = b.frame(Omega)
    Yb = _blocks(Y.double().cpu().numpy(), graphs, 2)
    Cb = _blocks(C.double().cpu().numpy(), graphs, 2)
    Ob = _blocks(Omega.double().cpu().numpy(), graphs, 2)
    anc = anc.cpu().numpy()
    ytol, ctol = (1e-12, 1e-9) if prec == "f64" else (1e-5, 1e-5)
    for i in range(len(Yb)):
        g = i // 2
        n, r = graphs[g]
        assert nrel(Yb[i], WS.sketch(a_in[g], Ob[i])) <= ytol, i
        # decisions taken on the device's own sketch
        K = WS.spa(WS.row_normalise(Yb[i], WS.row_sums(a_in[g])), r)
        assert list(anc[i, :r]) == K, i
        Co = WS.coords(Yb[i], K)
        rms = WS.rms_pos(Co)
        assert nrel(Cb[i], Co / rms) <= ctol, i
        assert np.allclose(Cb[i][K] * rms, np.eye(r), atol=1e-6 if prec == "f64" else 1e-3)
        assert abs(WS.rms_pos(Cb[i]) - 1.0) <= (1e-12 if prec == "f64" else 1e-6)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_targets_match_oracle(S, prec):
    dt = DT[prec]
    graphs, As, a_in, Omega = _setup(S, dt, seed=77)
    p = S.F64 if prec == "f64" else S.F32
    with S.Batch(As, [r for _, r in graphs], S.params(prec=p), restarts=2) as b:
        _, C, _ = b.frame(Omega)
        rng = np.random.default_rng(4)
        Cn = C.double().cpu().numpy()
        Hs = []
        for i, Ci in enumerate(_blocks(Cn, graphs, 2)):
            n, r = graphs[i // 2]
            Hs.append((np.abs(Ci[:, rng.permutation(r)]) * rng.uniform(0.5, 2, r)
                       + 1e-3 * rng.random((n, r))).ravel())
        Ht = torch.from_numpy(np.concatenate(Hs)).to(DEV, dt)
        T, perm = b.targets(C, Ht)
    Tb = _blocks(T.double().cpu().numpy(), graphs, 2)
    Hb = _blocks(Ht.double().cpu().numpy(), graphs, 2)
    Cb = _blocks(Cn, graphs, 2)
    perm = perm.cpu().numpy()
    for i in range(len(Tb)):
        g = i // 2
        n, r = graphs[g]
        To, pi = WS.targets(Cb[i], Hb[i])
        assert list(perm[i, :r]) == list(pi), i
        assert nrel(Tb[i], To) <= (1e-12 if prec == "f64" else 1e-6), i


def _rand_init(r, seed):
    rng = np.random.default_rng(seed)
    init = gen.mlp_init(r, 128, seed)
    init["b1"] = 0.1 * rng.standard_normal(128)
    init["M2"] = rng.standard_normal((r, 128)) * (0.5 / np.sqrt(128))
    init["b2"] = 0.3 * rng.standard_normal(r)
    return init


@pytest.mark.parametrize("r", [3, 8, 16, 32, 64])
def test_mlp_forward_matches_oracle(S, r):
    m = S.Mlp(_rand_init(r, 10 + r))
    rng = np.random.default_rng(r)
    N = 1000 + 37
    C = rng.standard_normal((N, r))
    sc = rng.uniform(0.5, 2.0, N)
    Ct = torch.from_numpy(C).to(DEV, torch.float32)
    Y = m.forward(Ct, torch.from_numpy(sc).to(DEV, torch.float32)).double().cpu().numpy()
    prm = m.params()
    yo, _ = WS.forward(prm, Ct.double().cpu().numpy())
    assert nrel(Y, sc.astype(np.float32).astype(np.float64)[:, None] * yo) <= 2e-6
    # the BF16 copies are the round-to-nearest-even values of the FP32 masters
    bits = m.M1h.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    assert np.array_equal(bits.view(np.float32).astype(np.float64), WS.bf16_round(prm["M1"]))


@pytest.mark.parametrize("r", [4, 16, 32])
def test_mlp_train_step_gradient_and_adam(S, r):
    m = S.Mlp(_rand_init(r, 40 + r))
    prm0 = m.params()
    rng = np.random.default_rng(7 + r)
    N, B, mu, lr = 900, 333, 0.5, 1e-3
    C = rng.standard_normal((N, r))
    T = rng.random((N, r))
    idx = rng.choice(N, size=B, replace=False).astype(np.int32)
    Ct = torch.from_numpy(C).to(DEV, torch.float32)
    Tt = torch.from_numpy(T).to(DEV, torch.float32)
    loss = m.train_step(Ct, Tt, torch.from_numpy(idx).to(DEV), mu, lr, want_loss=True)
    Cin, Tin = Ct.double().cpu().numpy()[idx], Tt.double().cpu().numpy()[idx]
    lo, go = WS.loss_and_grad(prm0, Cin, Tin, mu)
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    b1c = float(np.float32(1) - np.float32(0.9))       # (1 - beta1) and (1 - beta2) as the
    b2c = float(np.float32(1) - np.float32(0.999))     # device forms them in FP32
    gdev = m.adam_m.double().cpu().numpy() / b1c       # m = (1 - beta1) g after step 1
    H = 128
    parts = {"M1": gdev[:H * r].reshape(H, r), "b1": gdev[H * r:H * r + H],
             "M2": gdev[H * r + H:H * r + H + r * H].reshape(r, H), "b2": gdev[-r:]}
    for k in ("M1", "b1", "M2", "b2"):
        assert nrel(parts[k], go[k]) <= 1e-4, k
    prm1 = m.params()
    v = m.adam_v.double().cpu().numpy()
    mm = m.adam_m.double().cpu().numpy()
    assert np.allclose(v, b2c * (mm / b1c) ** 2, rtol=1e-5, atol=1e-30)
    flat0 = np.concatenate([prm0[k].ravel() for k in ("M1", "b1", "M2", "b2")])
    flat1 = np.concatenate([prm1[k].ravel() for k in ("M1", "b1", "M2", "b2")])
    ref, _, _ = WS.adam_step(flat0, mm / b1c, np.zeros_like(mm), np.zeros_like(mm), 1, lr)
    assert np.max(np.abs(flat1 - ref)) <= 1e-6
    bits = m.M2h.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    assert np.array_equal(bits.view(np.float32).astype(np.float64), WS.bf16_round(prm1["M2"]))


def test_batch_warmstart_end_to_end(S):
    graphs, As, a_in, Omega = _setup(S, torch.float32, seed=91)
    ranks = sorted({r for _, r in graphs})
    models = [S.Mlp(_rand_init(r, 200 + r)) for r in ranks]
    with S.Batch(As, [r for _, r in graphs], S.params(prec=S.F32), restarts=2) as b:
        _, C, _ = b.frame(Omega)
        W0 = b.warmstart(models, Omega)
    Cb = _blocks(C.double().cpu().numpy(), graphs, 2)
    Wb = _blocks(W0.double().cpu().numpy(), graphs, 2)
    for i in range(len(Cb)):
        g = i // 2
        n, r = graphs[g]
        prm = models[ranks.index(r)].params()
        s = WS.scale(np.sqrt(O.norm2_A(a_in[g])), n, r)
        yo, _ = WS.forward(prm, Cb[i])
        assert nrel(Wb[i], s * yo) <= 2e-6, i
        assert (Wb[i] >= 0).all() and np.array_equal(Wb[i] == 0, yo == 0)


def test_warmstart_error_codes(S):
    graphs, As, _, Omega = _setup(S, torch.float32, shapes=[(80, 4)], restarts=1)
    with S.Batch(As, [4], S.params(prec=S.F32), restarts=1) as b:
        with pytest.raises(S.SnmfError) as e:
            b.warmstart([S.Mlp(_rand_init(5, 1))], Omega)
        assert e.value.name == "E_ARG"
    _, As64, _, Om64 = _setup(S, torch.float64, shapes=[(80, 4)], restarts=1)
    with S.Batch(As64, [4], S.params(prec=S.F64), restarts=1) as b:
        with pytest.raises(S.SnmfError) as e:
            b.warmstart([S.Mlp(_rand_init(4, 1))], Om64)
        assert e.value.name == "E_UNSUPPORTED"
    A = torch.eye(40, dtype=torch.float32, device=DEV)
    with S.Batch([S.dense(A)], [4], S.params(prec=S.BF16X3), restarts=1) as b:
        with pytest.raises(S.SnmfError) as e:
            b.frame(torch.ones(160, dtype=torch.float32, device=DEV))
        assert e.value.name == "E_UNSUPPORTED"
    with pytest.raises(S.SnmfError) as e:                       # network rank != r
        S.warmstart(S.dense(A), torch.ones((40, 4), dtype=torch.float32, device=DEV),
                    S.Mlp(_rand_init(5, 1)))
    assert e.value.name == "E_SHAPE"
    with pytest.raises(S.SnmfError) as e:                       # network in F64
        S.warmstart(S.dense(A.double()), torch.ones((40, 4), dtype=torch.float64, device=DEV),
                    S.Mlp(_rand_init(4, 1)))
    assert e.value.name == "E_UNSUPPORTED"


def _single_problem(kind, dt, n=260, r=6, seed=5):
    """A planted symmetric nonnegative problem, dense or as CSR (an SBM graph), with its
    FP64 copy as the device holds it and a Gaussian sketch matrix."""
    rng = np.random.default_rng(seed)
    if kind == "dense":
        W = rng.random((n, r))
        a = W @ W.T
        At = torch.from_numpy(a).to(DEV, dt)
        ref = At.double().cpu().numpy()
        M = S_mod().dense(At)
    else:
        adj, _ = gen.sbm_adjacency(n, r, 0.3, 0.02, rng)
        a = gen.normalized_adjacency(adj)
        M = S_mod().csr_from_scipy(a, dt)
        ref = a.copy()
        ref.data = M.keep[2].double().cpu().numpy()
    Om = gen.sketch_matrix(n, r, 600 + seed)
    return M, ref, torch.from_numpy(Om).to(DEV, dt)


def S_mod():
    from paper_2606_02887_amd import snmf
    return snmf


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_problem_frame_start_matches_oracle(S, kind, prec):
    """snmf_warmstart without a network (the frame alone) for one dense or CSR problem:
    the oracle's frame_start on the same inputs (anchors are integer decisions taken in
    FP64 on both sides; the coordinates carry the FP32 sketch's rounding in F32)."""
    M, ref, Om = _single_problem(kind, DT[prec])
    W0 = S.warmstart(M, Om).double().cpu().numpy()
    Wo, _, _ = WS.frame_start(ref, Om.double().cpu().numpy(), np.sqrt(O.norm2_A(ref)))
    tol = 1e-10 if prec == "f64" else 2e-5
    assert nrel(W0, Wo) <= tol, nrel(W0, Wo)
    assert (W0 >= 0).all()


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_single_problem_learned_start_matches_oracle(S, kind):
    M, ref, Om = _single_problem(kind, torch.float32, r=8, seed=9)
    mlp = S.Mlp(_rand_init(8, 77))
    W0 = S.warmstart(M, Om, mlp).double().cpu().numpy()
    Wo, _, _ = WS.warm_start(mlp.params(), ref, Om.double().cpu().numpy(),
                             np.sqrt(O.norm2_A(ref)))
    assert nrel(W0, Wo) <= 2e-5, nrel(W0, Wo)
    assert (W0 >= 0).all()


def test_warm_start_gain_on_detectable_graphs(S):
    """Trained on 48 separately seeded SBM graphs (clusters detectable; every tenth held
    out for validation), the network's held-out loss falls below that of the frame's own
    start (the network's starting point) on the same targets; on 12 further graphs the
    learned start and the frame alone are closer to the end point after the first outer
    iteration than random starts (median over graphs of res_1 / best final - 1), and the
    learned start needs no more outer iterations to tau_g = (1 + 1e-4) x best final
    residual than the frame alone (median over graphs)."""
    from paper_2606_02887_amd import train_ws
    mk = lambda num, seed: gen.batched_sbm(num_graphs=num, n_lo=240, n_hi=480, ranks=(8,),
                                           restarts=3, p_in=0.2, p_out=0.01, seed=seed)
    train = mk(48, 30000)
    pools = train_ws.training_pools(S, torch, train, outer=120)
    log = []
    models = train_ws.train(S, torch, pools, epochs=12, batch=1024, lr=2e-3, log=log)
    for rec in log:
        print(rec)
    assert abs(log[0]["held_loss"] - log[0]["frame_held_loss"]) <= 1e-6 * log[0]["frame_held_loss"]
    assert log[-1]["held_loss"] < log[-1]["frame_held_loss"]
    test = mk(12, 31000)
    As = [S.csr_from_scipy(g["A"], torch.float32) for g in test]
    W0r = torch.from_numpy(np.concatenate([np.stack(g["W0"]).ravel() for g in test])).to(
        DEV, torch.float32)
    T = 200
    with S.Batch(As, [8] * len(test), S.params(prec=S.F32, max_outer=T), 3,
                 lam=train_ws.lambdas(test)) as b:
        Om = train_ws._sketch_buffer(torch, test, 3, 4242, DEV, torch.float32)
        starts = {"random": W0r, "frame": b.warmstart([], Om), "learned": b.warmstart([models[8]], Om)}
        runs = {k: b.solve(b.split(W), trace=True) for k, W in starts.items()}
    best = []
    for g in range(len(test)):
        best.append(min(runs[k][3][g * 3 + s, T - 1, 0] for k in runs for s in range(3)
                        if runs[k][2][g * 3 + s]["status"] == 0))
    gap, its = {}, {}
    for k, (_, _, infos, tr) in runs.items():
        for it in (1, 2, 4):
            per = [min(tr[g * 3 + s, it - 1, 0] for s in range(3)) / best[g] - 1.0
                   for g in range(len(test))]
            gap[(k, it)] = float(np.median(per))
        per = []
        for g in range(len(test)):
            hit = [np.nonzero(tr[g * 3 + s, :, 0] <= (1 + 1e-4) * best[g])[0] for s in range(3)
                   if infos[g * 3 + s]["status"] == 0]
            firsts = [h[0] + 1 for h in hit if h.size]
            per.append(min(firsts) if firsts else T + 1)
        its[k] = float(np.median(per))
    print("median gap after 1, 2, 4 outer iterations:", gap)
    print("median outer iterations to tau_g:", its)
    assert gap[("learned", 1)] < gap[("random", 1)]
    assert gap[("frame", 1)] < gap[("random", 1)]
    assert its["learned"] <= its["frame"]
