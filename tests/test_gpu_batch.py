"""Parity of the batching form (snmf_batch_*) on the GPU.

Every instance (problem g, restart s) of a batched solve must follow the oracle's single
solve of problem g from start s; instances must not see each other (identical starts give
bitwise identical results, equal to the single-solve path); the stacked CSR A-pass must
equal A_g P_s for every instance; per-instance stopping must match the instance's own
trajectory.
"""
import numpy as np
import pytest

import oracle as O
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


def _graphs(seed, shapes, restarts):
    """Small SBM graphs (n, r) with `restarts` random starts each, float64."""
    out = []
    for g, (n, r) in enumerate(shapes):
        rng = np.random.default_rng(seed + g)
        adj, _ = gen.sbm_adjacency(n, max(2, r), 0.25, 0.02, rng)
        a = gen.normalized_adjacency(adj)
        w0 = np.stack([gen.start_factor(rng, n, r, gen.mean_of_sparse(a))
                       for _ in range(restarts)])
        out.append((a, r, w0))
    return out


# ragged shapes: ranks of three tile classes (4, 8, 32 padded), n not a tile multiple
SHAPES = [(157, 3), (333, 8), (410, 20), (75, 8)]


def _batch_inputs(S, graphs, dt):
    As = [S.csr_from_scipy(a, dt) for a, _, _ in graphs]
    a_in = [sp_round(a, dt) for a, _, _ in graphs]
    W0s = [torch.from_numpy(w).to(DEV, dt).contiguous() for _, _, w in graphs]
    w_in = [w.double().cpu().numpy() for w in W0s]
    return As, a_in, W0s, w_in


def sp_round(a, dt):
    """The matrix as the device holds it (values rounded to dt), in float64."""
    b = a.copy().astype(np.float64)
    b.data = torch.from_numpy(a.data).to(dt).double().numpy()
    return b


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_instances_follow_the_oracle(S, prec):
    """Config-0-like budget (20 outer iterations, before rounding differences grow): every
    instance's residual and PG norm match the oracle's solve of its problem and start."""
    dt = DT[prec]
    graphs = _graphs(500, SHAPES, restarts=2)
    As, a_in, W0s, w_in = _batch_inputs(S, graphs, dt)
    lams = [O.default_lambda(a) for a in a_in]
    prm = S.params(prec=S.F64 if prec == "f64" else S.F32, max_outer=20)
    with S.Batch(As, [r for _, r, _ in graphs], prm, restarts=2, lam=lams) as b:
        Ws, Hs, infos, _ = b.solve(W0s)
    tol = 1e-9 if prec == "f64" else 1e-3
    for g, (a, r, _) in enumerate(graphs):
        for s in range(2):
            info = infos[g * 2 + s]
            _, _, hist = O.snmpbb(a_in[g], w_in[g][s], O.Params(lam=lams[g]), 20)
            ref = hist[-1]
            assert info["status"] == 0 and info["outer"] == 20
            assert abs(info["res_WH"] - ref["res_WH"]) <= tol * ref["res_WH"], (g, s)
            assert abs(info["pg_norm"] - ref["pg"]) <= tol * ref["pg"], (g, s)
            W = Ws[g][s].double().cpu().numpy()
            Ht = Hs[g][s].double().cpu().numpy()
            assert (W >= 0).all() and (Ht >= 0).all()
            direct = O.residual_WH(a_in[g], W, Ht)
            assert abs(info["res_WH"] - direct) <= (1e-10 if prec == "f64" else 1e-4) * direct


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_equal_starts_are_bitwise_equal_and_match_single_solve(S, prec):
    """Instances are isolated: S copies of one start give bitwise identical factors, and
    (dense A: the same kernels as the single path's two-kernel inner iterations,
    fuse_inner = 0) bitwise the single solve's factors."""
    dt = DT[prec]
    prob = gen.planted_dense(240, 6, 77)
    At = torch.from_numpy(prob["A"]).to(DEV, dt)
    W0 = torch.from_numpy(prob["W0"]).to(DEV, dt)
    lam = O.default_lambda(prob["A"])
    p = S.F64 if prec == "f64" else S.F32
    W1, H1, i1 = S.solve(S.dense(At), W0, S.params(lam=lam, prec=p, max_outer=30, fuse_inner=0))
    W0s = [W0.unsqueeze(0).repeat(3, 1, 1).contiguous()]
    with S.Batch([S.dense(At)], [6], S.params(lam=lam, prec=p, max_outer=30), restarts=3) as b:
        Ws, Hs, infos, _ = b.solve(W0s)
    for s in range(3):
        assert torch.equal(Ws[0][s], W1) and torch.equal(Hs[0][s], H1)
        assert infos[s]["res_WH"] == i1["res_WH"] and infos[s]["outer"] == i1["outer"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_stacked_apass(S, prec):
    dt = DT[prec]
    graphs = _graphs(900, SHAPES + [(64, 64)], restarts=3)
    As, a_in, _, _ = _batch_inputs(S, graphs, dt)
    prm = S.params(prec=S.F64 if prec == "f64" else S.F32, max_outer=1)
    with S.Batch(As, [r for _, r, _ in graphs], prm, restarts=3) as b:
        rng = np.random.default_rng(3)
        P = torch.from_numpy(rng.random(b.elements)).to(DEV, dt)
        B = torch.empty_like(P)
        b.apass(P, B)
        Pn, Bn = P.double().cpu().numpy(), B.double().cpu().numpy()
    off = 0
    tol = 1e-12 if prec == "f64" else 1e-5
    for g, (a, r, _) in enumerate(graphs):
        n = a.shape[0]
        for s in range(3):
            Pi = Pn[off: off + n * r].reshape(n, r)
            Bi = Bn[off: off + n * r].reshape(n, r)
            assert nrel(Bi, a_in[g] @ Pi) <= tol, (g, s)
            off += n * r
    assert off == Pn.size


def test_batch_per_instance_target_stop(S):
    """A residual target stops each instance at its own first monitored hit; the others
    keep iterating, and their trajectories are unchanged by the stop of the first."""
    graphs = _graphs(1300, [(200, 4), (260, 6)], restarts=2)
    As, a_in, W0s, _ = _batch_inputs(S, graphs, torch.float64)
    lams = [O.default_lambda(a) for a in a_in]
    rs = [r for _, r, _ in graphs]
    with S.Batch(As, rs, S.params(prec=S.F64, max_outer=30), restarts=2, lam=lams) as b:
        _, _, base, tr = b.solve(W0s, trace=True)
    tau = tr[0, 9, 0]          # instance 0's residual after 10 outer iterations
    with S.Batch(As, rs, S.params(prec=S.F64, max_outer=30, target_res=tau, check_every=4),
                 restarts=2, lam=lams) as b:
        _, _, infos, tr2 = b.solve(W0s, trace=True)
    for i in range(4):
        hits = np.nonzero(tr[i, :, 0] <= tau)[0]
        if hits.size:
            assert infos[i]["converged_at"] == hits[0] + 1
            assert infos[i]["outer"] == hits[0] + 1
            assert infos[i]["seconds_to_target"] > 0
        else:
            assert infos[i]["converged_at"] == 0 and infos[i]["outer"] == 30
        k = infos[i]["outer"]
        assert np.array_equal(tr2[i, :k, :5], tr[i, :k, :5])
    assert 1 <= infos[0]["converged_at"] <= 10


def test_batch_breakdown_stays_in_its_instance(S):
    """A zero start makes G = 0 and rho = 0 in restart 1 (a breakdown); restart 0 of the
    same problem and the other problem must still follow the oracle."""
    graphs = _graphs(1500, [(180, 5), (120, 4)], restarts=2)
    As, a_in, W0s, w_in = _batch_inputs(S, graphs, torch.float64)
    W0s[0][1].zero_()
    lams = [O.default_lambda(a) for a in a_in]
    with S.Batch(As, [5, 4], S.params(prec=S.F64, max_outer=15), restarts=2, lam=lams) as b:
        Ws, Hs, infos, _ = b.solve(W0s)
    names = {v: k for k, v in S.STATUS.items()}
    assert infos[1]["status"] == names["E_BREAKDOWN"]
    for i in (0, 2, 3):
        g, s = divmod(i, 2)
        _, _, hist = O.snmpbb(a_in[g], w_in[g][s], O.Params(lam=lams[g]), 15)
        assert infos[i]["status"] == 0 and infos[i]["outer"] == 15
        assert abs(infos[i]["res_WH"] - hist[-1]["res_WH"]) <= 1e-9 * hist[-1]["res_WH"]


def test_batch_graph_replay_equals_direct(S):
    graphs = _graphs(1700, SHAPES[:3], restarts=2)
    As, a_in, W0s, _ = _batch_inputs(S, graphs, torch.float32)
    rs = [r for _, r, _ in graphs]
    lams = [O.default_lambda(a) for a in a_in]
    out = []
    for ug in (1, 0):
        with S.Batch(As, rs, S.params(prec=S.F32, max_outer=12, use_graph=ug), restarts=2,
                     lam=lams) as b:
            out.append(b.solve(W0s))
    for g in range(len(graphs)):
        assert torch.equal(out[0][0][g], out[1][0][g]) and torch.equal(out[0][1][g], out[1][1][g])


def _dense_sym(rng, n):
    a = rng.random((n, n))
    return 0.5 * (a + a.T)


@pytest.mark.parametrize("shapes,restarts", [
    ([(260, 64), (197, 20), (70, 3)], 3),   # few (row tile, column block) pairs: K slices
    ([(1100, 64)], 57),                      # 9 x 57 pairs: one slice, written directly
])
def test_batch_bf16x3_stacked_apass(S, shapes, restarts):
    """BF16X3 batches run one stacked split-BF16 product per problem over its S r columns
    (A_hi P_hi + A_hi P_lo + A_lo P_hi); every instance's block must be A_g P_s to the
    split's accuracy (operands exact to ~2^-16 relative, FP32 accumulation), as for the
    single solve's split A-pass."""
    rng = np.random.default_rng(1300 + restarts)
    As = [torch.from_numpy(_dense_sym(rng, n)).to(DEV, torch.float32) for n, _ in shapes]
    a_in = [a.double().cpu().numpy() for a in As]
    prm = S.params(prec=S.BF16X3, max_outer=1)
    with S.Batch([S.dense(a) for a in As], [r for _, r in shapes], prm, restarts=restarts) as b:
        P = torch.from_numpy(rng.random(b.elements)).to(DEV, torch.float32)
        B = torch.full_like(P, float("nan"))
        b.apass(P, B)
        Pn, Bn = P.double().cpu().numpy(), B.double().cpu().numpy()
    off = 0
    for g, (n, r) in enumerate(shapes):
        for s in range(restarts):
            p_s = Pn[off: off + n * r].reshape(n, r)
            b_s = Bn[off: off + n * r].reshape(n, r)
            err = nrel(b_s, O.apply_A(a_in[g], p_s))
            assert err <= 2e-5, (g, s, err)
            off += n * r
    assert off == Bn.size


def test_batch_bf16x3_instances_follow_the_oracle(S):
    """A dense BF16X3 batch of config 0 (planted n = 500, r = 10) for 20 outer iterations,
    the budget of the single solve's config-0 test: restarts 0 and 2 start from config 0's
    W0 and must match the oracle's residual and PG norm to 1e-3, as the single solve does,
    and each other bitwise; restart 1 starts at random: residual to 1e-3, PG norm (the
    quantity most sensitive to rounding after 20 iterations; 1.4e-3 measured from another
    random start) to 1e-2."""
    prob = gen.config(0)
    At = torch.from_numpy(prob["A"]).to(DEV, torch.float32)
    a_in = At.double().cpu().numpy()
    lam = O.default_lambda(a_in)
    n, r = prob["W0"].shape
    w0 = [prob["W0"], gen.start_factor(np.random.default_rng(5), n, r, float(a_in.mean())),
          prob["W0"]]
    W0 = torch.from_numpy(np.stack(w0)).to(DEV, torch.float32).contiguous()
    w_in = W0.double().cpu().numpy()
    prm = S.params(lam=lam, prec=S.BF16X3, max_outer=20)
    with S.Batch([S.dense(At)], [r], prm, restarts=3) as b:
        Ws, Hs, infos, _ = b.solve([W0])
    for s in range(2):
        _, _, hist = O.snmpbb(a_in, w_in[s], O.Params(lam=lam), 20)
        ref = hist[-1]
        info = infos[s]
        assert info["status"] == 0 and info["outer"] == 20
        assert abs(info["res_WH"] - ref["res_WH"]) <= 1e-3 * ref["res_WH"], s
        assert abs(info["pg_norm"] - ref["pg"]) <= (1e-3 if s == 0 else 1e-2) * ref["pg"], s
        W = Ws[0][s].double().cpu().numpy()
        Ht = Hs[0][s].double().cpu().numpy()
        assert (W >= 0).all() and (Ht >= 0).all()
        # the monitor against A_hi + A_lo (2^-17 elementwise) vs the FP64 residual
        assert abs(info["res_WH"] - O.residual_WH(a_in, W, Ht)) <= 5e-4 * info["res_WH"]
    assert torch.equal(Ws[0][2], Ws[0][0]) and torch.equal(Hs[0][2], Hs[0][0])
    assert infos[2]["res_WH"] == infos[0]["res_WH"]


def test_batch_bf16x3_rho_beside_the_split(S):
    """Enough restarts of rank 64 at n = 1100 that the stacked product (9 row tiles x one
    column block per restart) and the restarts' rho workgroups exceed the two workgroup
    slots per CU (the restart count is derived from this device's CU count: 52 on 256
    CUs), so rho runs in the partner split's launch instead: the first and last restarts
    must follow the oracle's solve from their starts for 5 outer iterations."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    R = (2 * cus) // 10 + 1
    assert 9 * R + R > 2 * cus
    prob = gen.planted_dense(1100, 64, 57)
    At = torch.from_numpy(prob["A"]).to(DEV, torch.float32)
    a_in = At.double().cpu().numpy()
    lam = O.default_lambda(a_in)
    rng = np.random.default_rng(57)
    w0 = np.stack([gen.start_factor(rng, 1100, 64, float(a_in.mean())) for _ in range(R)])
    W0 = torch.from_numpy(w0).to(DEV, torch.float32).contiguous()
    w_in = W0.double().cpu().numpy()
    with S.Batch([S.dense(At)], [64], S.params(lam=lam, prec=S.BF16X3, max_outer=5),
                 restarts=R) as b:
        _, _, infos, _ = b.solve([W0])
    for s in (0, R - 1):
        _, _, hist = O.snmpbb(a_in, w_in[s], O.Params(lam=lam), 5)
        assert infos[s]["status"] == 0 and infos[s]["outer"] == 5
        assert abs(infos[s]["res_WH"] - hist[-1]["res_WH"]) <= 1e-3 * hist[-1]["res_WH"], s


def test_batch_bf16x3_stop_and_breakdown_stay_in_their_restart(S):
    """Restarts of one dense problem share the stacked split-BF16 product: restart 0 stops
    at its own first monitored hit of a target, restart 2 (zero start: G = 0, rho = 0)
    breaks down, and restart 1's trajectory is bitwise the same as without them."""
    prob = gen.planted_dense(240, 6, 77)
    At = torch.from_numpy(prob["A"]).to(DEV, torch.float32)
    lam = O.default_lambda(At.double().cpu().numpy())
    rng = np.random.default_rng(9)
    w0 = np.stack([prob["W0"], gen.start_factor(rng, 240, 6, float(prob["A"].mean())),
                   np.zeros((240, 6))])
    W0 = torch.from_numpy(w0).to(DEV, torch.float32).contiguous()
    names = {v: k for k, v in S.STATUS.items()}
    with S.Batch([S.dense(At)], [6], S.params(lam=lam, prec=S.BF16X3, max_outer=30),
                 restarts=3) as b:
        _, _, base, tr = b.solve([W0], trace=True)
    tau = tr[0, 9, 0]              # restart 0's residual after 10 outer iterations
    prm = S.params(lam=lam, prec=S.BF16X3, max_outer=30, target_res=tau, check_every=4)
    with S.Batch([S.dense(At)], [6], prm, restarts=3) as b:
        _, _, infos, tr2 = b.solve([W0], trace=True)
    assert base[2]["status"] == names["E_BREAKDOWN"] == infos[2]["status"]
    hits = np.nonzero(tr[0, :, 0] <= tau)[0]
    assert infos[0]["converged_at"] == hits[0] + 1 == infos[0]["outer"]
    assert 1 <= infos[0]["converged_at"] <= 10
    for i in (0, 1):
        k = infos[i]["outer"]
        assert np.array_equal(tr2[i, :k, :5], tr[i, :k, :5]), i
    assert base[1]["status"] == 0 and base[1]["outer"] == 30


def test_batch_error_codes(S):
    graphs = _graphs(2100, [(60, 3), (80, 4)], restarts=1)
    As, _, W0s, _ = _batch_inputs(S, graphs, torch.float64)
    with pytest.raises(S.SnmfError) as e:
        S.Batch(As, [3, 4], S.params(prec=S.BF16X3), restarts=1)
    assert e.value.name == "E_UNSUPPORTED"
    dense = S.dense(torch.eye(60, dtype=torch.float64, device=DEV))
    with pytest.raises(S.SnmfError) as e:
        S.Batch([As[0], dense], [3, 3], S.params(prec=S.F64), restarts=1)
    assert e.value.name == "E_UNSUPPORTED"
    with pytest.raises(S.SnmfError) as e:
        S.Batch(As, [3, 81], S.params(prec=S.F64), restarts=1)
    assert e.value.name == "E_SHAPE"
    with pytest.raises(S.SnmfError) as e:
        S.Batch(As, [3, 4], S.params(prec=S.F64), restarts=0)
    assert e.value.name == "E_ARG"
    with pytest.raises(S.SnmfError) as e:
        S.Batch(As, [3, 4], S.params(prec=S.F64), restarts=1, lam=[0.1, -1.0])
    assert e.value.name == "E_ARG"
    with S.Batch(As, [3, 4], S.params(prec=S.F64, max_outer=2), restarts=1) as b:
        bad = [W0s[0].clone(), W0s[1].clone()]
        bad[1][0, 3, 1] = -1.0
        with pytest.raises(S.SnmfError) as e:
            b.solve(bad)
        assert e.value.name == "E_NEGATIVE"


# ------------------------------------------------------------------ the 256-graph workload
@pytest.fixture(scope="module")
def c4_reference():
    """The oracle's solve of all 2048 instances (256 SBM graphs x 8 starts) for 20 outer
    iterations (tests/golden/c4_reference.json, written by make_c4_reference.py from the
    oracle alone): breakdowns, completed outer iterations, and the last monitor record."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "c4_reference.json")
    with open(path) as f:
        ref = json.load(f)
    assert ref["outer"] == 20
    return {(i["g"], i["s"]): i for i in ref["instances"]}


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_c4_workload_against_the_oracle(S, prec, c4_reference):
    """All 2048 instances of the batched workload for 20 outer iterations.  The oracle
    breaks down on 8 of them: on these graphs (below the detection threshold) the W-step
    or H-step projects a whole factor to zero within 5 outer iterations, so the next
    half-step has rho = ||P^T P||_2 = 0.  The GPU must report E_BREAKDOWN on exactly
    those instances, after the same number of completed outer iterations or up to two more
    (a factor that the oracle projects to exact zeros can keep a few entries of rounding
    size on the device, whose tiny rho then blows the next iterate up before a non-finite
    scalar stops it), with the same record of its last completed iteration; every other
    instance must match the oracle's record after 20 outer iterations."""
    dt = DT[prec]
    graphs = gen.config(4)
    S_ = len(graphs[0]["W0"])
    As = [S.csr_from_scipy(g["A"], dt) for g in graphs]
    lams = [0.01 * float(np.sqrt(np.sum(np.asarray(g["A"].data, np.float64) ** 2))) for g in graphs]
    W0s = [torch.from_numpy(np.stack(g["W0"])).to(DEV, dt).contiguous() for g in graphs]
    with S.Batch(As, [g["r"] for g in graphs], S.params(prec=S.F64 if prec == "f64" else S.F32,
                                                       max_outer=20, check_every=1 << 30),
                 S_, lam=lams) as b:
        _, _, infos, tr = b.solve(W0s, trace=True)
    broken_gpu = {divmod(i, S_) for i, inf in enumerate(infos) if inf["status"] != 0}
    broken_or = {k for k, v in c4_reference.items() if v["breakdown"]}
    assert len(broken_or) == 8
    assert broken_gpu == broken_or, (sorted(broken_gpu ^ broken_or))
    tol = 1e-9 if prec == "f64" else 1e-3
    for (g, s) in sorted(broken_or):
        inf, ref = infos[g * S_ + s], c4_reference[(g, s)]
        assert inf["status"] == 9
        assert ref["outer"] <= inf["outer"] <= ref["outer"] + 2, ((g, s), inf["outer"], ref["outer"])
        rec = tr[g * S_ + s, ref["outer"] - 1]
        assert abs(rec[0] - ref["res_WH"]) <= tol * ref["res_WH"], ((g, s), rec[0], ref["res_WH"])
    # every other instance: its record after 20 outer iterations, to tol plus three times
    # what rounding-size changes of the factors after every outer iteration (absolute, of
    # FP64 size for the FP64 solve, of FP32 size as well for the FP32 one) move the
    # oracle's own record.  Near a saddle point with whole columns of both factors at
    # zero, such changes revive them and the iteration leaves the saddle, a thousandfold
    # per outer iteration: there the oracle's perturbed runs differ by up to 1e-2 from its
    # unperturbed one, by 1e-16 elsewhere
    errs = {"res_WH": [], "objective": [], "pg": []}
    sens = {"res_WH": [], "objective": [], "pg": []}
    for i, inf in enumerate(infos):
        g, s = divmod(i, S_)
        ref = c4_reference[(g, s)]
        if ref["breakdown"]:
            continue
        assert inf["status"] == 0 and inf["outer"] == 20
        perts = [ref["perturbed"]] + ([ref["perturbed32"]] if prec == "f32" else [])
        for k, got in (("res_WH", inf["res_WH"]), ("objective", inf["objective"]),
                       ("pg", inf["pg_norm"])):
            errs[k].append(abs(got - ref[k]) / abs(ref[k]))
            sens[k].append(max(abs(p[k] - ref[k]) / abs(ref[k]) if not p["breakdown"] else np.inf
                               for p in perts))
    for k in errs:
        e, d = np.array(errs[k]), np.array(sens[k])
        print(f"{prec} {k}: relative error median {np.median(e):.2e} 99% {np.quantile(e, 0.99):.2e} "
              f"max {e.max():.2e}; oracle's own spread 99% {np.quantile(d[np.isfinite(d)], 0.99):.2e}; "
              f"instances beyond tol {int(np.sum(e > tol))}")
        if k != "pg":
            bad = np.nonzero(e > tol + 3.0 * d)[0]
            assert bad.size == 0, (k, [(int(j), e[j], d[j]) for j in bad[:5]])


# ------------------------------------------------------------------ launch-shape autotuner
def test_tuned_batches_agree_and_the_choice_is_cached(S, tmp_path):
    """Every launch shape gives the same iteration (FP64: the same records to 1e-12, the
    grouping of the partial sums being the only change); the tuner's choice lies in the
    candidate sets, and a second call with the same kind of batch reads it from the cache."""
    from paper_2606_02887_amd import autotune
    graphs = gen.batched_sbm(num_graphs=12, n_lo=300, n_hi=900, restarts=2, seed=4242)
    As = [S.csr_from_scipy(g["A"], torch.float64) for g in graphs]
    rs = [g["r"] for g in graphs]
    W0s = [torch.from_numpy(np.stack(g["W0"])).to(DEV, torch.float64).contiguous() for g in graphs]
    base = None
    for cfg in (None, {"tiles_per_wg": [1, 2, 16, 4], "spmm_rows_per_wg": 4},
                {"tiles_per_wg": [8, 1, 1, 4], "spmm_rows_per_wg": 64}):
        with S.Batch(As, rs, S.params(prec=S.F64, lam=0.05, max_outer=4, tuning=cfg), 2) as b:
            _, Hs, infos, _ = b.solve(W0s)
        res = np.array([i["res_WH"] for i in infos])
        if base is None:
            base = res
        else:
            assert np.max(np.abs(res - base) / base) <= 1e-12
    path = str(tmp_path / "tuning.json")
    log = []
    cfg, hit = autotune.tune(S, torch, As, rs, 2, W0s, S.F64, outer=3, reps=1, cache_path=path,
                             log=log)
    assert not hit and len(log) >= 5
    assert all(t in autotune.TILES for t in cfg["tiles_per_wg"])
    assert cfg["spmm_rows_per_wg"] in autotune.SPMM_ROWS
    cfg2, hit2 = autotune.tune(S, torch, As, rs, 2, W0s, S.F64, cache_path=path)
    assert hit2 and cfg2 == cfg
    with pytest.raises(S.SnmfError) as e:
        S.Batch(As, rs, S.params(prec=S.F64, tuning={"tiles_per_wg": [0, 4, 4, 4],
                                                     "spmm_rows_per_wg": 16}), 2)
    assert e.value.name == "E_ARG"
