"""Half-step parity at the benchmark sizes, in the launch configuration bench.py times.

The dense planted problem at n = 8192, r = 64 (the FP32 A-pass with its balanced split
over two workgroups per CU, and the split-BF16 A-pass, each with the fused rho workgroup),
the graph problem
at n = 20000, r = 20 (CSR A-pass and the Laplacian products of the H-step) and the
low-rank problem at n = 200000, ell = 64, r = 32 (the LAI products; the n x r arrays hold
more than 4 MiB, so step 2 forms D again).  The oracle's half-step at these sizes costs a
few dense or low-rank products on the CPU, so every entry of X+ is compared.

Tolerances (normwise on X+ after one half-step of five inner iterations): FP32 sums of
n = 8192 to 200000 terms carry about sqrt(n) 2^-24 = 5e-6 to 3e-5 relative rounding into
B, which the inner iterations pass on to X, so FP32 is held to 3e-5; split BF16 adds the
2^-17 element error of A_hi + A_lo, 5e-5.  Measured: 1.9e-6 (dense FP32), 2.5e-6 (split
BF16), 1.9e-7 (graph), 5.3e-7 (low rank).
"""
import numpy as np
import pytest

import oracle as O
from paper_2606_02887_amd import gen
from parity_util import elem_rel, nrel
from rounding_model import half_step_fp32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_02887_amd import snmf
    return snmf


# entrywise bound: |a - b| <= etol (|b| + 1e-3 max|b|) with etol = max(1e-4, 10 x the
# entrywise movement of the FP32 rounding model); an entry is formed from terms of the
# size of max|X|, whose FP32 rounding over five inner iterations, relative to the 1e-3
# floor, is about 1e-4 unless the BB steps amplify it (the model measures that)
ETOL = 1e-4


def _etol():
    return max(ETOL, 10.0 * _half_step.model[1])


def _t(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV, dtype)


def _half_step(S, Aop_gpu, Aop_oracle, X, P, prec, is_hstep, lam, gamma=0.0, L_gpu=None,
               L_or=None, fuse=1):
    Xt, Pt = _t(X, torch.float32), _t(P, torch.float32)
    X_in, P_in = Xt.double().cpu().numpy(), Pt.double().cpu().numpy()
    prm = S.params(lam=lam, gamma=gamma, prec=prec, inner_iters=5, max_outer=1, validate=0,
                   fuse_inner=fuse)
    pl = S.Plan(Aop_gpu, X.shape[1], prm, L_gpu)
    sc = pl.half_step(Xt, Pt, bool(is_hstep))
    pl.close()
    log = []
    oprm = O.Params(lam=lam, gamma=gamma, inner_iters=5)
    Xo = O.half_step(Aop_oracle, X_in, P_in, oprm, laplacian=L_or is not None, L=L_or, log=log)
    # what FP32 rounding of the gradient update alone moves X+ (tests/rounding_model.py)
    Xm = half_step_fp32(O.HalfStep(Aop_oracle, P_in, lam, gamma, L_or), X_in, oprm)
    _half_step.model = (nrel(Xm, Xo), elem_rel(Xm, Xo))
    return Xt.double().cpu().numpy(), Xo, sc, log


def _scalars(sc, log, tol):
    assert abs(sc["rho"] - log[0]["rho"]) <= 1e-10 * log[0]["rho"]
    assert abs(sc["alpha"] - log[-1]["alpha"]) <= tol * log[-1]["alpha"]
    assert abs(sc["beta"] - log[-1]["beta"]) <= tol
    assert abs(sc["ss"] - log[-1]["ss"]) <= tol * log[-1]["ss"]
    assert int(sc["ls_evals"]) == sum(e["evals"] for e in log)


@pytest.fixture(scope="module")
def dense_c1():
    p = gen.config(1)                                   # planted dense n = 8192, r = 64
    A = p["A"]
    At = _t(A, torch.float32)
    A_in = At.double().cpu().numpy()                    # the FP32-rounded input both sides see
    lam = 0.01 * float(np.sqrt(np.sum(A_in * A_in)))    # bench.py's lambda
    P = gen.start_factor(np.random.default_rng(3), A.shape[0], 64, float(A.mean()))
    return At, A_in, p["W0"], P, lam


@pytest.mark.parametrize("form,tol", [("f32", 3e-5), ("bf16x3", 5e-5)])
@pytest.mark.parametrize("is_hstep", [0, 1])
def test_dense_n8192_r64_half_step(S, dense_c1, form, tol, is_hstep):
    At, A_in, X, P, lam = dense_c1
    prec = S.F32 if form == "f32" else S.BF16X3
    Xg, Xo, sc, log = _half_step(S, S.dense(At), A_in, X, P, prec, is_hstep, lam)
    err = nrel(Xg, Xo)
    ee = elem_rel(Xg, Xo)
    print(f"dense n=8192 r=64 {form} is_hstep={is_hstep}: nrel {err:.3e} entrywise {ee:.3e}")
    assert ee <= _etol(), (ee, _half_step.model)
    assert err <= tol
    _scalars(sc, log, 1e-3)
    assert (Xg >= 0).all()


def test_graph_n20000_r20_hstep(S):
    p = gen.config(2)                                   # SBM n = 20000, 10-NN Laplacian
    A, L = p["A"], O.knn_laplacian(p["X"], p["knn"])
    r = 20
    Ag, Lg = S.csr_from_scipy(A, torch.float32), S.csr_from_scipy(L, torch.float32)
    import scipy.sparse as sp
    A_in = sp.csr_matrix((Ag.keep[2].double().cpu().numpy(), A.indices, A.indptr), A.shape)
    L_in = sp.csr_matrix((Lg.keep[2].double().cpu().numpy(), L.indices, L.indptr), L.shape)
    lam = 0.01 * float(np.sqrt(np.sum(A_in.data ** 2)))
    X = p["W0"]
    P = gen.start_factor(np.random.default_rng(4), A.shape[0], r, float(A_in.mean()))
    Xg, Xo, sc, log = _half_step(S, Ag, A_in, X, P, S.F32, 1, lam, gamma=0.2, L_gpu=Lg,
                                 L_or=L_in)
    err = nrel(Xg, Xo)
    ee = elem_rel(Xg, Xo)
    print(f"graph n=20000 r=20 H-step: nrel {err:.3e} entrywise {ee:.3e}")
    assert ee <= _etol(), (ee, _half_step.model)
    assert err <= 3e-5
    _scalars(sc, log, 1e-3)


@pytest.mark.parametrize("fuse", [1, 0])
def test_lowrank_n200000_r32_half_step(S, fuse):
    """fuse = 1: one kernel per inner iteration, two workgroups per CU (512).  fuse = 0:
    two kernels, three workgroups per CU (768), so every kernel re-reduces more than 512
    rows of partial sums, the loader's second pass."""
    q = gen.config(3)                                   # LAI n = 200000, ell = 64
    U, lamv = O.range_finder(q["A"], q["rank"], q["power_iters"], q["Omega"])
    r = 32
    Ut = _t(U, torch.float32)
    lr_in = O.LowRank(Ut.double().cpu().numpy(), lamv)
    lam = 0.01 * float(np.sqrt(np.sum(lamv ** 2)))     # bench.py's lambda
    X = q["W0"]
    P = np.random.default_rng(5).random(X.shape) * float(X.mean())
    Xg, Xo, sc, log = _half_step(S, S.lowrank(Ut, _t(lamv, torch.float64)), lr_in, X, P,
                                 S.F32, 0, lam, fuse=fuse)
    err = nrel(Xg, Xo)
    ee = elem_rel(Xg, Xo)
    print(f"low rank n=200000 r=32 fuse={fuse}: nrel {err:.3e} entrywise {ee:.3e}")
    assert ee <= _etol(), (ee, _half_step.model)
    assert err <= 3e-5
    _scalars(sc, log, 1e-3)


def test_dense_n8192_batched8_bf16x3_stacked_apass(S, dense_c1):
    """The stacked split-BF16 A-pass of bench.py's 8 batched restarts (8192 x 8192 times
    8 x (8192 x 64), one launch of 64 x 8 (row tile, column block) workgroups): every
    instance's block against the FP64 product, to the split's accuracy (3e-5: the
    single-solve split bound with FP32 sums over 8192 terms)."""
    At, A_in, _, _, _ = dense_c1
    rng = np.random.default_rng(1101)
    with S.Batch([S.dense(At)], [64], S.params(prec=S.BF16X3, max_outer=1), restarts=8) as b:
        P = torch.from_numpy(rng.random(b.elements)).to(DEV, torch.float32)
        B = torch.full_like(P, float("nan"))
        b.apass(P, B)
        Pn = P.double().cpu().numpy().reshape(8, 8192, 64)
        Bn = B.double().cpu().numpy().reshape(8, 8192, 64)
    for s in range(8):
        err = nrel(Bn[s], A_in @ Pn[s])
        print(f"batched8 bf16x3 restart {s}: nrel {err:.3e}")
        assert err <= 3e-5, (s, err)


def test_lowrank_n200000_device_sketch(S):
    """The surrogate of the LAI workload built on the device (snmf_lai_sketch: the
    power-law graph n = 200000, rank 64 + 10, two power iterations, FP32) against the
    oracle's range finder from the same Omega: eigenvalues within 1e-5 of |lam_1| and the
    subspaces within a sine of 1e-5 (as far as the oracle's own gap between the 64th and
    65th Ritz values allows: Davis-Kahan with 100 x 2^-24 |lam_1| / gap)."""
    q = gen.config(3)
    M = S.csr_from_scipy(q["A"], torch.float32)
    Om = _t(q["Omega"], torch.float32)
    U, lam = S.lai_sketch(M, q["rank"], q["power_iters"], Om)
    ref = q["A"].copy().astype(np.float64)
    ref.data = M.keep[2].double().cpu().numpy()
    om = Om.double().cpu().numpy()
    Uo, lo = O.range_finder(ref, q["rank"], q["power_iters"], om)
    _, ritz = O.range_finder(ref, om.shape[1], q["power_iters"], om)
    Ug, lg = U.double().cpu().numpy(), lam.cpu().numpy()
    lerr = np.abs(lg - lo).max() / abs(lo[0])
    ang = float(np.linalg.norm(Ug - Uo @ (Uo.T @ Ug), 2))
    gap = abs(ritz[q["rank"] - 1]) - abs(ritz[q["rank"]])
    bound = max(1e-5, 100 * 2.0 ** -24 * abs(ritz[0]) / gap)
    print(f"device sketch n=200000: eigenvalues {lerr:.2e}, sin angle {ang:.2e} (bound {bound:.1e})")
    assert lerr <= 1e-5
    assert ang <= bound


@pytest.mark.parametrize("form", ["f32", "bf16x3"])
def test_dense_n8192_r64_whole_solve_2000_outer(S, form):
    """The benchmark workload solved for its full budget of 2000 outer iterations, against
    the oracle's runs from the same start and from three rounding-level changes of it
    (tests/golden/c1_reference.json and c1_perturbed_*.json, written by
    make_c1_reference.py from the oracle alone).  Eight GPU starts (W0 and seven
    2^-22 changes of it, one batched solve): the residual from W0, and from every other
    start, within 1e-3 of the oracle's (the oracle's own four runs spread by 2.4e-4); the
    mean log projected-gradient norm within 4 standard errors of the oracle ensemble's
    (the oracle's runs: 878 to 1799, a factor 2 spread by 2000 iterations)."""
    import json
    import os
    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    runs = [json.load(open(os.path.join(gdir, "c1_reference.json")))]
    for s in (1, 2, 3):
        runs.append(json.load(open(os.path.join(gdir, f"c1_perturbed_{s}.json"))))
    res_ref = runs[0]["res_ref"]
    lam = runs[0]["lambda"]
    ores = np.array([r["res_ref"] for r in runs])
    opg = np.array([r["pg_ref"] for r in runs])
    p = gen.config(1)
    A = _t(p["A"], torch.float32)
    W0 = p["W0"]
    starts = np.stack([W0] + [W0 * (1.0 + 2.0 ** -22 * np.random.default_rng(300 + s).choice(
        [-1.0, 1.0], size=W0.shape)) for s in range(7)])
    prec = S.F32 if form == "f32" else S.BF16X3
    with S.Batch([S.dense(A)], [64], S.params(lam=lam, prec=prec, max_outer=2000,
                                             check_every=1 << 30), 8, lam=[lam]) as b:
        _, _, infos, _ = b.solve([_t(starts, torch.float32)])
    assert all(i["status"] == 0 and i["outer"] == 2000 for i in infos)
    gres = np.array([i["res_WH"] for i in infos])
    gpg = np.array([i["pg_norm"] for i in infos])
    lg, lo = np.log(gpg), np.log(opg)
    z = abs(lg.mean() - lo.mean()) / np.sqrt(lg.var(ddof=1) / lg.size + lo.var(ddof=1) / lo.size)
    print(f"2000 outer {form}: res from W0 {gres[0]:.8f} (oracle {res_ref:.8f}, rel "
          f"{abs(gres[0] - res_ref) / res_ref:.1e}); res over starts {gres.min():.8f}.."
          f"{gres.max():.8f}; PG {gpg.min():.0f}..{gpg.max():.0f} (oracle {opg.min():.0f}.."
          f"{opg.max():.0f}), z {z:.2f}")
    assert abs(gres[0] - res_ref) <= 1e-3 * res_ref
    assert np.all(np.abs(gres - ores.mean()) <= 1e-3 * ores.mean())
    assert z <= 4.0


def test_graph_n20000_device_laplacian(S):
    """The graph workload's Laplacian (10-NN over 16-dim features, n = 20000) built on the
    device: pattern identical to the oracle's, values within FP32 rounding."""
    p = gen.config(2)
    X = _t(p["X"], torch.float32)
    M = S.knn_graph(X, p["knn"])
    rowptr, col, val = (t.cpu().numpy() for t in M.keep)
    ref = O.knn_laplacian(X.double().cpu().numpy(), p["knn"])
    assert np.array_equal(rowptr, ref.indptr) and np.array_equal(col, ref.indices)
    assert np.abs(val.astype(np.float64) - ref.data).max() <= 2e-7
