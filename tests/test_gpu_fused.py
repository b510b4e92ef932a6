"""The fused inner iterations (fuse_inner = 1, the default) against the two-kernel path
(fuse_inner = 0) and the oracle.

A fused kernel runs the line search of inner iteration k, the update and direction k + 1;
it takes the BB step of iteration k + 1 from sums its predecessor prepared.  When the line
search accepts beta = 1 those are the update's own sums, formed with step 2's operations,
so a solve in which no trial backtracks (max_ls = 0) gives the same bits on both paths:
the factors, every info field but the clock and every trace column but the time stamp.
After a backtrack the sums come from S = dZ + phi beta D (unclipped for phi beta <= 1), the
same numbers up to rounding: the FP64 solves then match the oracle as closely as the
two-kernel path does (1e-9), and the two paths agree to 1e-10 in FP64.  Cases: dense FP32,
split BF16 and FP64, CSR, low rank; a strict monotone line search (theta = 0.5, eta = 0)
that backtracks often; one, three and five inner iterations; workgroups owning several row
tiles (n = 40000, r = 64); Graph-SNMPBB and the naive variant, whose W-steps take the fused
path and H-steps the two-kernel one.
"""
import numpy as np
import pytest

import oracle as O
from paper_2606_02887_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
CLOCK = ("seconds", "seconds_to_target")
TRACE_TIME = 5


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_02887_amd import snmf
    return snmf


def _t(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV, dt)


def _both(S, M, W0, L=None, **kw):
    kw.setdefault("max_ls", 0)   # no backtracking: the two paths give the same bits
    out = []
    for fuse in (1, 0):
        prm = S.params(fuse_inner=fuse, **kw)
        W, Ht, info = S.solve(M, W0, prm, L=L)
        torch.cuda.synchronize()
        out.append((W.cpu().numpy(), Ht.cpu().numpy(), info))
    return out


def _same(a, b):
    (Wa, Ha, ia), (Wb, Hb, ib) = a, b
    assert np.array_equal(Wa, Wb) and np.array_equal(Ha, Hb)
    for k in ia:
        if k in CLOCK or k == "trace":
            continue
        va, vb = ia[k], ib[k]
        assert (va == vb) or (va != va and vb != vb), (k, va, vb)
    ta, tb = ia["trace"], ib["trace"]
    keep = [c for c in range(ta.shape[1]) if c != TRACE_TIME]
    assert ta.shape == tb.shape
    assert np.array_equal(ta[:, keep], tb[:, keep], equal_nan=True)


def _planted(n, r, seed):
    p = gen.planted_dense(n, r, seed)
    return p["A"], p["W0"], O.default_lambda(p["A"])


@pytest.mark.parametrize("prec,n,r", [("f32", 700, 64), ("bf16x3", 700, 64), ("f32", 1000, 20),
                                      ("f64", 300, 5), ("f64", 520, 33)])
def test_fused_dense_same_bits(S, prec, n, r):
    A, W0, lam = _planted(n, r, 40 + r)
    dt = torch.float64 if prec == "f64" else torch.float32
    p = {"f32": S.F32, "bf16x3": S.BF16X3, "f64": S.F64}[prec]
    a, b = _both(S, S.dense(_t(A, dt)), _t(W0, dt), lam=lam, prec=p, max_outer=12)
    print(f"dense {prec} n={n} r={r}: res {a[2]['res_WH']:.6e}, line-search trials "
          f"{a[2]['ls_evals']} for {a[2]['inner_total']} inner iterations")
    _same(a, b)


def test_fused_backtracking_matches_oracle(S):
    """theta = 0.5, eta = 0: the acceptance test is monotone and strict, so many inner
    iterations backtrack and take the BB step from the polynomial sums."""
    A, W0, lam = _planted(600, 12, 77)
    outer = 15
    a, b = _both(S, S.dense(_t(A, torch.float64)), _t(W0, torch.float64), lam=lam,
                 prec=S.F64, max_outer=outer, theta=0.5, eta=0.0, max_ls=20)
    info = a[2]
    backtracked = info["ls_evals"] - info["inner_total"]
    _, _, hist = O.snmpbb(A, W0, O.Params(lam=lam, theta=0.5, eta=0.0), outer)
    res_o = np.array([h["res_WH"] for h in hist])
    pg_o = np.array([h["pg"] for h in hist])
    tr = info["trace"]
    e_res = np.abs(tr[:, 0] - res_o).max() / res_o.max()
    e_pg = np.abs(tr[:, 3] - pg_o).max() / pg_o.max()
    e_two = max(np.abs(a[0] - b[0]).max() / np.abs(b[0]).max(),
                np.abs(a[1] - b[1]).max() / np.abs(b[1]).max())
    print(f"{info['ls_evals']} trials for {info['inner_total']} inner iterations; oracle: "
          f"residual {e_res:.1e}, PG {e_pg:.1e}; two-kernel path {e_two:.1e}")
    assert backtracked >= 10
    assert e_res <= 1e-9 and e_pg <= 1e-9
    assert e_two <= 1e-10


@pytest.mark.parametrize("inner", [1, 3, 5])
def test_fused_inner_counts_same_bits(S, inner):
    A, W0, lam = _planted(500, 16, 5 + inner)
    a, b = _both(S, S.dense(_t(A, torch.float32)), _t(W0, torch.float32), lam=lam,
                 prec=S.F32, max_outer=10, inner_iters=inner)
    assert a[2]["inner_total"] == 2 * 10 * inner
    _same(a, b)


def test_fused_csr_several_tiles_per_workgroup(S):
    """n = 40000, r = 64: 1250 row tiles of 32 rows on 1024 workgroups.  (At r <= 32 in
    FP32 a fused plan keeps two workgroups per CU and a two-kernel plan three, so their
    partial sums are grouped differently there.)"""
    n, r = 40000, 64
    a_ = gen.random_symmetric_csr(n, 6.0, 3)
    rng = np.random.default_rng(2)
    W0 = gen.start_factor(rng, n, r, gen.mean_of_sparse(a_))
    M = S.csr_from_scipy(a_, torch.float32)
    lam = 0.01 * float(np.sqrt(np.sum(a_.data.astype(np.float32).astype(np.float64) ** 2)))
    a, b = _both(S, M, _t(W0, torch.float32), lam=lam, prec=S.F32, max_outer=4)
    _same(a, b)


@pytest.mark.parametrize("ntiles", [257, 513])
def test_fused_partial_grid_edges_same_bits(S, ntiles):
    """FP32 at r = 64: both forms launch one workgroup per 32-row tile (up to 1024), and
    every kernel re-reduces one row of partial sums per workgroup, thread t adding the rows
    t, t + 256, ... (two per pass).  257 rows: one thread has a second row; 513: one pass
    more.  The fused kernels' slot-major sums and the two-kernel form's row-major ones must
    add the same rows in the same order."""
    n, r = 32 * ntiles, 64
    a_ = gen.random_symmetric_csr(n, 6.0, 40 + ntiles)
    rng = np.random.default_rng(ntiles)
    W0 = gen.start_factor(rng, n, r, gen.mean_of_sparse(a_))
    M = S.csr_from_scipy(a_, torch.float32)
    lam = 0.01 * float(np.sqrt(np.sum(a_.data.astype(np.float32).astype(np.float64) ** 2)))
    a, b = _both(S, M, _t(W0, torch.float32), lam=lam, prec=S.F32, max_outer=4)
    _same(a, b)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_lowrank_same_bits(S, prec):
    n, ell, r = 4000, 24, 16
    rng = np.random.default_rng(12)
    U, _ = np.linalg.qr(rng.standard_normal((n, ell)))
    lam_ = np.sort(rng.random(ell))[::-1] * 50.0 + 1.0
    W0 = rng.random((n, r)) * 0.05
    dt = torch.float64 if prec == "f64" else torch.float32
    p = S.F64 if prec == "f64" else S.F32
    M = S.lowrank(_t(U, dt), _t(lam_, torch.float64))
    a, b = _both(S, M, _t(W0, dt), lam=O.default_lambda(O.LowRank(U, lam_)), prec=p,
                 max_outer=10)
    _same(a, b)


def test_fused_graph_and_naive_same_bits(S):
    """Graph-SNMPBB (the H-step carries the Laplacian term and keeps two kernels per inner
    iteration) and the naive variant (its H-step is H <- W)."""
    p = gen.sbm_problem(n=800, k=4, r=4, p_in=0.1, p_out=0.01, seed=21)
    A, L = p["A"], O.knn_laplacian(p["X"], p["knn"])
    rng = np.random.default_rng(3)
    W0 = gen.start_factor(rng, A.shape[0], 4, gen.mean_of_sparse(A))
    for prec, dt in ((S.F32, torch.float32), (S.F64, torch.float64)):
        Ag, Lg = S.csr_from_scipy(A, dt), S.csr_from_scipy(L, dt)
        a, b = _both(S, Ag, _t(W0, dt), L=Lg, lam=O.default_lambda(A), gamma=0.5, prec=prec,
                     max_outer=10)
        _same(a, b)
        a, b = _both(S, Ag, _t(W0, dt), lam=0.0, naive=1, prec=prec, max_outer=10)
        _same(a, b)


@pytest.mark.parametrize("prec,kind", [("f32", "dense"), ("f64", "dense"), ("f32", "csr")])
def test_fused_nmf_same_bits(S, prec, kind):
    """Rectangular NMF (eq. (1.1)) runs the same inner kernels: its W-step and H-step take
    the fused form too (arrays below 4 MiB) and give the two-kernel form's bits."""
    dt = torch.float64 if prec == "f64" else torch.float32
    p = S.F64 if prec == "f64" else S.F32
    if kind == "dense":
        m, n = 700, 450
        prob = gen.planted_rect(m, n, 12, 5)
        M = S.dense(_t(prob["V"], dt))
    else:
        m, n = 3000, 1700
        prob = gen.random_rect_csr(m, n, 0.02, 16, 6)
        M = S.csr_from_scipy(prob["V"], dt)
    W0, H0 = _t(prob["W0"], dt), _t(prob["Ht0"], dt)
    out = []
    for fuse in (1, 0):
        W, Ht, info = S.nmf_solve(M, n, W0, H0, S.params(prec=p, lam=0.0, max_outer=10, max_ls=0,
                                                         fuse_inner=fuse))
        torch.cuda.synchronize()
        out.append((W.cpu().numpy(), Ht.cpu().numpy(), info))
    _same(out[0], out[1])
