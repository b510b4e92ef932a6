"""Per-kernel parity of the HIP primitives against the FP64 oracle on identical inputs.

Tolerances: normwise relative error <= 1e-12 (FP64 kernels; 1e-13 where the operation
is a single reduction), <= 1e-5 (FP32), BF16 split bit-exact against a round-to-nearest-
even emulation, split-BF16 product stated per case (<= 2e-5).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2606_02887_amd import gen
from parity_util import comp_rel, nrel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_02887_amd import snmf
    return snmf


DEV = "cuda"


def _t(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV, dtype)


# ------------------------------------------------------------------ rho = ||G||_2
@pytest.mark.parametrize("r", [1, 2, 5, 10, 20, 31, 32, 33, 64])
def test_rho_matches_eigvalsh(S, r):
    rng = np.random.default_rng(r)
    P = rng.random((3 * r + 5, r))
    G = P.T @ P
    got = S.rho(_t(G, torch.float64))
    ref = O.spectral_norm_psd(G)
    assert abs(got - ref) <= 1e-13 * ref


def test_rho_near_degenerate_spectrum(S):
    """Equal-size clusters give G ~ c I: r nearly equal eigenvalues, still exact to 1e-13."""
    rng = np.random.default_rng(3)
    r, n = 20, 400
    P = 1e-8 * rng.random((n, r))
    P[np.arange(n), np.arange(n) % r] += 1.0 + 1e-6 * rng.random(n)
    G = P.T @ P
    ev = np.linalg.eigvalsh(G)
    assert (ev[-1] - ev[0]) / ev[-1] < 1e-5
    got = S.rho(_t(G, torch.float64))
    ref = O.spectral_norm_psd(G)
    assert abs(got - ref) <= 1e-13 * ref


# ------------------------------------------------------------------ Gram and A-pass
# (132, 34) and (260, 64): FP32 workgroup chunks longer than a tile's K (one workgroup
# spans several tiles); (2048, 64), (4100, 34), (4608, 64): chunks that end inside tiles
@pytest.mark.parametrize("n,r", [(1, 1), (37, 5), (132, 34), (260, 64), (500, 10), (1029, 33),
                                 (2048, 64), (4100, 34), (4608, 64)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gram_and_dense_apass(S, n, r, prec):
    rng = np.random.default_rng(n * 100 + r)
    A = rng.random((n, n))
    A = 0.5 * (A + A.T)
    P = rng.random((n, r))
    dt = torch.float64 if prec == "f64" else torch.float32
    At, Pt = _t(A, dt), _t(P, dt)
    A_in = At.double().cpu().numpy()       # identical (possibly rounded) inputs
    P_in = Pt.double().cpu().numpy()
    pl = S.Plan(S.dense(At), r, S.params(prec=S.F64 if prec == "f64" else S.F32, max_outer=1))
    G = pl.gram(Pt).cpu().numpy()
    assert nrel(G, P_in.T @ P_in) <= 1e-13
    B = torch.empty_like(Pt)
    pl.apass(Pt, B)
    tol = 1e-12 if prec == "f64" else 1e-5
    ref = O.apply_A(A_in, P_in)
    assert nrel(B.cpu().numpy(), ref) <= tol
    # A, P >= 0: every entry is a sum of nonnegative terms, |A||P| = A P
    assert comp_rel(B.cpu().numpy(), ref, ref) <= tol
    pl.close()


@pytest.mark.parametrize("n,r", [(64, 8), (500, 10), (1000, 32), (1100, 64), (2048, 40)])
def test_split_bf16_apass(S, n, r):
    rng = np.random.default_rng(7 + n)
    A = rng.random((n, n))
    A = 0.5 * (A + A.T)
    P = rng.random((n, r))
    At, Pt = _t(A, torch.float32), _t(P, torch.float32)
    A_in = At.double().cpu().numpy()
    P_in = Pt.double().cpu().numpy()
    pl = S.Plan(S.dense(At), r, S.params(prec=S.BF16X3, max_outer=1))
    B = torch.empty_like(Pt)
    pl.apass(Pt, B)
    ref = O.apply_A(A_in, P_in)
    err = nrel(B.cpu().numpy(), ref)
    # three-product split: operands exact to ~2^-16 relative, FP32 accumulation
    assert err <= 2e-5, err
    # entrywise: each operand's hi + lo is within 2^-17 of it, so every (nonnegative)
    # term is within ~2^-16 of its value, plus the FP32 sum: 3e-5 of A P per entry
    assert comp_rel(B.cpu().numpy(), ref, ref) <= 3e-5
    pl.close()


def _bf16_rne_bits(x32):
    u = x32.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r & 0xFFFF).astype(np.uint16)


def test_bf16_split_is_round_to_nearest_even(S):
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.random(5000), rng.standard_normal(5000) * 1e3,
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e-39]]).astype(np.float32)
    hi, lo = S.split_bf16(_t(x, torch.float32))
    hi = hi.cpu().numpy().view(np.uint16)
    lo = lo.cpu().numpy().view(np.uint16)
    ref_hi = _bf16_rne_bits(x)
    hi_f = (ref_hi.astype(np.uint32) << 16).view(np.float32)
    ref_lo = _bf16_rne_bits((x - hi_f).astype(np.float32))
    assert np.array_equal(hi, ref_hi)
    assert np.array_equal(lo, ref_lo)
    recon = hi_f.astype(np.float64) + (ref_lo.astype(np.uint32) << 16).view(np.float32)
    rel = np.abs(recon - x) / np.maximum(np.abs(x), 1e-30)
    assert rel[np.abs(x) > 1e-30].max() <= 2.0 ** -16


# ------------------------------------------------------------------ CSR SpMM
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("r", [1, 7, 20, 32, 64])
def test_csr_spmm(S, prec, r):
    rng = np.random.default_rng(r)
    n = 3001
    a = sp.random(n, n, density=0.003, random_state=5, format="csr")
    a = (a + a.T + sp.diags(rng.random(n))).tolil()
    a[11, :] = rng.random(n) * (rng.random(n) < 0.5)  # one long row (~n/2 nonzeros)
    a[7, :] = 0                                       # an empty row
    a = a.tocsr()
    a.eliminate_zeros()
    a.sort_indices()
    assert a.indptr[8] == a.indptr[7]
    dt = torch.float64 if prec == "f64" else torch.float32
    M = S.csr_from_scipy(a, dt)
    X = _t(rng.random((n, r)), dt)
    Y = S.spmm(M, X)
    a_in = sp.csr_matrix((M.keep[2].double().cpu().numpy(), a.indices, a.indptr), shape=a.shape)
    ref = a_in @ X.double().cpu().numpy()
    tol = 1e-13 if prec == "f64" else 1e-6
    assert nrel(Y.cpu().numpy(), ref) <= tol
    mag = abs(a_in) @ np.abs(X.double().cpu().numpy())
    assert comp_rel(Y.cpu().numpy(), ref, mag) <= (1e-13 if prec == "f64" else 2e-6)


# ------------------------------------------------------------------ LAI product
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,ell,r", [(997, 16, 5), (20000, 74, 32), (5000, 128, 64),
                                    (70000, 16, 16)])
def test_lai_apass(S, prec, n, ell, r):
    rng = np.random.default_rng(n + ell)
    U, _ = np.linalg.qr(rng.standard_normal((n, ell)))
    lam = rng.standard_normal(ell) * 10
    P = rng.random((n, r))
    dt = torch.float64 if prec == "f64" else torch.float32
    Ut, Pt = _t(U, dt), _t(P, dt)
    lamt = _t(lam, torch.float64)
    pl = S.Plan(S.lowrank(Ut, lamt), r, S.params(prec=S.F64 if prec == "f64" else S.F32,
                                                  max_outer=1, validate=0))
    B = torch.empty_like(Pt)
    pl.apass(Pt, B)
    ref = O.apply_A(O.LowRank(Ut.double().cpu().numpy(), lam), Pt.double().cpu().numpy())
    tol = 1e-12 if prec == "f64" else 2e-6
    assert nrel(B.cpu().numpy(), ref) <= tol
    # entrywise against |U| |lam| |U|^T |P| (U has mixed signs: the products cancel)
    Ua = np.abs(Ut.double().cpu().numpy())
    mag = Ua @ (np.abs(lam)[:, None] * (Ua.T @ np.abs(Pt.double().cpu().numpy())))
    assert comp_rel(B.cpu().numpy(), ref, mag) <= (1e-13 if prec == "f64" else 2e-6)
    pl.close()
