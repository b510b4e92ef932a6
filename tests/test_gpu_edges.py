"""Degenerate and edge cases of the range finder, rectangular NMF and the naive variant,
through the C ABI against the oracle."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2606_02887_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_02887_amd import snmf
    return snmf


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_range_finder_on_an_exactly_rank_deficient_matrix(S, prec):
    """A = W W^T of rank 3 sketched at rank 6 (+4 oversampling, two power iterations): the
    sketch loses rank, the shifted Cholesky QR absorbs it, the three nonzero eigenvalues
    match the oracle's (1e-10 / 1e-5 of |lam_1|) and the other three are rounding-size on
    both sides; U stays orthonormal.  Both sides see the same stored A."""
    dt = torch.float64 if prec == "f64" else torch.float32
    rng = np.random.default_rng(3)
    W = rng.random((300, 3))
    At = torch.from_numpy(W @ W.T).to(DEV, dt)
    Om = torch.from_numpy(gen.sketch_matrix(300, 10, 5)).to(DEV, dt)
    U, lam = S.lai_sketch(S.dense(At), 6, 2, Om)
    lg = lam.cpu().numpy()
    _, lo = O.range_finder(At.double().cpu().numpy(), 6, 2, Om.double().cpu().numpy())
    tol = 1e-10 if prec == "f64" else 1e-5
    assert np.abs(lg[:3] - lo[:3]).max() <= tol * abs(lo[0])
    # (A stored in FP32 is no longer exactly of rank 3: its other eigenvalues are of the
    # size of its rounding, 3e-9 |lam_1| here)
    tiny = 1e-12 if prec == "f64" else 1e-7
    assert np.abs(lg[3:]).max() <= tol * abs(lo[0]) and np.abs(lo[3:]).max() <= tiny * abs(lo[0])
    Ug = U.double().cpu().numpy()
    assert np.abs(Ug.T @ Ug - np.eye(6)).max() <= (1e-10 if prec == "f64" else 1e-4)


def _csr_with_empty_lines(m, n, seed):
    V = sp.random(m, n, density=0.1, random_state=seed, format="lil")
    V[5, :] = 0
    V[:, 7] = 0
    V = V.tocsr()
    V.eliminate_zeros()
    return V


@pytest.mark.parametrize("r", [1, 3])
def test_nmf_with_empty_rows_and_columns(S, r):
    """A sparse V with an empty row and an empty column (so V^T has an empty row too):
    FP64 over 10 outer iterations against the oracle, the empty row of W and of Ht at 0."""
    V = _csr_with_empty_lines(40, 30, 4)
    M = S.csr_from_scipy(V, torch.float64)
    rng = np.random.default_rng(r)
    W0, H0 = rng.random((40, r)), rng.random((30, r))
    W, Ht, info = S.nmf_solve(M, 30, torch.from_numpy(W0).to(DEV), torch.from_numpy(H0).to(DEV),
                              S.params(prec=S.F64, lam=0.0, max_outer=10))
    Wo, Ho, hist = O.nmf_solve(V, W0, H0, O.Params(), 10)
    Wg, Hg = W.cpu().numpy(), Ht.cpu().numpy()
    assert info["status"] == 0
    assert np.abs(Wg - Wo).max() <= 1e-12 * np.abs(Wo).max()
    assert np.abs(Hg - Ho).max() <= 1e-12 * np.abs(Ho).max()
    assert abs(info["res_WH"] - hist[-1]["res_WH"]) <= 1e-12 * hist[-1]["res_WH"]
    assert not Wg[5].any() and not Hg[7].any()


def test_nmf_minimal_dense_shape(S):
    """m = 2, n = 3, r = 2 (r = min(m, n)), FP64 over 5 outer iterations, to 1e-10."""
    rng = np.random.default_rng(8)
    V = rng.random((2, 3))
    W0, H0 = rng.random((2, 2)), rng.random((3, 2))
    W, Ht, info = S.nmf_solve(S.dense(torch.from_numpy(V).to(DEV)), 3,
                              torch.from_numpy(W0).to(DEV), torch.from_numpy(H0).to(DEV),
                              S.params(prec=S.F64, lam=0.0, max_outer=5))
    Wo, Ho, hist = O.nmf_solve(V, W0, H0, O.Params(), 5)
    assert info["status"] == 0
    # a 2 x 3 V of rank 2 is fitted exactly, and the BB steps near the exact fit carry the
    # 1e-16 differences of the summation order to about 1e-12
    assert np.abs(W.cpu().numpy() - Wo).max() <= 1e-10 * np.abs(Wo).max()
    assert np.abs(Ht.cpu().numpy() - Ho).max() <= 1e-10 * np.abs(Ho).max()
    assert abs(info["res_WH"] - hist[-1]["res_WH"]) <= 1e-10


def test_nmf_zero_partner_breaks_down_like_the_oracle(S):
    """Ht0 = 0: the first W-step's partner block vanishes (rho = ||Ht^T Ht||_2 = 0); the
    oracle raises and the library reports E_BREAKDOWN."""
    V = _csr_with_empty_lines(40, 30, 4)
    W0 = np.random.default_rng(1).random((40, 3))
    with pytest.raises(FloatingPointError):
        O.nmf_solve(V, W0, np.zeros((30, 3)), O.Params(), 3)
    with pytest.raises(S.SnmfError) as e:
        S.nmf_solve(S.csr_from_scipy(V, torch.float64), 30, torch.from_numpy(W0).to(DEV),
                    torch.zeros((30, 3), dtype=torch.float64, device=DEV),
                    S.params(prec=S.F64, lam=0.0, max_outer=3))
    assert e.value.name == "E_BREAKDOWN"


def test_naive_zero_start_breaks_down_like_the_oracle(S):
    rng = np.random.default_rng(3)
    W = rng.random((120, 3))
    A = W @ W.T
    with pytest.raises(FloatingPointError):
        O.naive(A, np.zeros((120, 3)), O.Params(lam=0.0), 3)
    with pytest.raises(S.SnmfError) as e:
        S.solve(S.dense(torch.from_numpy(A).to(DEV)),
                torch.zeros((120, 3), dtype=torch.float64, device=DEV),
                S.params(prec=S.F64, lam=0.0, naive=1, max_outer=3))
    assert e.value.name == "E_BREAKDOWN"
