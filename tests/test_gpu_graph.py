"""GPU parity of the graph preprocessing of Graph-SNMPBB (snmf_knn, snmf_knn_graph;
Section 2.2, eq. (2.3)) against the oracle (oracle/graph.py) on the same points.

Neighbour lists and the CSR pattern are integer results: they must be identical (both
sides rank by FP64 distance, ties to the lower index).  The values (Gaussian kernel,
normalised Laplacian) are FP64 on the device and rounded to the output type: within 1e-12
(F64) or 2^-24 plus one rounding (F32, bound 2e-7) of the entry, relative to max |entry|.
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


def _points(n, dim, k, seed):
    rng = np.random.default_rng(seed)
    labels = np.repeat(np.arange(k), n // k + 1)[:n]
    return gen.cluster_features(labels, k, dim, rng)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,dim,K", [(3000, 16, 10), (997, 3, 1), (1500, 64, 40), (400, 7, 64)])
def test_knn_matches_oracle(S, prec, n, dim, K):
    X = torch.from_numpy(_points(n, dim, 8, n + dim)).to(DEV, DT[prec])
    nbr = S.knn(X, K).cpu().numpy()
    idx, _ = O.knn(X.double().cpu().numpy(), K)
    assert np.array_equal(nbr, idx)


def test_knn_ties_go_to_the_lower_index(S):
    """Integer points on a line: exact ties everywhere; neighbours i - 1, i + 1, i - 2, ..."""
    X = torch.arange(300, dtype=torch.float64, device=DEV)[:, None].contiguous()
    nbr = S.knn(X, 4).cpu().numpy()
    idx, _ = O.knn(X.cpu().numpy(), 4)
    assert np.array_equal(nbr, idx)
    assert list(nbr[10]) == [9, 11, 8, 12]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("laplacian,sigma", [(True, 0.0), (False, 0.0), (True, 1.5), (False, 2.0)])
def test_knn_graph_matches_oracle(S, prec, laplacian, sigma):
    n, dim, K = 2500, 16, 10
    X = torch.from_numpy(_points(n, dim, 10, 5)).to(DEV, DT[prec])
    M = S.knn_graph(X, K, sigma=sigma, laplacian=laplacian)
    rowptr, col, val = (t.cpu().numpy() for t in M.keep)
    Xo = X.double().cpu().numpy()
    ref = O.knn_laplacian(Xo, K, sigma) if laplacian else O.similarity(Xo, K, sigma)
    assert np.array_equal(rowptr, ref.indptr) and np.array_equal(col, ref.indices)
    err = np.abs(val.astype(np.float64) - ref.data).max() / np.abs(ref.data).max()
    assert err <= (1e-12 if prec == "f64" else 2e-7), err


def test_graph_solve_on_the_device_laplacian(S):
    """Graph-SNMPBB with the Laplacian built on the device: the same solve as with the
    oracle's Laplacian (identical pattern, values to FP32 rounding), 30 outer iterations
    in FP64 from the same start, residual and projected-gradient norm to 1e-9."""
    p = gen.sbm_problem(n=1200, k=6, r=6, p_in=0.06, p_out=0.003, seed=41)
    A = p["A"]
    Xt = torch.from_numpy(p["X"]).to(DEV, torch.float64)
    Lg = S.knn_graph(Xt, p["knn"])
    Lo = O.knn_laplacian(p["X"], p["knn"])
    lam = O.default_lambda(A)
    W, Ht, info = S.solve(S.csr_from_scipy(A, torch.float64),
                          torch.from_numpy(p["W0"]).to(DEV, torch.float64),
                          S.params(lam=lam, gamma=0.2, prec=S.F64, max_outer=30), Lg)
    _, _, hist = O.snmpbb(A, p["W0"], O.Params(lam=lam, gamma=0.2), 30, L=Lo)
    assert abs(info["res_WH"] - hist[-1]["res_WH"]) <= 1e-9 * hist[-1]["res_WH"]
    assert abs(info["pg_norm"] - hist[-1]["pg"]) <= 1e-9 * hist[-1]["pg"]


def test_graph_error_codes(S):
    X = torch.rand((50, 4), dtype=torch.float32, device=DEV)
    bad = X.clone()
    bad[7, 2] = float("nan")
    with pytest.raises(S.SnmfError) as e:
        S.knn(bad, 3)
    assert e.value.name == "E_NONFINITE"
    with pytest.raises(S.SnmfError) as e:
        S.knn(X, 50)
    assert e.value.name == "E_SHAPE"
    with pytest.raises(S.SnmfError) as e:
        S.knn_graph(torch.rand((50, 65), dtype=torch.float32, device=DEV), 3)
    assert e.value.name == "E_SHAPE"
