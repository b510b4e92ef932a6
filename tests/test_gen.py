"""Checks of the seeded workload generators (input recipes, not solver arithmetic)."""
import numpy as np
import scipy.sparse as sp

from paper_2606_02887_amd import gen


def test_planted_dense_is_symmetric_nonnegative_and_seeded():
    p = gen.planted_dense(64, 4, 123)
    q = gen.planted_dense(64, 4, 123)
    A = p["A"]
    assert (A == A.T).all() and (A >= 0).all()
    assert np.array_equal(A, q["A"]) and np.array_equal(p["W0"], q["W0"])
    # noise is 1% of the mean: the planted product explains ~99% of A
    res = np.linalg.norm(A - p["Wstar"] @ p["Wstar"].T) / np.linalg.norm(A)
    assert 1e-3 < res < 2e-2


def test_sbm_structure():
    rng = np.random.default_rng(0)
    adj, labels = gen.sbm_adjacency(600, 6, 0.1, 0.005, rng)
    assert (adj != adj.T).nnz == 0 and adj.diagonal().sum() == 0
    rows, cols = adj.nonzero()
    same = labels[rows] == labels[cols]
    n_in = same.sum() / 2
    n_out = (~same).sum() / 2
    pairs_in = 6 * (100 * 99 / 2)
    pairs_out = 600 * 599 / 2 - pairs_in
    assert abs(n_in / pairs_in - 0.1) < 0.01
    assert abs(n_out / pairs_out - 0.005) < 0.001
    a = gen.normalized_adjacency(adj)
    d = np.asarray(adj.sum(1)).ravel()
    i, j = rows[0], cols[0]
    assert abs(a[i, j] - 1 / np.sqrt(d[i] * d[j])) < 1e-15


def test_tri_unrank_enumerates_all_pairs():
    m = 37
    i, j = gen._tri_unrank(np.arange(m * (m - 1) // 2), m)
    ref = [(a, b) for a in range(m) for b in range(a + 1, m)]
    assert list(zip(i.tolist(), j.tolist())) == ref


def test_powerlaw_mean_degree_and_symmetry():
    a = gen.powerlaw_csr(n=20000, seed=5)
    assert abs(a.nnz / a.shape[0] - 10) <= 0.2 + 1e-9
    assert abs(a - a.T).max() == 0
    assert a.data.min() > 0 and a.data.max() <= 1
    assert a.diagonal().sum() == 0


def test_random_symmetric_csr_and_lowrank():
    a = gen.random_symmetric_csr(5000, 12.0, 7)
    assert a.shape == (5000, 5000) and abs(a.nnz / 5000 - 12.0) < 1.0
    assert (a - a.T).nnz == 0 and a.diagonal().max() == 0.0
    assert a.data.min() > 0.0 and a.data.max() <= 1.0
    b = gen.random_symmetric_csr(5000, 12.0, 7)
    assert (a != b).nnz == 0
    U, lam = gen.random_lowrank(100, 8, 3)
    assert U.shape == (100, 8) and U.dtype == np.float32 and np.all(lam == 1.0)
