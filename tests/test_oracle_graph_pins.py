"""Pins of the oracle's graph preprocessing (oracle/graph.py): K-nearest neighbours on
points whose neighbours are known in closed form, agreement with a k-d tree (scipy's
cKDTree, a library routine) on tie-free random data, the Gaussian kernel values, and the
defining properties of the normalised Laplacian (symmetric, L D^{1/2} 1 = 0, spectrum in
[0, 2], unit diagonal).
"""
import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

import oracle as O


def test_knn_on_a_line_with_ties_to_the_lower_index():
    """Points 0, 1, ..., 9 on a line: the 2 nearest of an interior point i are i - 1 and
    i + 1 (equal distance: the lower index first); of point 0 they are 1 and 2."""
    X = np.arange(10.0)[:, None]
    idx, d2 = O.knn(X, 2)
    assert list(idx[0]) == [1, 2] and list(d2[0]) == [1.0, 4.0]
    for i in range(1, 9):
        assert list(idx[i]) == [i - 1, i + 1] and list(d2[i]) == [1.0, 1.0]
    assert list(idx[9]) == [8, 7]


def test_knn_agrees_with_a_kd_tree():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((600, 5))
    idx, d2 = O.knn(X, 7)
    dist, nb = cKDTree(X).query(X, k=8)
    assert np.array_equal(idx, nb[:, 1:])
    np.testing.assert_allclose(d2, dist[:, 1:] ** 2, rtol=1e-12)


def test_similarity_union_pattern_and_gaussian_values():
    """Three points at 0, 1, 3 with K = 1: 0 -> 1, 1 -> 0, 3 -> 1; the union pattern is
    {0-1, 1-3}; with sigma = 1 the values are exp(-d^2/2)."""
    X = np.array([[0.0], [1.0], [3.0]])
    V = O.similarity(X, 1).toarray()
    assert np.array_equal(V, np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], float))
    Vg = O.similarity(X, 1, sigma=1.0).toarray()
    np.testing.assert_allclose(Vg[0, 1], np.exp(-0.5), rtol=1e-15)
    np.testing.assert_allclose(Vg[1, 2], np.exp(-2.0), rtol=1e-15)
    assert np.array_equal(Vg, Vg.T)


def test_normalized_laplacian_properties():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((200, 3))
    for sigma in (0.0, 0.7):
        V = O.similarity(X, 6, sigma)
        L = O.normalized_laplacian(V).toarray()
        d = np.asarray(V.sum(axis=1)).ravel()
        assert np.abs(L - L.T).max() <= 1e-15
        np.testing.assert_allclose(np.diag(L), 1.0, atol=0)
        assert np.abs(L @ np.sqrt(d)).max() <= 1e-13 * np.sqrt(d).max()
        ev = np.linalg.eigvalsh(L)
        assert ev.min() >= -1e-12 and ev.max() <= 2 + 1e-12
    # an isolated point keeps L_ii = 1 and an empty off-diagonal row
    V = sp.csr_matrix(np.array([[0, 1, 0], [1, 0, 0], [0, 0, 0]], float))
    L = O.normalized_laplacian(V).toarray()
    assert L[2, 2] == 1.0 and not L[2, :2].any()
