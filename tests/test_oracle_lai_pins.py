"""Pins of the oracle's LAI sketch (oracle/lai.py) against facts fixed by the mathematics:
orthonormal output, exact recovery of a matrix of rank <= the sketch rank (then the
surrogate is A itself and lam are its nonzero eigenvalues), and an approximation error at
least and close to the best rank-k error (dense eigendecomposition, Eckart-Young).  The
SVD start is pinned by its closed form on an exactly low-rank planted problem.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2606_02887_amd import gen


def test_range_finder_orthonormal_and_near_optimal():
    rng = np.random.default_rng(2)
    n, k = 400, 10
    w = rng.random((n, k))
    A = sp.csr_matrix(w @ w.T + 0.01 * (lambda e: e + e.T)(rng.standard_normal((n, n))))
    U, lam = O.range_finder(A, k, 2, gen.sketch_matrix(n, k + 10, 7))
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-12
    Ad = A.toarray()
    ev = np.linalg.eigvalsh(Ad)
    best = np.sqrt(np.sort(ev ** 2)[:-k].sum())
    err = np.linalg.norm(Ad - (U * lam) @ U.T)
    assert best <= err <= 1.05 * best
    assert np.all(np.diff(np.abs(lam)) <= 0)


@pytest.mark.parametrize("dense", [True, False])
def test_range_finder_recovers_low_rank_exactly(dense):
    """rank(A) = 6 <= sketch rank 8: U diag(lam) U^T = A, and lam holds the six nonzero
    eigenvalues of A (then two zeros)."""
    rng = np.random.default_rng(3)
    n = 300
    w = rng.standard_normal((n, 6))
    Ad = w @ np.diag([5.0, -3.0, 2.0, 1.5, -1.0, 0.5]) @ w.T
    A = Ad if dense else sp.csr_matrix(Ad)
    U, lam = O.range_finder(A, 8, 1, gen.sketch_matrix(n, 12, 9))
    assert np.linalg.norm(Ad - (U * lam) @ U.T) <= 1e-10 * np.linalg.norm(Ad)
    ev = np.linalg.eigvalsh(Ad)
    top = ev[np.argsort(-np.abs(ev))[:6]]
    np.testing.assert_allclose(lam[:6], top, rtol=1e-10)
    assert np.abs(lam[6:]).max() <= 1e-10 * np.abs(lam).max()


def test_range_finder_power_iterations_sharpen_the_subspace():
    """Each round of products with A shrinks the angle between span(U) and the dominant
    eigenvectors when the spectrum decays slowly (the point of the power iterations)."""
    rng = np.random.default_rng(4)
    n, k = 500, 8
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = 1.0 / np.arange(1, n + 1) ** 0.5
    A = (V * ev) @ V.T
    Om = gen.sketch_matrix(n, k + 4, 11)
    angles = []
    for q in (0, 1, 2):
        U, _ = O.range_finder(A, k, q, Om)
        angles.append(np.linalg.norm(V[:, :k] - U @ (U.T @ V[:, :k]), 2))
    assert angles[2] < angles[1] < angles[0]


def test_svd_start_closed_form_on_planted_problem():
    """A = W* W*^T of rank r: the SVD start is |U E^(1/2)| with U, E the eigenpairs of A,
    and |U E^(1/2)| |U E^(1/2)|^T equals A wherever U E^(1/2) has one sign per row (here:
    W* with disjoint column supports, so A's eigenvectors are W*'s normalised columns)."""
    rng = np.random.default_rng(5)
    n, r = 120, 4
    W = np.zeros((n, r))
    for j, rows in enumerate(np.array_split(np.arange(n), r)):
        W[rows, j] = rng.random(rows.size) + 0.1
    A = W @ W.T
    W0 = O.svd_start(A, r, 1, gen.sketch_matrix(n, r + 4, 13))
    assert (W0 >= 0).all()
    np.testing.assert_allclose(W0 @ W0.T, A, atol=1e-10 * np.abs(A).max())
    # columns are W*'s up to order
    cols = sorted(range(r), key=lambda j: -np.linalg.norm(W[:, j]))
    np.testing.assert_allclose(np.sort(np.linalg.norm(W0, axis=0)), np.sort(np.linalg.norm(W, axis=0)),
                               rtol=1e-10)
