"""FP64 CPU reference of the LAI sketch -- TEST INFRASTRUCTURE ONLY.

LAI-SNMPBB (Section 2.3) replaces A by a low-rank surrogate A ~= U E U^T built from a
random sketch: the product of A with a random n x ell matrix is orthonormalised
(A S = Q R), the small matrix Q^T A Q is diagonalised (Q^T A Q = P E P^T), and U = Q P.
The paper leaves the sketch unspecified; the reading taken here (and by the GPU path):

* S = Omega is a Gaussian n x ell matrix with ell = rank + oversample (an input: the
  random numbers are drawn by the caller);
* power_iters rounds of two more products with A, an orthonormalisation after every
  product (the subspace iteration of Halko, Martinsson & Tropp, 2011, Algorithm 4.4):
  Y = A Omega, Q = orth(Y); then power_iters times Q = orth(A Q), Q = orth(A Q);
* T = Q^T A Q (symmetrised), T = P E P^T, and the rank eigenpairs of largest |E| are
  kept (ties in |E| keep the lower index): U = Q P_rank, lam = E_rank, in that order.

orth() is a thin QR (numpy's Householder QR); the result does not depend on which
orthonormal basis of the range it returns, since U and lam are those of A restricted to
span(Q).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _apply(A, X):
    if sp.issparse(A):
        return np.asarray(A @ X)
    return np.asarray(A, dtype=np.float64) @ X


def orth(Y):
    """An orthonormal basis of the columns of Y (thin QR)."""
    q, _ = np.linalg.qr(Y)
    return q


def range_finder(A, rank: int, power_iters: int, Omega):
    """(U, lam): U n x rank with orthonormal columns, lam the matching eigenvalues of
    Q^T A Q, ordered by decreasing |lam|."""
    Om = np.asarray(Omega, dtype=np.float64)
    q = orth(_apply(A, Om))
    for _ in range(power_iters):
        q = orth(_apply(A, q))
        q = orth(_apply(A, q))
    t = q.T @ _apply(A, q)
    t = 0.5 * (t + t.T)
    ev, p = np.linalg.eigh(t)
    order = np.argsort(-np.abs(ev), kind="stable")[:rank]
    return np.ascontiguousarray(q @ p[:, order]), ev[order].copy()


def svd_start(A, r: int, power_iters: int, Omega):
    """The SVD-based start of the numerical experiments (Section 4.2): with the leading
    r singular triplets A ~= U E V^T, W0 = |U E^(1/2)| and H0 = |E^(1/2) V^T|.  For a
    symmetric A the singular triplets are eigenpairs, E = |lam|, V = U sign(lam), so
    H0^T = W0; the triplets come from the range finder above (rank r)."""
    U, lam = range_finder(A, r, power_iters, Omega)
    return np.abs(U * np.sqrt(np.abs(lam))[None, :])
