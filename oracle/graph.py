"""FP64 CPU reference of the graph preprocessing of Graph-SNMPBB -- TEST INFRASTRUCTURE ONLY.

Section 2.2 builds the similarity matrix of data points as in Kuang et al.: a Gaussian
kernel with parameter sigma, keeping only each point's K nearest neighbours (all other
entries zero); the Laplacian of eq. (2.3) is L = I - D^{-1/2} V D^{-1/2} with
d_i = sum_j V_ij.  Readings taken here (and by the GPU path):

* neighbours by Euclidean distance, the point itself excluded, ties to the lower index;
* the kernel exp(-||x_i - x_j||^2 / (2 sigma^2)); sigma = 0 gives the unweighted graph
  (every kept entry 1), the Laplacian of the graph workload;
* the kept pattern is symmetrised by union: V_ij is kept when j is among the K nearest
  of i or i among the K nearest of j (the kernel value is symmetric);
* an isolated point (d_i = 0) gets D^{-1/2}_ii = 0, so L_ii = 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def knn(X, K: int, block: int = 1024):
    """Indices (n x K) and squared distances of every point's K nearest other points, by
    brute force in FP64: sorted by (distance, index)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    idx = np.empty((n, K), dtype=np.int64)
    dst = np.empty((n, K))
    cols = np.arange(n)
    for b0 in range(0, n, block):
        xb = X[b0:b0 + block]
        d2 = np.sum((xb[:, None, :] - X[None, :, :]) ** 2, axis=2)
        for t in range(xb.shape[0]):
            i = b0 + t
            d = d2[t].copy()
            d[i] = np.inf
            order = np.lexsort((cols, d))[:K]          # by distance, then index
            idx[i] = order
            dst[i] = d[order]
    return idx, dst


def similarity(X, K: int, sigma: float = 0.0):
    """The symmetric K-nearest-neighbour similarity matrix (CSR, sorted columns)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    idx, _ = knn(X, K)
    rows = np.repeat(np.arange(n), K)
    cols = idx.reshape(-1)
    pat = sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(n, n)).tocsr()
    pat = ((pat + pat.T) > 0).astype(np.float64).tocsr()
    pat.sort_indices()
    if sigma > 0:
        r_, c_ = pat.nonzero()
        d2 = np.sum((X[r_] - X[c_]) ** 2, axis=1)
        pat = sp.csr_matrix((np.exp(-d2 / (2.0 * sigma * sigma)), (r_, c_)), shape=(n, n))
        pat.sort_indices()
    return pat


def normalized_laplacian(V):
    """L = I - D^{-1/2} V D^{-1/2}, d_i = sum_j V_ij (d_i = 0: zero scale)."""
    V = sp.csr_matrix(V)
    n = V.shape[0]
    d = np.asarray(V.sum(axis=1)).ravel()
    s = np.zeros_like(d)
    s[d > 0] = 1.0 / np.sqrt(d[d > 0])
    L = sp.identity(n, format="csr") - sp.diags(s) @ V @ sp.diags(s)
    L = sp.csr_matrix(L)
    L.sum_duplicates()
    L.sort_indices()
    return L


def knn_laplacian(X, K: int, sigma: float = 0.0):
    """Normalised Laplacian of the symmetrised K-nearest-neighbour graph over X."""
    return normalized_laplacian(similarity(X, K, sigma))
