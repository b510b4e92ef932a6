"""Seeded synthetic inputs for the SNMPBB workloads.

This module builds inputs only: the symmetric nonnegative matrix A (dense or CSR), node
features, cluster labels, Gaussian sketch matrices and the starting factor W0.  It contains none of the solver's arithmetic, so both the HIP path and the
CPU reference consume identical bytes from it without sharing any solver code.

Recipes (all seeds go through numpy's PCG64 ``default_rng``):

* planted dense problem -- a random nonnegative ``W*`` gives ``W* W*^T``; symmetric
  Gaussian noise with standard deviation ``noise * mean(W* W*^T)`` is added to the upper
  triangle (diagonal included) and mirrored; the sum is clipped at zero.  This follows
  the synthetic experiment of the paper's Section 4 (there ``V = W W^T`` without noise).
* stochastic block model graphs with equal clusters, normalised as
  ``D^{-1/2} Adj D^{-1/2}`` (isolated nodes get a zero scale).
* Gaussian node features with cluster-shifted means, over which the graph workload's
  K-nearest-neighbour Laplacian (eq. (2.3)) is built by the method's preprocessing.
* a power-law CSR matrix (Chung-Lu-like sampling of row degrees with exponent 2.1).
* Gaussian sketch matrices (the random input of the range finder of Section 2.3 and of
  the warm start; the range finder itself is method arithmetic and lives with the solver).
* ``W0 = U[0,1] * sqrt(mean(A) / r)`` (Section 4.1 item (4) uses ``2*sqrt(mean/r)``;
  the workloads here use the factor 1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SEED_BASE = 1000


# --------------------------------------------------------------------------- dense
def planted_dense(n: int, r: int, seed: int, noise: float = 0.01):
    """Planted dense problem ``A = max(W* W*^T + E, 0)`` in float64.

    Returns a dict with ``A`` (n x n, float64, C order), ``Wstar`` (n x r) and
    ``W0`` (n x r).
    """
    rng = np.random.default_rng(seed)
    wstar = rng.random((n, r))
    a = wstar @ wstar.T
    if noise > 0.0:
        sigma = noise * float(a.mean())
        e = rng.standard_normal((n, n))
        e = np.triu(e)
        e += np.triu(e, 1).T
        e *= sigma
        a += e
        del e
    np.maximum(a, 0.0, out=a)
    a = 0.5 * (a + a.T)          # exact symmetry of the stored bytes
    w0 = start_factor(rng, n, r, float(a.mean()))
    return {"A": np.ascontiguousarray(a), "Wstar": wstar, "W0": w0}


def start_factor(rng, n: int, r: int, mean_a: float, scale: float = 1.0):
    """``W0 = U[0,1] * scale * sqrt(mean(A)/r)`` (random start of Section 4.1)."""
    return rng.random((n, r)) * (scale * np.sqrt(max(mean_a, 0.0) / r))


def mean_of_sparse(a: sp.csr_matrix) -> float:
    """Mean over all n*n entries of a sparse matrix (zeros included)."""
    n = a.shape[0]
    return float(a.data.sum()) / float(n) / float(n)


# --------------------------------------------------------------------------- graphs
def _tri_unrank(idx: np.ndarray, m: int):
    """Map ranks of pairs (i<j) of an m-set, enumerated row by row, to (i, j)."""
    idx = idx.astype(np.int64)
    b = 2 * m - 1
    i = np.floor((b - np.sqrt(np.maximum(b * b - 8.0 * idx, 0.0))) / 2.0).astype(np.int64)
    i = np.clip(i, 0, m - 2)
    start = i * (2 * m - i - 1) // 2
    over = start > idx
    while np.any(over):
        i[over] -= 1
        start = i * (2 * m - i - 1) // 2
        over = start > idx
    nxt = (i + 1) * (2 * m - i - 2) // 2
    under = nxt <= idx
    while np.any(under):
        i[under] += 1
        start = i * (2 * m - i - 1) // 2
        nxt = (i + 1) * (2 * m - i - 2) // 2
        under = nxt <= idx
    j = idx - start + i + 1
    return i, j


def sbm_adjacency(n: int, k: int, p_in: float, p_out: float, rng):
    """Unweighted SBM adjacency (CSR, symmetric, no self loops) and labels.

    Clusters are as equal as possible (sizes differ by at most one); every pair in a
    block is an independent Bernoulli draw, sampled as a binomial count followed by a
    uniform choice of distinct pairs.
    """
    sizes = np.full(k, n // k, dtype=np.int64)
    sizes[: n % k] += 1
    starts = np.concatenate([[0], np.cumsum(sizes)])
    labels = np.repeat(np.arange(k), sizes)
    rows, cols = [], []
    for a in range(k):
        na = int(sizes[a])
        for b in range(a, k):
            nb = int(sizes[b])
            if a == b:
                m = na * (na - 1) // 2
                if m == 0:
                    continue
                cnt = int(rng.binomial(m, p_in))
                if cnt == 0:
                    continue
                idx = rng.choice(m, size=cnt, replace=False)
                i, j = _tri_unrank(idx, na)
            else:
                m = na * nb
                cnt = int(rng.binomial(m, p_out))
                if cnt == 0:
                    continue
                idx = rng.choice(m, size=cnt, replace=False).astype(np.int64)
                i, j = idx // nb, idx % nb
            rows.append(i + starts[a])
            cols.append(j + starts[b])
    if rows:
        r_ = np.concatenate(rows)
        c_ = np.concatenate(cols)
    else:
        r_ = np.zeros(0, np.int64)
        c_ = np.zeros(0, np.int64)
    data = np.ones(2 * r_.size)
    adj = sp.coo_matrix((data, (np.concatenate([r_, c_]), np.concatenate([c_, r_]))),
                        shape=(n, n)).tocsr()
    adj.sum_duplicates()
    adj.data[:] = 1.0
    return adj, labels


def normalized_adjacency(adj: sp.csr_matrix) -> sp.csr_matrix:
    """``D^{-1/2} Adj D^{-1/2}`` with ``d^{-1/2} := 0`` for isolated nodes."""
    d = np.asarray(adj.sum(axis=1)).ravel()
    s = np.zeros_like(d)
    nz = d > 0
    s[nz] = 1.0 / np.sqrt(d[nz])
    out = sp.diags(s) @ adj @ sp.diags(s)
    out = sp.csr_matrix(out)
    out.sort_indices()
    return out


def cluster_features(labels: np.ndarray, k: int, dim: int, rng, spread: float = 2.0):
    """Gaussian node features ``x_i ~ N(mu_{c(i)}, I)`` with ``mu_c ~ N(0, spread^2 I)``."""
    mu = rng.standard_normal((k, dim)) * spread
    return mu[labels] + rng.standard_normal((labels.size, dim))


def sbm_problem(n: int = 20000, k: int = 20, r: int = 20, p_in: float = 0.02,
                p_out: float = 0.0005, seed: int = SEED_BASE + 2, knn: int = 10,
                feat_dim: int = 16):
    """Graph workload: normalised SBM adjacency, the node features over which the
    K-nearest-neighbour Laplacian is built (K = ``knn``), labels and W0."""
    rng = np.random.default_rng(seed)
    adj, labels = sbm_adjacency(n, k, p_in, p_out, rng)
    a = normalized_adjacency(adj)
    x = cluster_features(labels, k, feat_dim, rng)
    w0 = start_factor(rng, n, r, mean_of_sparse(a))
    return {"A": a, "X": x, "knn": knn, "labels": labels, "W0": w0, "k": k}


# --------------------------------------------------------------------------- power law
def _powerlaw_sample(n, xmin, exponent, cap, rng_seed):
    rng = np.random.default_rng(rng_seed)
    u = 1.0 - rng.random(n)                          # (0, 1]
    tail = exponent - 1.0
    deg = np.floor(xmin * u ** (-1.0 / tail)).astype(np.int64)
    deg = np.clip(deg, 1, cap)
    w = deg.astype(np.float64)
    p = w / w.sum()
    total = int(deg.sum())
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    cols = rng.choice(n, size=total, p=p)
    keep = rows != cols
    rows, cols = rows[keep], cols[keep]
    vals = 1.0 - rng.random(rows.size)               # U(0, 1]
    a = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    a.sum_duplicates()                               # repeated draws of one pair: keep one value
    a.data = np.minimum(a.data, 1.0)
    a = a.maximum(a.T).tocsr()
    a.sort_indices()
    return a


def powerlaw_csr(n: int = 200000, exponent: float = 2.1, mean_degree: float = 10.0,
                 seed: int = SEED_BASE + 3, tol: float = 0.02):
    """Symmetric nonnegative power-law CSR matrix with mean nnz per row ~= mean_degree.

    Target degrees are ``floor(xmin * u^{-1/(exponent-1)})`` capped at ``sqrt(n*mean)``;
    each row draws that many columns with probability proportional to the target
    degrees, values are U(0,1], and ``A <- max(A, A^T)`` symmetrises.  ``xmin`` is
    found by bisection so that the mean nnz per row after symmetrisation is within
    ``tol`` of ``mean_degree``.
    """
    cap = int(np.sqrt(n * mean_degree))
    lo, hi = 0.3, 8.0
    best = None
    for _ in range(30):
        mid = 0.5 * (lo + hi)
        a = _powerlaw_sample(n, mid, exponent, cap, seed)
        m = a.nnz / n
        best = a
        if abs(m - mean_degree) <= tol * mean_degree:
            break
        if m > mean_degree:
            hi = mid
        else:
            lo = mid
    return best


def lai_problem(n: int = 200000, rank: int = 64, oversample: int = 10, power_iters: int = 2,
                r: int = 32, seed: int = SEED_BASE + 3):
    """Low-rank input workload: the power-law CSR A, the Gaussian sketch matrix Omega
    (n x (rank + oversample)) from which the range finder builds the surrogate
    U diag(lam) U^T, the sketch sizes, and W0."""
    a = powerlaw_csr(n=n, seed=seed)
    omega = sketch_matrix(n, rank + oversample, seed + 17)
    rng = np.random.default_rng(seed + 29)
    w0 = start_factor(rng, n, r, mean_of_sparse(a))
    return {"A": a, "Omega": omega, "rank": rank, "power_iters": power_iters, "W0": w0}


# --------------------------------------------------------------------------- batches
def batched_sbm(num_graphs: int = 256, n_lo: int = 500, n_hi: int = 5000,
                ranks=(8, 16, 32), restarts: int = 8, p_in: float = 0.02,
                p_out: float = 0.0005, seed: int = SEED_BASE + 4):
    """A batch of independent SBM graphs of uneven size (k = r clusters each).

    Graph g uses seed ``seed + g``.  Each graph carries ``restarts`` random starts.
    """
    graphs = []
    for g in range(num_graphs):
        rng = np.random.default_rng(seed + g)
        n = int(rng.integers(n_lo, n_hi + 1))
        r = int(ranks[int(rng.integers(0, len(ranks)))])
        adj, labels = sbm_adjacency(n, r, p_in, p_out, rng)
        a = normalized_adjacency(adj)
        mean_a = mean_of_sparse(a)
        w0s = [start_factor(rng, n, r, mean_a) for _ in range(restarts)]
        graphs.append({"A": a, "labels": labels, "r": r, "n": n, "W0": w0s})
    return graphs


# --------------------------------------------------------------------------- named configs
def config(c: int, **over):
    """The five named workloads (c = 0..4) with their fixed seeds."""
    seed = SEED_BASE + c
    if c == 0:
        return planted_dense(over.get("n", 500), over.get("r", 10), seed)
    if c == 1:
        return planted_dense(over.get("n", 8192), over.get("r", 64), seed)
    if c == 2:
        return sbm_problem(seed=seed, **over)
    if c == 3:
        return lai_problem(seed=seed, **over)
    if c == 4:
        return batched_sbm(seed=seed, **over)
    raise ValueError(f"unknown workload {c}")


# --------------------------------------------------------------------------- warm start
def sketch_matrix(n: int, r: int, seed: int):
    """Gaussian sketch matrix Omega (n x r, float64): the random input of Y = A Omega in
    the range finder and the warm start."""
    return np.random.default_rng(seed).standard_normal((n, r))


def mlp_init(r: int, hidden: int = 128, seed: int = SEED_BASE + 16):
    """Initial weights of the residual warm-start network r -> hidden -> r: He-normal M1,
    zero b1, and zero M2 and b2, so that the untrained network returns its input's
    positive part (the start of the frame alone)."""
    rng = np.random.default_rng(seed)
    return {"M1": rng.standard_normal((hidden, r)) * np.sqrt(2.0 / r),
            "b1": np.zeros(hidden),
            "M2": np.zeros((r, hidden)),
            "b2": np.zeros(r)}


# --------------------------------------------------------------------------- HBM-sized inputs
def random_symmetric_csr(n: int, mean_degree: float, seed: int) -> sp.csr_matrix:
    """A symmetric CSR with about n * mean_degree nonzeros at uniform random positions and
    values uniform(0, 1] (both triangles stored, no self-loops): the shape of the graph
    products at sizes that do not fit the caches, for timing the sparse A-pass."""
    rng = np.random.default_rng(seed)
    m = int(n * mean_degree / 2)
    i = rng.integers(0, n, size=m, dtype=np.int64)
    j = rng.integers(0, n, size=m, dtype=np.int64)
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    key = np.unique(lo[lo != hi] * n + hi[lo != hi])   # each unordered pair once
    i, j = key // n, key % n
    v = 1.0 - rng.random(i.size)
    a = sp.coo_matrix((np.concatenate([v, v]), (np.concatenate([i, j]), np.concatenate([j, i]))),
                      shape=(n, n)).tocsr()
    a.sort_indices()
    return a


def random_lowrank(n: int, ell: int, seed: int):
    """(U, lam): a Gaussian n x ell factor and unit weights, for timing the LAI products at
    sizes that do not fit the caches (the timing does not depend on U being orthonormal)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, ell)).astype(np.float32), np.ones(ell)



# --------------------------------------------------------------------------- rectangular NMF
def planted_rect(m: int, n: int, r: int, seed: int, noise: float = 0.01):
    """Planted rectangular problem ``V = max(W* Ht*^T + E, 0)`` (m x n, float64) for NMF
    (eq. (1.1)): ``W*`` and ``Ht*`` uniform on [0, 1), E Gaussian with standard deviation
    ``noise * mean(W* Ht*^T)``.  Returns ``V``, ``W0`` (m x r) and ``Ht0`` (n x r), the
    starts drawn as ``start_factor`` from the mean of V."""
    rng = np.random.default_rng(seed)
    wstar, hstar = rng.random((m, r)), rng.random((n, r))
    v = wstar @ hstar.T
    if noise > 0.0:
        v += (noise * float(v.mean())) * rng.standard_normal((m, n))
    np.maximum(v, 0.0, out=v)
    mv = float(v.mean())
    return {"V": np.ascontiguousarray(v), "W0": start_factor(rng, m, r, mv),
            "Ht0": start_factor(rng, n, r, mv)}


def random_rect_csr(m: int, n: int, density: float, r: int, seed: int):
    """A sparse m x n nonnegative matrix with about density*m*n entries at uniform random
    positions, values uniform(0, 1] (a document-term-like count surrogate), and starts
    W0, Ht0 from its mean."""
    rng = np.random.default_rng(seed)
    nnz = int(density * m * n)
    key = np.unique(rng.integers(0, m * n, size=nnz, dtype=np.int64))
    v = 1.0 - rng.random(key.size)
    a = sp.csr_matrix((v, (key // n, key % n)), shape=(m, n))
    a.sort_indices()
    mv = float(a.data.sum()) / m / n
    return {"V": a, "W0": start_factor(rng, m, r, mv), "Ht0": start_factor(rng, n, r, mv)}
