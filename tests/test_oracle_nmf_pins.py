"""Pins of the oracle's NMPBB for rectangular NMF (oracle/nmf.py, eq. (1.1)): gradients
against finite differences of 1/2 ||V - W H||^2, the inner-loop limit against row-wise
NNLS (Lawson-Hanson), a planted exact factorisation as a fixed point, convergence back
to it from a perturbed start, and the trace-form residual on sparse input."""
import numpy as np
import scipy.optimize
import scipy.sparse as sp

import importlib

import oracle as O

N = importlib.import_module("oracle.nmf")


def _fd(fun, X, h=1e-6):
    g = np.zeros_like(X)
    for idx in np.ndindex(*X.shape):
        e = np.zeros_like(X)
        e[idx] = h
        g[idx] = (fun(X + e) - fun(X - e)) / (2 * h)
    return g


def test_gradients_match_fd_of_the_nmf_objective():
    rng = np.random.default_rng(1)
    m, n, r = 7, 5, 3
    V = rng.random((m, n))
    W, Ht = rng.random((m, r)), rng.random((n, r))
    f = lambda W_, Ht_: 0.5 * np.sum((V - W_ @ Ht_.T) ** 2)
    np.testing.assert_allclose(O.HalfStep(V, Ht, 0.0).grad(W), _fd(lambda X: f(X, Ht), W),
                               atol=1e-7)
    np.testing.assert_allclose(O.HalfStep(V.T, W, 0.0).grad(Ht), _fd(lambda X: f(W, X), Ht),
                               atol=1e-7)


def test_inner_limits_are_row_wise_nnls():
    """With H fixed the W-step is min_{W>=0} 1/2||V - W H||^2: row i solves
    nnls(Ht, V_i); the H-step's column j solves nnls(W, V_:,j)."""
    rng = np.random.default_rng(2)
    m, n, r = 12, 9, 3
    V = rng.random((m, n))
    W0, Ht0 = rng.random((m, r)), rng.random((n, r))
    prm = O.Params(inner_iters=4000)
    W = O.half_step(V, W0, Ht0, prm)
    for i in range(m):
        np.testing.assert_allclose(W[i], scipy.optimize.nnls(Ht0, V[i])[0], atol=1e-8)
    Ht = O.half_step(V.T, Ht0, W0, prm)
    for j in range(n):
        np.testing.assert_allclose(Ht[j], scipy.optimize.nnls(W0, V[:, j])[0], atol=1e-8)


def test_planted_exact_factorisation():
    rng = np.random.default_rng(3)
    m, n, r = 60, 40, 4
    Ws, Hs = rng.random((m, r)) + 0.1, rng.random((n, r)) + 0.1
    V = Ws @ Hs.T
    W, Ht, hist = N.nmf(V, Ws, Hs, O.Params(), 3)
    assert np.abs(W - Ws).max() <= 1e-12 and np.abs(Ht - Hs).max() <= 1e-12
    assert hist[-1]["res_WH"] <= 1e-14 and hist[-1]["pg"] <= 1e-10
    W, Ht, hist = N.nmf(V, np.maximum(Ws + 0.02 * rng.standard_normal((m, r)), 0),
                        np.maximum(Hs + 0.02 * rng.standard_normal((n, r)), 0), O.Params(), 300)
    assert hist[-1]["res_WH"] < 1e-6 and hist[-1]["res_WH"] < 1e-3 * hist[0]["res_WH"]


def test_sparse_residual_equals_dense():
    rng = np.random.default_rng(4)
    V = sp.random(30, 20, density=0.3, random_state=5, format="csr")
    W, Ht = rng.random((30, 3)), rng.random((20, 3))
    assert abs(N.residual(V, W, Ht) - N.residual(V.toarray(), W, Ht)) <= 1e-13
