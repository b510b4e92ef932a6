"""Pins of the oracle's naive symmetric variant (oracle.snmpbb.naive, Section 2.1: each
outer iteration solves for W with the partner held at the current W and no penalty, then
sets H <- W^T).

* The inner loop's limit is the W-step's own problem, min_{W >= 0} ||A - W W_i^T||, which
  splits into row-wise nonnegative least squares nnls(W_i, A_i) (Lawson-Hanson in scipy):
  over two outer iterations, so the partner of the second is the first's result.
* H = W after every outer iteration (sym_gap 0, res_WWt = res_WH).
* A planted exact factorisation A = W* W*^T with W* > 0 is a fixed point.
* Mutations (a partner frozen at W0; an H-step in place of H <- W^T) fail the first pin.
"""
import numpy as np
import scipy.optimize

import importlib

import oracle as O

SN = importlib.import_module("oracle.snmpbb")


def _sym(rng, n):
    B = rng.random((n, n))
    return B + B.T


def _nnls_pin(fn) -> bool:
    """Two outer iterations of fn with 4000 inner iterations each against row-wise NNLS
    with the partner of each outer iteration (W0, then the first result)."""
    rng = np.random.default_rng(5)
    n, r = 10, 3
    A = _sym(rng, n)
    W0 = rng.random((n, r))
    prm = O.Params(lam=0.0, inner_iters=4000)
    W1, _, _ = fn(A, W0, prm, 1)
    W2, _, _ = fn(A, W0, prm, 2)
    E1 = np.array([scipy.optimize.nnls(W0, A[i])[0] for i in range(n)])
    E2 = np.array([scipy.optimize.nnls(E1, A[i])[0] for i in range(n)])
    return np.abs(W1 - E1).max() <= 1e-7 and np.abs(W2 - E2).max() <= 1e-6


def test_inner_limit_is_nnls_with_the_current_partner():
    assert _nnls_pin(SN.naive)


def test_nnls_pin_catches_mutations():
    def frozen_partner(A, W0, prm, outer):   # partner stays W0
        W = W0.copy()
        for _ in range(outer):
            W = O.half_step(A, W, W0, prm)
        return W, W.copy(), []

    def with_h_step(A, W0, prm, outer):      # the penalty method's alternation at lam = 0
        return O.snmpbb(A, W0, prm, outer)

    assert not _nnls_pin(frozen_partner)
    assert not _nnls_pin(with_h_step)


def test_h_equals_w_after_every_outer_iteration():
    rng = np.random.default_rng(6)
    n, r = 40, 4
    A = _sym(rng, n)
    W0 = rng.random((n, r))
    W, Ht, hist = SN.naive(A, W0, O.Params(lam=0.0), 6)
    assert np.array_equal(W, Ht)
    for h in hist:
        assert h["sym_gap"] == 0.0 and h["res_WWt"] == h["res_WH"]
    res = np.linalg.norm(A - W @ W.T) / np.linalg.norm(A)
    assert abs(hist[-1]["res_WH"] - res) <= 1e-14 * res
    # the first W-step is the penalty method's at lam = 0 (both start from Ht = W0)
    W1, _, _ = SN.naive(A, W0, O.Params(lam=0.0), 1)
    assert np.array_equal(W1, O.half_step(A, W0, W0, O.Params(lam=0.0)))


def test_planted_fixed_point():
    rng = np.random.default_rng(7)
    n, r = 50, 4
    Ws = rng.random((n, r)) + 0.1
    A = Ws @ Ws.T
    W, Ht, hist = SN.naive(A, Ws, O.Params(lam=0.0), 3)
    assert np.abs(W - Ws).max() <= 1e-12
    assert hist[-1]["res_WH"] <= 1e-14 and hist[-1]["pg"] <= 1e-10


def test_lam_must_be_zero():
    import pytest
    with pytest.raises(ValueError):
        SN.naive(np.eye(3), np.ones((3, 1)), O.Params(lam=0.1), 1)
