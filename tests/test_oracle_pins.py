"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each compares it with something
independent -- finite differences of the literal objective (eq. (1.3)/(2.3)), a
textbook NNLS solver, a closed form, the exact planted solution, invariants proved in
Section 3, or brute-force evaluation on tiny inputs.
"""
import numpy as np
import pytest
import scipy.optimize
import scipy.sparse as sp

import oracle as O
from oracle import snmpbb as S
from paper_2606_02887_amd import gen


def _sym_nonneg(n, rng, rank=None):
    if rank is None:
        a = rng.random((n, n))
        return 0.5 * (a + a.T)
    w = rng.random((n, rank))
    return w @ w.T


def _small_laplacian(n, rng, knn=3):
    x = rng.standard_normal((n, 2))
    return O.knn_laplacian(x, knn)


# ------------------------------------------------------------------ gradients vs FD
def _fd_grad(fun, X, h=1e-5):
    g = np.zeros_like(X)
    for idx in np.ndindex(*X.shape):
        e = np.zeros_like(X)
        e[idx] = h
        g[idx] = (fun(X + e) - fun(X - e)) / (2 * h)
    return g


@pytest.mark.parametrize("lam,gamma", [(0.0, 0.0), (0.3, 0.0), (0.3, 0.7)])
def test_gradient_matches_fd_of_literal_objective(lam, gamma):
    rng = np.random.default_rng(1)
    n, r = 9, 3
    A = _sym_nonneg(n, rng)
    L = _small_laplacian(n, rng)
    W = rng.random((n, r))
    Ht = rng.random((n, r))
    Ld = L.toarray()
    # W-step: derivative of eq. (1.3)/(2.3) w.r.t. W with H fixed
    fw = lambda X: O.objective_direct(A, X, Ht, lam, gamma, Ld)
    hs_w = O.HalfStep(A, Ht, lam)
    np.testing.assert_allclose(hs_w.grad(W), _fd_grad(fw, W), rtol=0, atol=1e-7)
    # H-step: derivative w.r.t. Ht (= H^T) with W fixed; the Laplacian acts on H only
    fh = lambda X: O.objective_direct(A, W, X, lam, gamma, Ld)
    hs_h = O.HalfStep(A, W, lam, gamma, L if gamma else None)
    np.testing.assert_allclose(hs_h.grad(Ht), _fd_grad(fh, Ht), rtol=0, atol=1e-7)


def test_planted_mistake_in_gradient_is_caught():
    """A plausible slip (lam*(X+P) instead of lam*(X-P)) must fail the FD pin."""
    rng = np.random.default_rng(2)
    n, r, lam = 8, 2, 0.5
    A = _sym_nonneg(n, rng)
    W, Ht = rng.random((n, r)), rng.random((n, r))

    class Broken(O.HalfStep):
        def grad(self, X):
            return X @ self.G - self.B + self.lam * (X + self.P)

    fw = lambda X: O.objective_direct(A, X, Ht, lam)
    err = np.abs(Broken(A, Ht, lam).grad(W) - _fd_grad(fw, W)).max()
    assert err > 1e-2


# ------------------------------------------------------------------ objective forms
@pytest.mark.parametrize("gamma", [0.0, 0.4])
def test_trace_form_objective_equals_literal(gamma):
    rng = np.random.default_rng(3)
    n, r, lam = 40, 5, 0.2
    A = _sym_nonneg(n, rng)
    L = _small_laplacian(n, rng)
    W, Ht = rng.random((n, r)), rng.random((n, r))
    lit = O.objective_direct(A, W, Ht, lam, gamma, L)
    # W-step form (no Laplacian on W: the gamma term is a constant there)
    fw = O.HalfStep(A, Ht, lam).f(W) + (0.5 * gamma * np.sum(Ht * (L @ Ht)))
    fh = O.HalfStep(A, W, lam, gamma, L if gamma else None).f(Ht)
    assert abs(fw - lit) <= 1e-12 * abs(lit)
    assert abs(fh - lit) <= 1e-12 * abs(lit)


def test_trace_form_with_sparse_and_lowrank_operators():
    rng = np.random.default_rng(4)
    n, r, lam = 30, 4, 0.1
    Ad = _sym_nonneg(n, rng)
    ev, V = np.linalg.eigh(Ad)
    W, Ht = rng.random((n, r)), rng.random((n, r))
    lit = O.objective_direct(Ad, W, Ht, lam)
    assert abs(O.HalfStep(sp.csr_matrix(Ad), Ht, lam).f(W) - lit) <= 1e-12 * lit
    assert abs(O.HalfStep(O.LowRank(V, ev), Ht, lam).f(W) - lit) <= 1e-11 * lit


# ------------------------------------------------------------------ planted exact problem
def test_planted_exact_solution_is_a_fixed_point():
    rng = np.random.default_rng(5)
    n, r = 60, 4
    Wst = rng.random((n, r))
    A = Wst @ Wst.T
    prm = O.Params(lam=0.01 * np.linalg.norm(A))
    hs = O.HalfStep(A, Wst, prm.lam)
    assert np.abs(hs.grad(Wst)).max() <= 1e-12 * np.abs(hs.B).max()
    W, Ht, hist = O.snmpbb(A, Wst, prm, 3)
    assert np.abs(W - Wst).max() <= 1e-12
    assert hist[-1]["res_WH"] <= 1e-14
    assert hist[-1]["pg"] <= 1e-10


def test_planted_perturbed_start_converges_back():
    rng = np.random.default_rng(6)
    n, r = 80, 3
    Wst = rng.random((n, r))
    A = Wst @ Wst.T
    prm = O.Params(lam=0.01 * np.linalg.norm(A))
    W0 = np.maximum(Wst + 0.05 * rng.standard_normal((n, r)), 0)
    W, Ht, hist = O.snmpbb(A, W0, prm, 300)
    assert hist[-1]["res_WH"] < 1e-8
    assert hist[-1]["res_WH"] < hist[0]["res_WH"] * 1e-4


# ------------------------------------------------------------------ inner-solve limits
def test_inner_loop_limit_is_the_row_wise_nnls_solution():
    """With P fixed the half-step is min_{X>=0} 1/2||A - X P^T||^2 + lam/2||X-P||^2, whose
    rows solve nnls([P; sqrt(lam) I], [a_i; sqrt(lam) p_i]) (Lawson-Hanson)."""
    rng = np.random.default_rng(7)
    n, r, lam = 25, 4, 0.3
    A = _sym_nonneg(n, rng)
    P = rng.random((n, r))
    X0 = rng.random((n, r))
    prm = O.Params(lam=lam, inner_iters=3000)
    X = O.half_step(A, X0, P, prm)
    M = np.vstack([P, np.sqrt(lam) * np.eye(r)])
    for i in range(n):
        x_ref, _ = scipy.optimize.nnls(M, np.concatenate([A[i], np.sqrt(lam) * P[i]]))
        np.testing.assert_allclose(X[i], x_ref, atol=1e-8)
    assert (X >= 0).all()


def test_rank_one_inner_limit_closed_form():
    rng = np.random.default_rng(8)
    n, lam = 30, 0.2
    A = _sym_nonneg(n, rng) - 0.45          # some negative entries so the clip is active
    A = 0.5 * (A + A.T)
    p = rng.random((n, 1))
    x_cf = np.maximum(0.0, (A @ p + lam * p) / (float((p.T @ p)[0, 0]) + lam))
    X = O.half_step(A, rng.random((n, 1)), p, O.Params(lam=lam, inner_iters=400))
    assert (x_cf == 0).any() and (x_cf > 0).any()
    np.testing.assert_allclose(X, x_cf, atol=1e-10)


# ------------------------------------------------------------------ Section 3 invariants
def _run_logged(prm, n=50, r=5, seed=9, gamma_L=False):
    rng = np.random.default_rng(seed)
    A = _sym_nonneg(n, rng, rank=r) + 0.01 * _sym_nonneg(n, rng)
    L = _small_laplacian(n, rng) if gamma_L else None
    P = rng.random((n, r))
    X0 = rng.random((n, r))
    hs = O.HalfStep(A, P, prm.lam, prm.gamma if gamma_L else 0.0, L)
    log = []
    O.nmpbb(hs, X0, prm, log, keep_arrays=True)
    return hs, log


@pytest.mark.parametrize("gamma_L", [False, True])
def test_bb_curvature_identity_and_descent_lemma(gamma_L):
    prm = O.Params(lam=0.05, gamma=0.3, inner_iters=12)
    hs, log = _run_logged(prm, gamma_L=gamma_L)
    Mtot = hs.G + prm.lam * np.eye(hs.G.shape[0])
    for e in log:
        Sm = e["Xn"] - e["X"]
        # Y = S (H H^T + lam I) [+ gam L S]  (LAI curvature section)
        sy_id = np.sum((Sm @ Mtot) * Sm)
        if hs.L is not None:
            sy_id += prm.gamma * np.sum(Sm * (hs.L @ Sm))
        assert abs(e["sy"] - sy_id) <= 1e-10 * (abs(sy_id) + 1e-300)
        assert e["sy"] >= prm.lam * e["ss"] * (1 - 1e-12)
        # descent lemma: <grad f(Z), D_alpha(Z)> <= -||D_alpha||^2 / alpha
        assert e["delta"] <= -e["normD2"] / e["alpha"] + 1e-12 * abs(e["delta"])
        assert (e["Xn"] >= 0).all() and (e["Z"] >= 0).all()


def test_nonmonotone_reference_is_monotone_with_unit_relaxation():
    """f(W_k) <= F_k <= F_{k-1} <= ... (Section 3.1) for phi = 1 (no relaxation)."""
    prm = O.Params(lam=0.05, phi=1.0, inner_iters=30)
    hs, log = _run_logged(prm, seed=10)
    for a, b in zip(log[:-1], log[1:]):
        assert not a["exhausted"]
        assert b["fX"] <= b["F"] * (1 + 1e-13) + 1e-13
        assert b["F"] <= a["F"] * (1 + 1e-13) + 1e-13


def test_lipschitz_constant_of_the_gradient_is_attained():
    """||grad f(X1) - grad f(X2)|| <= (||H H^T||_2 + lam) ||X1 - X2||, with equality along
    the top eigenvector of H H^T (Section 3.1, proof of Theorem 3.1)."""
    rng = np.random.default_rng(11)
    n, r, lam = 20, 4, 0.3
    A = _sym_nonneg(n, rng)
    P = rng.random((n, r))
    hs = O.HalfStep(A, P, lam)
    Lc = hs.rho + lam
    for _ in range(5):
        X1, X2 = rng.random((n, r)), rng.random((n, r))
        lhs = np.linalg.norm(hs.grad(X1) - hs.grad(X2))
        assert lhs <= Lc * np.linalg.norm(X1 - X2) * (1 + 1e-12)
    ev, V = np.linalg.eigh(P.T @ P)
    dX = np.outer(rng.random(n), V[:, -1])
    X1 = rng.random((n, r))
    lhs = np.linalg.norm(hs.grad(X1 + dX) - hs.grad(X1))
    assert abs(lhs - Lc * np.linalg.norm(dX)) <= 1e-10 * lhs


def test_rho_is_the_spectral_norm():
    rng = np.random.default_rng(12)
    P = rng.random((30, 6))
    G = P.T @ P
    assert abs(O.spectral_norm_psd(G) - np.linalg.norm(P, 2) ** 2) <= 1e-12 * np.linalg.norm(G)


# ------------------------------------------------------------------ LAI
def test_lai_on_exactly_low_rank_input_equals_dense():
    rng = np.random.default_rng(13)
    n, ell, r = 70, 6, 3
    Wst = rng.random((n, ell))
    A = Wst @ Wst.T
    ev, V = np.linalg.eigh(A)
    keep = np.argsort(-np.abs(ev))[:ell]
    lr = O.LowRank(V[:, keep], ev[keep])
    prm = O.Params(lam=0.01 * np.linalg.norm(A))
    W0 = rng.random((n, r)) * np.sqrt(A.mean() / r)
    Wd, Hd, hd = O.snmpbb(A, W0, prm, 20)
    Wl, Hl, hl = O.snmpbb(lr, W0, prm, 20)
    np.testing.assert_allclose(Wl, Wd, rtol=0, atol=1e-10 * np.abs(Wd).max())
    assert abs(hl[-1]["res_WH"] - hd[-1]["res_WH"]) <= 1e-9


def test_lai_gradient_bias_and_bound():
    """grad_LAI - grad = (A - U E U^T) P  and  ||bias|| <= mu ||P|| (LAI curvature)."""
    rng = np.random.default_rng(14)
    n, ell, r, lam = 50, 8, 3, 0.1
    A = _sym_nonneg(n, rng)
    ev, V = np.linalg.eigh(A)
    keep = np.argsort(-np.abs(ev))[:ell]
    lr = O.LowRank(V[:, keep], ev[keep])
    Ad = (V[:, keep] * ev[keep]) @ V[:, keep].T
    P, X = rng.random((n, r)), rng.random((n, r))
    bias = O.HalfStep(lr, P, lam).grad(X) - O.HalfStep(A, P, lam).grad(X)
    np.testing.assert_allclose(bias, (A - Ad) @ P, atol=1e-11)
    mu = np.linalg.norm(A - Ad)
    assert np.linalg.norm(bias) <= mu * np.linalg.norm(P) * (1 + 1e-12)


# ------------------------------------------------------------------ monitor
def test_pg_norm_zero_iff_stationary_on_brute_force_tiny():
    rng = np.random.default_rng(15)
    n, r, lam = 6, 2, 0.2
    A = _sym_nonneg(n, rng)
    W, Ht = rng.random((n, r)), rng.random((n, r))
    prm = O.Params(lam=lam)
    # brute force: evaluate the projected gradient elementwise from the FD gradient
    gw = _fd_grad(lambda X: O.objective_direct(A, X, Ht, lam), W)
    gh = _fd_grad(lambda X: O.objective_direct(A, W, X, lam), Ht)
    bf = np.sqrt(sum(((np.maximum(x - g, 0) - x) ** 2).sum() for x, g in ((W, gw), (Ht, gh))))
    assert abs(O.pg_norm(A, W, Ht, prm) - bf) <= 1e-7 * bf


def test_residual_trace_form_equals_direct():
    rng = np.random.default_rng(16)
    n, r = 40, 3
    A = _sym_nonneg(n, rng)
    W, Ht = rng.random((n, r)), rng.random((n, r))
    d = O.residual_WH(A, W, Ht)
    s_ = O.residual_WH(sp.csr_matrix(A), W, Ht)
    assert abs(d - s_) <= 1e-12
    assert abs(d - np.linalg.norm(A - W @ Ht.T) / np.linalg.norm(A)) <= 1e-14
