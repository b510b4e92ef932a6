"""Pins of the individual steps of Algorithm 1 in the oracle, each with a mutation check.

Every pin compares the oracle with a fact fixed by the mathematics of the method, not
with a re-typed copy of its code:

* the Barzilai-Borwein step (Algorithm 1, step 3): on a partner block with orthogonal,
  equal-norm columns (G = c I) the gradient is affine with Hessian (c + lam) I, so every
  difference Y equals (c + lam) S and every BB step after the first is exactly
  1/(c + lam);
* the first projection with the fixed scale 1/rho0 (Algorithm 1, step 2; Section 2.4):
  on the same quadratic, a gradient step of length 1/c from an interior point X lands at
  x* - (lam/c)(X - x*), x* = (A P + lam P)/(c + lam) the unconstrained minimiser; with
  lam = 0 it lands on x* itself, so the next direction and the next step vanish;
* the acceptance test (Algorithm 1, step 4): the accepted beta is the first of
  1, s, s^2, ... for which the literal objective of eq. (1.3) at Z + beta D lies below
  F_k + theta beta <grad f(Z), D>, with the gradient taken by finite differences;
* the nonmonotone reference (Section 2.4): F_0 = f(X_0) and F_{k+1} = f(X_{k+1}) +
  eta (F_k - f(X_{k+1})) unrolled by hand into its closed form over three steps;
* the monitor: ||A - W W^T||/||A||, ||W - H^T||/||W|| and f(W, H) by explicit loops.

Each mutation check builds a variant of the oracle's inner loop with one plausible slip
(an inverted BB ratio, the BB step used in the first projection, the test made at the
relaxed point, a swapped memory weight) and shows that the pin turns red on it.
"""
import importlib
import inspect

import numpy as np
import pytest

import oracle as O

OS = importlib.import_module("oracle.snmpbb")   # the module (the package re-exports its names)


def mutant(old: str, new: str):
    """The oracle's inner loop with the one source fragment `old` replaced by `new`."""
    src = inspect.getsource(OS.nmpbb)
    assert src.count(old) == 1, old
    ns = dict(vars(OS))
    exec(compile(src.replace(old, new), "<nmpbb mutant>", "exec"), ns)
    return ns["nmpbb"]


def _isotropic(n=24, r=3, c=2.0, seed=0):
    """Symmetric positive A and a nonnegative partner P whose columns have disjoint
    supports and squared norm c each, so that G = P^T P = c I."""
    rng = np.random.default_rng(seed)
    a = rng.random((n, n)) + 0.5
    A = 0.5 * (a + a.T)
    P = np.zeros((n, r))
    blocks = np.array_split(np.arange(n), r)
    for j, rows in enumerate(blocks):
        v = rng.random(rows.size) + 0.2
        P[rows, j] = v * np.sqrt(c) / np.linalg.norm(v)
    assert np.allclose(P.T @ P, c * np.eye(r), atol=1e-14)
    return A, P, rng


# ------------------------------------------------------------------ BB step
def bb_pin_holds(nmpbb_fn) -> bool:
    c, lam = 2.0, 0.3
    A, P, rng = _isotropic(c=c)
    hs = O.HalfStep(A, P, lam)
    log = []
    nmpbb_fn(hs, rng.random(P.shape), O.Params(lam=lam, inner_iters=4), log)
    assert len(log) == 4
    want = 1.0 / (c + lam)
    # Y = gn - g cancels as the iterates converge: four iterations keep it to ~1e-14
    return all(abs(e["alpha"] - want) <= 1e-12 * want for e in log[1:])


def test_bb_step_is_inverse_curvature_on_isotropic_quadratic():
    assert bb_pin_holds(O.nmpbb)


@pytest.mark.parametrize("old,new", [
    ("ratio = ss / sy", "ratio = sy / ss"),                    # inverted ratio
    ("sy = float(np.sum(S * (gn - g)))", "sy = float(np.sum(S * gn))"),   # Y without -g
])
def test_bb_pin_catches_mutants(old, new):
    assert not bb_pin_holds(mutant(old, new))


# ------------------------------------------------------------------ first projection
def first_projection_pin_holds(nmpbb_fn) -> bool:
    c, lam = 2.0, 0.3
    A, P, rng = _isotropic(c=c, seed=1)
    hs = O.HalfStep(A, P, lam)
    xstar = (A @ P + lam * P) / (c + lam)
    X0 = xstar * (1.0 + 0.2 * (rng.random(P.shape) - 0.5))
    log = []
    nmpbb_fn(hs, X0, O.Params(lam=lam, inner_iters=6), log, keep_arrays=True)
    ok = len(log) == 6
    for e in log:
        ok &= bool((e["X"] > 0).all() and (e["Z"] > 0).all())   # interior: no clipping
        want = xstar - (lam / c) * (e["X"] - xstar)
        ok &= np.abs(e["Z"] - want).max() <= 1e-12 * np.abs(xstar).max()
    return bool(ok)


def test_first_projection_step_is_one_over_rho():
    assert first_projection_pin_holds(O.nmpbb)


def test_first_projection_lands_on_minimiser_without_penalty():
    """lam = 0, G = c I: Z_0 = x* = A P / c, so D_0 = 0, X_1 = x*, and every later step
    S is zero up to rounding (Algorithm 1 at a stationary point)."""
    c = 3.0
    A, P, rng = _isotropic(c=c, seed=2)
    hs = O.HalfStep(A, P, 0.0)
    log = []
    X = O.nmpbb(hs, rng.random(P.shape), O.Params(lam=0.0, inner_iters=6), log, keep_arrays=True)
    xstar = A @ P / c
    tol = 1e-13 * np.abs(xstar).max()
    assert np.abs(log[0]["Z"] - xstar).max() <= tol
    assert np.abs(log[0]["D"]).max() <= tol
    assert np.abs(X - xstar).max() <= tol
    assert all(e["ss"] <= (1e-13 * np.linalg.norm(xstar)) ** 2 for e in log[1:])


@pytest.mark.parametrize("old,new", [
    ("Z = proj(X - g / rho)", "Z = proj(X - alpha * g)"),          # BB step in place of 1/rho
    ("Z = proj(X - g / rho)", "Z = proj(X - g / (rho + hs.lam))"),  # lam not omitted
    ("Z = proj(X - g / rho)", "Z = proj(X - g * rho)"),             # inverted scale
])
def test_first_projection_pin_catches_mutants(old, new):
    assert not first_projection_pin_holds(mutant(old, new))


# ------------------------------------------------------------------ acceptance test
def _fd_dot(fun, X, V, h=1e-6):
    """<grad fun(X), V> by a central difference along V."""
    return (fun(X + h * V) - fun(X - h * V)) / (2.0 * h)


def _ls_case():
    """A tiny half-step with nearly collinear partner columns: the BB step overshoots
    along some directions, so the backtracking is active and the point at which f is
    tested changes the accepted beta."""
    rng = np.random.default_rng(0)
    n, lam = 8, 0.01
    a = rng.random((n, n))
    A = 0.5 * (a + a.T)
    p = rng.random(n)
    P = np.stack([p, p + 0.2 * rng.random(n)], 1)
    return A, P, rng.random((n, 2)), lam


def acceptance_pin_holds(nmpbb_fn) -> bool:
    A, P, X0, lam = _ls_case()
    prm = O.Params(lam=lam, inner_iters=8)
    log = []
    nmpbb_fn(O.HalfStep(A, P, lam), X0, prm, log, keep_arrays=True)
    fd = lambda X: O.objective_direct(A, X, P, lam)      # eq. (1.3) with H = P^T
    shrinks = 0
    for e in log:
        delta = _fd_dot(fd, e["Z"], e["D"])
        beta = 1.0
        for t in range(prm.max_ls + 1):
            if fd(e["Z"] + beta * e["D"]) <= e["F"] + prm.theta * beta * delta:
                break
            if t == prm.max_ls:
                break
            beta *= prm.beta_shrink
        if beta != e["beta"]:
            return False
        shrinks += beta < 1.0
    assert shrinks >= 1, "the case must exercise the backtracking"
    return True


def test_accepted_beta_follows_the_literal_test_at_z_plus_beta_d():
    assert acceptance_pin_holds(O.nmpbb)


@pytest.mark.parametrize("old,new", [
    ("trial = Z + beta * D", "trial = Z + prm.phi * beta * D"),     # test at the relaxed point
    ("<= F + prm.theta * beta * delta", "<= fX + prm.theta * beta * delta"),  # monotone test
])
def test_acceptance_pin_catches_mutants(old, new):
    assert not acceptance_pin_holds(mutant(old, new))


# ------------------------------------------------------------------ nonmonotone reference
def reference_pin_holds(nmpbb_fn) -> bool:
    A, P, X0, lam = _ls_case()
    eta = 0.85
    log = []
    nmpbb_fn(O.HalfStep(A, P, lam), X0, O.Params(lam=lam, eta=eta, inner_iters=4), log,
             keep_arrays=True)
    f = [O.objective_direct(A, X0, P, lam)] + [O.objective_direct(A, e["Xn"], P, lam)
                                               for e in log[:3]]
    # F_3 of the recursion, unrolled: a convex combination of f_0 .. f_3
    F3 = (1 - eta) * f[3] + eta * (1 - eta) * f[2] + eta ** 2 * (1 - eta) * f[1] + eta ** 3 * f[0]
    F1 = (1 - eta) * f[1] + eta * f[0]
    return (abs(log[0]["F"] - f[0]) <= 1e-13 * abs(f[0])
            and abs(log[1]["F"] - F1) <= 1e-12 * abs(F1)
            and abs(log[3]["F"] - F3) <= 1e-12 * abs(F3))


def test_nonmonotone_reference_three_steps_by_hand():
    assert reference_pin_holds(O.nmpbb)


@pytest.mark.parametrize("old,new", [
    ("F = fn + prm.eta * (F - fn)", "F = F + prm.eta * (fn - F)"),   # memory weights swapped
    ("F = fn + prm.eta * (F - fn)", "F = fn"),                      # monotone reference
])
def test_reference_pin_catches_mutants(old, new):
    assert not reference_pin_holds(mutant(old, new))


# ------------------------------------------------------------------ monitor
def test_monitor_by_explicit_loops():
    rng = np.random.default_rng(21)
    n, r, lam, gam = 7, 2, 0.3, 0.4
    a = rng.random((n, n))
    A = 0.5 * (a + a.T)
    x = rng.standard_normal((n, 2))
    from paper_2606_02887_amd import gen
    L = O.knn_laplacian(x, 2)
    Ld = L.toarray()
    W, Ht = rng.random((n, r)), rng.random((n, r))
    m = O.monitor(A, W, Ht, O.Params(lam=lam, gamma=gam), L)
    nA = sum(A[i, j] ** 2 for i in range(n) for j in range(n)) ** 0.5
    rww = sum((A[i, j] - sum(W[i, t] * W[j, t] for t in range(r))) ** 2
              for i in range(n) for j in range(n)) ** 0.5 / nA
    rwh = sum((A[i, j] - sum(W[i, t] * Ht[j, t] for t in range(r))) ** 2
              for i in range(n) for j in range(n))
    gap = sum((W[i, t] - Ht[i, t]) ** 2 for i in range(n) for t in range(r))
    nW = sum(W[i, t] ** 2 for i in range(n) for t in range(r))
    lap = sum(Ht[i, t] * Ld[i, j] * Ht[j, t] for i in range(n) for j in range(n) for t in range(r))
    f = 0.5 * rwh + 0.5 * lam * gap + 0.5 * gam * lap
    assert abs(m["res_WWt"] - rww) <= 1e-13 * rww
    assert abs(m["res_WH"] - rwh ** 0.5 / nA) <= 1e-13
    assert abs(m["sym_gap"] - (gap / nW) ** 0.5) <= 1e-13
    assert abs(m["objective"] - f) <= 1e-12 * f
    # the objective of a planted exact factorisation with lam, gam = 0 is zero
    Wst = rng.random((n, r))
    m0 = O.monitor(Wst @ Wst.T, Wst, Wst, O.Params())
    assert abs(m0["objective"]) <= 1e-12 and m0["res_WWt"] <= 1e-7
