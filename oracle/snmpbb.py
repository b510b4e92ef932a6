"""FP64 CPU reference ("oracle") of SNMPBB, Graph-SNMPBB and LAI-SNMPBB.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package; only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may call it.  It
shares no code with the HIP library: it is plain numpy/scipy in float64, written from
the paper (Swart & Brust, "A Nonmonotone Gradient-Based Algorithm for Symmetric
Nonnegative Matrix Factorization and Graph Clustering").

What it computes, with the passage each part follows:

* objective  f(W,H;lam,gam) = 1/2||A - W H||^2 + lam/2 ||W - H^T||^2 + gam/2 tr(H L H^T)
  -- eq. (1.3) (symmetric penalty) and eq. (2.3) (Graph-SNMPBB).  The factor H is
  stored transposed, ``Ht = H^T`` (n x r), so both half-steps have the same shape:
  W-step: variable X = W, partner P = Ht;  H-step: X = Ht, P = W.
* gradients  grad_W = W H H^T - A H^T + lam W - lam H^T               -- eq. (2.1)
             grad_H = W^T W H - W^T A + lam H - lam W^T (+ gam H L)     -- eq. (2.2)/(2.3)
  transposed into the common form  grad(X) = X G - A P + lam (X - P) [+ gam L X]  with
  G = P^T P (A and L symmetric).
* the inner loop is Algorithm 1 (NMPBB) with the choices of Section 2.4: first
  projection with 1/rho0, rho0 = ||H0 H0^T||_2 (lam omitted); Frobenius BB step
  clipped to [alpha_min, alpha_max]; nonmonotone reference F_k; backtracking from
  beta = 1; relaxed update Z + phi*beta*D.
* outer alternation W-step then H-step (Section 1, Section 2.1).
* LAI-SNMPBB (Section 2.3): every product A P becomes U (lam * (U^T P)).

Readings taken where the paper is silent (each is a field of ``Params``):
  inner_iters = 5 fixed inner iterations per half-step, early exit only when S = 0;
  alpha_0 = 1/rho for the first inner iteration (no S_{-1} exists);
  alpha_min = 1e-10, alpha_max = 1e10; eta = 0.85 constant; theta = 1e-3; phi = 1.7;
  backtracking factor 0.5 with at most ``max_ls`` reductions (the last beta is taken
  when the cap is hit);  the acceptance test evaluates f(Z + beta D) as Algorithm 1
  writes it (``accept_at_relaxed`` switches to the f(Z + phi beta D) reading of
  Section 2.4);  the relaxed point is projected, max(0, Z + phi beta D), so that the
  iterate stays feasible (``project_update``);  the H-step uses rho = ||W^T W||_2 and
  omits gam ||L|| just as lam is omitted.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Params:
    lam: float = 0.0                # symmetric penalty lambda of eq. (1.3)
    gamma: float = 0.0              # Laplacian weight gamma of eq. (2.3)
    eta: float = 0.85               # nonmonotone memory eta_k in [0, 1)
    theta: float = 1e-3             # Armijo parameter theta_k in (0, 1)
    phi: float = 1.7                # relaxation factor varphi
    alpha_min: float = 1e-10
    alpha_max: float = 1e10
    beta_shrink: float = 0.5
    max_ls: int = 20
    inner_iters: int = 5
    accept_at_relaxed: bool = False
    project_update: bool = True


class LowRank:
    """Low-rank input A ~= U diag(lam) U^T of Section 2.3 (U has orthonormal columns)."""

    def __init__(self, U, lam):
        self.U = np.asarray(U, dtype=np.float64)
        self.lam = np.asarray(lam, dtype=np.float64)
        self.shape = (self.U.shape[0], self.U.shape[0])


# --------------------------------------------------------------------------- A-operator
def apply_A(A, P):
    """A @ P for a dense array, a scipy sparse matrix or a LowRank operator.

    For LowRank the product is formed as U (lam * (U^T P)), with U^T P first
    (Section 2.3: the large n x n product is never formed)."""
    if isinstance(A, LowRank):
        t = A.U.T @ P
        return A.U @ (A.lam[:, None] * t)
    if sp.issparse(A):
        return np.asarray(A @ P)
    return A @ P


def norm2_A(A) -> float:
    """||A||_F^2; for LowRank the surrogate's norm sum(lam^2) (U orthonormal)."""
    if isinstance(A, LowRank):
        return float(np.sum(A.lam ** 2))
    if sp.issparse(A):
        return float(np.sum(np.asarray(A.data, dtype=np.float64) ** 2))
    return float(np.sum(np.asarray(A, dtype=np.float64) ** 2))


def spectral_norm_psd(G) -> float:
    """||G||_2 of a symmetric positive semidefinite r x r matrix = its largest eigenvalue."""
    return float(np.linalg.eigvalsh(G)[-1])


def proj(X):
    """Projection onto the nonnegative orthant (Section 1.1, Proj)."""
    return np.maximum(X, 0.0)


# --------------------------------------------------------------------------- objective
def objective_direct(A_dense, W, Ht, lam, gamma=0.0, L=None):
    """Eq. (1.3) / (2.3) evaluated literally from a dense A (small inputs only)."""
    H = Ht.T
    f = 0.5 * np.sum((A_dense - W @ H) ** 2) + 0.5 * lam * np.sum((W - H.T) ** 2)
    if gamma and L is not None:
        Ld = L.toarray() if sp.issparse(L) else L
        f += 0.5 * gamma * np.trace(H @ Ld @ H.T)
    return float(f)


class HalfStep:
    """f and its gradient with the partner block P fixed (one half-step).

    f(X) = 1/2||A||^2 - <A P, X> + 1/2 <X^T X, P^T P> + lam/2 ||X - P||^2
           [+ gam/2 <X, L X>]
    which equals eq. (1.3)/(2.3) with H = P^T (W-step) or W = P (H-step): expanding
    1/2||A - X P^T||^2 uses <A, X P^T> = <A P, X> and ||X P^T||^2 = <X^T X, P^T P>."""

    def __init__(self, A, P, lam, gamma=0.0, L=None, normA2=None):
        self.P = P
        self.lam = float(lam)
        self.gamma = float(gamma) if L is not None else 0.0
        self.L = L if self.gamma else None
        self.G = P.T @ P                                  # H H^T  (r x r)
        self.B = apply_A(A, P)                            # A H^T  (n x r)
        self.normA2 = norm2_A(A) if normA2 is None else normA2
        self.rho = spectral_norm_psd(self.G)              # rho0 = ||H0 H0^T||_2

    def grad(self, X):
        g = X @ self.G - self.B
        if self.lam:                     # (the penalty needs X and P of one shape)
            g = g + self.lam * (X - self.P)
        if self.L is not None:
            g = g + self.gamma * np.asarray(self.L @ X)
        return g

    def f(self, X):
        v = 0.5 * self.normA2 - np.sum(self.B * X) + 0.5 * np.sum((X.T @ X) * self.G)
        if self.lam:
            v += 0.5 * self.lam * np.sum((X - self.P) ** 2)
        if self.L is not None:
            v += 0.5 * self.gamma * np.sum(X * np.asarray(self.L @ X))
        return float(v)


# --------------------------------------------------------------------------- Algorithm 1
def nmpbb(hs: HalfStep, X0, prm: Params, log: Optional[list] = None, keep_arrays: bool = False):
    """Inner NMPBB iterations (Algorithm 1 with the Section 2.4 components).

    Returns the last iterate.  If ``log`` is a list, one dict per inner iteration is
    appended with the scalars of that iteration (for invariant and lockstep tests);
    ``keep_arrays`` also stores the iterate, Z, D and the gradients."""
    rho = hs.rho
    if not rho > 0.0:
        raise FloatingPointError("rho = ||P^T P||_2 is zero: the partner block vanished")
    X = np.array(X0, dtype=np.float64, copy=True)
    g = hs.grad(X)
    fX = hs.f(X)
    F = fX                                         # F_0 = f(W_0)
    alpha = 1.0 / rho
    ss = sy = None
    for k in range(prm.inner_iters):
        Z = proj(X - g / rho)                      # first projection, step 1/rho0
        gZ = hs.grad(Z)
        if k > 0:                                  # Frobenius BB step, clipped
            ratio = ss / sy if sy > 0.0 else np.inf   # sy >= lam*ss > 0 unless S = 0
            alpha = min(prm.alpha_max, max(prm.alpha_min, ratio))
        D = proj(Z - alpha * gZ) - Z               # second projection -> direction
        delta = float(np.sum(gZ * D))              # <grad f(Z_k), D_k>
        beta, t, exhausted, evals = 1.0, 0, False, 0
        while True:                                # nonmonotone backtracking from beta = 1
            if prm.accept_at_relaxed:
                trial = Z + prm.phi * beta * D
                if prm.project_update:
                    trial = proj(trial)
            else:
                trial = Z + beta * D
            evals += 1
            if hs.f(trial) <= F + prm.theta * beta * delta:
                break
            if t >= prm.max_ls:
                exhausted = True
                break
            beta *= prm.beta_shrink
            t += 1
        Xn = Z + prm.phi * beta * D                # relaxed update
        if prm.project_update:
            Xn = proj(Xn)
        gn = hs.grad(Xn)
        S = Xn - X
        ss = float(np.sum(S * S))
        sy = float(np.sum(S * (gn - g)))
        fn = hs.f(Xn)
        if log is not None:
            log.append(dict(k=k, alpha=alpha, beta=beta, ls=t, evals=evals,
                            exhausted=exhausted, delta=delta, F=F, fX=fX, fZ=hs.f(Z),
                            fn=fn, ss=ss, sy=sy, normD2=float(np.sum(D * D)),
                            rho=rho))
            if keep_arrays:
                log[-1].update(X=X.copy(), Z=Z, D=D, Xn=Xn.copy(), g=g.copy(), gZ=gZ,
                               gn=gn.copy())
        F = fn + prm.eta * (F - fn)                # F_{k+1} = f(W_{k+1}) + eta (F_k - f(W_{k+1}))
        X, g, fX = Xn, gn, fn
        if ss == 0.0:                              # stationary: nothing left to do
            break
    return X


def half_step(A, X, P, prm: Params, laplacian: bool = False, L=None, normA2=None, log=None):
    """One half-step: build f for the fixed partner P, run the inner loop from X."""
    hs = HalfStep(A, P, prm.lam, prm.gamma if laplacian else 0.0,
                  L if laplacian else None, normA2)
    return nmpbb(hs, X, prm, log)


# --------------------------------------------------------------------------- monitor
def residual_WH(A, W, Ht, normA2=None) -> float:
    """||A - W Ht^T||_F / ||A||_F (the residual of Section 4).  Dense A is evaluated
    directly; sparse / low-rank A via the exact expansion
    ||A||^2 - 2<A Ht, W> + <W^T W, Ht^T Ht>."""
    nA2 = norm2_A(A) if normA2 is None else normA2
    if isinstance(A, np.ndarray):
        return float(np.linalg.norm(A - W @ Ht.T) / np.sqrt(nA2))
    val = nA2 - 2.0 * np.sum(apply_A(A, Ht) * W) + np.sum((W.T @ W) * (Ht.T @ Ht))
    return float(np.sqrt(max(val, 0.0)) / np.sqrt(nA2))


def pg_norm(A, W, Ht, prm: Params, L=None) -> float:
    """Projected-gradient stationarity measure ||D_1|| for both blocks, where
    D_1(X) = Proj[X - grad f(X)] - X = -min(X, grad f(X)) vanishes exactly at
    stationary points (Section 3.1)."""
    gw = HalfStep(A, Ht, prm.lam).grad(W)
    gh = HalfStep(A, W, prm.lam, prm.gamma, L).grad(Ht)
    return float(np.sqrt(np.sum(np.minimum(W, gw) ** 2) + np.sum(np.minimum(Ht, gh) ** 2)))


def objective(A, W, Ht, prm: Params, L=None, normA2=None) -> float:
    """f(W, H) of eq. (1.3), plus gam/2 tr(H L H^T) of eq. (2.3) when L is given, in the
    trace form 1/2||A||^2 - <A Ht, W> + 1/2<W^T W, Ht^T Ht> + lam/2||W - Ht||^2
    [+ gam/2 <Ht, L Ht>] (for LowRank input ||A||^2 is the surrogate's sum(lam^2))."""
    nA2 = norm2_A(A) if normA2 is None else normA2
    v = (0.5 * nA2 - np.sum(apply_A(A, Ht) * W) + 0.5 * np.sum((W.T @ W) * (Ht.T @ Ht))
         + 0.5 * prm.lam * np.sum((W - Ht) ** 2))
    if L is not None and prm.gamma:
        v += 0.5 * prm.gamma * np.sum(Ht * np.asarray(L @ Ht))
    return float(v)


def monitor(A, W, Ht, prm: Params, L=None, normA2=None):
    """The per-outer-iteration record: residuals ||A - W H||/||A|| and ||A - W W^T||/||A||
    (Section 4), the symmetry gap ||W - H^T||/||W||, the projected-gradient norm and the
    objective f(W, H)."""
    nA2 = norm2_A(A) if normA2 is None else normA2
    out = dict(res_WH=residual_WH(A, W, Ht, nA2),
               res_WWt=residual_WH(A, W, W, nA2),
               sym_gap=float(np.linalg.norm(W - Ht) / max(np.linalg.norm(W), 1e-300)),
               pg=pg_norm(A, W, Ht, prm, L),
               objective=objective(A, W, Ht, prm, L, nA2))
    return out


# --------------------------------------------------------------------------- outer loop
def snmpbb(A, W0, prm: Params, max_outer: int, L=None, target_res: float = 0.0,
           monitor_every: int = 1, logs: Optional[list] = None):
    """SNMPBB outer alternation: W-step with H fixed, then H-step with W fixed.

    ``Ht`` starts at ``W0`` (H0 = W0^T, Section 4.1 item (4)).  With ``L`` and
    ``prm.gamma > 0`` this is Graph-SNMPBB (Laplacian on the H block, eq. (2.3)).
    Returns (W, Ht, history) where history holds one monitor dict per outer iteration
    (every ``monitor_every``-th); the loop stops after the first monitored outer
    iteration whose residual is <= target_res (when target_res > 0)."""
    nA2 = norm2_A(A)
    W = np.array(W0, dtype=np.float64, copy=True)
    Ht = W.copy()
    hist = []
    lap = L is not None and prm.gamma > 0
    for i in range(max_outer):
        lw = [] if logs is not None else None
        lh = [] if logs is not None else None
        W = half_step(A, W, Ht, prm, False, None, nA2, lw)
        Ht = half_step(A, Ht, W, prm, lap, L, nA2, lh)
        if logs is not None:
            logs.append((lw, lh))
        if (i + 1) % monitor_every == 0 or i + 1 == max_outer:
            m = monitor(A, W, Ht, prm, L if lap else None, nA2)
            m["outer"] = i + 1
            hist.append(m)
            if target_res > 0 and m["res_WH"] <= target_res:
                break
    return W, Ht, hist


def naive(A, W0, prm: Params, max_outer: int, target_res: float = 0.0):
    """The naive symmetric variant that Section 2.1 describes before the penalty method
    (and reports to perform poorly): every outer iteration runs Algorithm 1 on W alone for
    min ||A - W W_i^T||_F^2 / 2, the partner held at the current iterate W_i and no
    penalty, then sets H <- W^T.  prm.lam must be 0.  Returns (W, Ht, history) as snmpbb
    does, with Ht = W after every outer iteration."""
    if prm.lam != 0.0:
        raise ValueError("the naive variant has no penalty term (lam must be 0)")
    nA2 = norm2_A(A)
    W = np.array(W0, dtype=np.float64, copy=True)
    hist = []
    for i in range(max_outer):
        W = half_step(A, W, W.copy(), prm, False, None, nA2)
        Ht = W.copy()                                  # H <- W^T
        m = monitor(A, W, Ht, prm, None, nA2)
        m["outer"] = i + 1
        hist.append(m)
        if target_res > 0 and m["res_WH"] <= target_res:
            break
    return W, W.copy(), hist


def default_lambda(A) -> float:
    """lambda ~= 0.01 ||A||_F (Section 4.1, guideline (1))."""
    return 0.01 * float(np.sqrt(norm2_A(A)))
