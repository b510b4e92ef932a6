"""The property the fused inner kernels rely on after a backtrack, checked on the oracle's
own iterates (Algorithm 1 with the Section 2.4 update).

D = max(0, Z - alpha grad f(Z)) - Z makes Z + D >= 0, and Z >= 0, so for t = phi beta <= 1
the relaxed point Z + t D is a convex combination of two nonnegative points: the
projection max(0, .) leaves it unchanged and S = X_{k+1} - X_k = dZ + t D with dZ = Z - X_k.
Then <S,S>, <S,Y> = <S, S (G + lam I)> and <g,S> are polynomials in t whose coefficients
are sums over dZ, D, dZ G and D G; the fused kernels form those coefficients with the
direction and evaluate the polynomials once the line search has chosen beta.  With the
default phi = 1.7 and beta_shrink = 0.5 every backtracked trial has t <= 0.85.  The trial
beta = 1 (t = phi > 1) does get clipped, which is why its sums are formed from the clipped
update itself.
"""
import numpy as np

import oracle as O
from paper_2606_02887_amd import gen


def _iterations():
    p = gen.planted_dense(400, 10, 77)
    A, W0 = p["A"], p["W0"]
    prm = O.Params(lam=O.default_lambda(A), theta=0.5, eta=0.0)
    W, H = W0.copy(), W0.copy()
    out = []
    for _ in range(6):
        for hs in (0, 1):
            X, P = (W, H) if hs == 0 else (H, W)
            log = []
            hstep = O.HalfStep(A, P, prm.lam)
            X = O.nmpbb(hstep, X, prm, log=log, keep_arrays=True)
            G = P.T @ P
            out += [(e, G) for e in log]
            if hs == 0:
                W = X
            else:
                H = X
    return prm, out


def test_backtracked_updates_are_unclipped_polynomials():
    prm, its = _iterations()
    back = [(e, G) for e, G in its if e["beta"] < 1.0]
    assert len(back) >= 5                         # theta = 0.5, eta = 0 backtracks often
    for e, G in back:
        t = prm.phi * e["beta"]
        assert t <= 1.0
        X, Z, D, g = e["X"], e["Z"], e["D"], e["g"]
        assert (Z >= 0).all() and (Z + D >= -1e-15 * np.abs(Z).max()).all()
        S = e["Xn"] - X
        dZ = Z - X
        assert np.abs(S - (dZ + t * D)).max() <= 1e-14 * np.abs(X).max()
        ss = np.sum(dZ * dZ) + t * (2.0 * np.sum(dZ * D) + t * np.sum(D * D))
        sGs = np.sum(dZ * (dZ @ G)) + t * (2.0 * np.sum(dZ * (D @ G)) + t * np.sum(D * (D @ G)))
        gS = np.sum(g * dZ) + t * np.sum(g * D)
        assert abs(ss - e["ss"]) <= 1e-10 * e["ss"]
        assert abs(sGs + prm.lam * ss - e["sy"]) <= 1e-10 * e["sy"]
        assert abs(gS - np.sum(g * S)) <= 1e-10 * np.abs(g).sum() * np.abs(S).max()


def test_the_first_trial_is_clipped():
    """t = phi = 1.7 > 1: some accepted beta = 1 updates do leave the nonnegative orthant
    before the projection, so S differs from dZ + phi D there."""
    prm, its = _iterations()
    clipped = 0
    for e, _ in its:
        if e["beta"] == 1.0:
            clipped += int((e["Z"] + prm.phi * e["D"] < 0).any())
    assert clipped >= 5
