"""An FP32 rounding model of the GPU half-step, used only to size the FP32 parity bounds.

The HIP kernels run Algorithm 1 with FP32 arrays and FP64 scalars, and they carry the
gradient by linearity: g = X G + lam X - C once per half-step (C = A P + lam P), then
grad f(Z) = g + (Z - X)(G + lam I) [+ gam L (Z - X)] and g+ = g + S (G + lam I)
[+ gam L S].  The oracle forms every gradient directly in FP64.  Where the partner block
P has strongly correlated columns, the first projection Z = X - g/rho cancels most of X
and grad f(Z) is a small difference of two large terms, so the FP32 rounding of the
update (about 2^-24 |X G|) is large against grad f(Z); the nonmonotone BB steps, longer
than 1/rho, then carry it into X+.  This module repeats the half-step in numpy with every
stored array rounded to FP32 (scalars in FP64, the line search in the closed form of the
quadratic), so a test can measure how far that arithmetic alone moves X+ from the
oracle's, and bound the GPU by a small multiple of it.  It shares no code with the HIP
library and is not a reference: expected values always come from the oracle.
"""
import numpy as np


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def half_step_fp32(hs, X0, prm):
    """X+ after prm.inner_iters inner iterations, FP32 arrays; hs is the oracle's
    HalfStep (it supplies G, B, P, lam, gamma, L and rho)."""
    G32 = f32(hs.G)
    lam, gam, rho = hs.lam, hs.gamma, hs.rho
    L = hs.L

    def lap(V):
        return f32(L @ V) if L is not None else 0.0

    X = f32(X0)
    C = f32(hs.B + lam * hs.P) if lam else f32(hs.B)   # (NMF: P and X differ in shape)
    g = f32(f32(X @ G32) + f32(lam * X) - C)
    if L is not None:
        g = f32(g + f32(gam * lap(X)))
    F_minus_f = 0.0
    alpha = 1.0 / rho
    rinv = f32(1.0 / rho)
    ss = sy = None
    for k in range(prm.inner_iters):
        Z = f32(np.maximum(0.0, f32(X - f32(g * rinv))))
        dZ = f32(Z - X)
        gZ = f32(g + f32(f32(dZ @ G32) + f32(lam * dZ)))
        if L is not None:
            gZ = f32(gZ + f32(gam * lap(dZ)))
        if k > 0:
            alpha = min(prm.alpha_max, max(prm.alpha_min, ss / sy if sy > 0 else np.inf))
        D = f32(f32(np.maximum(0.0, f32(Z - f32(f32(alpha) * gZ)))) - Z)
        delta = float(np.sum(gZ * D))
        q = float(np.sum((D @ hs.G) * D)) + lam * float(np.sum(D * D))
        if L is not None:
            q += gam * float(np.sum(D * (L @ D)))
        fZ_minus_fX = float(np.sum(0.5 * (g + gZ) * dZ))
        beta = 1.0
        for t in range(prm.max_ls + 1):
            if fZ_minus_fX + (1.0 - prm.theta) * beta * delta + 0.5 * beta * beta * q <= F_minus_f:
                break
            if t == prm.max_ls:
                break
            beta *= prm.beta_shrink
        Xn = f32(np.maximum(0.0, f32(Z + f32(f32(prm.phi * beta) * D))))
        S = f32(Xn - X)
        gn = f32(g + f32(f32(S @ G32) + f32(lam * S)))
        if L is not None:
            gn = f32(gn + f32(gam * lap(S)))
        ss = float(np.sum(S * S))
        sy = float(np.sum((S @ hs.G) * S)) + lam * ss
        if L is not None:
            sy += gam * float(np.sum(S * (L @ S)))
        dlt = float(np.sum(g * S)) + 0.5 * sy          # f(X+) - f(X), exact for a quadratic
        F_minus_f = prm.eta * (F_minus_f - dlt)
        X, g = Xn, gn
        if ss == 0.0:
            break
    return X
