"""FP64 CPU reference of NMPBB for (unsymmetric) NMF -- TEST INFRASTRUCTURE ONLY.

The method's starting point (Section 1, eq. (1.1); Section 2.1): a nonnegative
V (m x n) ~= W H with W (m x r) >= 0 and H (r x n) >= 0, minimising 1/2 ||V - W H||_F^2 by
alternating a W-step (H fixed) and an H-step (W fixed), each a run of Algorithm 1 with
the components of Section 2.4.  With H stored transposed (Ht = H^T, n x r) both steps
take the form of snmpbb.HalfStep without the penalty (lam = 0): the W-step has
partner P = Ht and product V Ht, the H-step partner P = W and product V^T W.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .snmpbb import HalfStep, Params, nmpbb


def _norm2(V):
    if sp.issparse(V):
        return float(np.sum(np.asarray(V.data, dtype=np.float64) ** 2))
    return float(np.sum(np.asarray(V, dtype=np.float64) ** 2))


def residual(V, W, Ht, normV2=None) -> float:
    """||V - W Ht^T||_F / ||V||_F."""
    nV2 = _norm2(V) if normV2 is None else normV2
    if not sp.issparse(V):
        return float(np.linalg.norm(np.asarray(V) - W @ Ht.T) / np.sqrt(nV2))
    val = nV2 - 2.0 * np.sum(np.asarray(V @ Ht) * W) + np.sum((W.T @ W) * (Ht.T @ Ht))
    return float(np.sqrt(max(val, 0.0)) / np.sqrt(nV2))


def pg_norm(V, W, Ht) -> float:
    """||min(W, grad_W f)||^2 + ||min(Ht, grad_Ht f)||^2, square root (zero exactly at
    first-order stationary points)."""
    gw = HalfStep(V, Ht, 0.0).grad(W)
    gh = HalfStep(V.T, W, 0.0).grad(Ht)
    return float(np.sqrt(np.sum(np.minimum(W, gw) ** 2) + np.sum(np.minimum(Ht, gh) ** 2)))


def nmf(V, W0, Ht0, prm: Params, max_outer: int):
    """NMPBB on eq. (1.1): W-step then H-step per outer iteration.  prm.lam must be 0
    (there is no coupling between W and H^T).  Returns (W, Ht, history)."""
    if prm.lam != 0.0 or prm.gamma != 0.0:
        raise ValueError("NMF has no symmetric penalty or Laplacian term")
    nV2 = _norm2(V)
    Vt = V.T.tocsr() if sp.issparse(V) else np.asarray(V).T
    W = np.array(W0, dtype=np.float64, copy=True)
    Ht = np.array(Ht0, dtype=np.float64, copy=True)
    hist = []
    for i in range(max_outer):
        W = nmpbb(HalfStep(V, Ht, 0.0, normA2=nV2), W, prm)
        Ht = nmpbb(HalfStep(Vt, W, 0.0, normA2=nV2), Ht, prm)
        res = residual(V, W, Ht, nV2)
        hist.append({"outer": i + 1, "res_WH": res, "pg": pg_norm(V, W, Ht),
                     "objective": 0.5 * res * res * nV2})
    return W, Ht, hist
