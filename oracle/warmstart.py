"""FP64 CPU reference of the learned warm start -- TEST INFRASTRUCTURE ONLY.

The warm start is not in the paper (its closest analogue is the SVD-based start of the
numerical experiments, Section 4.2).  It maps a symmetric nonnegative A to a start W0 for
SNMPBB in three steps, each written here plainly in numpy float64:

1. sketch      Y = A Omega, Omega an n x r Gaussian matrix (an input: the random numbers
               are drawn by the caller).
2. frame       successive projection (SPA; Gillis & Vavasis, "Fast and robust recursive
               algorithms for separable nonnegative matrix factorization", 2014) on the
               sketch with row i divided by d_i = (A 1)_i picks r anchor rows K.  For
               A = W W^T with W >= 0, Y_i / d_i = W_i M / (W_i W^T 1) is a convex
               combination of the anchor rows Y_k / d_k -- the separable setting in which
               SPA finds the anchors (rows with d_i = 0 become zero).  The coordinates of
               every row in the anchor frame are C = Y Y_K^{-1}, computed as
               C = Y Y_K^T (Y_K Y_K^T + eps I)^{-1} with eps = 1e-12 tr(Y_K Y_K^T) / r.
               If Y = W M for some r x r M (as for A = W W^T), C = W W_K^{-1}: the frame
               removes the random mixing M that a row-wise map could not undo.  C is then
               divided by the entry RMS of relu(C), so that every problem's coordinates
               have the same scale (a row-wise map cannot see a per-problem scale).
3. network     W0_i = s relu(c_i + M2 relu(M1 c_i + b1) + b2), a row-wise residual MLP
               r -> H -> r with BF16 weights M1, M2 (FP32 biases), and the scale
               s = (sqrt(r) ||A||_F / (n r))^(1/2), the entry RMS of a W with
               ||W W^T||_F = ||A||_F and r equal orthogonal columns.  With M2 = 0 and
               b2 = 0 it is the start of the frame alone, s relu(c_i).

Training: targets are converged SNMPBB factors Ht whose columns are permuted to the
anchor order by a linear assignment (scipy's Hungarian solver) on the cosine similarity
of columns, divided by their entry RMS (the shape of the factor; s sets the scale); the
loss is the mean squared error plus a scale term mu (mean(y^2) - mean(t^2))^2; the
optimiser is Adam (Kingma & Ba, 2015).
"""
from __future__ import annotations

import numpy as np
import scipy.optimize as so
import scipy.sparse as sp

HIDDEN = 128


# --------------------------------------------------------------------------- sketch
def sketch(A, Omega):
    """Y = A Omega in float64 (dense or scipy sparse A)."""
    Om = np.asarray(Omega, dtype=np.float64)
    if sp.issparse(A):
        return np.asarray(A @ Om)
    return np.asarray(A, dtype=np.float64) @ Om


def row_sums(A):
    """d = A 1."""
    if sp.issparse(A):
        return np.asarray(A.sum(axis=1), dtype=np.float64).ravel()
    return np.asarray(A, dtype=np.float64).sum(axis=1)


def row_normalise(Y, d):
    """Row i divided by d_i (rows with d_i <= 0 become zero)."""
    out = np.zeros_like(Y)
    nz = d > 0
    out[nz] = Y[nz] / d[nz, None]
    return out


def spa(R0, r):
    """Successive projection: r times, take the row of largest norm (first index on ties)
    and project every row onto the orthogonal complement of that row."""
    R = np.array(R0, dtype=np.float64, copy=True)
    K = []
    for _ in range(r):
        nrm2 = np.sum(R * R, axis=1)
        k = int(np.argmax(nrm2))
        K.append(k)
        if nrm2[k] > 0:
            u = R[k] / np.sqrt(nrm2[k])
            R = R - np.outer(R @ u, u)
    return K


def coords(Y, K):
    """C = Y Y_K^T (Y_K Y_K^T + eps I)^{-1}, eps = 1e-12 tr(Y_K Y_K^T) / r."""
    YK = Y[K]
    r = len(K)
    Gk = YK @ YK.T
    eps = 1e-12 * np.trace(Gk) / r
    return np.linalg.solve(Gk + eps * np.eye(r), (Y @ YK.T).T).T


def rms_pos(C) -> float:
    """Entry RMS of relu(C)."""
    pos = np.maximum(C, 0.0)
    return float(np.sqrt(np.mean(pos * pos)))


def frame(A, Omega):
    """(C, K, Y): coordinates of every row in the SPA anchor frame of the sketch, divided
    by rms(relu(C)) (left as they are if relu(C) = 0)."""
    Y = sketch(A, Omega)
    K = spa(row_normalise(Y, row_sums(A)), Omega.shape[1])
    C = coords(Y, K)
    rms = rms_pos(C)
    return (C / rms if rms > 0 else C), K, Y


def scale(normA, n, r):
    """s = (sqrt(r) ||A||_F / (n r))^(1/2)."""
    return float(np.sqrt(np.sqrt(r) * normA / (n * r)))


# --------------------------------------------------------------------------- BF16
def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), through float32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------- network
def forward(params, C, quantize=True):
    """Rows of C (N x r) -> (y, cache): y = relu(c + M2 relu(M1 c + b1) + b2)."""
    M1 = bf16_round(params["M1"]) if quantize else np.asarray(params["M1"], np.float64)
    M2 = bf16_round(params["M2"]) if quantize else np.asarray(params["M2"], np.float64)
    b1 = np.asarray(params["b1"], np.float64)
    b2 = np.asarray(params["b2"], np.float64)
    a = C @ M1.T + b1
    h = np.maximum(a, 0.0)
    o = C + h @ M2.T + b2
    return np.maximum(o, 0.0), (C, a, h, o, M1, M2)


def loss(y, T, mu):
    """mean((y - t)^2) + mu (mean(y^2) - mean(t^2))^2 over all N x r entries."""
    d = (np.mean(y * y) - np.mean(T * T))
    return float(np.mean((y - T) ** 2) + mu * d * d)


def loss_and_grad(params, C, T, mu, quantize=True):
    """Loss and its gradient with respect to M1, b1, M2, b2 (straight through the BF16
    rounding of the weights)."""
    y, (C_, a, h, o, M1, M2) = forward(params, C, quantize)
    N = y.size
    d = np.mean(y * y) - np.mean(T * T)
    dy = 2.0 * (y - T) / N + mu * 2.0 * d * (2.0 * y / N)
    do = dy * (o > 0)
    gM2 = do.T @ h
    gb2 = do.sum(axis=0)
    dh = do @ M2
    da = dh * (a > 0)
    gM1 = da.T @ C_
    gb1 = da.sum(axis=0)
    return loss(y, T, mu), {"M1": gM1, "b1": gb1, "M2": gM2, "b2": gb2}


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------- targets
def match_columns(C, Ht):
    """Permutation p (anchor j <- column p[j] of Ht) maximising the summed cosine
    similarity of C[:, j] and Ht[:, p[j]] (linear assignment)."""
    cn = np.sqrt(np.sum(C * C, axis=0))
    hn = np.sqrt(np.sum(Ht * Ht, axis=0))
    cos = (C.T @ Ht) / np.maximum(np.outer(cn, hn), 1e-300)
    rows, cols = so.linear_sum_assignment(-cos)
    p = np.empty(C.shape[1], dtype=np.int64)
    p[rows] = cols
    return p


def targets(C, Ht):
    """Training targets of one problem: the columns of Ht in the anchor order
    (match_columns) divided by their entry RMS (zero if Ht = 0); and the permutation."""
    p = match_columns(C, Ht)
    T = np.asarray(Ht, dtype=np.float64)[:, p]
    rms = float(np.sqrt(np.mean(T * T)))
    return (T / rms if rms > 0 else T), p


def frame_start(A, Omega, normA):
    """The start of the frame alone (the ablation without the network):
    W0 = s relu(C) / rms(relu(C)), rms over all n r entries (W0 = s everywhere if
    relu(C) = 0; the frame's C has rms(relu(C)) = 1 already, up to rounding)."""
    C, K, _ = frame(A, Omega)
    n, r = C.shape
    s = scale(normA, n, r)
    pos = np.maximum(C, 0.0)
    rms = rms_pos(C)
    return (s * pos / rms if rms > 0 else np.full_like(C, s)), C, K


def warm_start(params, A, Omega, normA):
    """W0 = s * MLP(C) for one problem."""
    C, K, _ = frame(A, Omega)
    n, r = C.shape
    y, _ = forward(params, C)
    return scale(normA, n, r) * y, C, K
