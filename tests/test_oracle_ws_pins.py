"""Pins of the warm-start oracle (oracle/warmstart.py) against facts that do not depend
on it: finite differences, closed forms, planted separable structure, a library
assignment solver and torch's BF16 rounding."""
import numpy as np
import pytest

from oracle import warmstart as WS
from paper_2606_02887_amd import gen


def _separable(n, r, seed):
    """Rows of Y are convex combinations (row sums <= 0.9) of r anchor rows, plus the
    anchors themselves at known positions (Gillis & Vavasis' noiseless separable case)."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((r, r)) + 3 * np.eye(r)
    H = rng.random((n, r))
    H = 0.9 * H / H.sum(axis=1, keepdims=True) * rng.random((n, 1))
    pos = rng.choice(n, size=r, replace=False)
    H[pos] = np.eye(r)
    return H @ B, H, pos, B


def test_spa_recovers_planted_anchors():
    for seed in range(5):
        Y, H, pos, _ = _separable(300, 6, seed)
        K = WS.spa(Y, 6)
        assert sorted(K) == sorted(pos.tolist())


def test_coords_reproduce_planted_mixing():
    Y, H, pos, _ = _separable(200, 5, 11)
    K = WS.spa(Y, 5)
    C = WS.coords(Y, K)
    # C = Y Y_K^{-1} = H H_K^{-1}; H_K is a permutation (the anchors)
    assert np.max(np.abs(C - H @ np.linalg.inv(H[K]))) <= 1e-9
    assert np.allclose(C[K], np.eye(5), atol=1e-9)


def test_frame_undoes_sketch_mixing_for_exact_low_rank():
    """A = W W^T with W separable: Y = W (W^T Omega) and C = W W_K^{-1} for any Omega, up
    to the frame's scaling to rms(relu(C)) = 1."""
    rng = np.random.default_rng(5)
    n, r = 150, 4
    W = rng.random((n, r)) * 0.2
    pos = rng.choice(n, size=r, replace=False)
    W[pos] = np.eye(r) * 2.0
    A = W @ W.T
    for s in range(3):
        Om = gen.sketch_matrix(n, r, 100 + s)
        C, K, _ = WS.frame(A, Om)
        E = W @ np.linalg.inv(W[K])
        E /= np.sqrt(np.mean(np.maximum(E, 0.0) ** 2))
        assert np.max(np.abs(C - E)) <= 1e-7
        assert abs(np.sqrt(np.mean(np.maximum(C, 0.0) ** 2)) - 1.0) <= 1e-12


def _fd(fun, x, h=1e-6):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        xp = x.copy()
        xm = x.copy()
        xp[i] += h
        xm[i] -= h
        g[i] = (fun(xp) - fun(xm)) / (2 * h)
    return g


@pytest.mark.parametrize("mu", [0.0, 0.7])
def test_mlp_gradient_matches_finite_differences(mu):
    rng = np.random.default_rng(3)
    r, H, N = 4, 9, 13
    prm = {"M1": rng.standard_normal((H, r)), "b1": 0.1 * rng.standard_normal(H),
           "M2": rng.standard_normal((r, H)) * 0.3, "b2": rng.standard_normal(r) * 0.2}
    C = rng.standard_normal((N, r))
    T = rng.random((N, r))
    _, g = WS.loss_and_grad(prm, C, T, mu, quantize=False)
    for key in ("M1", "b1", "M2", "b2"):
        def f(val, key=key):
            q = dict(prm)
            q[key] = val
            y, _ = WS.forward(q, C, quantize=False)
            return WS.loss(y, T, mu)
        gfd = _fd(f, prm[key])
        assert np.max(np.abs(g[key] - gfd)) <= 1e-7 * max(1.0, np.max(np.abs(gfd))), key


def test_planted_gradient_mistake_is_caught():
    """A dropped output mask [o > 0] (a plausible slip) is visible to the FD check."""
    rng = np.random.default_rng(4)
    prm = {"M1": rng.standard_normal((5, 3)), "b1": np.zeros(5),
           "M2": rng.standard_normal((3, 5)), "b2": np.zeros(3)}
    C = rng.standard_normal((7, 3))
    T = rng.random((7, 3))
    y, (C_, a, h, o, M1, M2) = WS.forward(prm, C, quantize=False)
    assert (o < 0).any() and (o > 0).any()
    wrong = (2.0 * (y - T) / y.size).T @ h            # gM2 without the mask
    right = WS.loss_and_grad(prm, C, T, 0.0, quantize=False)[1]["M2"]
    assert np.max(np.abs(wrong - right)) > 1e-3


def test_residual_network_starts_at_the_frame():
    """With M2 = 0 and b2 = 0 the network is the frame's own start relu(c)."""
    rng = np.random.default_rng(8)
    r = 5
    prm = gen.mlp_init(r, 16, 3)
    assert not prm["M2"].any() and not prm["b2"].any()
    C = rng.standard_normal((40, r))
    y, _ = WS.forward(prm, C)
    assert np.array_equal(y, np.maximum(C, 0.0))


def test_targets_are_matched_and_unit_rms():
    rng = np.random.default_rng(12)
    C = rng.random((60, 4)) ** 3
    perm = rng.permutation(4)
    Ht = 7.0 * C[:, perm] + 1e-3 * rng.random((60, 4))
    T, p = WS.targets(C, Ht)
    assert np.array_equal(perm[p], np.arange(4))
    assert abs(np.sqrt(np.mean(T * T)) - 1.0) <= 1e-14
    assert np.allclose(T * np.sqrt(np.mean(Ht * Ht)), Ht[:, p], rtol=1e-14)


def test_adam_first_step_closed_form():
    """With m0 = v0 = 0 the bias-corrected first step is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = WS.adam_step(np.ones(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(th, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-6, 6, 5000),
                        [0.0, -0.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8)]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(WS.bf16_round(x), ref)


def test_match_columns_recovers_permutation():
    rng = np.random.default_rng(2)
    C = rng.random((80, 6)) ** 4
    perm = rng.permutation(6)
    Ht = C[:, perm] * rng.uniform(0.5, 2.0, 6) + 1e-3 * rng.random((80, 6))
    p = WS.match_columns(C, Ht)
    assert np.array_equal(Ht[:, p].argmax(axis=0), C.argmax(axis=0))
    assert np.array_equal(perm[p], np.arange(6))


def test_scale():
    # r orthogonal columns with entry RMS s have ||W W^T||_F = sqrt(r) n s^2 = ||A||_F
    n, r, normA = 100, 4, 7.0
    s = WS.scale(normA, n, r)
    W = np.zeros((n, r))
    for j in range(r):
        W[j * 25:(j + 1) * 25, j] = s * np.sqrt(n / 25)
    assert np.isclose(np.sqrt(np.mean(W * W)), s)
    assert np.isclose(np.linalg.norm(W @ W.T), normA)


def test_frame_start_scale_and_sign():
    """The frame-only start is nonnegative, zero exactly where the coordinate is negative,
    and its entry RMS is the scale s = (sqrt(r) ||A||_F / (n r))^(1/2) (closed form)."""
    rng = np.random.default_rng(77)
    n, r = 120, 5
    W = rng.random((n, r))
    A = W @ W.T
    Om = rng.standard_normal((n, r))
    nA = float(np.linalg.norm(A))
    W0, C, K = WS.frame_start(A, Om, nA)
    s = np.sqrt(np.sqrt(r) * nA / (n * r))
    assert (W0 >= 0).all()
    assert np.array_equal(W0 == 0, C <= 0)
    assert abs(np.sqrt(np.mean(W0 ** 2)) - s) <= 1e-13 * s
