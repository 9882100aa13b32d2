"""Pins of the learned-preconditioner oracle (oracle/mlp.py) against facts that do not come from it:
central finite differences, a hand-built network, Adam's first step in closed form, the exactness of
the correction on a small symmetric matrix, hand-computed features, and a planted mistake."""
import numpy as np
import pytest

from oracle import mlp
from oracle.davidson import davidson


def _random_net(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (mlp.N_IN, mlp.N_HID)) * np.sqrt(6 / mlp.N_IN) * scale
    W2 = rng.uniform(-1, 1, (mlp.N_HID, mlp.N_HID)) * np.sqrt(6 / mlp.N_HID) * scale
    b1 = rng.normal(0, 0.1, mlp.N_HID)
    b2 = rng.normal(0, 0.1, mlp.N_HID)
    w3 = rng.normal(0, 0.05, mlp.N_HID)
    return mlp.pack(W1, b1, W2, b2, w3, 0.03)


def _random_batch(seed, n=24):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (n, mlp.N_IN))
    A = np.stack([rng.normal(0, 1, n), rng.normal(0, 1, n), rng.uniform(0.5, 1.5, n)], axis=1)
    return X, A


def test_gradient_matches_central_differences():
    p = _random_net(0)
    X, A = _random_batch(1)
    g = mlp.grad(p, X, A)
    rng = np.random.default_rng(2)
    # every parameter group: a few entries of W1, b1, W2, b2, w3 and b3
    picks = np.concatenate([rng.integers(0, mlp.OFF_B1, 6), rng.integers(mlp.OFF_B1, mlp.OFF_W2, 4),
                            rng.integers(mlp.OFF_W2, mlp.OFF_B2, 8), rng.integers(mlp.OFF_B2, mlp.OFF_W3, 4),
                            rng.integers(mlp.OFF_W3, mlp.OFF_B3, 4), [mlp.OFF_B3]])
    h = 1e-6
    for k in picks:
        e = np.zeros(mlp.N_PARAMS)
        e[k] = h
        fd = (mlp.loss(p + e, X, A) - mlp.loss(p - e, X, A)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_gradient_directional_derivative():
    """<grad, v> equals the derivative of the loss along a random direction v (all parameters)."""
    p = _random_net(3)
    X, A = _random_batch(4)
    v = np.random.default_rng(5).normal(0, 1, mlp.N_PARAMS)
    h = 1e-6
    fd = (mlp.loss(p + h * v, X, A) - mlp.loss(p - h * v, X, A)) / (2 * h)
    assert abs(fd - np.dot(mlp.grad(p, X, A), v)) <= 1e-6 * abs(fd)


def test_planted_missing_relu_mask_is_caught(monkeypatch):
    """Backpropagating through relu without its 0/1 mask fails the finite-difference pin."""
    p = _random_net(0)
    X, A = _random_batch(1)
    monkeypatch.setattr(mlp, "relu_grad", lambda z: np.ones_like(z))
    g = mlp.grad(p, X, A)
    monkeypatch.undo()
    v = np.random.default_rng(5).normal(0, 1, mlp.N_PARAMS)
    h = 1e-6
    fd = (mlp.loss(p + h * v, X, A) - mlp.loss(p - h * v, X, A)) / (2 * h)
    assert abs(fd - np.dot(g, v)) > 1e-3 * abs(fd)


def test_forward_hand_built_network():
    """x0 -> unit 0 (weight 2, bias -0.5) -> unit 3 of layer 2 (weight 3, bias 0.25) -> output (0.5, 0.1)."""
    W1 = np.zeros((mlp.N_IN, mlp.N_HID))
    W2 = np.zeros((mlp.N_HID, mlp.N_HID))
    b1 = np.zeros(mlp.N_HID)
    b2 = np.zeros(mlp.N_HID)
    w3 = np.zeros(mlp.N_HID)
    W1[0, 0], b1[0] = 2.0, -0.5
    W2[0, 3], b2[3] = 3.0, 0.25
    w3[3] = 0.5
    p = mlp.pack(W1, b1, W2, b2, w3, 0.1)
    X = np.zeros((3, mlp.N_IN))
    X[:, 0] = [1.0, 0.1, -2.0]
    m, _ = mlp.forward(p, X)
    # row 0: h1 = 1.5, h2 = 4.75, m = 2.475; row 1: h1 = 0, h2 = 0.25, m = 0.225; row 2 likewise
    np.testing.assert_allclose(m, [0.5 * (3 * 1.5 + 0.25) + 0.1, 0.5 * 0.25 + 0.1, 0.5 * 0.25 + 0.1], rtol=0, atol=1e-15)


def test_zero_output_layer_is_the_diagonal_preconditioner():
    p = _random_net(7)
    p[mlp.OFF_W3:] = 0.0
    X, _ = _random_batch(8, n=50)
    t = np.random.default_rng(9).normal(0, 1, 50)
    assert np.array_equal(mlp.apply(p, X, t), t)
    A = np.stack([t, 0.7 * t, np.ones(50)], axis=1)
    assert mlp.loss(p, X, A) == pytest.approx(np.mean((0.3 * t) ** 2), rel=1e-14)


def test_adam_first_step_closed_form():
    """With zero moments, Adam's first bias-corrected step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(11)
    p = rng.normal(0, 1, 40)
    g = rng.normal(0, 1, 40)
    z = np.zeros(40)
    p1, m1, m2 = mlp.adam(p, g, z, z, 1, 1e-3)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-13)
    np.testing.assert_allclose(m2, 0.001 * g * g, rtol=1e-13)


def test_exact_correction_converges_in_one_step():
    """Rayleigh-Ritz on span{u, delta} gives the lowest eigenpair exactly, and delta is orthogonal to u."""
    rng = np.random.default_rng(13)
    n = 60
    H = rng.normal(0, 1, (n, n))
    H = 0.5 * (H + H.T) + np.diag(np.linspace(0, 8, n))
    evals, evecs = np.linalg.eigh(H)
    psi = evecs[:, 0]
    u = psi + 0.3 * rng.normal(0, 1, n) / np.sqrt(n)
    u /= np.linalg.norm(u)
    delta = mlp.exact_correction(u, psi)
    assert abs(np.dot(u, delta)) < 1e-13
    Q, _ = np.linalg.qr(np.stack([u, delta], axis=1))
    assert np.linalg.eigvalsh(Q.T @ H @ Q)[0] == pytest.approx(evals[0], abs=1e-12)
    # the same through the oracle Davidson: a "preconditioner" that returns delta converges in one step
    res = davidson(lambda x: H @ x, np.diag(H).copy(), u, tol=1e-10, max_iter=5,
                   precond=lambda r, theta, uu: mlp.exact_correction(uu, psi))
    assert res["converged"] and res["iters"] <= 2 and res["energy"] == pytest.approx(evals[0], abs=1e-10)


def test_pairs_unit_rms_sign_aligned():
    rng = np.random.default_rng(17)
    n = 40
    t = rng.normal(0, 1, n)
    psi = rng.normal(0, 1, n)
    psi /= np.linalg.norm(psi)
    u = psi + 0.2 * rng.normal(0, 1, n)
    u /= np.linalg.norm(u)
    A = mlp.pairs(t, u, psi, np.arange(n))
    a, b = A[:, 0], A[:, 1]
    delta = mlp.exact_correction(u, psi)
    # for V = [u]: a = t and b = +-delta at unit RMS, b pointing along a; diagonal loss 2 (1 - cos(t, delta))
    assert np.dot(a, a) == pytest.approx(n, rel=1e-12) and np.dot(b, b) == pytest.approx(n, rel=1e-12)
    assert np.allclose(b / np.linalg.norm(b), np.sign(np.dot(t, delta)) * delta / np.linalg.norm(delta))
    assert np.dot(a, b) >= 0
    cos = abs(np.dot(t, delta)) / np.linalg.norm(t) / np.linalg.norm(delta)
    assert mlp.loss(np.zeros(mlp.N_PARAMS), np.zeros((n, mlp.N_IN)), A) == pytest.approx(2 * (1 - cos), rel=1e-12)
    assert mlp.pairs(t, psi, psi, np.arange(n)) is None    # converged iteration: no rows


def test_target_completes_the_subspace():
    """Appending the target to V makes Rayleigh-Ritz exact, and the target is orthogonal to V."""
    rng = np.random.default_rng(29)
    n, k = 50, 6
    H = rng.normal(0, 1, (n, n))
    H = 0.5 * (H + H.T) + np.diag(np.linspace(0, 10, n))
    evals, evecs = np.linalg.eigh(H)
    V, _ = np.linalg.qr(rng.normal(0, 1, (n, k)))
    v = mlp.target(V, evecs[:, 0])
    assert np.abs(V.T @ v).max() < 1e-13
    Q, _ = np.linalg.qr(np.column_stack([V, v]))
    assert np.linalg.eigvalsh(Q.T @ H @ Q)[0] == pytest.approx(evals[0], abs=1e-12)
    # one vector short of it (V alone) is not exact
    assert np.linalg.eigvalsh(V.T @ H @ V)[0] > evals[0] + 1e-3


def test_features_hand_computed():
    # two blocks: (off 0, 2 x 3, b=1, c=2) and (off 6, 1 x 2, b=3, c=0); n = 8
    blocks = [(0, 2, 3, 1, 2), (6, 1, 2, 3, 0)]
    r = np.array([1.0, -1.0, 2.0, 0.0, 0.5, -0.5, 3.0, 1.0])
    u = np.array([0.5, 0.5, 0.5, 0.5, 0.0, 0.0, 0.0, 0.0])
    d = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0, -1.0, 0.0])
    theta = 0.0
    F = mlp.features(blocks, r, u, d, theta)
    sr = np.sqrt(8) / np.sqrt(1 + 1 + 4 + 0 + 0.25 + 0.25 + 9 + 1)
    su = np.sqrt(8) / 1.0
    assert F[2, 0] == pytest.approx(np.arcsinh(2.0 * sr), rel=1e-15)
    t = np.array([-1.0, 0.5, -2 / 3, 0.0, -0.1, 0.5 / 6, 3.0, 1.0 / 1e-8])   # r / (0 - d), floor at d = 0
    st = np.sqrt(8) / np.linalg.norm(t)
    np.testing.assert_allclose(F[:, 1], np.arcsinh(t * st), rtol=1e-14)
    assert F[0, 2] == pytest.approx(np.arcsinh(0.5 * su), rel=1e-15) and F[5, 2] == 0.0
    sd = np.sqrt(8) / np.sqrt(1 + 4 + 9 + 16 + 25 + 36 + 1 + 0)
    assert F[6, 3] == pytest.approx(np.arcsinh(-1.0 * sd), rel=1e-15)
    assert list(F[0, 4:12]) == [0, 1, 0, 0, 0, 0, 1, 0] and list(F[7, 4:12]) == [0, 0, 0, 1, 1, 0, 0, 0]
    rms_r0 = np.sqrt((1 + 1 + 4 + 0 + 0.25 + 0.25) / 6)
    assert F[3, 12] == pytest.approx(np.arcsinh(rms_r0 * sr), rel=1e-15)
    assert F[7, 13] == 0.0 and F[1, 13] == pytest.approx(np.arcsinh(np.sqrt(1 / 6) * su), rel=1e-15)
    assert F[4, 14] == pytest.approx(np.log(2) / 8) and F[4, 15] == pytest.approx(np.log(3) / 8)
    assert F[6, 14] == 0.0 and F[6, 15] == pytest.approx(np.log(2) / 8)


def test_bf16_round_matches_torch_cpu_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(19)
    x = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1e4, 500), rng.normal(0, 1e-5, 500),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, -(1.0 + 2.0 ** -8)]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)
    # ties go to the even neighbour: 1 + 2^-8 -> 1, 1 + 3*2^-8 -> 1 + 2^-6
    assert mlp.bf16_round(1.0 + 2.0 ** -8) == 1.0 and mlp.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_bf16_mode_equals_fp64_on_representable_network():
    """With weights, biases and inputs on coarse grids, every product in the network is exact in
    bfloat16, so BF16 mode must agree with FP64 mode exactly (forward and gradient)."""
    rng = np.random.default_rng(23)
    W1 = rng.integers(-2, 3, (mlp.N_IN, mlp.N_HID)) * 0.5
    W2 = rng.integers(-2, 3, (mlp.N_HID, mlp.N_HID)) * 0.0625
    b1 = rng.integers(-4, 5, mlp.N_HID) * 0.25
    b2 = rng.integers(-4, 5, mlp.N_HID) * 0.25
    w3 = rng.normal(0, 0.1, mlp.N_HID)
    p = mlp.pack(W1, b1, W2, b2, w3, 0.5)
    X = rng.integers(-2, 3, (40, mlp.N_IN)).astype(np.float64)
    A = np.stack([rng.normal(0, 1, 40), rng.normal(0, 1, 40), np.ones(40)], axis=1)
    _, (z1, h1, _, _) = mlp.forward(p, X)
    assert np.array_equal(mlp.bf16_round(h1), h1)          # the premise: h1 is representable
    np.testing.assert_array_equal(mlp.forward(p, X, bf16=True)[0], mlp.forward(p, X)[0])
    np.testing.assert_array_equal(mlp.grad(p, X, A, bf16=True), mlp.grad(p, X, A))
    # and a non-representable network does differ (the mode is not a no-op)
    p2 = p + rng.normal(0, 1e-3, p.size)
    assert np.abs(mlp.forward(p2, X, bf16=True)[0] - mlp.forward(p2, X)[0]).max() > 0
