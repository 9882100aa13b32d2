"""Learned Davidson preconditioner: FP64 reference of the features, the network, its loss, gradient
and Adam update, and of the training pairs. Test infrastructure (the oracle): only tests and
benchmarks import it; the library never does.

The paper's Davidson solver uses the diagonal preconditioner (Sections 2.1, 2.2.1). The learned
preconditioner multiplies the diagonal correction t = r / (theta - D) coefficient by coefficient by
(1 + m), where m is the output of one small MLP shared by all psi coefficients:

    h1 = relu(x W1 + b1)  (16 -> 256),   h2 = relu(h1 W2 + b2)  (256 -> 256),   m = h2 . w3 + b3.

A network with w3 = b3 = 0 is exactly the diagonal preconditioner. Parameters are one flat vector
[W1 (16 x 256, row = input), b1, W2 (256 x 256, row = input), b2, w3, b3].

Training pairs. Let V (orthonormal columns) be the subspace that an iteration's correction t is
about to be orthogonalized against and psi the converged eigenvector of the same solve. The ideal
correction is the part of psi outside span(V), P psi = psi - V V^T psi: appending it makes the
subspace contain psi, so the next Rayleigh-Ritz step is exact (for V = [u] it is the direction of
psi / <u, psi> - u). Davidson only uses the direction of t, so both sides are brought to unit RMS
and the target to the sign that points along t: a = t_i sqrt(n) / ||t||,
b = sign(<t, P psi>) (P psi)_i sqrt(n) / ||P psi||. Minibatch loss (1/B) sum w (a (1 + m) - b)^2;
for the diagonal preconditioner (m = 0) its mean over an iteration is 2 (1 - cos(t, P psi)), and a
network cannot lower it by shrinking the correction. Iterations with ||P psi|| < 1e-7 give no rows.

BF16 mode (bf16=True) is the network as the matrix-core kernels evaluate it: inputs, W1, W2 and the
first hidden layer are rounded to bfloat16 (round to nearest even, from float32) before they enter a
product, and the relu masks are taken on those products (a decision taken in floating point is
taken at the kernel's precision on both sides). Its gradient treats the rounding as the identity
(straight-through): dW2 uses the unrounded h1, dW1 the unrounded inputs, and the backward pass
through layer 2 uses the rounded W2.

Parity pins: finite differences (gradient), a hand-built network (forward), Adam's first step in
closed form, the exactness of the correction on a small symmetric matrix, hand-computed features,
bfloat16 rounding against torch's CPU conversion, and BF16 mode equal to FP64 mode on a network whose
values are all exactly representable in bfloat16.
"""
import numpy as np

N_IN = 16
N_HID = 256
OFF_B1 = N_IN * N_HID
OFF_W2 = OFF_B1 + N_HID
OFF_B2 = OFF_W2 + N_HID * N_HID
OFF_W3 = OFF_B2 + N_HID
OFF_B3 = OFF_W3 + N_HID
N_PARAMS = OFF_B3 + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    W1 = p[:OFF_B1].reshape(N_IN, N_HID)
    b1 = p[OFF_B1:OFF_W2]
    W2 = p[OFF_W2:OFF_B2].reshape(N_HID, N_HID)
    b2 = p[OFF_B2:OFF_W3]
    w3 = p[OFF_W3:OFF_B3]
    b3 = p[OFF_B3]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def bf16_round(x):
    """Round to bfloat16 (nearest, ties to even) via float32, returned as float64 (finite inputs)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def relu(z):
    return np.maximum(z, 0.0)


def relu_grad(z):
    """Derivative of relu, taken as 0 at z = 0."""
    return (z > 0.0).astype(np.float64)


def forward(p, X, bf16=False):
    """Network output m (n,) for feature rows X (n x 16), and the intermediates."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    q = bf16_round if bf16 else (lambda a: a)
    z1 = q(X) @ q(W1) + b1
    h1 = relu(z1)
    z2 = q(h1) @ q(W2) + b2
    h2 = relu(z2)
    m = h2 @ w3 + b3
    return m, (z1, h1, z2, h2)


def loss(p, X, A, bf16=False):
    """(1/B) sum w (a (1 + m) - b)^2 over the rows; A rows are (a, b, w)."""
    A = np.asarray(A, dtype=np.float64)
    m, _ = forward(p, X, bf16)
    e = A[:, 0] * (1.0 + m) - A[:, 1]
    return float(np.mean(A[:, 2] * e * e))


def grad(p, X, A, bf16=False):
    """Gradient of loss() with respect to the flat parameter vector (backpropagation)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    n = X.shape[0]
    m, (z1, h1, z2, h2) = forward(p, X, bf16)
    e = A[:, 0] * (1.0 + m) - A[:, 1]
    g = 2.0 * A[:, 2] * A[:, 0] * e / n          # d loss / d m
    dw3 = h2.T @ g
    db3 = g.sum()
    d2 = np.outer(g, w3) * relu_grad(z2)         # d loss / d z2
    dW2 = h1.T @ d2
    db2 = d2.sum(axis=0)
    W2b = bf16_round(W2) if bf16 else W2
    d1 = (d2 @ W2b.T) * relu_grad(z1)            # d loss / d z1
    dW1 = X.T @ d1
    db1 = d1.sum(axis=0)
    return pack(dW1, db1, dW2, db2, dw3, db3)


def adam(p, g, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015, bias-corrected moments); returns (p, m1, m2). step >= 1."""
    m1 = beta1 * m1 + (1.0 - beta1) * g
    m2 = beta2 * m2 + (1.0 - beta2) * g * g
    mh = m1 / (1.0 - beta1 ** step)
    vh = m2 / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, m2


def diag_correction(r, d, theta):
    """Davidson's diagonal correction r / (theta - D), |theta - D| floored at 1e-8 with its sign
    (a zero difference counts as positive)."""
    den = theta - np.asarray(d, dtype=np.float64)
    small = np.abs(den) < 1e-8
    den = np.where(small, np.where(den < 0.0, -1e-8, 1e-8), den)
    return np.asarray(r, dtype=np.float64) / den


def _inv_rms(x):
    nrm = np.linalg.norm(x)
    return np.sqrt(x.size) / nrm if nrm > 0.0 else 0.0


def features(blocks, r, u, d, theta):
    """Feature rows (n x 16, FP64) of every psi coefficient.

    blocks: iterable of (offset, m_a, m_d, b, c) for the psi blocks (a, b, c, d) of the layout.
    Per coefficient i of block (b, c) with s_x = sqrt(n) / ||x|| (0 for x = 0):
      asinh(r_i s_r), asinh(t_i s_t), asinh(u_i s_u), asinh((D_i - theta) s_D), one-hot b, one-hot c,
      asinh(rms_block(r) s_r), asinh(rms_block(u) s_u), ln(m_a) / 8, ln(m_d) / 8,
    with t = diag_correction(r, D, theta) and rms_block the root mean square over the block.
    """
    r = np.asarray(r, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    t = diag_correction(r, d, theta)
    sr, st, su, sd = _inv_rms(r), _inv_rms(t), _inv_rms(u), _inv_rms(d - theta)
    F = np.zeros((r.size, N_IN))
    F[:, 0] = np.arcsinh(r * sr)
    F[:, 1] = np.arcsinh(t * st)
    F[:, 2] = np.arcsinh(u * su)
    F[:, 3] = np.arcsinh((d - theta) * sd)
    for off, ma, md, b, c in blocks:
        sl = slice(off, off + ma * md)
        F[sl, 4 + b] = 1.0
        F[sl, 8 + c] = 1.0
        F[sl, 12] = np.arcsinh(np.sqrt(np.mean(r[sl] ** 2)) * sr)
        F[sl, 13] = np.arcsinh(np.sqrt(np.mean(u[sl] ** 2)) * su)
        F[sl, 14] = np.log(ma) / 8.0
        F[sl, 15] = np.log(md) / 8.0
    return F


def apply(p, X, t):
    """Learned correction t (1 + m)."""
    m, _ = forward(p, X)
    return np.asarray(t, dtype=np.float64) * (1.0 + m)


def exact_correction(u, psi):
    """psi / <u, psi> - u: the correction that makes span{u, t} contain psi."""
    return psi / np.dot(u, psi) - u


def target(V, psi):
    """Part of psi outside span(V) (V: n x k, orthonormal columns)."""
    V = np.asarray(V, dtype=np.float64).reshape(len(psi), -1)
    return psi - V @ (V.T @ psi)


def pairs(t, V, psi, idx):
    """Training rows (a, b, w) at coefficients idx for one iteration, or None when ||P psi|| < 1e-7."""
    t = np.asarray(t, dtype=np.float64)
    v = target(V, psi)
    dd = np.dot(v, v)
    if np.sqrt(dd) < 1e-7:
        return None
    sa = np.sqrt(t.size / np.dot(t, t))
    sb = np.sqrt(t.size / dd) * (-1.0 if np.dot(t, v) < 0.0 else 1.0)
    idx = np.asarray(idx)
    return np.stack([sa * t[idx], sb * v[idx], np.ones(idx.size)], axis=1)
