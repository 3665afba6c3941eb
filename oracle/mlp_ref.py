"""Plain FP64 reference of the small MLP that proposes annealing protocols.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): the tests use it to check the
GPU forward / backward / Adam kernels; the product never imports it.

Network: x -> a1 = tanh(W1 x + b1) -> a2 = tanh(W2 a1 + b2) -> y = W3 a2 + b3.
Parameter vector layout: W1[H][I], b1[H], W2[H][H], b2[H], W3[O][H], b3[O].
Loss used by the learner: L = sum_b w_b sum_o (y_bo - t_bo)^2 / B.
"""
import numpy as np


def n_params(I, H, O):
    return H * I + H + H * H + H + O * H + O


def unpack(p, I, H, O):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * I].reshape(H, I); o += H * I
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + O * H].reshape(O, H); o += O * H
    b3 = p[o:o + O]
    return W1, b1, W2, b2, W3, b3


def forward(p, I, H, O, x):
    W1, b1, W2, b2, W3, b3 = unpack(p, I, H, O)
    x = np.asarray(x, dtype=np.float64)
    a1 = np.tanh(x @ W1.T + b1)
    a2 = np.tanh(a1 @ W2.T + b2)
    y = a2 @ W3.T + b3
    return y, (a1, a2)


def backward(p, I, H, O, x, acts, dy):
    """Gradient of sum_b <dy_b, y_b> with respect to the parameters (chain rule)."""
    W1, b1, W2, b2, W3, b3 = unpack(p, I, H, O)
    x = np.asarray(x, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    a1, a2 = acts
    dW3 = dy.T @ a2
    db3 = dy.sum(axis=0)
    d2 = (dy @ W3) * (1.0 - a2 ** 2)
    dW2 = d2.T @ a1
    db2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1.0 - a1 ** 2)
    dW1 = d1.T @ x
    db1 = d1.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])


def mse_grad(y, t, w):
    """L = sum_b w_b sum_o (y - t)^2 / B and dL/dy."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    B = y.shape[0]
    r = y - t
    return float(np.sum(w[:, None] * r * r) / B), 2.0 * w[:, None] * r / B


def adam(p, g, m, v, lr, b1, b2, eps, t):
    """One Adam step (Kingma & Ba 2015) with bias correction; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
