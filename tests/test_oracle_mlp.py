"""Pins of the FP64 MLP reference: gradients against central finite differences of the
loss (the function, not its derivative, is what the network defines), closed forms
(zero hidden weights give constant activations; a one-hidden-unit chain), and Adam's
first step (bias-corrected: it moves every parameter by lr * sign(g))."""
import numpy as np

from oracle import mlp_ref


def _setup(I=5, H=7, O=3, B=11, seed=0):
    r = np.random.default_rng(seed)
    p = r.standard_normal(mlp_ref.n_params(I, H, O)) * 0.5
    x = r.standard_normal((B, I))
    t = r.standard_normal((B, O))
    w = r.uniform(0.5, 2.0, B)
    return p, x, t, w


def _loss(p, x, t, w, I, H, O):
    y, _ = mlp_ref.forward(p, I, H, O, x)
    return mlp_ref.mse_grad(y, t, w)[0]


def test_gradient_matches_finite_differences():
    I, H, O = 5, 7, 3
    p, x, t, w = _setup(I, H, O)
    y, acts = mlp_ref.forward(p, I, H, O, x)
    _, dy = mlp_ref.mse_grad(y, t, w)
    g = mlp_ref.backward(p, I, H, O, x, acts, dy)
    h = 1e-6
    for k in range(len(p)):
        e = np.zeros_like(p)
        e[k] = h
        fd = (_loss(p + e, x, t, w, I, H, O) - _loss(p - e, x, t, w, I, H, O)) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(fd)), (k, fd, g[k])


def test_closed_forms():
    I, H, O = 3, 4, 2
    p = np.zeros(mlp_ref.n_params(I, H, O))
    W1, b1, W2, b2, W3, b3 = mlp_ref.unpack(p, I, H, O)
    x = np.random.default_rng(1).standard_normal((6, I))
    # all zero but the output bias: constant output
    p[-O:] = [0.25, -1.5]
    y, (a1, a2) = mlp_ref.forward(p, I, H, O, x)
    assert np.allclose(y, [0.25, -1.5]) and np.all(a1 == 0) and np.all(a2 == 0)
    # one active path: y0 = v * tanh(u * tanh(w * x0))
    I, H, O = 1, 1, 1
    w_, u_, v_ = 0.7, -1.3, 2.1
    p = np.array([w_, 0.0, u_, 0.0, v_, 0.0])
    xs = np.linspace(-2, 2, 9)[:, None]
    y, _ = mlp_ref.forward(p, I, H, O, xs)
    assert np.allclose(y[:, 0], v_ * np.tanh(u_ * np.tanh(w_ * xs[:, 0])), atol=1e-15)


def test_adam_first_step_moves_by_lr_sign():
    r = np.random.default_rng(2)
    p = r.standard_normal(20)
    g = r.standard_normal(20)
    p1, m, v = mlp_ref.adam(p, g, np.zeros(20), np.zeros(20), 0.01, 0.9, 0.999, 1e-12, 1)
    assert np.allclose(p - p1, 0.01 * np.sign(g), atol=1e-9)
