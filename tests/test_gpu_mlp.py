"""GPU MLP kernels (forward, squared-error gradient, backward, Adam) against the FP64
reference oracle/mlp_ref.py on the same parameters and inputs (FP32 arithmetic on
the GPU: relative tolerances derived from ~1e-7 rounding per operation times the
depth and fan-in of the network)."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref
from paper_1006_4247_amd import schedule

pytestmark = pytest.mark.gpu


def _setup(I, H, O, B, seed):
    r = np.random.default_rng(seed)
    net = schedule.MLP(I, H, O, seed=seed, max_batch=B)
    p = net.params.cpu().numpy().astype(np.float64)
    p[-O:] = r.standard_normal(O) * 0.1  # nonzero output bias
    net.params.copy_(torch.from_numpy(p.astype(np.float32)))
    p = net.params.cpu().numpy().astype(np.float64)
    x = r.standard_normal((B, I)).astype(np.float32)
    t = r.standard_normal((B, O)).astype(np.float32)
    w = r.uniform(0.5, 2.0, B).astype(np.float32)
    return net, p, x, t, w


@pytest.mark.parametrize("I,H,O,B", [(7, 64, 1, 300), (5, 16, 3, 1), (3, 256, 2, 70)])
def test_forward_backward_match_reference(I, H, O, B):
    net, p, x, t, w = _setup(I, H, O, B, I + H)
    xd, td, wd = (torch.from_numpy(a).cuda() for a in (x, t, w))
    net.loss_and_grad(xd, td, wd)
    torch.cuda.synchronize()
    y_ref, acts = mlp_ref.forward(p, I, H, O, x.astype(np.float64))
    loss_ref, dy_ref = mlp_ref.mse_grad(y_ref, t, w)
    g_ref = mlp_ref.backward(p, I, H, O, x.astype(np.float64), acts, dy_ref)
    y = net.y[:B].cpu().numpy()
    assert np.max(np.abs(y - y_ref)) <= 2e-5 * max(1.0, np.abs(y_ref).max())
    assert abs(net.loss.item() - loss_ref) <= 1e-5 * max(1.0, loss_ref)
    g = net.grad.cpu().numpy()
    scale = max(1e-3, np.abs(g_ref).max())
    assert np.max(np.abs(g - g_ref)) <= 2e-5 * scale * max(1.0, np.sqrt(B)), np.max(np.abs(g - g_ref)) / scale


def test_adam_matches_reference():
    I, H, O, B = 7, 32, 1, 50
    net, p, x, t, w = _setup(I, H, O, B, 3)
    xd, td, wd = (torch.from_numpy(a).cuda() for a in (x, t, w))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    pr = p.copy()
    for step in range(1, 6):
        net.loss_and_grad(xd, td, wd)
        g = net.grad.cpu().numpy().astype(np.float64)
        pr, m, v = mlp_ref.adam(net.params.cpu().numpy().astype(np.float64), g, m, v, 1e-2, 0.9, 0.999, 1e-8, step)
        net.adam_step(1e-2, 0.9, 0.999, 1e-8)
        assert np.max(np.abs(net.params.cpu().numpy() - pr)) <= 1e-6


def test_training_fits_a_smooth_function():
    r = np.random.default_rng(4)
    x = r.uniform(-1, 1, (2000, 3)).astype(np.float32)
    y = (np.sin(2 * x[:, :1]) + x[:, 1:2] ** 2 - 0.5 * x[:, 2:3]).astype(np.float32)
    net, loss = schedule.train(x, y[:, 0], None, H=32, steps=1500, lr=1e-2)
    var = float(np.var(y))
    assert loss < 0.02 * var, (loss, var)
