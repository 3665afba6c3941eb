"""One persistent launch over an uneven batch (hsg_sweep_tuned with path 5): several
size classes in one kernel, L = 12..16 swept in LDS from a work counter, the others
in tiles half-sweep by half-sweep behind the barrier of their own part of the grid.
Against the same ensembles swept class by class with the default kernels: spins and
counters bit for bit, energies up to the order of their FP64 sums, no guard bit; at
several sweep compositions, sweeps per call and partition sizes."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1006_4247_amd as hsg
from paper_1006_4247_amd import _abi

pytestmark = pytest.mark.gpu


def _batch(shapes, seed, prec):
    out = []
    sb = cb = qb = 0
    for (L, S, R) in shapes:
        e = hsg.Ensemble(L, S, 2, hsg.geometric_betas(1.0, 8.0, R), seed, precision=prec,
                         sample_base=sb, chain_base=cb, slot_base=qb)
        e.init_couplings()
        e.init_spins()
        sb, cb, qb = sb + S, cb + 2 * S, qb + 2 * S * R
        out.append(e)
    torch.cuda.synchronize()
    return out


def _batch_sweep(ens, n, n_hb, n_or, g_str=0):
    descs = (_abi.HsgEnsemble * len(ens))(*[e.desc for e in ens])
    t = _abi.HsgTuning(5, int(g_str), 0, 0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _abi.check(_abi.lib().hsg_sweep_tuned(descs, len(ens), n, n_hb, n_or, ctypes.byref(t), stream))


SHAPES = [(8, 8, 4), (12, 4, 6), (16, 4, 4), (24, 2, 4), (32, 1, 4)]


@pytest.mark.parametrize("prec,shapes", [("fp32", SHAPES), ("fp64", [(12, 2, 4), (16, 2, 3), (20, 1, 4), (6, 4, 4)])])
@pytest.mark.parametrize("n,n_hb,n_or,g_str", [(1, 1, 3, 0), (2, 1, 3, 0), (1, 0, 2, 0), (1, 2, 1, 16), (3, 1, 3, 8)])
def test_batch_launch_equals_class_by_class(prec, shapes, n, n_hb, n_or, g_str):
    a, b = _batch(shapes, 0xBA7C, prec), _batch(shapes, 0xBA7C, prec)
    for _ in range(2):
        for e in a:
            e.sweep(n, n_hb, n_or)
        _batch_sweep(b, n, n_hb, n_or, g_str)
    torch.cuda.synchronize()
    for k, (x, y) in enumerate(zip(a, b)):
        assert torch.equal(x.spins, y.spins), (k, x.L)
        assert torch.equal(x.sweep_ctr, y.sweep_ctr), (k, x.L)
        ex, ey = x.energy.cpu().numpy(), y.energy.cpu().numpy()
        assert np.allclose(ex, ey, rtol=1e-12, atol=1e-9 * x.N), (k, x.L, np.abs(ex - ey).max())
        assert int(y.guard.item()) == 0, (k, int(y.guard.item()))
    for e in a + b:
        e.check()


def test_batch_launch_refuses_what_it_does_not_cover():
    e = _batch([(16, 1, 2)], 1, "fp32") + _batch([(8, 1, 2)], 2, "fp64")
    descs = (_abi.HsgEnsemble * 2)(*[x.desc for x in e])
    t = _abi.HsgTuning(5, 0, 0, 0)
    assert _abi.lib().hsg_sweep_tuned(descs, 2, 1, 1, 3, ctypes.byref(t), None) == _abi.HSG_ERR_UNSUPPORTED
