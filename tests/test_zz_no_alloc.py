"""hsg_sweep_static (the sweep entry point for callers that cannot allocate) against
hsg_sweep, through the C ABI: bit-for-bit equal spins, counters and energies on two
consecutive calls, the second with a smaller ensemble (the library's device array
keeps the first call's sums; nothing may depend on them), on the streaming path
(whose per-tile sums use that array) and on the LDS-resident path; sizes beyond the
array are refused before anything runs."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1006_4247_amd as hsg
from paper_1006_4247_amd import _abi

pytestmark = pytest.mark.gpu


def _pair(L, S, C, R, seed, prec="fp32"):
    out = []
    for _ in range(2):
        e = hsg.Ensemble(L, S, C, hsg.geometric_betas(1.0, 8.0, R), seed, precision=prec)
        e.init_couplings()
        e.init_spins()
        out.append(e)
    torch.cuda.synchronize()
    return out


def _static(e, n_sweeps, n_hb, n_or, scratch=True):
    d = _abi.HsgEnsemble.from_buffer_copy(e.desc)
    if not scratch:
        d.scratch = None
    return _abi.lib().hsg_sweep_static(ctypes.byref(d), 1, n_sweeps, n_hb, n_or, e._stream())


def _same(a, b):
    torch.cuda.synchronize()
    assert torch.equal(a.spins, b.spins)
    assert torch.equal(a.sweep_ctr, b.sweep_ctr)
    assert torch.equal(a.energy, b.energy)


@pytest.mark.parametrize("shapes", [
    [(24, 4, 2, 6, "fp32"), (20, 1, 2, 3, "fp32")],   # streaming, then a smaller streaming ensemble
    [(32, 2, 2, 8, "fp64"), (18, 1, 1, 2, "fp64")],
    [(16, 4, 2, 6, "fp32"), (8, 2, 2, 4, "fp32")],    # LDS-resident (no device array needed)
])
def test_static_sweep_equals_sweep_twice(shapes):
    for k, (L, S, C, R, prec) in enumerate(shapes):
        a, b = _pair(L, S, C, R, 0x5A7 + k, prec)
        a.sweep(2, 1, 3)
        _abi.check(_static(b, 2, 1, 3, scratch=False))
        _same(a, b)
        a.sweep(1, 0, 2)
        _abi.check(_static(b, 1, 0, 2, scratch=False))
        _same(a, b)
        b.check()


def test_static_sweep_refuses_sizes_beyond_its_array():
    """640 slots at L = 64 need 640 x 1024 per-tile sums, beyond the 2^19 doubles of the
    library's array: refused during validation, before any device work (the descriptor's
    pointers are never touched)."""
    d = _abi.HsgEnsemble()
    d.L, d.n_samples, d.n_chains, d.n_temps, d.precision = 64, 16, 2, 20, _abi.HSG_FP32
    for name in ["spins", "couplings", "betas", "temp_of_slot", "slot_of_temp", "energy", "sweep_ctr",
                 "swap_ctr", "swap_stats", "rt_state", "rt_trips", "guard"]:
        setattr(d, name, 4096)
    code = _abi.lib().hsg_sweep_static(ctypes.byref(d), 1, 1, 1, 3, None)
    assert code == _abi.HSG_ERR_INVALID
    assert b"device array" in _abi.lib().hsg_last_error()
    d.n_samples = 1  # 40 slots fit: validation passes (n_sweeps = 0 enqueues nothing)
    assert _abi.lib().hsg_sweep_static(ctypes.byref(d), 1, 0, 1, 3, None) == _abi.HSG_OK
