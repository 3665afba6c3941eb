"""Host-side checks of the HIP library and its binding (no GPU needed): the
library loads and exports every entry point of include/hsgpt.h, the struct
mirror matches the header, argument validation rejects bad calls before any
launch, and the layout conversion agrees with the oracle's site indexing."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import hsgref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsgpt.h")


def _lib_or_skip():
    from paper_1006_4247_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libhsgpt.so not built: run __graft_entry__.build()")
    return _abi


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:hsg_status|int|const char\*|size_t)\s+(hsg_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for need in ["hsg_init_couplings", "hsg_init_spins", "hsg_sweep", "hsg_energy", "hsg_swap",
                 "hsg_anneal_swap", "hsg_measure", "hsg_sweep_measure", "hsg_check", "hsg_mlp_forward",
                 "hsg_mlp_backward", "hsg_mlp_adam"]:
        assert need in names


def test_library_exports_every_declared_symbol():
    _abi = _lib_or_skip()
    lib = ctypes.CDLL(_abi.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _abi.SIGNATURES, name


def test_struct_layout_matches_header():
    _abi = _lib_or_skip()
    # int32 x6, uint32 x4, uint64, 12 pointers, 2 pointers, 2 int32, 5 pointers
    expected = 6 * 4 + 4 * 4 + 8 + 12 * 8 + 2 * 8 + 2 * 4 + 5 * 8
    assert ctypes.sizeof(_abi.HsgEnsemble) == expected
    assert _abi.HsgEnsemble.spins.offset == 48
    assert ctypes.sizeof(_abi.HsgTuning) == 16


def test_abi_version_and_validation_without_gpu():
    _abi = _lib_or_skip()
    lib = _abi.lib()
    assert lib.hsg_abi_version() == 1
    d = _abi.HsgEnsemble()
    d.L, d.n_samples, d.n_chains, d.n_temps, d.precision = 5, 1, 1, 2, 1
    assert lib.hsg_scratch_bytes(ctypes.byref(d)) == 0  # odd L
    assert lib.hsg_sweep(ctypes.byref(d), 1, 1, 1, 3, None) == _abi.HSG_ERR_INVALID
    assert b"even" in lib.hsg_last_error()
    d.L = 8
    assert lib.hsg_scratch_bytes(ctypes.byref(d)) > 2 * 3 * 512 * 4
    assert lib.hsg_sweep(ctypes.byref(d), 1, 1, 1, 3, None) == _abi.HSG_ERR_INVALID
    assert b"NULL" in lib.hsg_last_error()
    assert lib.hsg_sweep(ctypes.byref(d), 1, 1, -1, 3, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_swap(ctypes.byref(d), 1, 7, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_anneal_swap(ctypes.byref(d), 1, 2, 1, 3, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_sweep(None, 0, 1, 1, 3, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_sweep_measure(ctypes.byref(d), 1, -1, 1, 3, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_sweep_measure(ctypes.byref(d), 1, 1, 0, 0, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_sweep_measure(ctypes.byref(d), 1, 1, 1, 3, None) == _abi.HSG_ERR_INVALID
    assert b"NULL" in lib.hsg_last_error()
    assert lib.hsg_sweep_measure(None, 0, 1, 1, 3, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_coolheat_swap_pairs(ctypes.byref(d), 1, 0, None, None) == _abi.HSG_ERR_INVALID
    assert b"eps" in lib.hsg_last_error()
    assert lib.hsg_coolheat_swap_pairs(ctypes.byref(d), 1, 5, None, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_coolheat_swap(ctypes.byref(d), 1, 0, -1.0, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_mlp_forward(None, 0, 64, 2, None, 1, None, None, None) == _abi.HSG_ERR_INVALID
    sink = ctypes.c_void_p(64)  # never dereferenced: each call below fails its checks first
    assert lib.hsg_probe_issue(5, 1, 64, 1, sink, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_probe_issue(0, 1, 96, 1, sink, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_probe_issue(0, 1, 2048, 1, sink, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_probe_issue(0, 0, 64, 1, sink, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_probe_issue(0, 1, 64, 0, sink, None) == _abi.HSG_ERR_INVALID
    assert lib.hsg_probe_issue(0, 1, 64, 1, None, None) == _abi.HSG_ERR_INVALID


@pytest.mark.parametrize("L", [2, 4, 6, 8])
def test_layout_conversion_matches_oracle_indexing(L):
    from paper_1006_4247_amd.ensemble import (device_to_natural, natural_to_device,
                                              natural_to_device_index)
    N = L ** 3
    perm = natural_to_device_index(L)
    for x in range(N):
        assert perm[x] == hsgref.parity(L, x) * (N // 2) + hsgref.compressed_index(L, x)
    a = np.random.default_rng(L).standard_normal((2, 3, N, 3))
    b = natural_to_device(a, L)
    assert b.shape == (2, 3, 3, 2, N // 2)
    assert np.array_equal(device_to_natural(b, L), a)


def test_plan_settings_are_validated_without_gpu():
    """hsg_plan_create parses and checks its JSON settings before touching the device:
    malformed or unknown settings return HSG_ERR_INVALID with a message."""
    _abi = _lib_or_skip()
    lib = _abi.lib()
    d = (_abi.HsgEnsemble * 1)()
    plan = ctypes.c_void_p()
    bad = [b'{"exchange": "bogus"}', b'{"nope": 1}', b'{"pairing": 1.5}',
           b'{"exchange": "anneal", "pairing": 0}', b'[1]', b'{"eps": [0.1, 0.2]}',
           b'{"n_hb": 0, "n_or": 0}', b'{"exchange": "coolheat", "eps": -1}', b'{"path": [1, 2]}',
           b'{"exchange": "plain"} x', b'{"split": 0}', b'{"split": 17}',
           b'{"split": 2, "path": 2}', b'{"split": 2, "path": 5}',
           b'{"stream": [1]}', b'{"stream": [0, 0]}', b'{"stream": [-1]}', b'{"stream": [0], "split": 2}']
    for js in bad:
        assert lib.hsg_plan_create(d, 1, js, ctypes.byref(plan)) == _abi.HSG_ERR_INVALID, js
        assert lib.hsg_last_error(), js
        assert not plan.value
    assert lib.hsg_plan_create(d, 0, b"{}", ctypes.byref(plan)) == _abi.HSG_ERR_INVALID
    assert lib.hsg_plan_run(None, 1, None) == _abi.HSG_ERR_INVALID
