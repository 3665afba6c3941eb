"""The issue-rate probe behind the roofline peaks (hsg_probe_issue): every kind runs,
and the LDS kinds read the words they are meant to read."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1006_4247_amd import _abi

pytestmark = pytest.mark.gpu


def _expected_lds_sums(kind, groups, threads, iters):
    t = np.tile(np.arange(threads), groups)
    lane, w = t & 63, (t >> 6) & 3
    x = (t.astype(np.float32) * np.float32(1e-7)).astype(np.float64)
    total = np.zeros(t.shape, np.float64)
    for c in range(16):
        if kind == 3:
            word = w * 64 + lane + 256 * c
        else:
            word = 4 * (w * 64 + lane + 256 * (c // 4)) + (c % 4)
        total += 2.0 * (c * 1e-3 + x) + iters * word * 1e-3
    return total


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_probe_issue_kinds(kind):
    lib = _abi.lib()
    groups, threads, iters = 4, 256, 10
    sink = torch.zeros(groups * threads, dtype=torch.float32, device="cuda:0")
    _abi.check(lib.hsg_probe_issue(kind, groups, threads, iters, ctypes.c_void_p(sink.data_ptr()), None))
    torch.cuda.synchronize()
    v = sink.cpu().numpy()
    assert np.all(np.isfinite(v))
    if kind in (3, 4):
        np.testing.assert_allclose(v, _expected_lds_sums(kind, groups, threads, iters), rtol=1e-5)
