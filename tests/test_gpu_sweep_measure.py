"""Sweeps followed by the measurement in one call (hsg_sweep_measure), on the GPU.

* Oracle parity: the spins, energies and counters after the call meet the sweep bars
  against the oracle's sweep (paper Sec. III.C), and Q, chi and the energies per site
  equal the oracle's measurement (Sec. IV) of the GPU's own final configurations.
* Equality with the two calls it stands for (hsg_sweep, then hsg_measure): identical
  spins and counters, energies and measurements up to the rounding order of FP64 sums,
  on the fused launches (two chains: binary32 L <= 10 and binary64 L <= 12 with both
  replicas side by side, binary32 L = 16 with the two swept in sequence by one
  workgroup) and on cases that take the two launches (other L, one or three chains,
  streaming sizes), and at two full shapes (L = 8, 128 x 2 x 8; L = 16, 64 x 2 x 24,
  the benchmark's launch), where the fused measurement also meets the oracle's.
"""
import numpy as np
import pytest
import torch

from gpu_pair import make_pair, sweep_and_check
from oracle import hsgref

import paper_1006_4247_amd as hsg

pytestmark = pytest.mark.gpu

SEED = 0x100642470C00


def _betas(R, lo=1.0, hi=8.0):
    return hsg.geometric_betas(lo, hi, R)


def _scramble_labels(gpu, ref, rng):
    """Give every (sample, chain) its own random slot order, on both sides."""
    S, C, R = ref.S, ref.C, ref.R
    for s in range(S):
        for c in range(C):
            perm = rng.permutation(R).astype(np.int32)  # temp_of_slot
            inv = np.argsort(perm).astype(np.int32)
            ref.temp_of_slot[s, c] = perm
            ref.slot_of_temp[s, c] = inv
            gpu.temp_of_slot[s, c] = torch.from_numpy(perm).to(gpu.device)
            gpu.slot_of_temp[s, c] = torch.from_numpy(inv).to(gpu.device)


def _set_counters(gpu, ref, base):
    ctr = (base + np.arange(ref.sweep_ctr.size, dtype=np.uint32) * 5).reshape(ref.sweep_ctr.shape)
    ref.sweep_ctr[...] = ctr
    gpu.sweep_ctr.copy_(torch.from_numpy(ctr.view(np.int32)))


def _oracle_measure_of(gpu):
    """The oracle's measurement of the GPU ensemble's current state (spins, energies,
    labels)."""
    ref = hsgref.RefEnsemble(gpu.L, gpu.S, gpu.C, gpu.betas.cpu().numpy(), 0)
    ref.spins[...] = gpu.spins_natural()
    ref.energy[...] = gpu.energy.cpu().numpy()
    ref.slot_of_temp[...] = gpu.slot_of_temp.cpu().numpy()
    return ref.measure()


@pytest.mark.parametrize("prec,L", [("fp32", 2), ("fp32", 4), ("fp32", 8), ("fp32", 10), ("fp32", 16),
                                    ("fp64", 6), ("fp64", 10), ("fp64", 12), ("fp64", 14)])
@pytest.mark.parametrize("kind", ["hb", "or", "hb+3or"])
def test_sweep_measure_parity(prec, L, kind):
    S, C, R = 3, 2, 4
    n_hb, n_or = {"hb": (1, 0), "or": (0, 1), "hb+3or": (1, 3)}[kind]
    gpu, ref = make_pair(L, S, C, _betas(R), SEED + L, prec=prec)
    _scramble_labels(gpu, ref, np.random.default_rng(L))
    _set_counters(gpu, ref, 300 + L)
    out = {}

    def launch():
        out["m"] = gpu.sweep_measure(1, n_hb, n_or)
        out["m"] = tuple(t.clone() for t in out["m"])

    what = "sweep_measure L=%d %s %s" % (L, prec, kind)
    rep = sweep_and_check(gpu, n_hb, n_or, launch=launch, what=what)
    print("[parity] %s: %s" % (what, rep.summary()), flush=True)
    Q, chi, e = out["m"]
    # the measurement of the launch's own final configurations (the replay of a
    # composite step leaves the same spins and energies)
    rQ, rchi, re = _oracle_measure_of(gpu)
    assert np.max(np.abs(Q.cpu().numpy() - rQ)) <= 1e-10
    assert np.max(np.abs(chi.cpu().numpy() - rchi)) <= 1e-10 * max(1.0, float(np.max(rchi)))
    assert np.array_equal(e.cpu().numpy(), re)


def _twins(L, S, C, R, prec, seed):
    """Two GPU ensembles in one state (the oracle's initial one, labels scrambled)."""
    a, ref = make_pair(L, S, C, _betas(R), seed, prec=prec)
    b = hsg.Ensemble(L, S, C, _betas(R), seed, precision=prec)
    for name in ("spins", "couplings", "energy", "sweep_ctr"):
        getattr(b, name).copy_(getattr(a, name))
    rng = np.random.default_rng(seed & 0xFFFF)
    for s in range(S):
        for c in range(C):
            perm = torch.from_numpy(rng.permutation(R).astype(np.int32)).to(a.device)
            for e in (a, b):
                e.temp_of_slot[s, c] = perm
                e.slot_of_temp[s, c] = torch.argsort(perm).to(torch.int32)
    torch.cuda.synchronize()
    return a, b


def _assert_same(a, b, fused_energy_bitwise):
    torch.cuda.synchronize()
    assert torch.equal(a.spins, b.spins)
    assert torch.equal(a.sweep_ctr, b.sweep_ctr)
    if fused_energy_bitwise:
        assert torch.equal(a.energy, b.energy)
    else:
        assert torch.allclose(a.energy, b.energy, rtol=1e-13, atol=1e-9)
    assert torch.allclose(a.e_temp, b.e_temp, rtol=1e-13, atol=1e-12)
    if a.C >= 2:
        assert torch.allclose(a.Q, b.Q, rtol=0, atol=1e-9)
        assert torch.allclose(a.chi, b.chi, rtol=1e-12, atol=1e-12)
    a.check()
    b.check()


@pytest.mark.parametrize("prec,L,C,n_sweeps", [
    ("fp32", 10, 2, 3),   # one launch
    ("fp32", 8, 2, 2),
    ("fp64", 8, 2, 1),
    ("fp64", 12, 2, 2),   # one launch with 256 threads per replica (the sweep alone: 448)
    ("fp32", 16, 2, 2),   # one launch, the two replicas in sequence
    ("fp32", 12, 2, 1),   # two launches from here on
    ("fp32", 8, 1, 1),    # one chain: no overlap
    ("fp32", 8, 3, 2),    # three chains: Q of chains 0 and 1
    ("fp64", 16, 2, 1),
    ("fp32", 20, 2, 1),   # streaming size: the measurement finishes the sweep's energies
    ("fp32", 20, 2, 3),   # ... of the last of three sweeps
    ("fp64", 18, 2, 2),
    ("fp32", 18, 1, 1),   # ... with one chain (no overlap)
    ("fp32", 20, 3, 1),
    ("fp32", 20, 2, 0),   # no sweep: the measurement alone
    ("fp32", 8, 2, 0),    # no sweep: the measurement alone
])
def test_sweep_measure_equals_sweep_then_measure(prec, L, C, n_sweeps):
    a, b = _twins(L, 2, C, 5, prec, SEED + 100 + L + C)
    a.sweep(n_sweeps, 1, 3)
    a.measure()
    b.sweep_measure(n_sweeps, 1, 3)
    _assert_same(a, b, fused_energy_bitwise=not (prec == "fp64" and L == 12 and C == 2 and n_sweeps > 0))


@pytest.mark.parametrize("L,S,R", [(8, 128, 8), (16, 64, 24)])
def test_sweep_measure_full_shape(L, S, R):
    """Full binary32 shapes (the smallest class of the uneven batch; the L = 16
    benchmark shape and launch), 1 HB + 3 OR, two steps in a row with a plain exchange
    between."""
    C = 2
    a = hsg.Ensemble(L, S, C, _betas(R), SEED + 7, precision="fp32")
    b = hsg.Ensemble(L, S, C, _betas(R), SEED + 7, precision="fp32")
    for e in (a, b):
        e.init_couplings()
        e.init_spins()
    for _ in range(2):
        a.sweep(1, 1, 3)
        a.measure()
        a.swap(0)
        b.sweep_measure(1, 1, 3)
        b.swap(0)
    _assert_same(a, b, fused_energy_bitwise=True)
    assert torch.equal(a.slot_of_temp, b.slot_of_temp)
    # one more fused launch, its measurement against the oracle's measurement of its own
    # final configurations (no exchange after it), every (sample, temperature)
    b.sweep_measure(1, 1, 3)
    torch.cuda.synchronize()
    rQ, rchi, re = _oracle_measure_of(b)
    assert np.max(np.abs(b.Q.cpu().numpy() - rQ)) <= 1e-10
    assert np.max(np.abs(b.chi.cpu().numpy() - rchi)) <= 1e-10 * max(1.0, float(np.max(rchi)))
    assert np.array_equal(b.e_temp.cpu().numpy(), re)
