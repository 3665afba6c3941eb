"""Cooling / heating exchange (paper Sec. III.B) on the GPU against the oracle.

FP64: the log Jacobians of both maps to 1e-9 (relative), decisions, labels, counters
and statistics bit for bit, spins to 1e-12, energies to 1e-9, over several calls in all
three pair orders; L <= 16 runs the LDS-resident legs, L = 20 the generic ones.

FP32 (maps and site log Jacobians in binary32, their sums, energies and ln A in
binary64): each site is moved once per map, like one lattice sweep, so the transformed
spins meet the lattice-sweep bar (1e-5 per component).  From it: per site
|d ln det| <= 4 k/(1-k)^2 |ds|-scale terms plus ~2.4e-7 for the binary32 logarithm,
bounded here by N (4 k_max/(1-k_max)^2 * 1e-5 + 2.4e-7), and |d ln A| <= that bound for
both maps + max(beta) * (energy bound of the candidates).  Decisions are compared where
|ln A - ln u| exceeds it, pair by pair with disjoint pairings.
"""
import numpy as np
import pytest
import torch

import paper_1006_4247_amd as hsg
from oracle import hsgref
from tests import closed_forms as cf
from tests import inputs
from tests.gpu_pair import LATTICE_BAR, compare_ints, energy_bound, make_pair
from tests.test_gpu_decimate import _exact_forest, _log_u

pytestmark = pytest.mark.gpu
SEED = 0xC0DE
EPS = 0.017


def _betas(R, lo=0.5, hi=3.0):
    return hsgref.geometric_betas(lo, hi, R)


@pytest.mark.parametrize("L", [4, 6, 12, 16, 20])
@pytest.mark.parametrize("pairing", [0, 1, 2])
def test_coolheat_parity_fp64(L, pairing):
    S, C, R = 2, 2, 5
    gpu, ref = make_pair(L, S, C, _betas(R), SEED + 10 * L + pairing, prec="fp64")
    for call in range(2):
        w = gpu.coolheat_swap(EPS, pairing)
        lnA, ld = ref.coolheat_swap(EPS, pairing)
        torch.cuda.synchronize()
        wg = w.cpu().numpy()
        what = "coolheat fp64 L=%d pairing %d call %d" % (L, pairing, call)
        assert np.max(np.abs(wg - ld)) <= 1e-9 * max(1.0, np.abs(ld).max()), what
        st = compare_ints(gpu, ref, what)
        assert np.max(np.abs(st["spins"] - ref.spins)) <= 1e-12, what
        assert np.max(np.abs(st["energy"] - ref.energy)) <= 1e-9, what
    assert 0 < ref.stats[..., 1].sum() < ref.stats[..., 0].sum()
    gpu.check()


@pytest.mark.parametrize("R", [2, 3, 4])
def test_coolheat_short_ladders_fp64(R):
    """Ladders with at most one selected pair per chain and call (and, at R = 2 with odd
    pairs, none): a sequence of pairings, each call's diagnostics (zeros where not
    attempted, whatever an earlier call left there), labels, counters, spins and
    energies against the oracle."""
    L, S, C = 4, 2, 2
    gpu, ref = make_pair(L, S, C, _betas(R), SEED + 500 + R, prec="fp64")
    for call, pairing in enumerate([1, 2, 0, 2, 1, 0]):
        w = gpu.coolheat_swap(EPS, pairing)
        _, ld = ref.coolheat_swap(EPS, pairing)
        torch.cuda.synchronize()
        what = "coolheat fp64 R=%d call %d pairing %d" % (R, call, pairing)
        assert np.max(np.abs(w.cpu().numpy() - ld)) <= 1e-9 * max(1.0, np.abs(ld).max()), what
        st = compare_ints(gpu, ref, what)
        assert np.max(np.abs(st["spins"] - ref.spins)) <= 1e-12, what
        assert np.max(np.abs(st["energy"] - ref.energy)) <= 1e-9, what
    gpu.check()


def _max_k(ref, eps):
    L = ref.L
    k = 0.0
    for s in range(ref.S):
        for c in range(ref.C):
            for r in range(ref.R):
                for z in range(0, L ** 3, 7):
                    k = max(k, eps * np.linalg.norm(hsgref.local_field(L, ref.J[s], ref.spins[s, c, r], z)))
    return min(k * 1.5, 0.95)


@pytest.mark.parametrize("L", [4, 8, 16, 24])
@pytest.mark.parametrize("pairing", [1, 2])
def test_coolheat_parity_fp32(L, pairing):
    S, C, R = 2, 3, 7
    eps = EPS if L <= 16 else 0.01
    gpu, ref = make_pair(L, S, C, _betas(R), SEED + 100 + L + pairing, prec="fp32")
    before = ref.spins.copy()
    sot = ref.slot_of_temp.copy()
    n0 = ref.swap_ctr.copy()
    kmax = _max_k(ref, eps)
    w = gpu.coolheat_swap(eps, pairing)
    lnA, ld = ref.coolheat_swap(eps, pairing)
    torch.cuda.synchronize()
    wg = w.cpu().numpy()
    N = L ** 3
    bar = LATTICE_BAR["fp32"]
    tol_ld = N * (4.0 * kmax / (1.0 - kmax) ** 2 * bar + 2.4e-7)
    assert np.all(np.abs(wg - ld) <= tol_ld), (np.abs(wg - ld).max(), tol_ld)
    ebound = energy_bound(L, ref.J, np.full(ref.spins.shape[:-1], np.sqrt(3.0) * bar), "fp32")
    tol_lnA = 2.0 * tol_ld + ref.betas.max() * 2.0 * ebound.max()
    st = gpu.host_state()
    assert np.array_equal(st["swap_ctr"], ref.swap_ctr)
    checked = 0
    for s in range(S):
        for c in range(C):
            for i in range(pairing - 1, R - 1, 2):
                if abs(lnA[s, c, i] - _log_u(ref, s * C + c, i, int(n0[s, c]))) <= tol_lnA:
                    continue  # ambiguous in binary32
                checked += 1
                x, y = sot[s, c, i], sot[s, c, i + 1]
                assert np.array_equal(st["stats"][s, c, i], ref.stats[s, c, i])
                for slot in (x, y):
                    assert st["temp_of_slot"][s, c, slot] == ref.temp_of_slot[s, c, slot]
                    d = np.abs(st["spins"][s, c, slot] - ref.spins[s, c, slot]).max()
                    assert d <= bar, (s, c, slot, d)
    assert checked >= S * C * len(range(pairing - 1, R - 1, 2)) // 2, checked
    assert ref.stats[..., 1].sum() > 0
    # rejected pairs left both configurations bit-identical
    for s in range(S):
        for c in range(C):
            for i in range(pairing - 1, R - 1, 2):
                if st["stats"][s, c, i, 1] == 0:
                    for slot in (sot[s, c, i], sot[s, c, i + 1]):
                        assert np.array_equal(st["spins"][s, c, slot], before[s, c, slot])
    gpu.check()


@pytest.mark.parametrize("L", [8, 16, 18])
def test_coolheat_ascending_fp32(L):
    """All pairs in ascending order (one round of legs per pair), FP32.  A
    configuration can be mapped by several consecutive accepted pairs, so the
    per-pair bars above are tripled.  Along each chain the pairs are compared in order
    until the first decision binary32 cannot settle; the rest of that chain is skipped."""
    S, C, R = 2, 3, 7
    eps = EPS if L <= 8 else 0.006
    gpu, ref = make_pair(L, S, C, _betas(R), SEED + 400 + L, prec="fp32")
    N = L ** 3
    bar = LATTICE_BAR["fp32"]
    checked = full = 0
    for call in range(2):
        kmax = _max_k(ref, eps)
        tol_ld = 3.0 * N * (4.0 * kmax / (1.0 - kmax) ** 2 * bar + 2.4e-7)
        ebound = energy_bound(L, ref.J, np.full(ref.spins.shape[:-1], 3.0 * np.sqrt(3.0) * bar), "fp32")
        tol_lnA = 2.0 * tol_ld + ref.betas.max() * 2.0 * ebound.max()
        n0 = ref.swap_ctr.copy()
        stats0 = ref.stats.copy()
        w = gpu.coolheat_swap(eps, 0)
        lnA, ld = ref.coolheat_swap(eps, 0)
        torch.cuda.synchronize()
        wg = w.cpu().numpy()
        st = gpu.host_state()
        assert np.array_equal(st["swap_ctr"], ref.swap_ctr)
        for s in range(S):
            for c in range(C):
                clean = True
                for i in range(R - 1):
                    if abs(lnA[s, c, i] - _log_u(ref, s * C + c, i, int(n0[s, c]))) <= tol_lnA:
                        clean = False
                        break
                    checked += 1
                    assert np.all(np.abs(wg[s, c, i] - ld[s, c, i]) <= tol_ld), (s, c, i, wg[s, c, i], ld[s, c, i])
                    assert np.array_equal(st["stats"][s, c, i] - stats0[s, c, i], ref.stats[s, c, i] - stats0[s, c, i])
                if clean:
                    full += 1
                    assert np.array_equal(st["temp_of_slot"][s, c], ref.temp_of_slot[s, c])
                    # round trips: the chain kernel (L <= 16) and the split pass's
                    # finishing launch update them, one thread per slot
                    assert np.array_equal(st["rt_state"][s, c], ref.rt_state[s, c])
                    assert np.array_equal(st["rt_trips"][s, c], ref.rt_trips[s, c])
                    assert np.abs(st["spins"][s, c] - ref.spins[s, c]).max() <= 3.0 * bar
        ref.set_state(spins=st["spins"].astype(np.float64))
        for k in ("temp_of_slot", "slot_of_temp", "stats", "rt_state", "rt_trips"):
            getattr(ref, k)[...] = st[k]
    assert checked >= S * C * (R - 1) and full >= S * C, (checked, full)
    assert ref.stats[..., 1].sum() > 0
    gpu.check()


def test_coolheat_eps_zero_equals_plain_exchange_on_gpu():
    L, S, C, R = 8, 2, 2, 6
    a, _ = make_pair(L, S, C, _betas(R), SEED + 3, prec="fp32")
    b, _ = make_pair(L, S, C, _betas(R), SEED + 3, prec="fp32")
    for it in range(4):
        a.sweep(1, 1, 3)
        b.sweep(1, 1, 3)
        a.swap(it % 3)
        b.coolheat_swap(0.0, it % 3)
    torch.cuda.synchronize()
    sa, sb = a.host_state(), b.host_state()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k


def test_coolheat_non_bijective_eps_rejects_and_trips_guard():
    L, S, C, R = 4, 1, 2, 4
    gpu, _ = make_pair(L, S, C, _betas(R), SEED + 5, prec="fp64")
    st0 = gpu.host_state()
    gpu.coolheat_swap(50.0, 0)
    torch.cuda.synchronize()
    st = gpu.host_state()
    assert np.array_equal(st["spins"], st0["spins"])
    assert st["stats"][..., 1].sum() == 0 and np.all(st["swap_ctr"] == 1)
    with pytest.raises(hsg.HsgError) as ei:
        gpu.check()
    assert ei.value.code == 3


def test_coolheat_full_shape_sampled_pairs():
    """L = 16, 64 samples x 2 chains x 24 temperatures (FP32), eps = 0.017: sampled pairs
    recomputed by the oracle from the GPU's state before the call."""
    L, S, C, R = 16, 64, 2, 24
    betas = hsgref.geometric_betas(1.0, 8.0, R)
    gpu = hsg.Ensemble(L, S, C, betas, 0x100642470002, precision="fp32")
    gpu.init_couplings()
    gpu.init_spins()
    gpu.sweep(20, 1, 3)
    torch.cuda.synchronize()
    st0 = gpu.host_state()
    J = gpu.couplings_natural()
    w = gpu.coolheat_swap(EPS, 1)
    torch.cuda.synchronize()
    wg = w.cpu().numpy()
    st = gpu.host_state()
    rng = np.random.default_rng(5)
    N = L ** 3
    bar = LATTICE_BAR["fp32"]
    for k in range(6):
        s, c = int(rng.integers(S)), int(rng.integers(C))
        i = 2 * int(rng.integers(R // 2))
        x, y = st0["slot_of_temp"][s, c, i], st0["slot_of_temp"][s, c, i + 1]
        cx = st0["spins"][s, c, x].astype(np.float64)
        cy = st0["spins"][s, c, y].astype(np.float64)
        ldx = hsgref.coolheat(L, J[s], cx, EPS, False)
        ldy = hsgref.coolheat(L, J[s], cy, EPS, True)
        kmax = 0.6
        tol_ld = N * (4.0 * kmax / (1.0 - kmax) ** 2 * bar + 2.4e-7)
        assert abs(wg[s, c, i, 0] - ldx) <= tol_ld and abs(wg[s, c, i, 1] - ldy) <= tol_ld, (k, wg[s, c, i], ldx, ldy)
        accepted = st["stats"][s, c, i, 1] - st0["stats"][s, c, i, 1]
        if accepted:
            assert np.abs(st["spins"][s, c, x] - cx).max() <= bar
            assert np.abs(st["spins"][s, c, y] - cy).max() <= bar
        else:
            assert np.array_equal(st["spins"][s, c, x], st0["spins"][s, c, x])
            assert np.array_equal(st["spins"][s, c, y], st0["spins"][s, c, y])
    assert np.all(st["swap_ctr"] == st0["swap_ctr"] + 1)
    gpu.check()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_forest_law_stationary_under_gpu_coolheat(prec):
    L, C = 4, 256
    betas = np.array([0.5, 1.0, 2.0, 4.0])
    R = len(betas)
    rng = np.random.default_rng(93)
    J = inputs.forest_couplings(L, 1, 94)[0]
    spins = np.zeros((1, C, R, L ** 3, 3))
    for c in range(C):
        for r in range(R):
            spins[0, c, r] = _exact_forest(L, J, betas[r], rng)
    gpu, _ = make_pair(L, 1, C, betas, 0xC0F, prec=prec, J=J[None], spins=spins)
    for t in range(100):
        gpu.coolheat_swap(0.15, t % 3)
    torch.cuda.synchronize()
    st = gpu.host_state()
    acc = st["stats"][..., 1].sum() / st["stats"][..., 0].sum()
    assert acc > 0.1
    Jb = np.array([b[2] for b in cf.forest_bonds(L, J)])
    for r in range(R):
        H = np.array([st["energy"][0, c, st["slot_of_temp"][0, c, r]] for c in range(C)])
        mean, var = cf.forest_mean_H(betas[r], Jb), cf.forest_var_H(betas[r], Jb)
        z = (H.mean() - mean) / np.sqrt(var / C)
        assert abs(z) < 4.0, (r, H.mean(), mean, z)
        zv = (H.var(ddof=1) - var) / (var * np.sqrt(2.0 / (C - 1)))
        assert abs(zv) < 4.5, (r, H.var(ddof=1), var, zv)
    gpu.check()


@pytest.mark.parametrize("L", [4, 16, 20])
@pytest.mark.parametrize("pairing", [0, 1, 2])
def test_coolheat_per_pair_eps_parity_fp64(L, pairing):
    """One map parameter per pair of temperatures (Sec. IV), through
    hsg_coolheat_swap_pairs: the LDS-resident legs (L = 4, 16; at 16 ascending pairs
    decide inside the next pair's launch) and the split pass (L = 20) against the
    oracle, two calls."""
    S, C, R = 2, 2, 5
    eps = np.array([0.005, 0.02, 0.0, 0.012])
    gpu, ref = make_pair(L, S, C, _betas(R), SEED + 700 + 10 * L + pairing, prec="fp64")
    for call in range(2):
        w = gpu.coolheat_swap(eps, pairing)
        _, ld = ref.coolheat_swap(eps, pairing)
        torch.cuda.synchronize()
        what = "per-pair eps fp64 L=%d pairing %d call %d" % (L, pairing, call)
        assert np.max(np.abs(w.cpu().numpy() - ld)) <= 1e-9 * max(1.0, np.abs(ld).max()), what
        st = compare_ints(gpu, ref, what)
        assert np.max(np.abs(st["spins"] - ref.spins)) <= 1e-12, what
        assert np.max(np.abs(st["energy"] - ref.energy)) <= 1e-9, what
    gpu.check()


@pytest.mark.parametrize("L", [16, 24])
def test_coolheat_equal_per_pair_eps_equals_one_eps(L):
    """Equal per-pair parameters give the single-parameter exchange bit for bit
    (binary32; L = 16 LDS-resident, L = 24 split pass), ascending and even pairs."""
    S, C, R = 4, 2, 9
    a = hsg.Ensemble(L, S, C, _betas(R, 0.8, 2.0), SEED + 800 + L, precision="fp32")
    b = hsg.Ensemble(L, S, C, _betas(R, 0.8, 2.0), SEED + 800 + L, precision="fp32")
    for e in (a, b):
        e.init_couplings()
        e.init_spins()
        e.sweep(2, 1, 3)
    eps_t = torch.full((R - 1,), 0.01, dtype=torch.float64, device=b.device)
    for pairing in (0, 1, 0):
        a.coolheat_swap(0.01, pairing)
        b.coolheat_swap(eps_t, pairing)
    torch.cuda.synchronize()
    for k in ("spins", "temp_of_slot", "slot_of_temp", "energy", "swap_stats", "work", "rt_trips"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    a.check()
    b.check()


def test_coolheat_per_pair_eps_in_graph_replay():
    """PTRun with per-pair parameters prepared on the device: replays of a captured
    step equal eager steps."""
    from paper_1006_4247_amd import runtime
    L, S, C, R = 8, 3, 2, 6
    eps = [0.02, 0.015, 0.01, 0.008, 0.006]
    ens = [hsg.Ensemble(L, S, C, _betas(R, 0.8, 3.0), SEED + 900, precision="fp32") for _ in range(2)]
    for e in ens:
        e.init_couplings()
        e.init_spins()
    ra = runtime.PTRun([ens[0]], 1, 3, mode="coolheat", eps=eps)
    rb = runtime.PTRun([ens[1]], 1, 3, mode="coolheat", eps=eps)
    rb.capture()
    for _ in range(3):
        ra.step(rb.graph_steps)
        rb.replay()
        ra.synchronize()
        for k in ("spins", "slot_of_temp", "energy", "swap_stats"):
            assert torch.equal(getattr(ens[0], k), getattr(ens[1], k)), k
    assert ens[0].swap_stats[..., 1].sum() > 0
    ra.check()
    rb.check()
