"""Plans (hsg_plan_create / hsg_plan_run / hsg_plan_destroy): one cycle of several
ensembles captured into HIP graphs inside the library and replayed.  Through the C ABI,
n replayed cycles equal n eager cycles of the same calls bit for bit (spins, energies,
labels, counters, statistics, round trips, measurements), for every exchange, with
size classes on the LDS-resident and the streaming paths in one plan, odd cycle counts
(alternating exchanges keep their parity across runs) and zero cycles."""
import ctypes
import json

import numpy as np
import pytest
import torch

import paper_1006_4247_amd as hsg
from paper_1006_4247_amd import _abi

pytestmark = pytest.mark.gpu

SHAPES = [(8, 4, 2, 6, "fp32"), (24, 1, 2, 4, "fp32"), (6, 2, 2, 5, "fp64")]


def _batch(seed, K_max=0):
    out = []
    sb = cb = qb = 0
    for k, (L, S, C, R, prec) in enumerate(SHAPES):
        e = hsg.Ensemble(L, S, C, hsg.geometric_betas(1.0, 3.0, R), seed, precision=prec, K_max=K_max,
                         sample_base=sb, chain_base=cb, slot_base=qb)
        e.init_couplings()
        e.init_spins()
        sb, cb, qb = sb + S, cb + S * C, qb + S * C * R
        out.append(e)
    torch.cuda.synchronize()
    return out


def _state(ens):
    torch.cuda.synchronize()
    return [{k: getattr(e, k).detach().cpu().numpy().copy() for k in
             ("spins", "energy", "temp_of_slot", "slot_of_temp", "sweep_ctr", "swap_ctr", "swap_stats",
              "rt_state", "rt_trips", "Q", "chi", "e_temp", "guard")} for e in ens]


def _eager_cycle(e, settings, parity):
    ex = settings["exchange"]
    e.sweep_measure(1, settings.get("n_hb", 1), settings.get("n_or", 3))
    pairing = settings.get("pairing", 0 if ex == "plain" else -1)
    pairing = pairing if pairing >= 0 else parity + 1
    if ex == "plain":
        e.swap(pairing)
    elif ex == "decimate":
        e.decimate_swap(pairing)
    elif ex == "coolheat":
        e.coolheat_swap(settings["eps"], pairing)
    elif ex == "anneal":
        e.anneal_swap(parity, settings.get("anneal_n_hb", 1), settings.get("anneal_n_or", 3))


SETTINGS = [
    {"exchange": "plain", "pairing": 0},
    {"exchange": "plain", "pairing": 2, "n_hb": 1, "n_or": 2},
    {"exchange": "decimate"},
    {"exchange": "decimate", "pairing": 0},
    {"exchange": "coolheat", "eps": 0.004},
    {"exchange": "anneal", "anneal_n_hb": 1, "anneal_n_or": 1},
]


@pytest.mark.parametrize("settings", SETTINGS, ids=[json.dumps(s) for s in SETTINGS])
def test_plan_replay_equals_eager_cycles(settings):
    K_max = 3 if settings["exchange"] == "anneal" else 0
    a, b = _batch(0x9A11, K_max), _batch(0x9A11, K_max)
    if K_max:
        for e in a + b:
            e.set_schedule(np.array([1, 3, 0, 2, 1][:e.R - 1], dtype=np.int32))
    descs = (_abi.HsgEnsemble * len(b))(*[e.desc for e in b])
    plan = ctypes.c_void_p()
    _abi.check(_abi.lib().hsg_plan_create(descs, len(b), json.dumps(settings).encode(), ctypes.byref(plan)))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    try:
        parity = 0
        for n in (3, 0, 19, 2):
            for _ in range(n):
                for e in a:
                    _eager_cycle(e, settings, parity)
                parity ^= 1
            _abi.check(_abi.lib().hsg_plan_run(plan, n, stream))
            sa, sb = _state(a), _state(b)
            for k, (x, y) in enumerate(zip(sa, sb)):
                for name in x:
                    assert np.array_equal(x[name], y[name]), (settings, k, name, n)
        alternating = settings["exchange"] != "plain" and settings.get("pairing", -1) < 0
        assert _abi.lib().hsg_plan_next_parity(plan) == (parity if alternating else 0)
    finally:
        _abi.lib().hsg_plan_destroy(plan)
    for e in a + b:
        e.check()


def test_plan_per_pair_eps_and_tuned_paths():
    """Per-pair cooling / heating parameters (one list over every ensemble's pairs) and
    sweep tunings per ensemble."""
    a, b = _batch(0x9A12), _batch(0x9A12)
    eps = []
    for e in b:
        eps += list(np.linspace(0.002, 0.005, e.R - 1))
    tunings = [{"path": 1}, {"path": 4}, {"path": 3}]
    settings = {"exchange": "coolheat", "eps": eps, "path": [t["path"] for t in tunings]}
    descs = (_abi.HsgEnsemble * len(b))(*[e.desc for e in b])
    plan = ctypes.c_void_p()
    _abi.check(_abi.lib().hsg_plan_create(descs, len(b), json.dumps(settings).encode(), ctypes.byref(plan)))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    off = 0
    per = []
    for e in a:
        per.append(np.array(eps[off:off + e.R - 1]))
        off += e.R - 1
    for c in range(3):
        for e, t, ep in zip(a, tunings, per):
            e.sweep(1, 1, 3, tuning=t)
            e.measure()
            e.coolheat_swap(ep, 1 + c % 2)
    _abi.check(_abi.lib().hsg_plan_run(plan, 3, stream))
    _abi.lib().hsg_plan_destroy(plan)
    for x, y in zip(_state(a), _state(b)):
        for name in x:
            assert np.array_equal(x[name], y[name]), name


SPLIT_SHAPES = [(16, 5, 2, 6, "fp32"), (8, 3, 2, 4, "fp64"), (4, 1, 2, 3, "fp32")]
SPLIT_EXCHANGES = ["plain", "none", "decimate", "coolheat", "coolheat_pairs", "anneal"]


@pytest.mark.parametrize("split", [2, 3, 16])
@pytest.mark.parametrize("exchange", SPLIT_EXCHANGES)
def test_split_plan_equals_eager_cycles(split, exchange):
    """A split plan runs each ensemble as parts of consecutive samples (uneven parts, more
    parts asked for than samples, a one-sample ensemble left whole), each on a stream of
    its own, the parts' scratch the plan's own: n replayed cycles equal n eager cycles of
    the whole ensembles bit for bit, for every exchange."""
    K_max = 3 if exchange == "anneal" else 0

    def batch():
        out, sb, cb, qb = [], 0, 0, 0
        for L, S, C, R, prec in SPLIT_SHAPES:
            e = hsg.Ensemble(L, S, C, hsg.geometric_betas(1.0, 4.0, R), 0x9A13, precision=prec, K_max=K_max,
                             sample_base=sb, chain_base=cb, slot_base=qb)
            e.init_couplings()
            e.init_spins()
            if K_max:
                e.set_schedule(np.array([1, 3, 0, 2, 1][:R - 1], dtype=np.int32))
            sb, cb, qb = sb + S, cb + S * C, qb + S * C * R
            out.append(e)
        torch.cuda.synchronize()
        return out
    a, b = batch(), batch()
    eps_pairs = [list(np.linspace(0.002, 0.006, e.R - 1)) for e in a]
    if exchange == "coolheat_pairs":
        settings = {"exchange": "coolheat", "eps": [v for x in eps_pairs for v in x]}
    elif exchange == "coolheat":
        settings = {"exchange": "coolheat", "eps": 0.004}
    else:
        settings = {"exchange": exchange}
    settings.update(split=split, unroll=4)
    if exchange == "anneal":
        settings.update(anneal_n_hb=1, anneal_n_or=1)
    descs = (_abi.HsgEnsemble * len(b))(*[e.desc for e in b])
    plan = ctypes.c_void_p()
    _abi.check(_abi.lib().hsg_plan_create(descs, len(b), json.dumps(settings).encode(), ctypes.byref(plan)))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    try:
        parity = 0
        for n in (1, 9):
            for _ in range(n):
                for k, e in enumerate(a):
                    if exchange == "none":
                        e.sweep_measure(1, 1, 3)
                    elif exchange == "coolheat_pairs":
                        e.sweep_measure(1, 1, 3)
                        e.coolheat_swap(np.array(eps_pairs[k]), parity + 1)
                    else:
                        _eager_cycle(e, settings, parity)
                if exchange != "plain" and exchange != "none":
                    parity ^= 1
            _abi.check(_abi.lib().hsg_plan_run(plan, n, stream))
            for k, (x, y) in enumerate(zip(_state(a), _state(b))):
                for name in x:
                    assert np.array_equal(x[name], y[name]), (split, exchange, k, name, n)
    finally:
        _abi.lib().hsg_plan_destroy(plan)
    for e in a + b:
        e.check()


@pytest.mark.parametrize("groups", [[1, 0, 1], [0, 0, 0], [2, 1, 0]])
def test_stream_groups_equal_eager_cycles(groups):
    """Ensembles grouped onto capture streams (the ensembles of one group one after
    another, the groups side by side): replayed cycles equal eager cycles bit for bit."""
    a, b = _batch(0x9A14), _batch(0x9A14)
    settings = {"exchange": "plain", "stream": groups, "unroll": 4}
    descs = (_abi.HsgEnsemble * len(b))(*[e.desc for e in b])
    plan = ctypes.c_void_p()
    _abi.check(_abi.lib().hsg_plan_create(descs, len(b), json.dumps(settings).encode(), ctypes.byref(plan)))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    try:
        for _ in range(7):
            for e in a:
                e.sweep_measure(1, 1, 3)
                e.swap(0)
        _abi.check(_abi.lib().hsg_plan_run(plan, 7, stream))
        for k, (x, y) in enumerate(zip(_state(a), _state(b))):
            for name in x:
                assert np.array_equal(x[name], y[name]), (groups, k, name)
    finally:
        _abi.lib().hsg_plan_destroy(plan)
