"""GPU tests of the runtime layer: HIP-graph replays equal eager steps (checked after
every replay, with eager work between replays), several size classes on their own
streams equal the same classes run alone, the sweep kernel variants give the same
spins, and the autotuner picks a supported variant."""
import json

import numpy as np
import pytest
import torch

import paper_1006_4247_amd as hsg
from paper_1006_4247_amd import autotune, runtime

pytestmark = pytest.mark.gpu
SEED = 0x100642470005


def _classes(K_max=0):
    return runtime.uneven_batch([8, 4, 16], [3, 5, 2], [4, 6, 5], SEED, K_max=K_max)


def _init(ens_list, K=None):
    for e in ens_list:
        e.init_couplings()
        e.init_spins()
        if K is not None:
            e.set_schedule(np.full(e.R - 1, K, dtype=np.int32))


def _state(e):
    st = e.host_state()
    st["chi"] = e.chi.cpu().numpy()
    st["e_temp"] = e.e_temp.cpu().numpy()
    return st


def _equal(a, b):
    for ea, eb in zip(a, b):
        sa, sb = _state(ea), _state(eb)
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), k


@pytest.mark.parametrize("mode,concurrent", [("plain", False), ("anneal", False), ("plain", True),
                                             ("anneal", True)])
def test_graph_replay_equals_eager(mode, concurrent):
    K = 2 if mode == "anneal" else None
    a = _classes(K_max=2)
    b = _classes(K_max=2)
    _init(a, K)
    _init(b, K)
    ra = runtime.PTRun(a, mode=mode, concurrent=concurrent)
    rb = runtime.PTRun(b, mode=mode, concurrent=concurrent)
    rb.capture()
    per = rb.graph_steps
    for it in range(4):
        ra.step(per)
        rb.replay()
        # eager work of the program between replays
        junk = b[0].energy_from_scratch()
        ra.synchronize()
        rb.synchronize()
        assert junk.isfinite().all()
        _equal(a, b)
    ra.check()
    rb.check()


def test_classes_on_streams_equal_classes_alone():
    together = _classes()
    _init(together)
    alone = _classes()
    _init(alone)
    runtime.PTRun(together, concurrent=True).step(3)
    for e in alone:
        runtime.PTRun([e]).step(3)
    torch.cuda.synchronize()
    _equal(together, alone)


@pytest.mark.parametrize("prec,L", [("fp32", 8), ("fp32", 16), ("fp64", 8), ("fp32", 24), ("fp64", 18)])
def test_sweep_variants_agree(prec, L):
    """Sites of one sublattice do not interact, so every kernel variant (tile shape,
    workgroup order, persistence) must produce the same spins bit for bit."""
    out = []
    for tune in [{"path": 3}, {"path": 4}, {"path": 1}, {"path": 2, "block_threads": 128, "replicas_per_block": 4},
                 {"path": 2, "block_threads": 256, "replicas_per_block": 2},
                 {"path": 3, "block_threads": 256}, {"path": 3, "block_threads": 1024}]:
        e = hsg.Ensemble(L, 2, 2, hsg.geometric_betas(1.0, 8.0, 3), SEED, precision=prec)
        e.init_couplings()
        e.init_spins()
        try:
            e.sweep(2, 1, 3, tuning=tune)
        except hsg.HsgError as err:
            assert err.code == 4  # unsupported instance
            continue
        torch.cuda.synchronize()
        out.append((tune, e.spins.cpu().numpy(), e.energy.cpu().numpy()))
    assert len(out) >= 3
    if L > 16:
        assert [t for t, _, _ in out if t.get("path") == 4], "wavefront path did not run"
    for tune, s, en in out[1:]:
        assert np.array_equal(s, out[0][1]), tune
        assert np.allclose(en, out[0][2], rtol=1e-12, atol=1e-9), tune


def test_autotuner_picks_supported_variant(tmp_path, monkeypatch):
    monkeypatch.setenv("HSGPT_TUNING_CACHE", str(tmp_path / "tune.json"))
    best, times = autotune.tune(8, 4, 2, 4, "fp32", reps=3)
    assert json.dumps(best, sort_keys=True) in times
    again, _ = autotune.tune(8, 4, 2, 4, "fp32")  # served from the cache
    assert again == best
    e = hsg.Ensemble(8, 4, 2, hsg.geometric_betas(1.0, 8.0, 4), SEED)
    e.init_couplings()
    e.init_spins()
    e.sweep(1, 1, 3, tuning=best)
    e.check()


def test_concurrency_autotuning_keeps_the_chain():
    """concurrent='auto' times captured cycles both ways on the run's own steps; those
    steps are real (counted), and the run then continues exactly like a run that took
    the same number of steps."""
    a = _classes()
    _init(a)
    b = _classes()
    _init(b)
    ra = runtime.PTRun(a, concurrent="auto")
    assert ra.concurrent in (False, True)
    rb = runtime.PTRun(b)
    rb.step(ra.steps_done)
    ra.step(3)
    rb.step(3)
    ra.synchronize()
    _equal(a, b)


def test_stream_groups_in_the_runtime():
    """A batch of both kinds: the streaming class on one stream beside the LDS-resident
    ones (eager steps and captured cycles) continues exactly like the classes one after
    another; concurrent='auto' also times that grouping."""
    def mixed():
        ens = runtime.uneven_batch([8, 24, 12], [2, 1, 2], [4, 4, 5], SEED)
        _init(ens)
        return ens
    a, b = mixed(), mixed()
    ra = runtime.PTRun(a, concurrent=[1, 0, 1])
    assert ra.kind_groups() == [1, 0, 1]
    rb = runtime.PTRun(b)
    ra.step(2)
    rb.step(2)
    ra.capture()
    ra.replay(5)
    rb.step(5)
    ra.synchronize()
    _equal(a, b)
    c, d = mixed(), mixed()
    rc = runtime.PTRun(c, concurrent="auto")
    assert rc.groups in (None, [1, 0, 1])
    rd = runtime.PTRun(d)
    rd.step(rc.steps_done)
    rc.step(3)
    rd.step(3)
    rc.synchronize()
    _equal(c, d)
