"""Checkpoint / resume: a saved ensemble reloads bit for bit (host-side, no GPU), and a
run resumed from a checkpoint continues exactly as the uninterrupted run (GPU): every
random number is addressed by counters that live in the saved state."""
import numpy as np
import pytest
import torch

import paper_1006_4247_amd as hsg
from paper_1006_4247_amd import runtime


def _fill(e, seed):
    g = torch.Generator().manual_seed(seed)
    for k in e._STATE:
        t = getattr(e, k)
        if t.dtype.is_floating_point:
            t.copy_(torch.randn(t.shape, generator=g, dtype=torch.float64).to(t.dtype))
        else:
            t.copy_(torch.randint(0, 1000, t.shape, generator=g).to(t.dtype))


def test_save_load_roundtrip_host(tmp_path):
    e = hsg.Ensemble(4, 2, 2, hsg.geometric_betas(0.5, 2.0, 5), 0xABC, precision="fp32", device="cpu",
                     sample_base=3, chain_base=6, slot_base=30, K_max=4)
    _fill(e, 1)
    e.set_schedule(np.arange(4) % 3, np.linspace(0.6, 1.9, 16).reshape(4, 4))
    path = str(tmp_path / "ens.safetensors")
    e.save(path)
    f = hsg.Ensemble.load(path, device="cpu")
    assert f.meta() == e.meta()
    for k in e._STATE + ["anneal_lambda"]:
        assert torch.equal(getattr(f, k), getattr(e, k)), k
    d, d2 = e.desc, f.desc
    assert (d2.seed, d2.sample_base, d2.chain_base, d2.slot_base, d2.anneal_K_max) == \
        (d.seed, d.sample_base, d.chain_base, d.slot_base, d.anneal_K_max)
    assert bool(d2.anneal_lambda) and f._use_lambda


def test_load_rejects_other_shape(tmp_path):
    e = hsg.Ensemble(4, 1, 2, hsg.geometric_betas(0.5, 2.0, 3), 1, device="cpu")
    path = str(tmp_path / "a.safetensors")
    e.save(path)
    other = hsg.Ensemble(6, 1, 2, hsg.geometric_betas(0.5, 2.0, 3), 1, device="cpu")
    sd = {"meta": e.meta(), "tensors": e.state_dict()["tensors"]}
    with pytest.raises(ValueError):
        other.load_state_dict(sd)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["plain", "decimate", "coolheat"])
def test_resume_is_bitwise_identical(tmp_path, mode):
    def make():
        e = hsg.Ensemble(8, 2, 2, hsg.geometric_betas(0.8, 3.0, 6), 0x5A17, precision="fp32")
        e.init_couplings()
        e.init_spins()
        return e

    a = make()
    run_a = runtime.PTRun([a], 1, 3, mode=mode, eps=0.01)
    run_a.step(7)
    prefix = str(tmp_path / "ckpt")
    run_a.save(prefix)
    run_a.step(9)
    run_a.synchronize()
    b = make()  # fresh start, then the checkpoint
    b.sweep(3, 1, 3)
    run_b = runtime.PTRun([b], 1, 3, mode=mode, eps=0.01)
    run_b.restore(prefix)
    assert run_b.parity == run_a.parity ^ (9 % 2) and run_b.steps_done == 7
    run_b.step(9)
    run_b.synchronize()
    for k in a._STATE:
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    a.check()


@pytest.mark.gpu
def test_restore_refuses_other_dynamics(tmp_path):
    """A checkpoint resumes only the run it came from: another exchange, pairing, sweep
    composition or cooling / heating parameter raises instead of silently continuing a
    different Markov chain."""
    e = hsg.Ensemble(4, 1, 2, hsg.geometric_betas(0.8, 3.0, 4), 0x5A18, precision="fp32")
    e.init_couplings()
    e.init_spins()
    run = runtime.PTRun([e], 1, 3, mode="coolheat", eps=0.01)
    run.step(2)
    prefix = str(tmp_path / "ckpt")
    run.save(prefix)
    for kw in (dict(mode="coolheat", eps=0.02), dict(mode="decimate"), dict(mode="coolheat", eps=0.01, pairing=0)):
        other = runtime.PTRun([e], 1, 3, **kw)
        with pytest.raises(ValueError):
            other.restore(prefix)
    with pytest.raises(ValueError):
        runtime.PTRun([e], 1, 5, mode="coolheat", eps=0.01).restore(prefix)
    runtime.PTRun([e], 1, 3, mode="coolheat", eps=0.01).restore(prefix)
