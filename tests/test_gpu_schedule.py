"""The learned annealing schedule on the GPU: data from the method's own annealed
exchanges, surrogate trained with the project's kernels, per-pair protocols chosen
to maximise accepted exchanges per unit of sweep work (or, at the L = 32 workload, the
least predicted GPU time per round trip), frozen for a production segment.  The first
test shows what the network gains over the method without it: the fallback (linear
protocol, the same K for every pair) and a single protocol length for all pairs, at
L = 8, 16 samples x 2 chains x 12 temperatures, beta geometric 1..8 (plain exchange
acceptance ~0.01 on this ladder); the second runs the schedule at its own workload and
checks the chosen protocols against the oracle."""
import numpy as np
import pytest
import torch

import paper_1006_4247_amd as hsg
from paper_1006_4247_amd import schedule as sch

pytestmark = pytest.mark.gpu
K_GRID = [1, 2, 3, 4, 6, 8, 12, 16]


def _production(ens, K, G, steps):
    ens.set_schedule(K, sch.protocol(ens.betas_host, K, G, ens.K_max))
    st0 = ens.swap_stats.cpu().numpy().copy()
    for t in range(steps):
        ens.sweep(1, 1, 3)
        ens.anneal_swap(t % 2)
    torch.cuda.synchronize()
    st = ens.swap_stats.cpu().numpy() - st0
    acc = st[..., 1].sum(axis=(0, 1)) / np.maximum(st[..., 0].sum(axis=(0, 1)), 1)
    return acc, sch.ladder_efficiency(acc, K)


def test_learned_schedule_beats_the_fixed_fallback():
    L, S, C, R = 8, 16, 2, 12
    betas = hsg.geometric_betas(1.0, 8.0, R)
    ens = hsg.Ensemble(L, S, C, betas, 0xABCD, precision="fp32", K_max=16)
    ens.init_couplings()
    ens.init_spins()
    ens.sweep(200, 1, 3)
    rng = np.random.default_rng(0)
    x, y, w = sch.generate_data(ens, 200, K_GRID, rng)
    n = len(x)
    idx = rng.permutation(n)
    tr, te = idx[: int(0.8 * n)], idx[int(0.8 * n):]
    net, loss = sch.train(x[tr], y[tr], w[tr], steps=3000)
    p = sch.predict(net, x[te])
    r2 = 1 - np.sum((p - y[te]) ** 2) / np.sum((y[te] - y[te].mean()) ** 2)
    assert r2 > 0.7, r2
    _, _, e = ens.measure()
    ebar = e.mean(dim=(0, 1)).cpu().numpy()  # running means of the previous segment
    K, G, pred = sch.select_schedule(net, betas, ebar, L, K_GRID)
    acc_l, eff_l = _production(ens, K, G, 600)
    acc_f, eff_f = _production(ens, *sch.fixed_schedule(R, 4), 600)
    eff_u = {k: _production(ens, *sch.fixed_schedule(R, k), 600)[1] for k in (1, 8, 16)}
    ens.check()
    assert eff_l > 1.08 * eff_f, (eff_l, eff_f)          # beats the fallback K = 4
    assert eff_l > 2.0 * eff_u[1], (eff_l, eff_u)         # and a plain-like K = 1
    assert eff_l > 0.93 * max(eff_u.values()), (eff_l, eff_u)  # about as good as the best uniform K
    # no pair blocks the ladder: the selection keeps every predicted acceptance at
    # or above 0.05, and the surrogate's prediction error on single pairs is ~0.01-0.02
    # (plain exchange on this ladder accepts ~0.01 at the cold end)
    assert acc_l.min() >= 0.03, acc_l


def test_learned_schedule_at_its_workload_shape():
    """The learned schedule at its own workload (L = 32, 16 samples x 2 chains x 10
    temperatures, beta geometric 1..8, FP32): data generated on that ensemble with the
    project's kernels, protocols chosen for the least predicted GPU time per round trip
    from the measured cost of a step and of an annealing sweep, a production segment
    with them on the full ensemble; then one annealed exchange of each parity with the
    chosen protocols against the oracle on one sample (both chains), pair by pair."""
    from gpu_pair import anneal_and_check, make_pair

    L, S, C, R = 32, 16, 2, 10
    betas = hsg.geometric_betas(1.0, 8.0, R)
    grid = [0, 1, 2, 4, 8, 16, 32]
    leg = (1, 1)
    ens = hsg.Ensemble(L, S, C, betas, 0x3232, precision="fp32", K_max=32)
    ens.init_couplings()
    ens.init_spins()
    ens.sweep(30, 1, 3)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step_ms(K):
        ens.set_schedule(np.full(R - 1, K, np.int32))
        ev[0].record()
        for t in range(6):
            ens.sweep(1, 1, 3)
            ens.anneal_swap(t % 2, *leg)
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / 6

    t_base = step_ms(0)
    t_leg = max((step_ms(8) - t_base) / (8 * (R - 1) / 2.0), 1e-6)
    rng = np.random.default_rng(3)
    x, y, w = sch.generate_data(ens, 16, grid, rng, leg=leg)
    net, _ = sch.train(x, y, w, steps=1500)
    _, _, e = ens.measure()
    ebar = e.mean(dim=(0, 1)).cpu().numpy()
    K, G, pred = sch.select_schedule_round_trips(net, betas, ebar, L, grid, t_base, t_leg)
    assert np.all((K >= 0) & (K <= 32)), K
    lam = sch.protocol(betas, K, G, 32)
    for i in range(R - 1):
        pts = lam[i, : K[i]]
        assert np.all(np.diff(pts) > 0) and np.all(pts > betas[i]) and np.all(pts < betas[i + 1]), (i, pts)
    # production with the chosen protocols on the full ensemble
    ens.set_schedule(K, lam)
    st0 = ens.swap_stats.cpu().numpy().copy()
    for t in range(40):
        ens.sweep(1, 1, 3)
        ens.anneal_swap(t % 2, *leg)
    torch.cuda.synchronize()
    st = ens.swap_stats.cpu().numpy() - st0
    assert st[..., 0].sum() > 0
    ens.check()
    # oracle parity of the chosen protocols, one sample with two chains
    gpu, ref = make_pair(L, 1, 2, betas, 0x3233, prec="fp32", K_max=32)
    gpu.sweep(3, 1, 3)
    torch.cuda.synchronize()
    for parity in (0, 1):
        n_dec, n_cmp, worst = anneal_and_check(gpu, ref, parity, K, lam, *leg,
                                               what="L=32 learned protocols parity %d" % parity)
        print("[parity] L=32 learned K=%s parity %d: %d pairs, %d decisions compared, p99 / bar %.3f"
              % (list(K), parity, n_dec, n_cmp, worst), flush=True)
    gpu.check()
