"""Statistical parity of the GPU path.

* Open-chain forest on the GPU: per-temperature <H> and <chi> of plain and annealed PT
  equal their closed forms (tests/closed_forms.py), FP64 and FP32 - a check of the
  whole GPU chain (sweeps, exchange, annealing, measurement) against mathematics.
* Long runs at the shape of the small FP64 workload (L = 4, 2 chains, 8 temperatures,
  beta geometric 1..6, 1 HB + 3 OR + exchange every step): per-temperature energy
  density and overlap susceptibility of the GPU agree with the oracle's (different
  random streams, same couplings) within 3 sigma of the block-jackknife errors.
* The same comparison for binary32 spins at L = 8 (beta geometric 0.5..3, where
  these runs equilibrate): the GPU's FP32 chains against the FP64 oracle's.
"""
import numpy as np
import pytest
import torch

import closed_forms as cf
import inputs
import stat_util as su
from oracle import hsgref

import paper_1006_4247_amd as hsg
from paper_1006_4247_amd import runtime

pytestmark = pytest.mark.gpu


def _replicated(L, S, C, betas, seed, prec, J, K_max=0):
    e = hsg.Ensemble(L, S, C, betas, seed, precision=prec, K_max=K_max)
    e.init_spins()
    e.set_couplings_natural(np.broadcast_to(J, (S,) + J.shape))
    e.energy_from_scratch(out=e.energy)
    return e


@pytest.mark.parametrize("prec,mode", [("fp64", "plain"), ("fp32", "plain"), ("fp32", "anneal")])
def test_forest_closed_forms_on_gpu(prec, mode):
    L, S, C = 4, 64, 2
    betas = np.array([0.7, 1.6, 3.0])
    J = inputs.forest_couplings(L, 1, 101)[0]
    if prec == "fp32":
        J = J.astype(np.float32).astype(np.float64)
    Jb = np.array([b[2] for b in cf.forest_bonds(L, J)])
    e = _replicated(L, S, C, betas, 0xF0 + len(prec), prec, J, K_max=2)
    if mode == "anneal":
        e.set_schedule(np.array([2, 2], dtype=np.int32))
    n, burn = 3000, 300
    run = runtime.PTRun([e], n_hb=1, n_or=1, mode=mode, series_len=n)
    run.step(n)
    chi, et = run.series(0)  # [T][S][R], [T][S][C][R]
    run.check()
    H = et[burn:] * L ** 3
    for b, beta in enumerate(betas):
        m, err = su.block_mean_err(H[:, :, :, b].mean(axis=(1, 2)))
        expect = cf.forest_mean_H(beta, Jb)
        assert abs(m - expect) < 5 * err, (b, m, err, expect)
        mc, ec = su.block_mean_err(chi[burn:, :, b].mean(axis=1))
        cexp = cf.forest_chi(L, J, beta)
        assert abs(mc - cexp) < 5 * ec, (b, mc, ec, cexp)
    acc = e.swap_stats.cpu().numpy().sum(axis=(0, 1))
    assert np.all(acc[:, 1] > 0)


def _long_run_compare(L, R, betas, prec, n, burn, S_gpu, S_ref, seeds):
    ref0 = hsgref.RefEnsemble(L, 1, 2, betas, seeds[0], prec="fp64")
    ref0.init_couplings()
    J = ref0.J[0].copy()
    if prec == "fp32":
        J = J.astype(np.float32).astype(np.float64)
    C = 2
    # GPU: S_gpu replicas of the same coupling set (independent streams)
    g = _replicated(L, S_gpu, C, betas, seeds[1], prec, J)
    run = runtime.PTRun([g], n_hb=1, n_or=3, series_len=n)
    run.step(n)
    chi_g, e_g = run.series(0)
    run.check()
    # oracle (FP64): S_ref replicas of the same coupling set, other seed
    ref = hsgref.RefEnsemble(L, S_ref, C, betas, seeds[2], prec="fp64")
    ref.init_spins()
    ref.set_state(J=np.broadcast_to(J, (S_ref,) + J.shape))
    chi_r = np.zeros((n, S_ref, R))
    e_r = np.zeros((n, S_ref, C, R))
    for t in range(n):
        ref.sweep(1, 1, 3)
        ref.swap(0)
        _, chi_r[t], e_r[t] = ref.measure()
    z = []
    for b in range(R):
        for name, xg, xr in [("e", e_g[burn:, :, :, b].mean(axis=(1, 2)), e_r[burn:, :, :, b].mean(axis=(1, 2))),
                             ("chi", chi_g[burn:, :, b].mean(axis=1), chi_r[burn:, :, b].mean(axis=1))]:
            mg, sg = su.jackknife_mean_err(xg)
            mr, sr = su.jackknife_mean_err(xr)
            zz = (mg - mr) / np.sqrt(sg ** 2 + sr ** 2)
            print("L=%d %s %s beta_%d gpu %.6f +- %.6f oracle %.6f +- %.6f z %+.2f" % (
                L, prec, name, b, mg, sg, mr, sr, zz), flush=True)
            assert abs(zz) < 3.0, (name, b, mg, sg, mr, sr)
            z.append(zz)
    z = np.array(z)
    # the combined chi-square of the 2R comparisons stays plausible
    assert np.sum(z ** 2) < 2 * R + 6 * np.sqrt(4 * R), np.sum(z ** 2)


def test_long_run_matches_oracle():
    R = 8
    _long_run_compare(4, R, hsgref.geometric_betas(1.0, 6.0, R), "fp64", 1500, 300, 32, 8,
                      (0x1006, 0x2006, 0x3006))


def test_long_run_fp32_l8_matches_oracle():
    """FP32 spins (FP64 energies and observables) at L = 8 against the FP64 oracle."""
    R = 8
    _long_run_compare(8, R, hsgref.geometric_betas(0.5, 3.0, R), "fp32", 2000, 400, 32, 8,
                      (0x1008, 0x2008, 0x3008))
