"""Pins of the oracle's checkerboard sweeps (paper Sec. III.A W/B split, Sec. III.C
heat-bath and overrelaxation, hybrid sweep).

* a half-sweep's result does not depend on the order of the sites (sites of one
  sublattice do not interact), bit for bit;
* overrelaxation half-sweeps conserve H; every sweep keeps unit spins;
* beta = 0: <H> = 0 and Var(H) = sum_b J_b^2 / 3;
* small beta: <H> = -(beta/3) sum_b J_b^2 + O(beta^3);
* open-chain forest: <H>, Var(H) and <chi> equal their closed forms at any beta.
"""
import numpy as np
import pytest

import closed_forms as cf
import inputs
import stat_util as su
from oracle import hsgref

SEED = 0x1234


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("par", [0, 1])
@pytest.mark.parametrize("L", [2, 4, 6])
def test_halfsweep_is_order_independent(L, par, kind):
    N = L ** 3
    J = inputs.gaussian_couplings(L, 1, 40 + L)[0]
    s0 = inputs.unit_spins((), N, 50 + L)
    a = s0.copy()
    hsgref.halfsweep(L, J, a, par, kind, 1.7, SEED, 3, 5, par)
    sites = np.array([x for x in range(N) if hsgref.parity(L, x) == par], dtype=np.int32)
    for rep in range(3):
        order = inputs.rng(rep).permutation(sites).astype(np.int32)
        b = s0.copy()
        hsgref.halfsweep(L, J, b, par, kind, 1.7, SEED, 3, 5, par, order=order)
        assert np.array_equal(a, b)
    # the other sublattice is untouched
    other = np.array([hsgref.parity(L, x) != par for x in range(N)])
    assert np.array_equal(a[other], s0[other])


@pytest.mark.parametrize("rng32", [False, True])
def test_overrelaxation_conserves_energy_and_norm(rng32):
    L = 6
    N = L ** 3
    J = inputs.gaussian_couplings(L, 1, 60)[0]
    s = inputs.unit_spins((), N, 61)
    H0 = hsgref.energy(L, J, s)
    for par in [0, 1, 0, 1, 1]:
        hsgref.halfsweep(L, J, s, par, 1, 2.0, SEED, 0, 0, 0, rng32)
        assert abs(hsgref.energy(L, J, s) - H0) < 1e-11 * N
    hsgref.sweep(L, J, s, 1, 3, 2.0, SEED, 1, 1, rng32=rng32)
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-13)
    assert hsgref.energy(L, J, s) != H0


def test_adjoint_sweep_reverses_half_sweeps():
    """F* applies the same half-sweeps as F in reverse order."""
    L = 4
    N = L ** 3
    J = inputs.gaussian_couplings(L, 1, 62)[0]
    s0 = inputs.unit_spins((), N, 63)
    a = s0.copy()
    hsgref.sweep(L, J, a, 1, 2, 1.3, SEED, 7, 9, adjoint=True)
    b = s0.copy()
    for par, kind, hs in [(1, 1, 0), (0, 1, 0), (1, 1, 0), (0, 1, 0), (1, 0, 1), (0, 0, 0)]:
        hsgref.halfsweep(L, J, b, par, kind, 1.3, SEED, 7, 9, hs)
    assert np.array_equal(a, b)


def _run(L, J, beta, n_sweeps, n_hb=1, n_or=3, C=1, rng32=False, measure=False):
    ens = hsgref.RefEnsemble(L, 1, C, [beta], SEED, prec="fp32" if rng32 else "fp64")
    ens.init_spins()
    ens.set_state(J=J[None])
    H = np.zeros((n_sweeps, C))
    chi = np.zeros(n_sweeps)
    for t in range(n_sweeps):
        ens.sweep(1, n_hb, n_or)
        H[t] = ens.energy[0, :, 0]
        if measure:
            chi[t] = ens.measure()[1][0, 0]
    return H, chi


def test_beta_zero_energy_moments():
    L = 4
    J = inputs.gaussian_couplings(L, 1, 70)[0]
    H, _ = _run(L, J, 0.0, 6000, n_hb=1, n_or=0)
    h = H[:, 0]
    var_expect = np.sum(J ** 2) / 3.0
    assert abs(h.mean()) < 5 * np.sqrt(var_expect / h.size)
    assert abs(h.var() - var_expect) < 6 * np.sqrt(2.0 / h.size) * var_expect


def test_high_temperature_slope():
    L = 4
    beta = 0.05
    J = inputs.gaussian_couplings(L, 1, 71)[0]
    H, _ = _run(L, J, beta, 8000)
    m, e = su.block_mean_err(H[:, 0])
    expect = -(beta / 3.0) * np.sum(J ** 2)
    assert abs(m - expect) < 5 * e + abs(expect) * 0.01, (m, e, expect)


@pytest.mark.slow
@pytest.mark.parametrize("beta,rng32", [(1.5, False), (4.0, False), (2.0, True)])
def test_forest_closed_forms(beta, rng32):
    L = 4
    J = inputs.forest_couplings(L, 1, 72)[0]
    Jb = np.array([b[2] for b in cf.forest_bonds(L, J)])
    n = 12000
    H, chi = _run(L, J, beta, n, C=2, rng32=rng32, measure=True)
    burn = 200
    h = H[burn:].ravel()
    mH, eH = su.block_mean_err(H[burn:].mean(axis=1))
    assert abs(mH - cf.forest_mean_H(beta, Jb)) < 5 * eH, (mH, eH, cf.forest_mean_H(beta, Jb))
    vH, evH = su.block_var_err(H[burn:, 0])
    assert abs(vH - cf.forest_var_H(beta, Jb)) < 5 * evH, (vH, evH)
    mC, eC = su.block_mean_err(chi[burn:])
    cexp = cf.forest_chi(L, J, beta)
    assert abs(mC - cexp) < 5 * eC, (mC, eC, cexp)
    assert h.size > 0


def test_forest_detects_wrong_sign():
    """Sanity of the pin itself: the closed form at -beta is far from the run at beta."""
    L = 4
    beta = 1.5
    J = inputs.forest_couplings(L, 1, 72)[0]
    Jb = np.array([b[2] for b in cf.forest_bonds(L, J)])
    H, _ = _run(L, J, beta, 2000)
    mH, eH = su.block_mean_err(H[100:, 0])
    assert abs(mH - cf.forest_mean_H(-beta, Jb)) > 20 * eH
