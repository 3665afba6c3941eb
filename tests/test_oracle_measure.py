"""Pins of the oracle's measurements (paper Sec. II): overlap q_{ab,x} between the
two chains at one temperature, chi = (1/N) sum_ab (sum_x q_ab,x)^2, and the energy
per site e = H/N (the paper's E is -e).

Closed forms: aligned and orthogonal uniform states, chi invariance under a global
rotation of one replica, <chi> = 1 at beta = 0 (independent uniform spins).
"""
import numpy as np

import inputs
import stat_util as su
from oracle import hsgref


def _ens(L, R=2):
    ens = hsgref.RefEnsemble(L, 1, 2, np.linspace(0.5, 1.0, R), 7)
    ens.init_couplings()
    return ens


def test_aligned_and_orthogonal_states():
    L = 4
    N = L ** 3
    ens = _ens(L)
    ens.spins[0, 0, :, :, :] = [1.0, 0.0, 0.0]
    ens.spins[0, 1, 0, :, :] = [1.0, 0.0, 0.0]
    ens.spins[0, 1, 1, :, :] = [0.0, 1.0, 0.0]
    ens.compute_energy()
    Q, chi, e = ens.measure()
    expect0 = np.zeros((3, 3))
    expect0[0, 0] = N
    expect1 = np.zeros((3, 3))
    expect1[0, 1] = N
    assert np.array_equal(Q[0, 0], expect0) and np.array_equal(Q[0, 1], expect1)
    assert chi[0, 0] == N and chi[0, 1] == N
    assert np.allclose(e[0, 0, 0], -ens.J[0].sum() / N)


def test_measure_follows_temperature_labels():
    L = 2
    ens = _ens(L, R=3)
    ens.init_spins()
    ens.compute_energy()
    ens.temp_of_slot[0, 1] = [2, 0, 1]
    ens.slot_of_temp[0, 1] = [1, 2, 0]
    Q, chi, e = ens.measure()
    for b in range(3):
        s1 = ens.spins[0, 0, b]
        s2 = ens.spins[0, 1, ens.slot_of_temp[0, 1, b]]
        assert np.allclose(Q[0, b], s1.T @ s2, atol=1e-13)
        assert e[0, 1, b] == ens.energy[0, 1, ens.slot_of_temp[0, 1, b]] / 8


def test_chi_invariant_under_rotation_of_one_replica():
    L = 4
    ens = _ens(L)
    ens.init_spins()
    ens.compute_energy()
    _, chi, _ = ens.measure()
    q, _ = np.linalg.qr(inputs.rng(3).standard_normal((3, 3)))
    ens.spins[0, 1] = ens.spins[0, 1] @ q.T
    _, chi2, _ = ens.measure()
    assert np.allclose(chi, chi2, rtol=1e-12)


def test_chi_is_one_at_beta_zero():
    L = 4
    ens = hsgref.RefEnsemble(L, 1, 2, [0.0], 11)
    ens.init_couplings()
    ens.init_spins()
    vals = []
    for _ in range(3000):
        ens.sweep(1, 1, 0)
        vals.append(ens.measure()[1][0, 0])
    m, e = su.block_mean_err(np.array(vals))
    assert abs(m - 1.0) < 5 * e, (m, e)
