"""Pins of the oracle's replica exchange (paper Sec. I Eq. (1)) and round-trip
bookkeeping (paper Sec. IV.B).

* the acceptance frequency is min[1, exp(dbeta dH)];
* plain PT on the open-chain forest: per-temperature <H> equals the closed form
  at every beta (stationarity of the joint chain), and each configuration visits
  all temperatures;
* even/odd pairings touch only their pairs;
* the round-trip counter on scripted label sequences.
"""
import numpy as np
import pytest

import closed_forms as cf
import inputs
import stat_util as su
from oracle import hsgref

SEED = 0xBEEF


def test_acceptance_frequency_is_min_1_exp_delta():
    C = 6000
    betas = np.array([1.0, 1.5])
    for dH, expect in [(-2.0, np.exp(-1.0)), (-0.2, np.exp(-0.1)), (0.5, 1.0), (0.0, 1.0)]:
        ens = hsgref.RefEnsemble(2, 1, C, betas, SEED)
        ens.energy[0, :, 0] = 10.0
        ens.energy[0, :, 1] = 10.0 + dH  # H_{i+1} - H_i = dH, dbeta = 0.5
        ens.swap(0)
        acc = ens.stats[0, :, 0, 1].mean()
        assert np.all(ens.stats[0, :, 0, 0] == 1)
        assert abs(acc - expect) < 5 * np.sqrt(expect * (1 - expect) / C) + 1e-12, (dH, acc)
        swapped = ens.temp_of_slot[0, :, 0] == 1
        assert np.array_equal(swapped, ens.stats[0, :, 0, 1] == 1)
        # labels stay a permutation and the inverse map is consistent
        for c in range(0, C, 997):
            tos, sot = ens.temp_of_slot[0, c], ens.slot_of_temp[0, c]
            assert np.array_equal(sot[tos], np.arange(2))


def test_pairings_touch_only_their_pairs():
    R = 7
    ens = hsgref.RefEnsemble(2, 1, 50, hsgref.geometric_betas(1.0, 2.0, R), SEED)
    ens.energy[...] = inputs.synthetic_energies(1, 50, R, 3)
    ens.swap(1)
    assert np.all(ens.stats[0, :, 1::2, 0] == 0) and np.all(ens.stats[0, :, 0::2, 0] == 1)
    ens.swap(2)
    assert np.all(ens.stats[0, :, 1::2, 0] == 1) and np.all(ens.stats[0, :, 0::2, 0] == 1)
    assert np.all(ens.swap_ctr == 2)


def test_sequential_pairing_can_carry_a_configuration_across():
    """Ascending sequential pairs: a low-energy configuration at beta_0 can reach beta_{R-1}
    in one pass (each pair sees the labels left by the previous pair)."""
    R = 5
    ens = hsgref.RefEnsemble(2, 1, 1, hsgref.geometric_betas(1.0, 4.0, R), SEED)
    ens.energy[0, 0, :] = [-100.0, 0.0, 0.0, 0.0, 0.0]
    ens.swap(0)
    assert ens.temp_of_slot[0, 0, 0] == R - 1


@pytest.mark.slow
def test_forest_parallel_tempering_is_stationary():
    L = 4
    R = 4
    betas = hsgref.geometric_betas(0.5, 3.0, R)
    J = inputs.forest_couplings(L, 1, 80)[0]
    Jb = np.array([b[2] for b in cf.forest_bonds(L, J)])
    ens = hsgref.RefEnsemble(L, 1, 2, betas, SEED)
    ens.init_spins()
    ens.set_state(J=J[None])
    n = 8000
    Ht = np.zeros((n, 2, R))
    occ = np.zeros((2, R, R))
    for t in range(n):
        ens.sweep(1, 1, 1)
        ens.swap(0)
        _, _, e = ens.measure()
        Ht[t] = e[0] * L ** 3
        for c in range(2):
            occ[c, np.arange(R), ens.temp_of_slot[0, c]] += 1
    burn = 200
    for b in range(R):
        m, err = su.block_mean_err(Ht[burn:, :, b].mean(axis=1))
        expect = cf.forest_mean_H(betas[b], Jb)
        assert abs(m - expect) < 5 * err, (b, m, err, expect)
    acc = ens.stats[0].sum(axis=0)
    assert np.all(acc[:, 1] > 0.05 * acc[:, 0])
    frac = occ / n
    assert np.all(frac > 0.1), frac
    assert ens.rt_trips.sum() > 10


def test_round_trip_counter_scripted():
    R = 3
    tos = np.array([0, 1, 2], dtype=np.int32)
    state = np.array([1, 0, 0], dtype=np.int32)
    trips = np.zeros(3, dtype=np.int64)
    seq = [
        [1, 0, 2],  # slot1 reaches T_max -> state 1
        [2, 0, 1],  # slot0 reaches T_min
        [2, 1, 0],  # slot2 reaches T_max
        [0, 2, 1],  # slot0 back at T_max: trip; slot1 at T_min
        [1, 0, 2],  # slot1 back at T_max: trip
        [0, 1, 2],  # slot0 at T_max again without visiting T_min: no trip
    ]
    for lab in seq:
        tos[:] = lab
        hsgref.lib().hsgref_roundtrip_update(R, hsgref.i32p(tos), hsgref.i32p(state),
                                             hsgref.i64p(trips))
    assert list(trips) == [1, 1, 0]
    assert list(state) == [1, 1, 2]
