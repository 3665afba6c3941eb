"""Pins of the oracle's annealed (nonequilibrium-switch) replica exchange, the
prior-art variant cited in the paper's Sec. I (Opps & Schofield; Ballard &
Jarzynski), in the protocol the oracle states.

* K = 0 reproduces the plain exchange of Eq. (1) bit for bit;
* the work of a leg at K = 0 is (b - a) H(x) up and (a - b) H(y) down;
* an explicit protocol table equal to the linear one changes nothing;
* a rejected exchange leaves both configurations as they were; counters advance by K;
* Jarzynski's equality on the open-chain forest: <exp(-W_up)> = Z(b)/Z(a)
  with the closed-form ln Z;
* annealed PT on the forest is stationary: per-temperature <H> equals the
  closed form at every beta.
"""
import numpy as np
import pytest

import closed_forms as cf
import inputs
import stat_util as su
from oracle import hsgref

SEED = 0xA11EA1


def _ensemble(L, C, betas, J=None, seed=SEED, prec="fp64"):
    ens = hsgref.RefEnsemble(L, 1, C, betas, seed, prec=prec)
    if J is None:
        ens.init_couplings()
        ens.init_spins()
    else:
        ens.init_spins()
        ens.set_state(J=J[None])
    return ens


@pytest.mark.parametrize("parity", [0, 1])
def test_K0_is_plain_swap(parity):
    L, C, R = 4, 3, 6
    betas = hsgref.geometric_betas(0.5, 3.0, R)
    a = _ensemble(L, C, betas)
    b = _ensemble(L, C, betas)
    for _ in range(5):
        a.sweep(1, 1, 3)
        b.sweep(1, 1, 3)
        a.swap(parity + 1)
        w = b.anneal_swap(parity, np.zeros(R - 1, dtype=np.int32))
        for name in ["spins", "temp_of_slot", "slot_of_temp", "stats", "rt_state", "rt_trips",
                     "sweep_ctr", "swap_ctr", "energy"]:
            assert np.array_equal(getattr(a, name), getattr(b, name)), name
    # K = 0 works: (b - a) H(x) and (a - b) H(y)
    e_before = b.energy.copy()
    sot = b.slot_of_temp.copy()
    w = b.anneal_swap(parity, np.zeros(R - 1, dtype=np.int32))
    for c in range(C):
        for i in range(parity, R - 1, 2):
            x, y = sot[0, c, i], sot[0, c, i + 1]
            dB = betas[i + 1] - betas[i]
            assert w[0, c, i, 0] == dB * e_before[0, c, x]
            assert w[0, c, i, 1] == -dB * e_before[0, c, y]


def test_protocol_table_equal_to_linear_changes_nothing():
    L, C, R = 4, 2, 5
    betas = hsgref.geometric_betas(0.5, 3.0, R)
    K = np.array([3, 3, 2, 3], dtype=np.int32)
    lam = np.zeros((R - 1, 3))
    for i in range(R - 1):
        for k in range(1, K[i] + 1):
            lam[i, k - 1] = betas[i] + k * (betas[i + 1] - betas[i]) / (K[i] + 1)
    a = _ensemble(L, C, betas)
    b = _ensemble(L, C, betas)
    wa = a.anneal_swap(0, K)
    wb = b.anneal_swap(0, K, lam)
    assert np.array_equal(wa, wb)
    assert np.array_equal(a.spins, b.spins)


def test_reject_restores_and_counters_advance():
    L, C, R = 4, 8, 3
    betas = np.array([0.3, 2.0, 6.0])
    ens = _ensemble(L, C, betas)
    for _ in range(3):
        ens.sweep(1, 1, 3)
    before = ens.spins.copy()
    sot = ens.slot_of_temp.copy()
    ctr = ens.sweep_ctr.copy()
    K = np.array([4, 4], dtype=np.int32)
    ens.anneal_swap(0, K)
    acc = ens.stats[0, :, 0, 1]
    for c in range(C):
        x, y = sot[0, c, 0], sot[0, c, 1]
        z = sot[0, c, 2]
        assert ens.sweep_ctr[0, c, x] == ctr[0, c, x] + 4
        assert ens.sweep_ctr[0, c, y] == ctr[0, c, y] + 4
        assert ens.sweep_ctr[0, c, z] == ctr[0, c, z]  # idle in this phase
        assert np.array_equal(ens.spins[0, c, z], before[0, c, z])
        if acc[c] == 0:
            assert np.array_equal(ens.spins[0, c, x], before[0, c, x])
            assert np.array_equal(ens.spins[0, c, y], before[0, c, y])
        else:
            assert not np.array_equal(ens.spins[0, c, x], before[0, c, x])
            assert ens.temp_of_slot[0, c, x] == 1 and ens.temp_of_slot[0, c, y] == 0
        for q in range(R):
            assert abs(ens.energy[0, c, q] - hsgref.energy(L, ens.J[0], ens.spins[0, c, q])) < 1e-9


@pytest.mark.slow
def test_jarzynski_on_forest():
    L = 4
    a, b = 1.0, 1.6
    J = inputs.forest_couplings(L, 1, 90)[0]
    Jb = np.array([x[2] for x in cf.forest_bonds(L, J)])
    C = 64
    ens = _ensemble(L, C, np.array([a, b]), J=J)
    for _ in range(50):
        ens.sweep(1, 1, 1)
    Wup, Wdn = [], []
    for _ in range(120):
        ens.sweep(2, 1, 1)
        w = ens.anneal_swap(0, np.array([3], dtype=np.int32), n_hb=1, n_or=1)
        Wup.append(w[0, :, 0, 0].copy())
        Wdn.append(w[0, :, 0, 1].copy())
    Wup = np.concatenate(Wup)
    Wdn = np.concatenate(Wdn)
    dlnZ = cf.forest_log_Z(b, Jb) - cf.forest_log_Z(a, Jb)
    for W, expect in [(Wup, dlnZ), (Wdn, -dlnZ)]:
        ew = np.exp(-W)
        m, e = su.block_mean_err(ew)
        assert abs(np.log(m) - expect) < 5 * e / m, (np.log(m), e / m, expect)
    # Jensen (second law): <W_up> >= -ln(Z(b)/Z(a)) and <W_dn> >= +ln(Z(b)/Z(a))
    assert Wup.mean() >= -dlnZ - 0.05 and Wdn.mean() >= dlnZ - 0.05


@pytest.mark.slow
def test_forest_annealed_tempering_is_stationary():
    L = 4
    R = 4
    betas = hsgref.geometric_betas(0.5, 4.0, R)
    J = inputs.forest_couplings(L, 1, 91)[0]
    Jb = np.array([x[2] for x in cf.forest_bonds(L, J)])
    ens = _ensemble(L, 2, betas, J=J)
    n = 3000
    Ht = np.zeros((n, 2, R))
    K = np.full(R - 1, 2, dtype=np.int32)
    for t in range(n):
        ens.sweep(1, 1, 1)
        ens.anneal_swap(t % 2, K, n_hb=1, n_or=1)
        Ht[t] = ens.measure()[2][0] * L ** 3
    burn = 100
    for bidx in range(R):
        m, err = su.block_mean_err(Ht[burn:, :, bidx].mean(axis=1))
        expect = cf.forest_mean_H(betas[bidx], Jb)
        assert abs(m - expect) < 5 * err, (bidx, m, err, expect)
    st = ens.stats[0].sum(axis=0)
    assert np.all(st[:, 1] > 0)


def test_down_leg_inverts_up_leg_for_overrelaxation_sweeps():
    """With overrelaxation only, a sweep is a product of involutions, so its adjoint
    (the reversed product) is its inverse.  Two accepted exchanges of the same pair
    (nearly equal betas, so acceptance ~ 1) must return both configurations to their
    starting states: the down-leg undoes the up-leg."""
    L, C = 4, 4
    betas = np.array([1.0, 1.0 + 1e-12])
    ens = _ensemble(L, C, betas)
    ens.sweep(2, 1, 3)
    start = ens.spins.copy()
    K = np.array([3], dtype=np.int32)
    ens.anneal_swap(0, K, n_hb=0, n_or=2)
    assert np.all(ens.stats[0, :, 0, 1] == 1)
    assert not np.allclose(ens.spins, start)
    ens.anneal_swap(0, K, n_hb=0, n_or=2)
    assert np.all(ens.stats[0, :, 0, 1] == 2)
    assert np.allclose(ens.spins, start, atol=1e-11)
