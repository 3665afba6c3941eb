"""Pins of the oracle's lattice, local field and Hamiltonian (paper Sec. I Eq. (2),
Sec. III.A Eq. (bigS) and the W/B split).

The local field is pinned to the Hamiltonian through S_x = -dH/ds_x (H is linear
in each spin, so a central difference is exact up to rounding); the two
sublattice sums -sum_{x in p} s_x.S_x must both equal the bond sum; H must be
invariant under global rotations and s -> -s and linear in J.
"""
import numpy as np
import pytest

import inputs
from oracle import hsgref

SIZES = [2, 4, 6]


@pytest.mark.parametrize("L", SIZES)
def test_neighbors_and_parity(L):
    N = L ** 3
    seen = {0: set(), 1: set()}
    for x in range(N):
        p = hsgref.parity(L, x)
        seen[p].add(hsgref.compressed_index(L, x))
        for d in range(6):
            y = hsgref.neighbor(L, x, d)
            assert hsgref.neighbor(L, y, d ^ 1) == x
            assert hsgref.parity(L, y) == 1 - p
    assert seen[0] == set(range(N // 2)) == seen[1]


@pytest.mark.parametrize("L", SIZES)
def test_local_field_is_minus_gradient_of_H(L):
    N = L ** 3
    J = inputs.gaussian_couplings(L, 1, 1)[0]
    s = inputs.unit_spins((), N, 2)
    for x in range(0, N, max(1, N // 17)):
        S = hsgref.local_field(L, J, s, x)
        for a in range(3):
            sp, sm = s.copy(), s.copy()
            sp[x, a] += 0.5
            sm[x, a] -= 0.5
            grad = hsgref.energy(L, J, sp) - hsgref.energy(L, J, sm)
            assert abs(S[a] + grad) < 1e-12 * max(1.0, abs(grad))


@pytest.mark.parametrize("L", SIZES)
def test_two_sublattice_energy_identity(L):
    N = L ** 3
    J = inputs.gaussian_couplings(L, 1, 3)[0]
    s = inputs.unit_spins((), N, 4)
    H = hsgref.energy(L, J, s)
    HW = hsgref.sublattice_energy(L, J, s, 0)
    HB = hsgref.sublattice_energy(L, J, s, 1)
    assert abs(H - HW) < 1e-12 * N and abs(H - HB) < 1e-12 * N


def test_energy_symmetries():
    L = 4
    N = L ** 3
    J = inputs.gaussian_couplings(L, 1, 5)[0]
    J2 = inputs.gaussian_couplings(L, 1, 6)[0]
    s = inputs.unit_spins((), N, 7)
    H = hsgref.energy(L, J, s)
    q, _ = np.linalg.qr(inputs.rng(8).standard_normal((3, 3)))
    assert abs(hsgref.energy(L, J, s @ q.T) - H) < 1e-12 * N
    assert abs(hsgref.energy(L, J, -s) - H) < 1e-12 * N
    lin = 2.5 * H - 1.5 * hsgref.energy(L, J2, s)
    assert abs(hsgref.energy(L, 2.5 * J - 1.5 * J2, s) - lin) < 1e-12 * N


def test_energy_of_aligned_state_is_minus_bond_sum():
    L = 4
    J = inputs.gaussian_couplings(L, 1, 9)[0]
    s = np.zeros((L ** 3, 3))
    s[:, 1] = 1.0
    assert abs(hsgref.energy(L, J, s) + J.sum()) < 1e-12


def test_L2_has_doubled_bonds():
    """At L = 2 the bonds (x, mu) and (x - e_mu, mu) join the same two sites and both count."""
    L = 2
    J = inputs.gaussian_couplings(L, 1, 10)[0]
    s = inputs.unit_spins((), 8, 11)
    x = 0
    S = hsgref.local_field(L, J, s, x)
    expect = np.zeros(3)
    for mu in range(3):
        y = hsgref.neighbor(L, x, 2 * mu)
        assert y == hsgref.neighbor(L, x, 2 * mu + 1)
        expect += (J[x, mu] + J[y, mu]) * s[y]
    assert np.allclose(S, expect, atol=1e-14)
