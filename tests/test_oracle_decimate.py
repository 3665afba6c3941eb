"""Pins of the oracle's decimated exchange (paper Sec. III.A, Eqs. (xxxY), (HI),
(eq:aswap)), each against something other than the oracle's own formula:

* h(u) = ln(sinh(u)/u) against quadrature of the defining integral of Eq. (HI);
* ln A = 0 exactly when the two temperatures coincide;
* ln A against brute force: each decimated spin integrated numerically over the
  unit sphere with the full Hamiltonian Eq. (2) (fields taken from energy
  differences, not from the local-field routine);
* pointwise detailed balance of the whole move (swap of the kept sublattice +
  heat-bath re-insertion) with the closed-form heat-bath density;
* stationarity of the exact equilibrium law on the open-chain forest under
  decimated exchanges alone (wrong re-insertion temperature, a wrong sign or a
  wrong sublattice all bias the energies by many standard errors);
* the sublattice role alternates along the ladder from a random first pair.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import hsgref
from tests import closed_forms as cf
from tests import inputs

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _sphere_rule(n_c=64, n_phi=64):
    """Gauss-Legendre in cos(theta) times the trapezoid rule in phi: nodes [n][3], weights
    summing to 4 pi."""
    c, wc = np.polynomial.legendre.leggauss(n_c)
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1.0 - c ** 2)
    nodes = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)),
                      np.outer(c, np.ones(n_phi))], axis=-1).reshape(-1, 3)
    w = np.outer(wc, np.full(n_phi, 2.0 * np.pi / n_phi)).reshape(-1)
    return nodes, w


def _field_from_energy(L, J, s, z):
    """S_z from H: with every spin of z's sublattice set to zero, H is linear in s_z,
    H = -s_z . S_z (every bond has one end on each sublattice)."""
    par = np.array([hsgref.parity(L, x) for x in range(L ** 3)])
    base = s.copy()
    base[par == par[z]] = 0.0
    S = np.zeros(3)
    for a in range(3):
        t = base.copy()
        t[z, a] = 1.0
        S[a] = -hsgref.energy(L, J, t)
    return S


@pytest.mark.parametrize("u", [1e-6, 1e-3, 0.1, 0.7, 1.0, 3.0, 10.0, 40.0])
def test_log_sinhc_is_the_integral_of_eq_HI(u):
    # (1/2) int_{-1}^{1} exp(u c) dc = sinh(u)/u; scaled by exp(-u) to stay finite
    val, err = integrate.quad(lambda c: np.exp(u * (c - 1.0)), -1.0, 1.0, epsabs=0, epsrel=1e-13)
    ref = u + np.log(0.5 * val)
    assert abs(hsgref.log_sinhc(u) - ref) <= 3e-13 * max(1.0, abs(ref))


def test_log_sinhc_limits():
    assert hsgref.log_sinhc(0.0) == 0.0
    for u in (1e-5, 1e-4):
        assert abs(hsgref.log_sinhc(u) - u * u / 6.0) <= 1e-15
    for u in (25.0, 100.0):  # sinh(u)/u -> e^u/(2u)
        assert abs(hsgref.log_sinhc(u) - (u - np.log(2.0 * u))) <= 1e-13 * u


def test_equal_temperatures_give_ratio_one():
    L = 4
    J = inputs.gaussian_couplings(L, 1, 5)[0]
    sp = inputs.unit_spins((2,), L ** 3, 6)
    for d in (0, 1):
        assert hsgref.decimated_log_ratio(L, J, sp[0], sp[1], d, 1.7, 1.7) == 0.0


@pytest.mark.parametrize("L,d", [(2, 0), (2, 1), (4, 0), (4, 1)])
def test_log_ratio_equals_sphere_quadrature(L, d):
    J = inputs.gaussian_couplings(L, 1, 10 + L + d)[0]
    sp = inputs.unit_spins((2,), L ** 3, 20 + L + d)
    b1, b2 = 0.8, 1.9
    nodes, w = _sphere_rule()

    def log_integral(s, z, beta):
        # ln int dOmega exp(-beta H) over s_z with the rest of z's sublattice at zero
        S = _field_from_energy(L, J, s, z)
        e = beta * nodes @ S
        m = e.max()
        return m + np.log(np.sum(w * np.exp(e - m)))

    brute = 0.0
    for z in range(L ** 3):
        if hsgref.parity(L, z) != d:
            continue
        brute += (log_integral(sp[0], z, b2) - log_integral(sp[0], z, b1)
                  + log_integral(sp[1], z, b1) - log_integral(sp[1], z, b2))
    got = hsgref.decimated_log_ratio(L, J, sp[0], sp[1], d, b1, b2)
    assert abs(got - brute) <= 1e-10 * max(1.0, abs(brute)), (got, brute)


def _log_hb_density(L, J, s_new, s_fields, d, beta):
    """ln of the heat-bath density of the parity-d spins of s_new given the other
    sublattice of s_fields: prod_z R e^{beta s.S} / (4 pi sinh R), R = beta |S|."""
    out = 0.0
    for z in range(L ** 3):
        if hsgref.parity(L, z) != d:
            continue
        S = _field_from_energy(L, J, s_fields, z)
        R = beta * np.linalg.norm(S)
        out += beta * s_new[z] @ S - np.log(4.0 * np.pi) - cf.log_sinhc(R)
    return out


@pytest.mark.parametrize("d", [0, 1])
def test_pointwise_detailed_balance(d):
    """pi(X) T(X->Y) = pi(Y) T(Y->X) for X = (c1 at b1, c2 at b2), Y = ((w2, b1') at b1,
    (w1, b2') at b2): Metropolis on the decimated weights times the re-insertion
    densities, for random configurations (log form)."""
    L = 2
    J = inputs.gaussian_couplings(L, 1, 40 + d)[0]
    par = np.array([hsgref.parity(L, x) for x in range(L ** 3)])
    b1, b2 = 0.6, 1.5
    for trial in range(5):
        c = inputs.unit_spins((4,), L ** 3, 100 * trial + d)
        c1, c2 = c[0].copy(), c[1].copy()
        # Y: kept sublattice (parity 1 - d) exchanged, decimated spins new
        y1 = np.where((par == d)[:, None], c[2], c2)
        y2 = np.where((par == d)[:, None], c[3], c1)
        lnA_X = hsgref.decimated_log_ratio(L, J, c1, c2, d, b1, b2)
        lnA_Y = hsgref.decimated_log_ratio(L, J, y1, y2, d, b1, b2)
        lhs = (-b1 * hsgref.energy(L, J, c1) - b2 * hsgref.energy(L, J, c2) + min(0.0, lnA_X)
               + _log_hb_density(L, J, y1, c2, d, b1) + _log_hb_density(L, J, y2, c1, d, b2))
        rhs = (-b1 * hsgref.energy(L, J, y1) - b2 * hsgref.energy(L, J, y2) + min(0.0, lnA_Y)
               + _log_hb_density(L, J, c1, y2, d, b1) + _log_hb_density(L, J, c2, y1, d, b2))
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs)), (trial, lhs, rhs)


def _exact_forest_samples(L, J, beta, rng):
    """Exact sample of the open-chain forest at beta: along each chain, s_0 uniform and
    s_{k+1} drawn from exp(beta J_k s_k . s) (a tree: sequential conditionals are exact)."""
    N = L ** 3
    s = np.zeros((N, 3))
    for row in range(L * L):
        x0 = row * L
        v = rng.normal(size=3)
        s[x0] = v / np.linalg.norm(v)
        for i in range(1, L):
            x = x0 + i
            a = beta * J[x - 1, 0]
            n = s[x - 1] * np.sign(a) if a != 0 else np.array([0.0, 0.0, 1.0])
            R = abs(a)
            r = rng.uniform()
            cth = 1.0 + np.log(r + (1.0 - r) * np.exp(-2.0 * R)) / R if R > 0 else 2.0 * r - 1.0
            cth = min(1.0, max(-1.0, cth))
            # orthonormal pair around n
            t = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
            e1 = np.cross(n, t)
            e1 /= np.linalg.norm(e1)
            e2 = np.cross(n, e1)
            ph = 2.0 * np.pi * rng.uniform()
            s[x] = cth * n + np.sqrt(max(0.0, 1.0 - cth * cth)) * (np.cos(ph) * e1 + np.sin(ph) * e2)
    return s


def test_forest_law_is_stationary_under_decimated_exchange():
    L, C = 4, 96
    betas = np.array([0.5, 1.0, 2.0, 4.0])
    R = len(betas)
    rng = np.random.default_rng(77)
    J = inputs.forest_couplings(L, 1, 78)[0]
    ref = hsgref.RefEnsemble(L, 1, C, betas, 0x5EED)
    spins = np.zeros((1, C, R, L ** 3, 3))
    for c in range(C):
        for r in range(R):
            spins[0, c, r] = _exact_forest_samples(L, J, betas[r], rng)
    ref.set_state(J=J[None], spins=spins)
    for t in range(60):
        ref.decimate_swap(0)
    acc = ref.stats[..., 1].sum() / ref.stats[..., 0].sum()
    assert acc > 0.2  # the exchanges really moved configurations
    Jb = np.array([b[2] for b in cf.forest_bonds(L, J)])
    for r in range(R):
        H = np.array([ref.energy[0, c, ref.slot_of_temp[0, c, r]] for c in range(C)])
        mean, var = cf.forest_mean_H(betas[r], Jb), cf.forest_var_H(betas[r], Jb)
        z = (H.mean() - mean) / np.sqrt(var / C)
        assert abs(z) < 4.0, (r, H.mean(), mean, z)
        # spread as well as location (a re-insertion at a wrong temperature also shows here)
        zv = (H.var(ddof=1) - var) / (var * np.sqrt(2.0 / (C - 1)))
        assert abs(zv) < 4.5, (r, H.var(ddof=1), var, zv)


def test_role_alternates_from_a_random_first_pair():
    L, S, C = 2, 1, 40
    betas = hsgref.geometric_betas(1.0, 2.0, 6)
    ref = hsgref.RefEnsemble(L, S, C, betas, 123)
    ref.init_couplings()
    ref.init_spins()
    firsts = []
    for call in range(3):
        n0 = ref.swap_ctr.copy()
        _, role = ref.decimate_swap(0)
        for c in range(C):
            d0 = hsgref.decimate_role(ref.seed, ref.chain_base + c, int(n0[0, c]))
            assert np.array_equal(role[0, c], (d0 + np.arange(5)) % 2)
            firsts.append(d0)
    assert 0 < np.mean(firsts) < 1
    _, role = ref.decimate_swap(1)
    assert np.all(role[..., 1::2] == -1) and np.all(role[..., 0::2] >= 0)


def test_rejected_pairs_change_nothing_and_accepted_pairs_reinsert():
    """Pairs with ln u >= ln A leave both configurations bit-identical; accepted pairs keep
    the exchanged kept sublattice bit-identical and draw the other one anew."""
    L, S, C = 4, 1, 6
    betas = hsgref.geometric_betas(0.5, 3.0, 5)
    ref = hsgref.RefEnsemble(L, S, C, betas, 99)
    ref.init_couplings()
    ref.init_spins()
    ref.sweep(3, 1, 3)
    par = np.array([hsgref.parity(L, x) for x in range(L ** 3)])
    before = ref.spins.copy()
    sot = ref.slot_of_temp.copy()
    st0 = ref.stats.copy()
    n0 = ref.swap_ctr.copy()
    _, role = ref.decimate_swap(1)  # disjoint pairs: each configuration in one pair at most
    acc = ref.stats[..., 1] - st0[..., 1]
    assert 0 < acc.sum() < acc.size
    for c in range(C):
        for i in range(0, len(betas) - 1, 2):
            x, y = sot[0, c, i], sot[0, c, i + 1]
            d = role[0, c, i]
            if acc[0, c, i]:
                keep = par != d
                assert ref.temp_of_slot[0, c, x] == i + 1 and ref.temp_of_slot[0, c, y] == i
                for slot, beta in ((x, betas[i + 1]), (y, betas[i])):
                    new, old = ref.spins[0, c, slot], before[0, c, slot]
                    assert np.array_equal(new[keep], old[keep])
                    assert abs(ref.energy[0, c, slot] - hsgref.energy(L, ref.J[0], new)) < 1e-12
                    # each decimated spin is the heat-bath draw at the new temperature from
                    # the fields of the (unchanged) kept sublattice
                    g = ref.slot_base + c * len(betas) + slot
                    for z in np.flatnonzero(~keep):
                        S = hsgref.local_field(L, ref.J[0], old, z)
                        r1, r2 = hsgref.decimate_uniforms(L, False, ref.seed, g, int(n0[0, c]), i, z)
                        want = hsgref.heatbath_spin(S, beta, r1, r2)
                        assert np.allclose(new[z], want, rtol=0, atol=1e-14), (slot, z)
            else:
                assert np.array_equal(ref.spins[0, c, x], before[0, c, x])
                assert np.array_equal(ref.spins[0, c, y], before[0, c, y])


def test_reinsertion_draws_differ_between_pairs_calls_and_slots():
    """A configuration can be re-inserted after two pairs of one ascending call: its draws
    must differ between pairs, as well as between calls and configurations."""
    for rng32 in (False, True):
        base = hsgref.decimate_uniforms(4, rng32, 5, 10, 3, 2, 7)
        for args in ((10, 3, 3, 7), (10, 4, 2, 7), (11, 3, 2, 7)):
            assert hsgref.decimate_uniforms(4, rng32, 5, *args) != base
