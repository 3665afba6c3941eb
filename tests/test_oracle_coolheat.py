"""Pins of the oracle's cooling / heating exchange (paper Sec. III.B), each against
something other than the oracle's own formulas:

* the single-site map turns s towards S by alpha = eps |S| sin(theta), in the plane
  of s and S (geometry computed independently);
* heating inverts cooling (site and lattice), with the same log Jacobian;
* the Jacobian of the site map by the change-of-variables identity on the sphere,
  int g(f(s)) det J_f(s) dOmega = int g dOmega, with quadrature;
* the Jacobian of the lattice map by finite differences of the whole map (L = 2,
  16 tangent coordinates), so the two-sublattice composition is checked too;
* eps = 0 is the plain exchange of Eq. (1), bit for bit;
* ln A(T z) = -ln A(z) for the involution T (x, y) -> (C^-1 y, C x): the Jacobian is
  the involution's (a Jacobian taken at the untransformed state fails this);
* the exact open-chain forest law is stationary under cooling / heating exchanges.
"""
import numpy as np
import pytest

from oracle import hsgref
from tests import closed_forms as cf
from tests import inputs
from tests.test_oracle_decimate import _exact_forest_samples, _sphere_rule

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rand_unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_cooling_turns_towards_the_field_by_alpha():
    rng = np.random.default_rng(1)
    for _ in range(200):
        s = _rand_unit(rng, 1)[0]
        S = rng.normal(size=3) * rng.uniform(0.1, 5.0)
        eps = rng.uniform(0.0, 0.9) / np.linalg.norm(S)
        out, _ = hsgref.cool_spin(s, S, eps)
        n = S / np.linalg.norm(S)
        th = np.arctan2(np.linalg.norm(np.cross(s, n)), s @ n)
        thp = np.arctan2(np.linalg.norm(np.cross(out, n)), out @ n)
        assert abs(np.linalg.norm(out) - 1.0) < 1e-14
        assert abs(thp - (th - eps * np.linalg.norm(S) * np.sin(th))) < 1e-12
        assert abs(np.linalg.det(np.stack([s, out, n]))) < 1e-12  # coplanar


def test_heating_inverts_cooling_sites_and_poles():
    rng = np.random.default_rng(2)
    S = np.array([0.3, -1.2, 2.0])
    n = S / np.linalg.norm(S)
    spins = list(_rand_unit(rng, 300)) + [n, -n]
    for eps in (0.0, 0.05, 0.2, 0.99 / np.linalg.norm(S)):
        for s in spins:
            c, ld = hsgref.cool_spin(s, S, eps)
            b, ld2 = hsgref.heat_spin(c, S, eps)
            assert np.abs(b - s).max() < 1e-12
            assert abs(ld - ld2) < 1e-12
    k = 0.7
    for s in (n, -n):  # poles: det -> (1 - k cos(theta))^2
        _, ld = hsgref.cool_spin(s, S, k / np.linalg.norm(S))
        assert abs(ld - 2.0 * np.log(1.0 - k * (s @ n))) < 1e-12
    # zero field: identity
    out, ld = hsgref.cool_spin(spins[0], np.zeros(3), 0.3)
    assert np.array_equal(out, spins[0]) and ld == 0.0
    # not a bijection beyond k = 1
    assert np.isnan(hsgref.cool_spin(spins[0], S, 1.01 / np.linalg.norm(S))[1])


@pytest.mark.parametrize("k", [0.05, 0.3, 0.8])
def test_site_jacobian_by_change_of_variables(k):
    nodes, w = _sphere_rule(96, 96)
    S = np.array([0.4, 0.9, -1.7])
    eps = k / np.linalg.norm(S)
    mapped = np.zeros_like(nodes)
    ld = np.zeros(len(nodes))
    for j, s in enumerate(nodes):
        mapped[j], ld[j] = hsgref.cool_spin(s, S, eps)
    rng = np.random.default_rng(3)
    for _ in range(3):
        a = rng.normal(size=3) * 1.5
        g = lambda v: np.exp(v @ a) + (v[:, 0] ** 2) * v[:, 2]
        lhs = np.sum(w * g(mapped) * np.exp(ld))
        rhs = np.sum(w * g(nodes))
        assert abs(lhs - rhs) <= 2e-9 * abs(rhs), (lhs, rhs)


def _tangent_basis(v):
    t = np.array([1.0, 0.0, 0.0]) if abs(v[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(v, t)
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(v, e1)


def test_lattice_jacobian_by_finite_differences():
    L, N = 2, 8
    J = inputs.gaussian_couplings(L, 1, 7)[0]
    s0 = inputs.unit_spins((1,), N, 8)[0]
    eps = 0.08
    out0 = s0.copy()
    ld = hsgref.coolheat(L, J, out0, eps, False)
    basis_in = [_tangent_basis(v) for v in s0]
    basis_out = [_tangent_basis(v) for v in out0]
    h = 1e-6
    M = np.zeros((2 * N, 2 * N))
    for col in range(2 * N):
        site, d = divmod(col, 2)
        cols = []
        for sgn in (+1, -1):
            s = s0.copy()
            v = s[site] + sgn * h * basis_in[site][d]
            s[site] = v / np.linalg.norm(v)
            hsgref.coolheat(L, J, s, eps, False)
            cols.append(s)
        ds = (cols[0] - cols[1]) / (2 * h)
        for site2 in range(N):
            M[2 * site2, col] = ds[site2] @ basis_out[site2][0]
            M[2 * site2 + 1, col] = ds[site2] @ basis_out[site2][1]
    assert abs(np.log(abs(np.linalg.det(M))) - ld) < 1e-6, (np.log(abs(np.linalg.det(M))), ld)


def test_lattice_heating_inverts_cooling():
    L = 4
    J = inputs.gaussian_couplings(L, 1, 9)[0]
    s = inputs.unit_spins((1,), L ** 3, 10)[0]
    c = s.copy()
    ld = hsgref.coolheat(L, J, c, 0.02, False)
    assert hsgref.energy(L, J, c) < hsgref.energy(L, J, s)  # cooling lowers H
    b = c.copy()
    ld2 = hsgref.coolheat(L, J, b, 0.02, True)
    assert np.abs(b - s).max() < 1e-12 and abs(ld - ld2) < 1e-10


@pytest.mark.parametrize("pairing", [0, 1, 2])
def test_eps_zero_is_the_plain_exchange(pairing):
    L, S, C = 4, 2, 3
    betas = hsgref.geometric_betas(0.5, 2.0, 6)
    a = hsgref.RefEnsemble(L, S, C, betas, 31)
    b = hsgref.RefEnsemble(L, S, C, betas, 31)
    for e in (a, b):
        e.init_couplings()
        e.init_spins()
        e.sweep(2, 1, 3)
    spins0 = a.spins.copy()
    for _ in range(3):
        a.coolheat_swap(0.0, pairing)
        b.swap(pairing)
    for k in ("temp_of_slot", "slot_of_temp", "swap_ctr", "stats", "rt_state", "rt_trips", "energy"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert np.array_equal(a.spins, spins0)
    assert a.stats[..., 1].sum() > 0


def test_log_ratio_is_antisymmetric_under_the_involution():
    L = 4
    J = inputs.gaussian_couplings(L, 1, 11)[0]
    betas = np.array([1.1, 1.4])
    eps = 0.03
    x = inputs.unit_spins((1,), L ** 3, 12)[0]
    y = inputs.unit_spins((1,), L ** 3, 13)[0]
    xt = y.copy()
    hsgref.coolheat(L, J, xt, eps, True)   # C^-1 y, to beta_1
    yt = x.copy()
    hsgref.coolheat(L, J, yt, eps, False)  # C x, to beta_2

    def log_ratio(a, b):
        ref = hsgref.RefEnsemble(L, 1, 1, betas, 5)
        ref.set_state(J=J[None], spins=np.stack([a, b])[None, None])
        lnA, _ = ref.coolheat_swap(eps, 0)
        return lnA[0, 0, 0]

    l1, l2 = log_ratio(x, y), log_ratio(xt, yt)
    assert abs(l1 + l2) < 1e-9 * max(1.0, abs(l1)), (l1, l2)
    assert abs(l1) > 1e-3  # not trivially zero


def test_non_bijective_map_rejects():
    L, S, C = 4, 1, 2
    betas = hsgref.geometric_betas(1.0, 1.5, 4)
    ref = hsgref.RefEnsemble(L, S, C, betas, 41)
    ref.init_couplings()
    ref.init_spins()
    spins0 = ref.spins.copy()
    lnA, ld = ref.coolheat_swap(10.0, 0)
    assert np.all(np.isnan(lnA)) and ref.stats[..., 1].sum() == 0
    assert np.array_equal(ref.spins, spins0) and np.all(ref.swap_ctr == 1)


def test_forest_law_is_stationary_under_coolheat_exchange():
    L, C = 4, 96
    betas = np.array([0.5, 1.0, 2.0, 4.0])
    R = len(betas)
    rng = np.random.default_rng(17)
    J = inputs.forest_couplings(L, 1, 18)[0]
    ref = hsgref.RefEnsemble(L, 1, C, betas, 0xC001)
    spins = np.zeros((1, C, R, L ** 3, 3))
    for c in range(C):
        for r in range(R):
            spins[0, c, r] = _exact_forest_samples(L, J, betas[r], rng)
    ref.set_state(J=J[None], spins=spins)
    for t in range(60):
        ref.coolheat_swap(0.15, t % 3)
    acc = ref.stats[..., 1].sum() / ref.stats[..., 0].sum()
    assert acc > 0.1
    Jb = np.array([b[2] for b in cf.forest_bonds(L, J)])
    for r in range(R):
        H = np.array([ref.energy[0, c, ref.slot_of_temp[0, c, r]] for c in range(C)])
        mean, var = cf.forest_mean_H(betas[r], Jb), cf.forest_var_H(betas[r], Jb)
        z = (H.mean() - mean) / np.sqrt(var / C)
        assert abs(z) < 4.0, (r, H.mean(), mean, z)
        zv = (H.var(ddof=1) - var) / (var * np.sqrt(2.0 / (C - 1)))
        assert abs(zv) < 4.5, (r, H.var(ddof=1), var, zv)


def _fresh(L, S, C, betas, seed):
    ref = hsgref.RefEnsemble(L, S, C, betas, seed)
    ref.init_couplings()
    ref.init_spins()
    ref.sweep(2, 1, 3)
    return ref


@pytest.mark.parametrize("pairing", [0, 1, 2])
def test_per_pair_eps_constant_equals_one_eps(pairing):
    """One parameter per pair of temperatures (Sec. IV), all equal: the same exchange
    as the single parameter, bit for bit."""
    L, S, C = 4, 2, 2
    betas = hsgref.geometric_betas(0.5, 2.0, 6)
    a, b = _fresh(L, S, C, betas, 51), _fresh(L, S, C, betas, 51)
    for _ in range(3):
        la, da = a.coolheat_swap(0.03, pairing)
        lb, db = b.coolheat_swap(np.full(5, 0.03), pairing)
        assert np.array_equal(la, lb) and np.array_equal(da, db)
    for k in ("spins", "temp_of_slot", "slot_of_temp", "swap_ctr", "stats", "rt_state", "rt_trips", "energy"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k


def test_per_pair_eps_zero_pairs_are_plain_exchanges():
    """Disjoint (even) pairs with their own parameters: a pair with eps_i = 0 has the
    plain acceptance ln A = (b2 - b1)(H(y) - H(x)) of Eq. (1) and zero Jacobians, a pair
    with eps_i > 0 the cooling / heating one, which differs from it."""
    L, S, C = 4, 2, 2
    betas = hsgref.geometric_betas(0.5, 2.0, 6)
    ref = _fresh(L, S, C, betas, 52)
    eps = np.array([0.0, 0.0, 0.04, 0.0, 0.0])
    H = ref.energy.copy()
    sot = ref.slot_of_temp.copy()
    lnA, ld = ref.coolheat_swap(eps, 1)
    for s in range(S):
        for c in range(C):
            for i in (0, 4):
                x, y = sot[s, c, i], sot[s, c, i + 1]
                plain = (betas[i + 1] - betas[i]) * (H[s, c, y] - H[s, c, x])
                assert abs(lnA[s, c, i] - plain) <= 1e-10 * max(1.0, abs(plain))
                assert np.all(ld[s, c, i] == 0.0)
            x, y = sot[s, c, 2], sot[s, c, 3]
            plain = (betas[3] - betas[2]) * (H[s, c, y] - H[s, c, x])
            assert abs(lnA[s, c, 2] - plain) > 1e-6 and np.all(ld[s, c, 2] != 0.0)
    with pytest.raises(ValueError):
        ref.coolheat_swap(np.zeros(3), 1)
