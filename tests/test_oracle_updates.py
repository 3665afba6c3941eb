"""Pins of the oracle's single-site updates (paper Sec. III.C).

Heat-bath: the new spin's component c along S must follow the density
proportional to exp(R c) on [-1, 1] (R = beta |S|), checked with a KS test of
its closed-form distribution function in every regime of R, its mean (the
Langevin function), the paper's own inverse-CDF expression where that is
numerically safe, and rotational symmetry about S.  Overrelaxation: exact
invariants (s'.S = s.S, |s'| = |s|, involution).
"""
import numpy as np
import pytest
from scipy import stats

import closed_forms as cf
import inputs
from oracle import hsgref


def _frame_free_direction(seed):
    v = inputs.rng(seed).standard_normal(3)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("R", [0.0, 1e-8, 1e-3, 1.0, 10.0, 100.0, 700.0, 1e4])
def test_heatbath_cdf_all_regimes(R):
    n = 4000
    nhat = _frame_free_direction(int(R * 7) + 1)
    beta = 2.0
    S = nhat * (R / beta)
    r1 = inputs.uniforms(n, 11)
    r2 = inputs.uniforms(n, 12)
    out = np.array([hsgref.heatbath_spin(S, beta, a, b) for a, b in zip(r1, r2)])
    assert np.allclose(np.linalg.norm(out, axis=1), 1.0, atol=1e-14)
    c = out @ nhat
    p = stats.kstest(c, lambda v: cf.hb_cdf(np.clip(v, -1, 1), R)).pvalue
    assert p > 1e-4, (R, p)
    # Langevin mean <c> = coth R - 1/R, and the width from the closed form
    mean_expect = float(cf.langevin(np.array([R]))[0])
    sd = np.sqrt(float(cf.langevin_var(np.array([R]))[0]))
    assert abs(c.mean() - mean_expect) < 5 * sd / np.sqrt(n) + 1e-15


@pytest.mark.parametrize("R", [0.05, 0.7, 3.0, 17.5, 30.0])
def test_heatbath_matches_paper_inverse_cdf(R):
    """c = ln(z + (1/z - z) r)/R with z = exp(-R): the paper's expression, same r."""
    nhat = np.array([0.36, -0.48, 0.8])
    beta = 1.3
    S = nhat * (R / beta)
    for r in [1e-6, 0.01, 0.2, 0.5, 0.77, 0.99, 1 - 1e-9]:
        c = hsgref.heatbath_spin(S, beta, r, 0.3) @ nhat
        z = np.exp(-R)
        c_paper = np.log(z + (1.0 / z - z) * r) / R
        assert abs(c - c_paper) < 1e-10, (R, r, c, c_paper)


def test_heatbath_orthogonal_part_is_isotropic():
    nhat = np.array([0.0, 0.6, 0.8])
    u = np.array([1.0, 0.0, 0.0])
    v = np.cross(nhat, u)
    S = nhat * 2.0
    n = 6000
    r1 = inputs.uniforms(n, 21)
    r2 = inputs.uniforms(n, 22)
    out = np.array([hsgref.heatbath_spin(S, 1.0, a, b) for a, b in zip(r1, r2)])
    pu, pv = out @ u, out @ v
    sig = np.sqrt(np.mean(pu ** 2) / n)
    assert abs(pu.mean()) < 5 * sig and abs(pv.mean()) < 5 * sig
    assert abs(np.mean(pu ** 2) - np.mean(pv ** 2)) < 5 * np.sqrt(2.0 / n) * np.mean(pu ** 2)
    ang = np.arctan2(pv, pu)
    assert stats.kstest(ang, "uniform", args=(-np.pi, 2 * np.pi)).pvalue > 1e-4


@pytest.mark.parametrize("nz", [1.0, -1.0, 0.0, -0.0, 1e-12, -1e-12])
def test_heatbath_frame_edge_directions(nz):
    """Directions on and near the poles and the equator give unit spins with the right c."""
    rest = np.sqrt(max(0.0, 1.0 - nz * nz))
    nhat = np.array([rest * 0.6, rest * 0.8, nz])
    for r1 in [0.1, 0.5, 0.9]:
        out = hsgref.heatbath_spin(nhat * 1.5, 2.0, r1, 0.37)
        assert abs(np.linalg.norm(out) - 1.0) < 1e-14
        R = 3.0
        z = np.exp(-R)
        c_paper = np.log(z + (1.0 / z - z) * r1) / R
        assert abs(out @ nhat - c_paper) < 1e-12


def test_heatbath_zero_field_is_uniform():
    n = 4000
    r1 = inputs.uniforms(n, 31)
    r2 = inputs.uniforms(n, 32)
    out = np.array([hsgref.heatbath_spin(np.zeros(3), 1.0, a, b) for a, b in zip(r1, r2)])
    assert np.allclose(out[:, 2], 2 * r1 - 1, atol=1e-15)
    assert stats.kstest(out[:, 0], "uniform", args=(-1, 2)).pvalue > 1e-4


def test_overrelaxation_invariants():
    r = inputs.rng(5)
    for _ in range(500):
        s = r.standard_normal(3)
        s /= np.linalg.norm(s)
        S = r.standard_normal(3) * r.uniform(0.01, 6)
        s1 = hsgref.overrelax_spin(s, S)
        assert abs(s1 @ S - s @ S) < 1e-13 * max(1.0, np.linalg.norm(S))
        assert abs(np.linalg.norm(s1) - 1.0) < 1e-14
        s2 = hsgref.overrelax_spin(s1, S)
        assert np.allclose(s2, s, atol=1e-14)
        # the component orthogonal to S flips sign
        sh = S / np.linalg.norm(S)
        assert np.allclose(s1 - (s1 @ sh) * sh, -(s - (s @ sh) * sh), atol=1e-14)


def test_overrelaxation_zero_field_is_identity():
    s = np.array([0.6, 0.0, 0.8])
    assert np.array_equal(hsgref.overrelax_spin(s, np.zeros(3)), s)
