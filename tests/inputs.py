"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds none of the method's arithmetic: only random arrays and structural
masks, in the natural layouts (J [S][N][3], spins [...][N][3]).
"""
import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def gaussian_couplings(L, n_samples, seed, dtype=np.float64):
    """J ~ N(0,1), one per forward bond (x, mu), like the quenched couplings of the model."""
    g = rng(seed).standard_normal((n_samples, L ** 3, 3))
    return round_to(g, dtype)


def unit_spins(shape_prefix, N, seed, dtype=np.float64):
    """Random unit vectors (normalised Gaussian triples), shape prefix + (N, 3)."""
    g = rng(seed).standard_normal(tuple(shape_prefix) + (N, 3))
    g /= np.linalg.norm(g, axis=-1, keepdims=True)
    return round_to(g, dtype)


def round_to(a, dtype):
    """Round to the storage precision (values returned as float64)."""
    return np.asarray(a, dtype=dtype).astype(np.float64)


def forest_mask(L):
    """Mask [N][3] that keeps only the x-bonds of each row except the wrap-around bond.

    The lattice then splits into L^2 open chains of L sites (a forest), for which
    equilibrium averages have closed forms.
    """
    N = L ** 3
    m = np.zeros((N, 3))
    x = np.arange(N)
    i = x % L
    m[:, 0] = (i != L - 1).astype(np.float64)
    return m


def forest_couplings(L, n_samples, seed, dtype=np.float64):
    return gaussian_couplings(L, n_samples, seed, dtype) * forest_mask(L)[None]


def uniforms(n, seed):
    """Uniforms in the open interval (0, 1)."""
    u = rng(seed).random(n)
    u = np.where(u == 0.0, 0.5, u)
    return u


def synthetic_energies(S, C, R, seed, scale=3.0):
    """Per-slot energies for swap-only tests."""
    return rng(seed).standard_normal((S, C, R)) * scale
