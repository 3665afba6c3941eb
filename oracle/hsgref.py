"""ctypes wrapper around the FP64 CPU oracle (oracle/hsgref.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It
shares no code with the HIP library or its Python binding.

Layouts are the natural ones (all float64 unless noted):
  J      [S][N][3]        J[x][mu] couples x and x + e_mu, x = i + L(j + L k)
  spins  [S][C][R][N][3]  by slot (a physical configuration)
  temp_of_slot, slot_of_temp, rt_state int32 [S][C][R]; energy [S][C][R];
  sweep_ctr uint32 [S][C][R]; swap_ctr uint32 [S][C]; stats int64 [S][C][R-1][2];
  rt_trips int64 [S][C][R].
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_c_int = ctypes.c_int
_c_u32 = ctypes.c_uint32
_c_u64 = ctypes.c_uint64
_c_dbl = ctypes.c_double


def lib():
    """Load (building first if needed) the oracle library."""
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        sigs = {
            "hsgref_philox4x32_10": (None, [_u32p, _u32p, _u32p]),
            "hsgref_u01_24": (_c_dbl, [_c_u32]),
            "hsgref_u01_52": (_c_dbl, [_c_u32, _c_u32]),
            "hsgref_parity": (_c_int, [_c_int, _c_int]),
            "hsgref_compressed_index": (_c_int, [_c_int, _c_int]),
            "hsgref_neighbor": (_c_int, [_c_int, _c_int, _c_int]),
            "hsgref_init_couplings": (None, [_c_int, _c_int, _c_u32, _c_u64, _c_int, _dp]),
            "hsgref_init_spins": (None, [_c_int, _c_int, _c_u32, _c_u64, _c_int, _c_int, _dp]),
            "hsgref_local_field": (None, [_c_int, _dp, _dp, _c_int, _dp]),
            "hsgref_heatbath_spin": (None, [_dp, _c_dbl, _c_dbl, _c_dbl, _dp]),
            "hsgref_overrelax_spin": (None, [_dp, _dp, _dp]),
            "hsgref_hb_uniforms": (None, [_c_int, _c_int, _c_u64, _c_u32, _c_u32, _c_u32, _c_int,
                                          _dp, _dp]),
            "hsgref_fields": (None, [_c_int, _dp, _dp, _c_int, _dp]),
            "hsgref_hb_uniforms_all": (None, [_c_int, _c_int, _c_u64, _c_u32, _c_u32, _c_u32,
                                              _c_int, _dp, _dp]),
            "hsgref_heatbath_many": (None, [_c_int, _dp, _dp, _dp, _dp, _dp]),
            "hsgref_overrelax_many": (None, [_c_int, _dp, _dp, _dp]),
            "hsgref_energy": (_c_dbl, [_c_int, _dp, _dp]),
            "hsgref_sublattice_energy": (_c_dbl, [_c_int, _dp, _dp, _c_int]),
            "hsgref_halfsweep": (None, [_c_int, _dp, _dp, _c_int, _c_int, _c_dbl, _c_u64, _c_u32,
                                        _c_u32, _c_u32, _c_int, _i32p]),
            "hsgref_sweep": (None, [_c_int, _dp, _dp, _c_int, _c_int, _c_int, _c_dbl, _c_u64,
                                    _c_u32, _c_u32, _c_int]),
            "hsgref_sweep_batch": (None, [_c_int, _c_int, _c_int, _c_int, _dp, _dp, _dp, _i32p,
                                          _u32p, _c_u32, _c_u64, _c_int, _c_int, _c_int, _c_int,
                                          _dp]),
            "hsgref_swap_batch": (None, [_c_int, _c_int, _c_int, _dp, _dp, _i32p, _i32p, _u32p,
                                         _i64p, _i32p, _i64p, _c_u32, _c_u64, _c_int]),
            "hsgref_anneal_batch": (None, [_c_int, _c_int, _c_int, _c_int, _dp, _dp, _dp, _i32p,
                                           _i32p, _u32p, _u32p, _dp, _i64p, _i32p, _i64p, _c_u32,
                                           _c_u32, _c_u64, _c_int, _i32p, _dp, _c_int, _c_int,
                                           _c_int, _c_int, _dp]),
            "hsgref_log_sinhc": (_c_dbl, [_c_dbl]),
            "hsgref_decimated_log_ratio": (_c_dbl, [_c_int, _dp, _dp, _dp, _c_int, _c_dbl, _c_dbl]),
            "hsgref_decimate_uniforms": (None, [_c_int, _c_int, _c_u64, _c_u32, _c_u32, _c_u32,
                                                _c_int, _dp, _dp]),
            "hsgref_decimate_role": (_c_int, [_c_u64, _c_u32, _c_u32]),
            "hsgref_decimate_batch": (None, [_c_int, _c_int, _c_int, _c_int, _dp, _dp, _dp, _i32p,
                                             _i32p, _u32p, _dp, _i64p, _i32p, _i64p, _c_u32,
                                             _c_u32, _c_u64, _c_int, _c_int, _dp, _i32p]),
            "hsgref_cool_spin": (_c_dbl, [_dp, _dp, _c_dbl, _dp]),
            "hsgref_heat_spin": (_c_dbl, [_dp, _dp, _c_dbl, _dp]),
            "hsgref_coolheat": (_c_dbl, [_c_int, _dp, _dp, _c_dbl, _c_int]),
            "hsgref_coolheat_batch": (None, [_c_int, _c_int, _c_int, _c_int, _dp, _dp, _dp, _i32p,
                                             _i32p, _u32p, _dp, _i64p, _i32p, _i64p, _c_u32,
                                             _c_u64, _c_int, _c_dbl, _dp, _dp, _dp]),
            "hsgref_measure_batch": (None, [_c_int, _c_int, _c_int, _c_int, _dp, _dp, _i32p, _dp,
                                            _dp, _dp]),
            "hsgref_roundtrip_update": (None, [_c_int, _i32p, _i32p, _i64p]),
            "hsgref_num_threads": (_c_int, []),
            "hsgref_set_num_threads": (None, [_c_int]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a, ctype):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def dp(a):
    assert a.dtype == np.float64
    return _p(a, ctypes.c_double)


def i32p(a):
    assert a.dtype == np.int32
    return _p(a, ctypes.c_int32)


def u32p(a):
    assert a.dtype == np.uint32
    return _p(a, ctypes.c_uint32)


def i64p(a):
    assert a.dtype == np.int64
    return _p(a, ctypes.c_int64)


# ---------------------------------------------------------------- primitives
def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().hsgref_philox4x32_10(u32p(c), u32p(k), u32p(out))
    return out


def u01_24(w):
    return lib().hsgref_u01_24(int(w))


def u01_52(w0, w1):
    return lib().hsgref_u01_52(int(w0), int(w1))


def heatbath_spin(S, beta, r1, r2):
    S = np.ascontiguousarray(S, dtype=np.float64)
    out = np.zeros(3)
    lib().hsgref_heatbath_spin(dp(S), float(beta), float(r1), float(r2), dp(out))
    return out


def overrelax_spin(s, S):
    s = np.ascontiguousarray(s, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    out = np.zeros(3)
    lib().hsgref_overrelax_spin(dp(s), dp(S), dp(out))
    return out


def neighbor(L, x, d):
    return lib().hsgref_neighbor(L, x, d)


def parity(L, x):
    return lib().hsgref_parity(L, x)


def compressed_index(L, x):
    return lib().hsgref_compressed_index(L, x)


def init_couplings(L, n_samples, seed, sample_base=0, round_f32=False):
    N = L ** 3
    J = np.zeros((n_samples, N, 3))
    lib().hsgref_init_couplings(L, n_samples, sample_base, seed, int(round_f32), dp(J))
    return J


def init_spins(L, n_slots, seed, slot_base=0, cold=False, round_f32=False):
    N = L ** 3
    s = np.zeros((n_slots, N, 3))
    lib().hsgref_init_spins(L, n_slots, slot_base, seed, int(cold), int(round_f32), dp(s))
    return s


def local_field(L, J, s, x):
    J = np.ascontiguousarray(J, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    S = np.zeros(3)
    lib().hsgref_local_field(L, dp(J), dp(s), int(x), dp(S))
    return S


def energy(L, J, s):
    J = np.ascontiguousarray(J, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    return lib().hsgref_energy(L, dp(J), dp(s))


def sublattice_energy(L, J, s, par):
    J = np.ascontiguousarray(J, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    return lib().hsgref_sublattice_energy(L, dp(J), dp(s), int(par))


def hb_uniforms(L, rng32, seed, slot_global, t, hs, x):
    r1 = ctypes.c_double()
    r2 = ctypes.c_double()
    lib().hsgref_hb_uniforms(L, int(rng32), seed, slot_global, t, hs, int(x),
                             ctypes.byref(r1), ctypes.byref(r2))
    return r1.value, r2.value


def fields(L, J, s, par):
    """Local fields [N][3] of the sites of parity `par` (zeros at the other sites)."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    out = np.zeros((L ** 3, 3))
    lib().hsgref_fields(L, dp(J), dp(s), int(par), dp(out))
    return out


def hb_uniforms_all(L, rng32, seed, slot_global, t, hs, par):
    """Heat-bath uniforms (r1 [N], r2 [N]) of the sites of parity `par` (zeros elsewhere)."""
    r1 = np.zeros(L ** 3)
    r2 = np.zeros(L ** 3)
    lib().hsgref_hb_uniforms_all(L, int(rng32), seed, slot_global, t, hs, int(par), dp(r1), dp(r2))
    return r1, r2


def heatbath_many(S, beta, r1, r2):
    """Heat-bath updates, one per row of S [n][3] with beta, r1, r2 [n]."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    n = S.shape[0]
    b = np.ascontiguousarray(np.broadcast_to(beta, (n,)), dtype=np.float64)
    r1 = np.ascontiguousarray(r1, dtype=np.float64)
    r2 = np.ascontiguousarray(r2, dtype=np.float64)
    out = np.zeros((n, 3))
    lib().hsgref_heatbath_many(n, dp(S), dp(b), dp(r1), dp(r2), dp(out))
    return out


def overrelax_many(s, S):
    """Overrelaxation updates, one per row of s, S [n][3]."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    out = np.zeros(S.shape)
    lib().hsgref_overrelax_many(S.shape[0], dp(s), dp(S), dp(out))
    return out


def halfsweep(L, J, s, par, kind, beta, seed, slot_global, t, hs, rng32=False, order=None):
    """In-place half-sweep of one replica s [N][3]; kind 0 heat-bath, 1 overrelaxation."""
    assert s.dtype == np.float64 and s.flags["C_CONTIGUOUS"]
    J = np.ascontiguousarray(J, dtype=np.float64)
    o = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
    lib().hsgref_halfsweep(L, dp(J), dp(s), int(par), int(kind), float(beta), seed, slot_global,
                           t, hs, int(rng32), None if o is None else i32p(o))


def sweep(L, J, s, n_hb, n_or, beta, seed, slot_global, t, adjoint=False, rng32=False):
    assert s.dtype == np.float64 and s.flags["C_CONTIGUOUS"]
    J = np.ascontiguousarray(J, dtype=np.float64)
    lib().hsgref_sweep(L, dp(J), dp(s), int(n_hb), int(n_or), int(adjoint), float(beta), seed,
                       slot_global, t, int(rng32))


def log_sinhc(u):
    """h(u) = ln(sinh(u)/u), h(0) = 0."""
    return lib().hsgref_log_sinhc(float(u))


def decimated_log_ratio(L, J, sx, sy, d, b1, b2):
    """ln A of the decimated exchange (paper Eq. (eq:aswap)): x at b1, y at b2, parity d
    integrated out."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    sx = np.ascontiguousarray(sx, dtype=np.float64)
    sy = np.ascontiguousarray(sy, dtype=np.float64)
    return lib().hsgref_decimated_log_ratio(L, dp(J), dp(sx), dp(sy), int(d), float(b1), float(b2))


def decimate_uniforms(L, rng32, seed, slot_global, n, pair, x):
    r1 = ctypes.c_double()
    r2 = ctypes.c_double()
    lib().hsgref_decimate_uniforms(L, int(rng32), seed, slot_global, n, pair, x,
                                   ctypes.byref(r1), ctypes.byref(r2))
    return r1.value, r2.value


def decimate_role(seed, chain_global, n):
    return lib().hsgref_decimate_role(seed, chain_global, n)


def cool_spin(s, S, eps):
    """Cooling map of one spin (paper Sec. III.B): (new spin, log Jacobian)."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    out = np.zeros(3)
    ld = lib().hsgref_cool_spin(dp(s), dp(S), float(eps), dp(out))
    return out, ld


def heat_spin(s, S, eps):
    """Inverse of cool_spin: (pre-image, log Jacobian of cooling at the pre-image)."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    out = np.zeros(3)
    ld = lib().hsgref_heat_spin(dp(s), dp(S), float(eps), dp(out))
    return out, ld


def coolheat(L, J, s, eps, heat):
    """Lattice cooling (heat=False) or heating in place; returns the log Jacobian of cooling."""
    assert s.dtype == np.float64 and s.flags["C_CONTIGUOUS"]
    J = np.ascontiguousarray(J, dtype=np.float64)
    return lib().hsgref_coolheat(L, dp(J), dp(s), float(eps), int(heat))


def geometric_betas(bmin, bmax, R):
    """beta_r = bmin (bmax/bmin)^(r/(R-1)), ascending (the paper's ladder family, Sec. IV)."""
    r = np.arange(R, dtype=np.float64)
    return bmin * (bmax / bmin) ** (r / (R - 1))


class RefEnsemble:
    """One size class of S samples x C chains x R temperature slots, in natural layout.

    prec: 'fp64' (52-bit uniforms, FP64 inputs) or 'fp32' (24-bit uniforms, and the
    initial couplings and spins rounded to binary32, exactly as an FP32-spin run
    starts); the arithmetic is FP64 in both cases.
    """

    def __init__(self, L, n_samples, n_chains, betas, seed, prec="fp64", sample_base=0,
                 chain_base=0, slot_base=0):
        self.L = int(L)
        self.N = self.L ** 3
        self.S = int(n_samples)
        self.C = int(n_chains)
        self.betas = np.ascontiguousarray(betas, dtype=np.float64)
        self.R = len(self.betas)
        self.seed = int(seed)
        self.prec = prec
        self.rng32 = prec == "fp32"
        self.sample_base = int(sample_base)
        self.chain_base = int(chain_base)
        self.slot_base = int(slot_base)
        S, C, R, N = self.S, self.C, self.R, self.N
        self.J = np.zeros((S, N, 3))
        self.spins = np.zeros((S, C, R, N, 3))
        self.temp_of_slot = np.ascontiguousarray(np.broadcast_to(np.arange(R, dtype=np.int32), (S, C, R)))
        self.slot_of_temp = self.temp_of_slot.copy()
        self.energy = np.zeros((S, C, R))
        self.sweep_ctr = np.zeros((S, C, R), dtype=np.uint32)
        self.swap_ctr = np.zeros((S, C), dtype=np.uint32)
        self.stats = np.zeros((S, C, R - 1, 2), dtype=np.int64)
        self.rt_state = np.zeros((S, C, R), dtype=np.int32)
        self.rt_trips = np.zeros((S, C, R), dtype=np.int64)
        self.rt_state[..., 0] = 1

    # -- initialisation
    def init_couplings(self):
        lib().hsgref_init_couplings(self.L, self.S, self.sample_base, self.seed, int(self.rng32),
                                    dp(self.J))

    def init_spins(self, cold=False):
        flat = self.spins.reshape(self.S * self.C * self.R, self.N, 3)
        lib().hsgref_init_spins(self.L, self.S * self.C * self.R, self.slot_base, self.seed,
                                int(cold), int(self.rng32), dp(flat))
        self.compute_energy()

    def set_state(self, J=None, spins=None):
        if J is not None:
            self.J[...] = J
        if spins is not None:
            self.spins[...] = spins
        self.compute_energy()

    def compute_energy(self):
        for s in range(self.S):
            for c in range(self.C):
                for r in range(self.R):
                    self.energy[s, c, r] = energy(self.L, self.J[s], self.spins[s, c, r])
        return self.energy

    # -- the hot path
    def sweep(self, n_sweeps=1, n_hb=1, n_or=3):
        lib().hsgref_sweep_batch(self.L, self.S, self.C, self.R, dp(self.J), dp(self.spins),
                                 dp(self.betas), i32p(self.temp_of_slot), u32p(self.sweep_ctr),
                                 self.slot_base, self.seed, n_sweeps, n_hb, n_or,
                                 int(self.rng32), dp(self.energy))

    def swap(self, pairing=0):
        lib().hsgref_swap_batch(self.S, self.C, self.R, dp(self.betas), dp(self.energy),
                                i32p(self.temp_of_slot), i32p(self.slot_of_temp),
                                u32p(self.swap_ctr), i64p(self.stats), i32p(self.rt_state),
                                i64p(self.rt_trips), self.chain_base, self.seed, pairing)

    def anneal_swap(self, parity, K, lam=None, n_hb=1, n_or=3):
        """Annealed swap of the pairs i with i % 2 == parity; K: [R-1] int; lam: [R-1][K_max]."""
        Kv = np.ascontiguousarray(np.broadcast_to(np.asarray(K, dtype=np.int32), (self.R - 1,)))
        if lam is None:
            K_max = 0
            lp = None
        else:
            lam = np.ascontiguousarray(lam, dtype=np.float64)
            K_max = lam.shape[1]
            lp = dp(lam)
        work = np.zeros((self.S, self.C, self.R - 1, 2))
        lib().hsgref_anneal_batch(self.L, self.S, self.C, self.R, dp(self.J), dp(self.spins),
                                  dp(self.betas), i32p(self.temp_of_slot), i32p(self.slot_of_temp),
                                  u32p(self.sweep_ctr), u32p(self.swap_ctr), dp(self.energy),
                                  i64p(self.stats), i32p(self.rt_state), i64p(self.rt_trips),
                                  self.slot_base, self.chain_base, self.seed, int(parity),
                                  i32p(Kv), lp, K_max, n_hb, n_or, int(self.rng32), dp(work))
        return work

    def decimate_swap(self, pairing=0):
        """Decimated exchange (paper Sec. III.A) of the selected pairs (pairing as in swap).
        Returns ln A [S][C][R-1] (0 where not attempted) and the decimated parity
        [S][C][R-1] (-1 where not attempted)."""
        lnA = np.zeros((self.S, self.C, self.R - 1))
        role = np.zeros((self.S, self.C, self.R - 1), dtype=np.int32)
        lib().hsgref_decimate_batch(self.L, self.S, self.C, self.R, dp(self.J), dp(self.spins),
                                    dp(self.betas), i32p(self.temp_of_slot),
                                    i32p(self.slot_of_temp), u32p(self.swap_ctr), dp(self.energy),
                                    i64p(self.stats), i32p(self.rt_state), i64p(self.rt_trips),
                                    self.slot_base, self.chain_base, self.seed, int(pairing),
                                    int(self.rng32), dp(lnA), i32p(role))
        return lnA, role

    def coolheat_swap(self, eps, pairing=0):
        """Cooling / heating exchange (paper Sec. III.B) of the selected pairs; eps is one
        map parameter for every pair or an array of R-1, one per pair of temperatures
        (Sec. IV).  Returns ln A [S][C][R-1] and the log Jacobians of cooling at x and at
        C^-1 y [S][C][R-1][2] (zeros where not attempted)."""
        lnA = np.zeros((self.S, self.C, self.R - 1))
        ld = np.zeros((self.S, self.C, self.R - 1, 2))
        if np.ndim(eps) == 0:
            eps0, eps_pair = float(eps), None
        else:
            eps_pair = np.ascontiguousarray(eps, dtype=np.float64)
            if eps_pair.shape != (self.R - 1,):
                raise ValueError("per-pair eps must have R - 1 = %d entries" % (self.R - 1))
            eps0 = 0.0
        lib().hsgref_coolheat_batch(self.L, self.S, self.C, self.R, dp(self.J), dp(self.spins),
                                    dp(self.betas), i32p(self.temp_of_slot),
                                    i32p(self.slot_of_temp), u32p(self.swap_ctr), dp(self.energy),
                                    i64p(self.stats), i32p(self.rt_state), i64p(self.rt_trips),
                                    self.chain_base, self.seed, int(pairing), eps0, dp(lnA),
                                    dp(ld), dp(eps_pair) if eps_pair is not None else None)
        return lnA, ld

    def measure(self):
        Q = np.zeros((self.S, self.R, 3, 3))
        chi = np.zeros((self.S, self.R))
        e = np.zeros((self.S, self.C, self.R))
        lib().hsgref_measure_batch(self.L, self.S, self.C, self.R, dp(self.spins), dp(self.energy),
                                   i32p(self.slot_of_temp), dp(Q), dp(chi), dp(e))
        return Q, chi, e
