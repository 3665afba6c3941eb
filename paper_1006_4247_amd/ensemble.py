"""Torch-owned device buffers of one size class, driven through the C ABI.

PyTorch provides device memory, host<->device copies and the stream; every step
of the hot path runs in the HIP kernels of libhsgpt.so.  Layout helpers convert
between the device layout ([..][3][2][N/2], by component, parity and
sublattice index) and the natural one ([..][N][3], x = i + L(j + L k)).
"""
import ctypes

import numpy as np
import torch

from . import _abi

_NT = {"fp64": torch.float64, "fp32": torch.float32}


def geometric_betas(bmin, bmax, R):
    """beta_r = bmin (bmax/bmin)^(r/(R-1)): the geometric ladder family of the paper (Sec. IV)."""
    r = np.arange(R, dtype=np.float64)
    return bmin * (bmax / bmin) ** (r / (R - 1))


def natural_to_device_index(L):
    """perm[x] = p(x) * N/2 + h(x): position of natural site x in the [2][N/2] parity layout."""
    N = L ** 3
    x = np.arange(N)
    i = x % L
    row = x // L
    j = row % L
    k = row // L
    p = (i + j + k) & 1
    h = i // 2 + (L // 2) * row
    return p * (N // 2) + h


def device_to_natural(arr, L):
    """[..., 3, 2, N/2] -> [..., N, 3] (numpy)."""
    a = np.asarray(arr)
    N = L ** 3
    flat = a.reshape(a.shape[:-3] + (3, N))
    perm = natural_to_device_index(L)
    return np.ascontiguousarray(np.swapaxes(flat[..., perm], -1, -2))


def natural_to_device(arr, L):
    """[..., N, 3] -> [..., 3, 2, N/2] (numpy)."""
    a = np.asarray(arr)
    N = L ** 3
    perm = natural_to_device_index(L)
    out = np.empty(a.shape[:-2] + (3, N), dtype=a.dtype)
    out[..., perm] = np.swapaxes(a, -1, -2)
    return out.reshape(a.shape[:-2] + (3, 2, N // 2))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Ensemble:
    """One size class: S samples x C chains x R temperatures on one GPU.

    precision 'fp32' stores spins and couplings in binary32 (energies, works and
    observables stay FP64); 'fp64' stores everything in binary64.
    """

    def __init__(self, L, n_samples, n_chains, betas, seed, precision="fp32", device="cuda",
                 sample_base=0, chain_base=0, slot_base=0, K_max=0, stream=None):
        lib = _abi.lib()
        self.L = int(L)
        self.N = self.L ** 3
        self.S = int(n_samples)
        self.C = int(n_chains)
        betas = np.asarray(betas, dtype=np.float64)
        self.R = len(betas)
        self.seed = int(seed)
        self.precision = precision
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.K_max = int(K_max)
        self.stream = stream
        dt = _NT[precision]
        S, C, R, N = self.S, self.C, self.R, self.N
        z = dict(device=self.device)
        self.spins = torch.zeros((S, C, R, 3, 2, N // 2), dtype=dt, **z)
        self.couplings = torch.zeros((S, 3, 2, N // 2), dtype=dt, **z)
        self.betas = torch.tensor(betas, dtype=torch.float64, **z)
        self.betas_host = betas.copy()
        self.temp_of_slot = torch.zeros((S, C, R), dtype=torch.int32, **z)
        self.slot_of_temp = torch.zeros((S, C, R), dtype=torch.int32, **z)
        self.energy = torch.zeros((S, C, R), dtype=torch.float64, **z)
        self.sweep_ctr = torch.zeros((S, C, R), dtype=torch.int32, **z)
        self.swap_ctr = torch.zeros((S, C), dtype=torch.int32, **z)
        self.swap_stats = torch.zeros((S, C, R - 1, 2), dtype=torch.int64, **z)
        self.rt_state = torch.zeros((S, C, R), dtype=torch.int32, **z)
        self.rt_trips = torch.zeros((S, C, R), dtype=torch.int64, **z)
        self.guard = torch.zeros((1,), dtype=torch.int32, **z)
        self.anneal_K = torch.zeros((R - 1,), dtype=torch.int32, **z)
        self.anneal_lambda = (torch.zeros((R - 1, self.K_max), dtype=torch.float64, **z)
                              if self.K_max > 0 else None)
        self._use_lambda = False
        self.work = torch.zeros((S, C, R - 1, 2), dtype=torch.float64, **z)
        self.Q = torch.zeros((S, R, 3, 3), dtype=torch.float64, **z)
        self.chi = torch.zeros((S, R), dtype=torch.float64, **z)
        self.e_temp = torch.zeros((S, C, R), dtype=torch.float64, **z)
        self.desc = _abi.HsgEnsemble()
        d = self.desc
        d.L, d.n_samples, d.n_chains, d.n_temps = self.L, S, C, R
        d.precision = _abi.HSG_FP32 if precision == "fp32" else _abi.HSG_FP64
        d.sample_base, d.chain_base, d.slot_base = int(sample_base), int(chain_base), int(slot_base)
        d.seed = self.seed
        nbytes = lib.hsg_scratch_bytes(ctypes.byref(d))
        if nbytes == 0:
            raise _abi.HsgError(_abi.HSG_ERR_INVALID, "invalid ensemble shape")
        self.scratch = torch.zeros((nbytes,), dtype=torch.uint8, **z)
        self._fill_desc()

    # ------------------------------------------------------------ plumbing
    def _fill_desc(self):
        d = self.desc
        for name in ["spins", "couplings", "betas", "temp_of_slot", "slot_of_temp", "energy",
                     "sweep_ctr", "swap_ctr", "swap_stats", "rt_state", "rt_trips", "guard",
                     "anneal_K", "scratch", "work", "Q", "chi", "e_temp"]:
            setattr(d, name, _ptr(getattr(self, name)).value)
        d.anneal_lambda = _ptr(self.anneal_lambda if self._use_lambda else None).value
        d.anneal_K_max = self.K_max

    def _stream(self):
        s = self.stream if self.stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(s.cuda_stream)

    @property
    def n_slots(self):
        return self.S * self.C * self.R

    # ------------------------------------------------------------ the hot path
    def init_couplings(self):
        _abi.check(_abi.lib().hsg_init_couplings(ctypes.byref(self.desc), 1, self._stream()))

    def init_spins(self, cold=False):
        _abi.check(_abi.lib().hsg_init_spins(ctypes.byref(self.desc), 1, int(cold), self._stream()))

    def sweep(self, n_sweeps=1, n_hb=1, n_or=3, tuning=None):
        if tuning is None:
            _abi.check(_abi.lib().hsg_sweep(ctypes.byref(self.desc), 1, n_sweeps, n_hb, n_or,
                                            self._stream()))
        else:
            t = _abi.HsgTuning(int(tuning.get("path", 0)), int(tuning.get("block_threads", 0)),
                               int(tuning.get("replicas_per_block", 0)), int(tuning.get("flags", 0)))
            _abi.check(_abi.lib().hsg_sweep_tuned(ctypes.byref(self.desc), 1, n_sweeps, n_hb, n_or,
                                                  ctypes.byref(t), self._stream()))

    def energy_from_scratch(self, out=None):
        """Standalone bond-sum H of every slot (FP64); returns a new [S][C][R] tensor."""
        if out is None:
            out = torch.empty((self.S, self.C, self.R), dtype=torch.float64, device=self.device)
        if (tuple(out.shape) != (self.S, self.C, self.R) or out.dtype != torch.float64
                or not out.is_contiguous() or out.device != self.device):
            raise ValueError("out must be a contiguous float64 [S][C][R] tensor on %s" % self.device)
        _abi.check(_abi.lib().hsg_energy(ctypes.byref(self.desc), 1, _ptr(out), self._stream()))
        return out

    def swap(self, pairing=0):
        _abi.check(_abi.lib().hsg_swap(ctypes.byref(self.desc), 1, int(pairing), self._stream()))

    def set_schedule(self, K, lam=None):
        """Protocol lengths K [R-1] and optional interior betas lam [R-1][K_max] (device copies)."""
        K = np.broadcast_to(np.asarray(K, dtype=np.int32), (self.R - 1,))
        if int(K.max(initial=0)) > self.K_max:
            raise ValueError("K exceeds K_max = %d" % self.K_max)
        self.anneal_K.copy_(torch.from_numpy(np.array(K, dtype=np.int32)))
        if lam is not None:
            lam = np.asarray(lam, dtype=np.float64)
            if self.anneal_lambda is None or lam.shape != tuple(self.anneal_lambda.shape):
                raise ValueError("lambda must have shape [R-1][K_max]")
            self.anneal_lambda.copy_(torch.from_numpy(np.ascontiguousarray(lam)))
            self._use_lambda = True
        else:
            self._use_lambda = False
        self._fill_desc()

    def anneal_swap(self, parity, n_hb=1, n_or=3):
        _abi.check(_abi.lib().hsg_anneal_swap(ctypes.byref(self.desc), 1, int(parity), n_hb, n_or,
                                              self._stream()))

    def decimate_swap(self, pairing=0):
        """Decimated exchange (paper Sec. III.A) of the selected pairs; afterwards
        work[..., i, 0] holds ln A and work[..., i, 1] the decimated sublattice of pair i
        (0 and -1 where not attempted)."""
        _abi.check(_abi.lib().hsg_decimate_swap(ctypes.byref(self.desc), 1, int(pairing),
                                                self._stream()))
        return self.work

    def coolheat_swap(self, eps, pairing=0):
        """Cooling / heating exchange (paper Sec. III.B) of the selected pairs; eps is one
        map parameter for every pair, or R - 1 of them, one per pair of temperatures
        (Sec. IV; a sequence or a float64 tensor on this device).  Afterwards
        work[..., i, 0] and work[..., i, 1] hold ln det J_C(x) and ln det J_C(C^-1 y) of
        pair i (zeros where not attempted)."""
        if isinstance(eps, torch.Tensor) or np.ndim(eps) > 0:
            t = self.eps_pairs_tensor(eps)
            self._eps_pairs = t  # kept alive while the launch may still read it
            _abi.check(_abi.lib().hsg_coolheat_swap_pairs(ctypes.byref(self.desc), 1, int(pairing),
                                                          _ptr(t), self._stream()))
        else:
            _abi.check(_abi.lib().hsg_coolheat_swap(ctypes.byref(self.desc), 1, int(pairing),
                                                    float(eps), self._stream()))
        return self.work

    def eps_pairs_tensor(self, eps):
        """Per-pair map parameters as the float64 device tensor the exchange reads: a
        tensor already in that form is used as it is; anything else (a sequence, an
        array, a tensor elsewhere) is copied once and the copy waited for."""
        if (isinstance(eps, torch.Tensor) and eps.dtype == torch.float64 and eps.device == self.device
                and eps.is_contiguous()):
            t = eps
        else:
            a = eps.detach().cpu().numpy() if isinstance(eps, torch.Tensor) else np.asarray(eps)
            t = torch.tensor(a.astype(np.float64), device=self.device)
            torch.cuda.synchronize(self.device)
        if tuple(t.shape) != (self.R - 1,):
            raise ValueError("per-pair eps must have R - 1 = %d entries" % (self.R - 1))
        return t

    def measure(self):
        _abi.check(_abi.lib().hsg_measure(ctypes.byref(self.desc), 1, self._stream()))
        return self.Q, self.chi, self.e_temp

    def sweep_measure(self, n_sweeps=1, n_hb=1, n_or=3):
        """sweep(n_sweeps, n_hb, n_or) then measure(); one launch where the ensemble has
        two chains whose replicas fit one workgroup's LDS together."""
        _abi.check(_abi.lib().hsg_sweep_measure(ctypes.byref(self.desc), 1, n_sweeps, n_hb, n_or,
                                                self._stream()))
        return self.Q, self.chi, self.e_temp

    def check(self):
        _abi.check(_abi.lib().hsg_check(ctypes.byref(self.desc), 1, self._stream()))

    # ------------------------------------------------------------ checkpoint / resume
    # Every random number is a Philox block addressed by (site, sweep or exchange
    # counter, slot or chain, tag) under the seed, and the counters live in the state
    # arrays, so a run resumed from a checkpoint continues bit for bit as if it had
    # never stopped.
    _STATE = ["spins", "couplings", "betas", "temp_of_slot", "slot_of_temp", "energy", "sweep_ctr",
              "swap_ctr", "swap_stats", "rt_state", "rt_trips", "guard", "anneal_K", "work", "Q",
              "chi", "e_temp"]

    def meta(self):
        d = self.desc
        return {"L": self.L, "n_samples": self.S, "n_chains": self.C, "n_temps": self.R,
                "seed": self.seed, "precision": self.precision, "sample_base": int(d.sample_base),
                "chain_base": int(d.chain_base), "slot_base": int(d.slot_base), "K_max": self.K_max,
                "use_lambda": bool(self._use_lambda)}

    def state_dict(self):
        """Host copies of every state array (device layout) and the shape metadata."""
        st = {k: getattr(self, k).detach().cpu().clone() for k in self._STATE}
        if self.anneal_lambda is not None:
            st["anneal_lambda"] = self.anneal_lambda.detach().cpu().clone()
        return {"meta": self.meta(), "tensors": st}

    def load_state_dict(self, sd):
        m = sd["meta"]
        mine = self.meta()
        for k in ("L", "n_samples", "n_chains", "n_temps", "precision", "K_max"):
            if m[k] != mine[k]:
                raise ValueError("checkpoint %s = %r does not match this ensemble's %r" % (k, m[k], mine[k]))
        t = sd["tensors"]
        for k in self._STATE:
            getattr(self, k).copy_(t[k].to(self.device))
        if self.anneal_lambda is not None and "anneal_lambda" in t:
            self.anneal_lambda.copy_(t["anneal_lambda"].to(self.device))
        self._use_lambda = bool(m.get("use_lambda", False))
        self.seed = int(m["seed"])
        d = self.desc
        d.seed = self.seed
        d.sample_base, d.chain_base, d.slot_base = m["sample_base"], m["chain_base"], m["slot_base"]
        self._fill_desc()

    def save(self, path):
        """Checkpoint to a safetensors file (tensors; metadata as JSON in its header)."""
        import json
        from safetensors.torch import save_file
        sd = self.state_dict()
        save_file({k: v.contiguous() for k, v in sd["tensors"].items()}, path,
                  metadata={"hsg_meta": json.dumps(sd["meta"])})

    @classmethod
    def load(cls, path, device="cuda", stream=None):
        """A new ensemble holding the state saved by save()."""
        import json
        from safetensors import safe_open
        with safe_open(path, framework="pt") as f:
            m = json.loads(f.metadata()["hsg_meta"])
            tensors = {k: f.get_tensor(k) for k in f.keys()}
        betas = tensors["betas"].double().numpy()
        e = cls(m["L"], m["n_samples"], m["n_chains"], betas, m["seed"], precision=m["precision"],
                device=device, sample_base=m["sample_base"], chain_base=m["chain_base"],
                slot_base=m["slot_base"], K_max=m["K_max"], stream=stream)
        e.load_state_dict({"meta": m, "tensors": tensors})
        return e

    # ------------------------------------------------------------ host views (tests, I/O)
    def spins_natural(self):
        return device_to_natural(self.spins.detach().cpu().double().numpy(), self.L)

    def couplings_natural(self):
        return device_to_natural(self.couplings.detach().cpu().double().numpy(), self.L)

    def set_spins_natural(self, arr):
        dev = natural_to_device(np.asarray(arr, dtype=np.float64), self.L)
        self.spins.copy_(torch.from_numpy(dev).to(self.spins.dtype))

    def set_couplings_natural(self, arr):
        dev = natural_to_device(np.asarray(arr, dtype=np.float64), self.L)
        self.couplings.copy_(torch.from_numpy(dev).to(self.couplings.dtype))

    def reset_labels(self):
        """Identity labels and zero counters without touching spins (host-side setup)."""
        R = self.R
        ident = torch.arange(R, dtype=torch.int32, device=self.device).expand(self.S, self.C, R)
        self.temp_of_slot.copy_(ident)
        self.slot_of_temp.copy_(ident)
        self.sweep_ctr.zero_()
        self.swap_ctr.zero_()
        self.swap_stats.zero_()
        self.rt_trips.zero_()
        self.rt_state.zero_()
        self.rt_state[..., 0] = 1
        self.guard.zero_()

    def host_state(self):
        """Dict of numpy copies of every state array (natural spin layout)."""
        out = {
            "spins": self.spins_natural(),
            "temp_of_slot": self.temp_of_slot.cpu().numpy(),
            "slot_of_temp": self.slot_of_temp.cpu().numpy(),
            "energy": self.energy.cpu().numpy(),
            "sweep_ctr": self.sweep_ctr.cpu().numpy().view(np.uint32),
            "swap_ctr": self.swap_ctr.cpu().numpy().view(np.uint32),
            "stats": self.swap_stats.cpu().numpy(),
            "rt_state": self.rt_state.cpu().numpy(),
            "rt_trips": self.rt_trips.cpu().numpy(),
        }
        return out
