"""Drivers for parallel-tempering runs on one GPU.

`PTRun` steps one or several size classes (`Ensemble`s) through the hot path:
sweep and measurement of the swept configurations (one launch where an ensemble's two
chains fit one workgroup per temperature) -> exchange (plain, Eq. (1), annealed,
decimated or cooling / heating).  Each size class runs
on its own HIP stream if asked (concurrent=True), so the kernels of an uneven batch
(several L, sample counts and ladders) overlap on the chip; `capture()` builds a plan of
the library
(hsg_plan_create: the library captures one cycle of every class into a HIP graph,
each class on a capture stream of its own) and `replay()` runs it (hsg_plan_run, one
graph launch per cycle).  Observables are copied into device-resident time series.
"""
import ctypes
import json

import numpy as np
import torch

from . import _abi
from .ensemble import Ensemble


class PTRun:
    """mode 'plain': exchange every step with `pairing` (0 = all pairs ascending);
    mode 'anneal': annealed exchange alternating even / odd pairs (schedules must be
    set on the ensembles); mode 'decimate': decimated exchange (paper Sec. III.A),
    alternating even / odd pairs, or all pairs ascending every step if pairing == 0;
    mode 'coolheat': cooling / heating exchange (paper Sec. III.B) with parameter
    `eps` (one number, R - 1 per-pair values, or one such sequence per ensemble),
    pairs as for 'decimate'.  tunings: None (the library's default kernels), 'auto' (the
    autotuner's fastest sweep variant per ensemble shape, cached per device), or one
    tuning dict (or None) per ensemble.  concurrent: size classes one after another on
    the current stream (False), each on a stream of its own so that their kernels
    overlap (True), whichever of the two runs the cycle faster ('auto', timed on
    the run's own steps), or a list with one stream index per ensemble (the ensembles
    of one index one after another on one stream, the streams side by side).  split:
    in captured cycles (plans), each ensemble runs as `split` parts of consecutive
    samples on streams of their own, so that one part's exchange and launch edges
    overlap another's sweep; the results are the same bit for bit (L <= 16)."""

    def __init__(self, ensembles, n_hb=1, n_or=3, mode="plain", pairing=None, measure=True,
                 series_len=0, tunings=None, anneal_sweep=None, eps=0.0, concurrent=False, split=1):
        if mode not in ("plain", "anneal", "decimate", "coolheat"):
            raise ValueError("mode must be 'plain', 'anneal', 'decimate' or 'coolheat'")
        # cooling / heating parameter: one number, R - 1 per-pair values shared by the
        # ensembles, or one such sequence per ensemble (prepared on the device here, so
        # that steps and graph captures copy nothing)
        scalar = not isinstance(eps, (list, tuple, torch.Tensor)) and np.ndim(eps) == 0
        self.eps = eps if scalar else None
        if pairing is None:
            pairing = 0 if mode == "plain" else -1
        if isinstance(ensembles, Ensemble):
            ensembles = [ensembles]
        self.ens = list(ensembles)
        if self.eps is not None:
            self.eps = float(self.eps)
            self.eps_of = [self.eps] * len(self.ens)
        else:
            nested = (isinstance(eps, (list, tuple)) and len(eps) == len(self.ens)
                      and (isinstance(eps[0], torch.Tensor) or np.ndim(eps[0]) > 0))
            per = list(eps) if nested else [eps] * len(self.ens)
            self.eps_of = [e.eps_pairs_tensor(x) for e, x in zip(self.ens, per)]
        self.n_hb, self.n_or = n_hb, n_or
        self.split = int(split)
        if self.split < 1:
            raise ValueError("split must be >= 1")
        self.mode = mode
        self.pairing = pairing
        self.measure = measure
        if isinstance(tunings, str):
            if tunings != "auto":
                raise ValueError("tunings must be None, 'auto' or one tuning dict (or None) per ensemble")
            from .autotune import tune_ensemble
            tunings = [tune_ensemble(e, n_hb, n_or)[0] for e in self.ens]
        self.tunings = list(tunings) if tunings else [None] * len(self.ens)
        self.anneal_sweep = anneal_sweep or (n_hb, n_or)
        dev = self.ens[0].device
        self.device = dev
        # stream groups: a list with one index per ensemble puts the ensembles of one index
        # one after another on one stream and the groups side by side
        self.groups = None
        if isinstance(concurrent, (list, tuple)):
            if len(concurrent) != len(self.ens) or any(int(g) < 0 or int(g) >= len(self.ens) for g in concurrent):
                raise ValueError("concurrent as a list needs one stream index in [0, n) per ensemble")
            self.groups = [int(g) for g in concurrent]
            concurrent = True
        elif concurrent not in (False, True, "auto"):
            raise ValueError("concurrent must be False, True, 'auto' or one stream index per ensemble")
        self.concurrent = bool(concurrent) and len(self.ens) > 1
        n_streams = (max(self.groups) + 1) if self.groups else len(self.ens)
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(n_streams)] if len(self.ens) > 1 else []
        self.parity = 0
        self.steps_done = 0
        self.graph = None
        self.plan = None
        self.graph_steps = 0
        self.series_len = int(series_len)
        self.series_pos = 0
        if self.series_len:
            self.chi_series = [torch.zeros((self.series_len,) + tuple(e.chi.shape), dtype=torch.float64,
                                           device=dev) for e in self.ens]
            self.e_series = [torch.zeros((self.series_len,) + tuple(e.e_temp.shape), dtype=torch.float64,
                                         device=dev) for e in self.ens]
        for e in self.ens:
            e.stream = None  # steps run on the current stream, or on self.streams when concurrent
        if concurrent == "auto" and len(self.ens) > 1 and not self.series_len:
            choice = self._pick_concurrency()
            self.groups = choice if isinstance(choice, list) else None
            self.concurrent = bool(choice)

    # ------------------------------------------------------------ one step
    def _step_one(self, i, parity, slot):
        e = self.ens[i]
        if self.measure and self.tunings[i] is None:
            e.sweep_measure(1, self.n_hb, self.n_or)
        else:
            e.sweep(1, self.n_hb, self.n_or, tuning=self.tunings[i])
            if self.measure:
                e.measure()
        if self.measure and self.series_len and slot is not None:
            self.chi_series[i][slot].copy_(e.chi)
            self.e_series[i][slot].copy_(e.e_temp)
        if self.mode == "plain":
            e.swap(self.pairing)
        elif self.mode == "decimate":
            e.decimate_swap(self.pairing if self.pairing >= 0 else parity + 1)
        elif self.mode == "coolheat":
            e.coolheat_swap(self.eps_of[i], self.pairing if self.pairing >= 0 else parity + 1)
        else:
            e.anneal_swap(parity, *self.anneal_sweep)

    def _fork(self, fn):
        if not self.concurrent:
            for i in range(len(self.ens)):
                fn(i)
            return
        cur = torch.cuda.current_stream(self.device)
        for s in self.streams:
            s.wait_stream(cur)
        for i in range(len(self.ens)):
            with torch.cuda.stream(self.streams[self.groups[i] if self.groups else i]):
                fn(i)
        for s in self.streams:
            cur.wait_stream(s)

    def kind_groups(self):
        """Stream groups by kind: the streaming classes (HBM-bound) on stream 0, one after
        another so that each has the MALL to itself, the LDS-resident classes
        (compute-bound) beside them on stream 1; None if the batch has one kind only."""
        res = []
        for e, t in zip(self.ens, self.tunings):
            path = (t or {}).get("path", 0)
            res.append(e.L <= 16 if not path else path in (1, 3, 6))
        if all(res) or not any(res):
            return None
        return [1 if r else 0 for r in res]

    def _pick_concurrency(self, steps=20):
        """Autotuning of the batch's order: time captured cycles with the size classes one
        after another, with each on its own stream, and (batches of both kinds) with the
        streaming classes on one stream beside the LDS-resident ones (real steps of the
        run, counted), and keep the fastest.  Returns the choice for `concurrent`."""
        import time
        best, best_t = False, None
        candidates = [False, True]
        if self.kind_groups() is not None:
            candidates.append(self.kind_groups())
        for conc in candidates:
            self.groups = conc if isinstance(conc, list) else None
            self.concurrent = bool(conc)
            self.capture()
            self.replay(2)
            self.synchronize()
            t0 = time.perf_counter()
            self.replay(steps)
            self.synchronize()
            dt = time.perf_counter() - t0
            self.release()
            if best_t is None or dt < best_t:
                best, best_t = conc, dt
        return best

    def step(self, n=1):
        """n eager steps (asynchronous)."""
        if self.graph is not None:
            raise RuntimeError("this run replays a captured graph; call replay()")
        for _ in range(n):
            slot = self._next_slot()
            par = self.parity
            self._fork(lambda i: self._step_one(i, par, slot))
            self.parity ^= 1
            self.steps_done += 1

    def _next_slot(self):
        if not self.series_len:
            return None
        if self.series_pos >= self.series_len:
            raise RuntimeError("time series full; read it with series() and reset_series()")
        p = self.series_pos
        self.series_pos += 1
        return p

    # ------------------------------------------------------------ graphs
    def plan_settings(self):
        """The cycle as the library's plan settings (hsg_plan_create's JSON)."""
        names = {"plain": "plain", "anneal": "anneal", "decimate": "decimate", "coolheat": "coolheat"}
        st = {"exchange": names[self.mode], "n_hb": int(self.n_hb), "n_or": int(self.n_or),
              "measure": int(bool(self.measure))}
        if self.mode == "plain":
            st["pairing"] = int(self.pairing)
        elif self.mode in ("decimate", "coolheat"):
            st["pairing"] = int(self.pairing) if self.pairing >= 0 else -1
        if self.mode == "anneal":
            st["anneal_n_hb"], st["anneal_n_or"] = int(self.anneal_sweep[0]), int(self.anneal_sweep[1])
        if self.mode == "coolheat":
            if self.eps is not None:
                st["eps"] = float(self.eps)
            else:
                st["eps"] = [float(v) for t in self.eps_of for v in t.detach().cpu().numpy()]
        st["streams"] = int(self.concurrent or self.split > 1)
        if self.groups and self.concurrent:
            st["stream"] = list(self.groups)
        if self.split > 1:
            st["split"] = self.split
        if any(t is not None for t in self.tunings):
            for k in ("path", "block_threads", "replicas_per_block"):
                st[k] = [int((t or {}).get(k, 0)) for t in self.tunings]
        return st

    def capture(self, n_steps=None, unroll=None):
        """Build the library plan of one cycle of every size class (captured into HIP
        graphs inside the library).  Time series are not recorded by plans.  The plan
        reads the ensembles' descriptors as they are now (schedules included)."""
        if self.series_len:
            raise RuntimeError("plans do not record time series (series_len must be 0)")
        self.release()
        torch.cuda.synchronize(self.device)
        for e in self.ens:
            e._fill_desc()
        descs = (_abi.HsgEnsemble * len(self.ens))(*[e.desc for e in self.ens])
        plan = ctypes.c_void_p()
        st = self.plan_settings()
        if unroll is not None:
            st["unroll"] = int(unroll)
        txt = json.dumps(st).encode()
        _abi.check(_abi.lib().hsg_plan_create(descs, len(self.ens), txt, ctypes.byref(plan)))
        self.plan = plan
        self._plan_descs = descs
        _abi.check(_abi.lib().hsg_plan_set_next_parity(self.plan, int(self.parity)))
        self.graph = plan
        self.graph_steps = 1
        return plan

    def replay(self, n=1):
        """Run n cycles of the plan (on the current stream)."""
        st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        _abi.check(_abi.lib().hsg_plan_run(self.plan, int(n), st))
        self.steps_done += int(n)
        self.parity = int(_abi.lib().hsg_plan_next_parity(self.plan))

    def release(self):
        """Destroy the plan (if any); eager steps are possible again."""
        if getattr(self, "plan", None) is not None:
            torch.cuda.synchronize(self.device)
            _abi.lib().hsg_plan_destroy(self.plan)
        self.plan = None
        self.graph = None

    def __del__(self):
        try:
            self.release()
        except Exception:  # interpreter shutdown
            pass

    # ------------------------------------------------------------ checkpoint / resume
    def save(self, prefix):
        """Checkpoint every size class (prefix + '.<i>.safetensors') and the run's own
        position (which parity the alternating exchanges take next) in prefix + '.json'."""
        import json
        self.synchronize()
        for i, e in enumerate(self.ens):
            e.save("%s.%d.safetensors" % (prefix, i))
        with open(prefix + ".json", "w") as fh:
            json.dump({"parity": self.parity, "steps_done": self.steps_done, "n_classes": len(self.ens),
                       "mode": self.mode, "pairing": self.pairing, "n_hb": self.n_hb, "n_or": self.n_or,
                       "eps": self.eps if self.eps is not None
                       else [t.cpu().numpy().tolist() for t in self.eps_of]}, fh)

    def restore(self, prefix):
        """Load the state written by save() into this run's ensembles (same shapes).  The
        run's own dynamics (exchange mode, pairing, sweep composition, cooling / heating
        parameters) must be those of the saved run: a resumed run that silently changed
        them would not continue the same Markov chain, so a mismatch raises."""
        import json
        from safetensors import safe_open
        with open(prefix + ".json") as fh:
            pos = json.load(fh)
        if pos["n_classes"] != len(self.ens):
            raise ValueError("checkpoint holds %d size classes, this run %d" % (pos["n_classes"], len(self.ens)))
        mine = {"mode": self.mode, "pairing": self.pairing, "n_hb": self.n_hb, "n_or": self.n_or}
        for k, v in mine.items():
            if pos.get(k) != v:
                raise ValueError("checkpoint %s = %r, this run %r" % (k, pos.get(k), v))
        eps = (self.eps if self.eps is not None else [t.cpu().numpy().tolist() for t in self.eps_of])
        if self.mode == "coolheat" and not np.allclose(np.asarray(pos.get("eps"), dtype=np.float64),
                                                       np.asarray(eps, dtype=np.float64), rtol=0, atol=0):
            raise ValueError("checkpoint eps = %r, this run %r" % (pos.get("eps"), eps))
        # kernels of this run may still be in flight on the classes' streams
        self.synchronize()
        for i, e in enumerate(self.ens):
            with safe_open("%s.%d.safetensors" % (prefix, i), framework="pt") as f:
                m = json.loads(f.metadata()["hsg_meta"])
                e.load_state_dict({"meta": m, "tensors": {k: f.get_tensor(k) for k in f.keys()}})
        self.parity = int(pos["parity"])
        self.steps_done = int(pos["steps_done"])
        self.synchronize()

    # ------------------------------------------------------------ results
    def synchronize(self):
        torch.cuda.synchronize(self.device)

    def check(self):
        self.synchronize()
        for e in self.ens:
            e.check()

    def series(self, i=0):
        """(chi [T][S][R], e [T][S][C][R]) recorded so far for size class i (host copies)."""
        self.synchronize()
        n = self.series_pos
        return self.chi_series[i][:n].cpu().numpy(), self.e_series[i][:n].cpu().numpy()

    def reset_series(self):
        self.series_pos = 0

    def site_updates_per_step(self):
        return sum(e.n_slots * e.N * (self.n_hb + self.n_or) for e in self.ens)

    def anneal_updates_per_step(self):
        """Site updates spent in one annealed exchange pass (both legs of every selected
        pair), averaged over the two parities."""
        tot = 0.0
        for e in self.ens:
            K = e.anneal_K.cpu().numpy()
            for par in (0, 1):
                tot += 0.5 * 2 * K[par::2].sum() * e.S * e.C * e.N * sum(self.anneal_sweep)
        return tot


def uneven_batch(Ls, samples, temps, seed, chains=2, precision="fp32", bmin=1.0, bmax=8.0,
                 device="cuda", K_max=0):
    """Size classes L[i] with samples[i] samples x chains x temps[i] temperatures on one
    geometric beta ladder bmin..bmax each, with disjoint random streams."""
    from .ensemble import geometric_betas
    ens = []
    sb = cb = qb = 0
    for L, S, R in zip(Ls, samples, temps):
        e = Ensemble(L, S, chains, geometric_betas(bmin, bmax, R), seed, precision=precision,
                     device=device, sample_base=sb, chain_base=cb, slot_base=qb, K_max=K_max)
        sb += S
        cb += S * chains
        qb += S * chains * R
        ens.append(e)
    return ens


def linear_schedule(betas, K):
    """Interior points of the linear protocol l_k = a + k (b - a)/(K + 1), k = 1..K, per pair."""
    betas = np.asarray(betas, dtype=np.float64)
    K = np.broadcast_to(np.asarray(K, dtype=np.int64), (len(betas) - 1,))
    K_max = int(K.max(initial=0))
    lam = np.zeros((len(betas) - 1, max(K_max, 1)))
    for i in range(len(betas) - 1):
        a, b = betas[i], betas[i + 1]
        for k in range(1, K[i] + 1):
            lam[i, k - 1] = a + k * (b - a) / (K[i] + 1)
    return lam


def tune_coolheat_eps(ens, grid, steps=200, n_hb=1, n_or=3, pairing=-1):
    """The paper's tuning of the cooling / heating parameter (Sec. III.B): short runs at
    each eps of `grid` (in order, on the ensemble itself, so they also serve as
    equilibration), keeping the eps with the highest mean acceptance over the ladder.
    Returns (eps, {eps: mean acceptance})."""
    table = {}
    for eps in grid:
        run = PTRun([ens], n_hb, n_or, mode="coolheat", eps=eps, measure=False, pairing=pairing)
        st0 = ens.swap_stats.cpu().numpy().copy()
        run.step(steps)
        run.synchronize()
        st = ens.swap_stats.cpu().numpy() - st0
        acc = st[..., 1].sum(axis=(0, 1)) / np.maximum(st[..., 0].sum(axis=(0, 1)), 1)
        table[float(eps)] = float(acc.mean())
    best = max(table, key=table.get)
    return best, table


def tune_coolheat_eps_pairs(ens, grid, steps=200, n_hb=1, n_or=3, pairing=-1):
    """Per-pair tuning, as the paper suggests (Sec. IV): the same short runs at each
    eps of `grid`, keeping for every pair of temperatures the eps with its highest
    acceptance (a pair's acceptance depends on its own parameter).  Returns (eps per
    pair [R-1], {eps: acceptance per pair})."""
    table = {}
    for eps in grid:
        run = PTRun([ens], n_hb, n_or, mode="coolheat", eps=eps, measure=False, pairing=pairing)
        st0 = ens.swap_stats.cpu().numpy().copy()
        run.step(steps)
        run.synchronize()
        st = ens.swap_stats.cpu().numpy() - st0
        table[float(eps)] = st[..., 1].sum(axis=(0, 1)) / np.maximum(st[..., 0].sum(axis=(0, 1)), 1)
    keys = list(table)
    acc = np.stack([table[k] for k in keys])  # [grid][R-1]
    best = np.array([keys[j] for j in np.argmax(acc, axis=0)], dtype=np.float64)
    return best, {k: v.tolist() for k, v in table.items()}
