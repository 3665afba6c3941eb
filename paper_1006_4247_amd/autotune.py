"""Autotuner for the sweep kernels.

For an ensemble shape it times every supported kernel variant (LDS-resident with
one workgroup per replica at several block sizes, persistent double-buffered
workgroups, streaming half-sweeps at several block sizes and replicas per
workgroup) on a throwaway ensemble of the same shape (the caller's Markov chains
are not touched), and keeps the fastest.  Results are cached per device and shape
in a JSON file (default ~/.cache/hsgpt/tuning.json, override with HSGPT_TUNING_CACHE).
"""
import json
import os

import numpy as np
import torch

from . import _abi
from .ensemble import Ensemble, geometric_betas

CANDIDATES = (
    [{"path": 3, "block_threads": nt} for nt in (0, 256, 512)]
    + [{"path": 1, "block_threads": 0}]
    + [{"path": 6, "block_threads": 0}]
    + [{"path": 4, "block_threads": 0}]
    + [{"path": 2, "block_threads": nt, "replicas_per_block": rb}
       for nt in (128, 256, 512) for rb in (1, 2, 4)]
)


def _cache_path():
    return os.environ.get("HSGPT_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "hsgpt", "tuning.json"))


def _key(L, S, C, R, precision, n_hb, n_or, device):
    name = torch.cuda.get_device_properties(device).name.replace(" ", "_")
    return "%s/L%d/S%d/C%d/R%d/%s/%d+%d" % (name, L, S, C, R, precision, n_hb, n_or)


def _time(ens, tuning, n_hb, n_or, reps):
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    ens.sweep(1, n_hb, n_or, tuning=tuning)
    torch.cuda.synchronize(ens.device)
    for a, b in ev:
        a.record()
        ens.sweep(1, n_hb, n_or, tuning=tuning)
        b.record()
    torch.cuda.synchronize(ens.device)
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def tune(L, S, C, R, precision="fp32", n_hb=1, n_or=3, device="cuda", reps=8, use_cache=True,
         candidates=CANDIDATES):
    """Return (best tuning dict, {candidate: ms}) for this shape; cached by default."""
    device = torch.device(device)
    key = _key(L, S, C, R, precision, n_hb, n_or, device)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]["best"], cache[key]["times"]
    ens = Ensemble(L, S, C, geometric_betas(1.0, 8.0, R), 0x70E, precision=precision, device=device)
    ens.init_couplings()
    ens.init_spins()
    times = {}
    for cand in candidates:
        try:
            times[json.dumps(cand, sort_keys=True)] = _time(ens, cand, n_hb, n_or, reps)
        except _abi.HsgError as err:
            if err.code not in (_abi.HSG_ERR_UNSUPPORTED, _abi.HSG_ERR_INVALID):
                raise
    ens.check()
    best = json.loads(min(times, key=times.get))
    if use_cache:
        cache[key] = {"best": best, "times": times}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return best, times


def tune_ensemble(ens, n_hb=1, n_or=3, **kw):
    return tune(ens.L, ens.S, ens.C, ens.R, ens.precision, n_hb, n_or, ens.device, **kw)
