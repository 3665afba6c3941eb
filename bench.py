"""Benchmark of the parallel-tempering hot path on one MI355X.

One step = one pass of the whole hot path over the batch: one sweep of every
replica (1 heat-bath + 3 overrelaxation lattice sweeps, energy fused), one
replica-exchange pass over all neighbouring temperature pairs, and the overlap /
energy measurement.  Default workload: L = 16, 64 disorder samples x 2 chains x
24 temperatures (beta geometric 1..8), FP32 spins with FP64 energies, Gaussian
couplings and random unit spins from a fixed seed, inputs resident in HBM.

Prints one JSON line:  value = site-updates/ns over the timed steps; roofline =
the sweep kernel's algorithmic rate against the chip peak (durations from HIP
events on the launch stream); cpu_baseline = the FP64 oracle on the host cores
on a bounded sample of the same workload.
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and the chip's unit counts.  VALU: 256 CUs x 4 SIMDs, each
# accepting a wave64 binary32 instruction every two clocks (32 lanes per clock), at
# 2.4 GHz = 78.6 T lane-instructions/s, the published 157.3 TFLOP/s binary32 vector peak
# with an FMA counted as two (transcendentals issue at a quarter of that rate).
# `--issue-probe` measures these rates on the device.
HBM_PEAK_GBS = 8000.0
N_CU, CLOCK_GHZ, SIMDS_PER_CU, LANES_PER_SIMD_CLOCK = 256, 2.4, 4, 32
VALU_PEAK_TOPS = N_CU * SIMDS_PER_CU * LANES_PER_SIMD_CLOCK * CLOCK_GHZ / 1e3  # 78.6 T lane-instr/s
WAVE_INSTR_PER_CU_CLOCK = SIMDS_PER_CU * LANES_PER_SIMD_CLOCK / 64  # 2 wave64 instructions

# Algorithmic VALU operations per site update, the op model of the scope table's
# measurement row (one add/mul/FMA/compare, one transcendental or one integer op = 1):
# heat-bath ~150 (18 FMA for the field; norm, direction and R; the angles with their
# exp/log/sqrt/reciprocals; the frame; sin/cos of the azimuth; the rotation; ~50 integer
# ops of Philox per two uniforms), overrelaxation ~30 (field 18, reflection 12).
OPS_HEATBATH_UPDATE = 150
OPS_OVERRELAX_UPDATE = 30

WORKLOADS = {
    "plain-pt-L16-S64-C2-R24": dict(L=16, S=64, C=2, R=24, bmin=1.0, bmax=8.0, prec="fp32",
                                    n_hb=1, n_or=3, seed=0x100642470002),
    "plain-pt-L4-S1-C2-R8-fp64": dict(L=4, S=1, C=2, R=8, bmin=1.0, bmax=6.0, prec="fp64",
                                      n_hb=1, n_or=3, seed=0x100642470001),
}
DEFAULT = "plain-pt-L16-S64-C2-R24"

# cooling / heating parameter: the paper's per lattice size (Sec. IV), and the grid the
# short tuning runs scan
COOLHEAT_EPS_PAPER = {16: 0.017, 24: 0.01}
COOLHEAT_EPS_GRID = (0.001, 0.002, 0.003, 0.004, 0.005, 0.006, 0.008)
# the best eps falls with L (0.003 at L = 16, 0.002 at L = 24, the grid's 0.001 at
# L = 32), so the L = 32 study's grid reaches below 0.001; the others keep the grid above
COOLHEAT_EPS_GRID_STUDY = {32: (0.0004, 0.0006, 0.0008, 0.001, 0.0015, 0.002, 0.003)}
# the per-pair tuner's finer grid (each pair keeps its best)
COOLHEAT_EPS_GRID_PAIRS = (0.001, 0.0015, 0.002, 0.0025, 0.003, 0.0035, 0.004, 0.005, 0.006)


def algorithmic_ops_per_update(n_hb, n_or):
    return (n_hb * OPS_HEATBATH_UPDATE + n_or * OPS_OVERRELAX_UPDATE) / (n_hb + n_or)


def hbm_bytes_per_launch(w, measure=False):
    """Algorithmic HBM bytes of one LDS-resident sweep launch: every replica written
    once and read once, where a sweep that opens with a heat-bath half-sweep needs only
    the sublattice that half-sweep does not update (the other one is redrawn unread);
    the couplings of every sample read once.  With the measurement in the same launch
    (measure=True), the chain-0 replica of every (sample, temperature) is read once more
    for the overlap (the chain-1 replica is still in LDS)."""
    t = 4 if w["prec"] == "fp32" else 8
    N = w["L"] ** 3
    slots = w["S"] * w["C"] * w["R"]
    read = 3 * (N // 2) * t if w["n_hb"] > 0 else 3 * N * t
    extra = w["S"] * w["R"] * 3 * N * t if measure else 0
    return slots * (read + 3 * N * t) + w["S"] * 3 * N * t + extra


def step_kernel(w, fused_ok=True):
    """The kernel of the workload's step that sweeps every replica (the step's dominant
    kernel), as the library picks it: (name, whether it also measures).  With two
    chains at binary32 L = 16 the sweep and the measurement are one launch, unless
    the step is asked for unfused (the measurement as a launch of its own)."""
    if fused_ok and w["prec"] == "fp32" and w["L"] == 16 and w["C"] == 2:
        return "k_resident_mseq<float,16,512>", True
    nq = w["L"] ** 3 // 4
    nt = min(1024, (nq + 63) // 64 * 64)
    nt = 512 if nt >= 1024 else nt
    return "k_resident<%s,%d,%d>" % ("float" if w["prec"] == "fp32" else "double", w["L"], nt), False


OPS_OVERLAP_SITE = 9  # the overlap tensor: nine products per site of a (sample, temperature)


# Sources of the sweep kernel whose HBM traffic the counter summary records; the
# summary is used only while they and the compiler flags are unchanged.
KERNEL_SOURCES = ["paper_1006_4247_amd/csrc/sweep_resident.hip", "paper_1006_4247_amd/csrc/resident_body.h",
                  "paper_1006_4247_amd/csrc/hsg_device.h"]


def kernel_sources_sha256():
    import hashlib
    from paper_1006_4247_amd import build as hip_build
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    # the flags without the include directory, whose absolute path differs between hosts
    h.update(repr([f for f in hip_build.FLAGS if not f.startswith("-I")]).encode())
    return h.hexdigest()


def _kernel_base(kernel):
    return kernel.split("<")[0]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary in profiles/ (each counter scaled by its reading on a plain copy of known
    size), or None if the summary was taken on other kernel sources, for another
    workload or another kernel."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_%s_%s.md" % (_kernel_base(kernel), workload))
    if not os.path.exists(path):
        return None
    digest = kernel_sources_sha256()
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic:"):
                kv = dict(tok.split("=", 1) for tok in line.split()[1:] if "=" in tok)
                if (kv.get("workload") == workload and kv.get("sources_sha256") == digest
                        and kv.get("kernel") == kernel.replace(" ", "")):
                    return int(kv["bytes_per_launch"])
    return None


def measured_valu_instructions(workload, kernel):
    """VALU wave-instructions per launch of `kernel` from the rocprofv3 SQ_INSTS_VALU
    summary in profiles/ (its 'valu:' line), or None if it was taken on other kernel
    sources or for another workload."""
    if workload is None:
        return None
    path = os.path.join(ROOT, "profiles", "valu_lds_counters_%s_%s.md" % (_kernel_base(kernel), workload))
    if not os.path.exists(path):
        return None
    digest = kernel_sources_sha256()
    with open(path) as fh:
        for line in fh:
            if line.startswith("valu:"):
                kv = dict(tok.split("=", 1) for tok in line.split()[1:] if "=" in tok)
                if (kv.get("workload") == workload and kv.get("sources_sha256") == digest
                        and kv.get("kernel") == kernel.replace(" ", "")):
                    return int(kv["insts_valu_per_launch"])
    return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle(hsgref, w, S, budget_s):
    """Steps of the oracle on S samples of the workload for about budget_s seconds:
    (site updates per ns, steps, seconds)."""
    betas = hsgref.geometric_betas(w["bmin"], w["bmax"], w["R"])
    ens = hsgref.RefEnsemble(w["L"], S, w["C"], betas, w["seed"], prec=w["prec"])
    ens.init_couplings()
    ens.init_spins()
    per = S * w["C"] * w["R"] * w["L"] ** 3 * (w["n_hb"] + w["n_or"])
    n = 0
    t0 = time.perf_counter()
    while True:
        ens.sweep(1, w["n_hb"], w["n_or"])
        ens.measure()
        ens.swap(0)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s or n >= 100000:
            break
    return n * per / dt / 1e9, n, dt


def cpu_baseline(w, budget_s):
    """The FP64 oracle, as it stands, on a bounded sample of the workload: on every host
    thread (the reported value) and on one thread."""
    from oracle import hsgref
    S = min(2, w["S"])
    threads = int(hsgref.lib().hsgref_num_threads())
    v, n, dt = _time_oracle(hsgref, w, S, budget_s)
    hsgref.lib().hsgref_set_num_threads(1)
    try:
        v1, n1, dt1 = _time_oracle(hsgref, w, 1, budget_s / 3.0)
    finally:
        hsgref.lib().hsgref_set_num_threads(threads)
    return {"value": v, "unit": "site-updates/ns", "cores": threads, "kind": "oracle",
            "sample": "%d of %d samples x %d chains x %d temps, L=%d, %d steps (sweep + measurement + "
                      "exchange), %.1f s" % (S, w["S"], w["C"], w["R"], w["L"], n, dt),
            "value_one_thread": v1,
            "sample_one_thread": "1 sample, %d steps, %.1f s" % (n1, dt1),
            "cpu": _cpu_model()}


def exchange_comparison(torch, hsg, w, steps_plain, steps_anneal, seed=0x5EED):
    """Accepted exchanges and round trips per GPU-second at matched acceptance (~0.1) on
    the workload's lattice and beta range: plain PT on a ladder dense enough for
    acceptance ~0.1 versus annealed exchanges on the workload's own ladder with (a) one
    protocol length for every pair, chosen for acceptance ~0.1, and (b) the learned
    per-pair schedule; the decimated exchange (paper Sec. III.A) on the dense ladder
    (acceptance against plain PT at equal spacing) and on the workload's own ladder; and
    the cooling / heating exchange (paper Sec. III.B) on the dense ladder.
    Steps are replayed from a HIP graph; the learner's data generation and training are
    timed separately."""
    from paper_1006_4247_amd import runtime
    from paper_1006_4247_amd import schedule as sch

    L, S, C, bmin, bmax = w["L"], w["S"], w["C"], w["bmin"], w["bmax"]
    R0 = w["R"]
    R_dense = int(round(0.9 * np.sqrt(L ** 3) + 1))  # acceptance ~0.1 (erfc estimate)

    def make(R, K_max=32):
        betas = hsg.geometric_betas(bmin, bmax, R)
        e = hsg.Ensemble(L, S, C, betas, seed + R, precision=w["prec"], K_max=K_max)
        e.init_couplings()
        e.init_spins()
        return e

    def timed(e, mode, steps, eps=0.0, **kw):
        run = runtime.PTRun([e], w["n_hb"], w["n_or"], mode=mode, eps=eps, **kw)
        run.step(max(300, steps // 10))  # equilibration, also of the round-trip state
        run.synchronize()
        # read before the capture: host reads between warm and timed replays slow the
        # replays that follow
        st0 = e.swap_stats.cpu().numpy().copy()
        rt0 = e.rt_trips.cpu().numpy().copy()
        run.capture()
        run.synchronize()
        t0 = time.perf_counter()
        run.replay(max(1, steps // run.graph_steps))
        run.synchronize()
        dt = time.perf_counter() - t0
        e.check()
        st = e.swap_stats.cpu().numpy() - st0
        rt = e.rt_trips.cpu().numpy() - rt0
        acc = st[..., 1].sum(axis=(0, 1)) / np.maximum(st[..., 0].sum(axis=(0, 1)), 1)
        n = max(1, steps // run.graph_steps) * run.graph_steps
        return {"temperatures": e.R, "steps": n, "gpu_s": round(dt, 3), "ms_per_step": round(dt / n * 1e3, 4),
                "acceptance_min": round(float(acc.min()), 4), "acceptance_mean": round(float(acc.mean()), 4),
                "accepted_swaps_per_gpu_s": round(float(st[..., 1].sum()) / dt, 1),
                "round_trips": int(rt.sum()), "round_trips_per_gpu_s": round(float(rt.sum()) / dt, 2),
                # counting error of the round trips (Poisson)
                "round_trips_per_gpu_s_err": round(float(np.sqrt(max(rt.sum(), 1))) / dt, 2),
                "_acc": acc}

    out = {"lattice": "L=%d, %d samples x %d chains, beta %.1f..%.1f" % (L, S, C, bmin, bmax)}
    out["plain_dense_ladder"] = timed(make(R_dense), "plain", steps_plain)
    out["plain_own_ladder"] = timed(make(R0), "plain", steps_anneal)
    e = make(R0)
    K_uni = 12
    e.set_schedule(np.full(R0 - 1, K_uni, np.int32))
    r = timed(e, "anneal", steps_anneal)
    r["K"] = K_uni
    out["annealed_uniform_K"] = r
    # the learned schedule: legs of 1 HB + 1 OR lattice sweeps per annealing step, per-pair
    # protocols chosen to minimise the predicted GPU time per round trip from the step's
    # and one annealing sweep's measured cost
    e = make(R0)
    t0 = time.perf_counter()
    rng = np.random.default_rng(1)
    K_grid = [0, 1, 2, 3, 4, 6, 8, 12, 16, 24, 32]
    leg = (1, 1)
    e.sweep(100, w["n_hb"], w["n_or"])

    def step_ms(K):
        e.set_schedule(np.full(R0 - 1, K, np.int32))
        run = runtime.PTRun([e], w["n_hb"], w["n_or"], mode="anneal", anneal_sweep=leg)
        run.capture()
        run.replay(10)
        run.synchronize()
        t1 = time.perf_counter()
        run.replay(100)
        run.synchronize()
        dt = (time.perf_counter() - t1) / 100 * 1e3
        run.release()
        return dt

    t_base = step_ms(0)
    t_leg = (step_ms(4) - t_base) / (4 * (R0 - 1) / 2.0)
    x, y, wt = sch.generate_data(e, 120, K_grid, rng, n_hb=w["n_hb"], n_or=w["n_or"], leg=leg)
    net, loss = sch.train(x, y, wt, steps=3000)
    _, _, et = e.measure()
    ebar = et.mean(dim=(0, 1)).cpu().numpy()
    K, G, pred = sch.select_schedule_round_trips(net, e.betas_host, ebar, L, K_grid, t_base, t_leg)
    learn_s = time.perf_counter() - t0
    e.set_schedule(K, sch.protocol(e.betas_host, K, G, e.K_max))
    r = timed(e, "anneal", steps_anneal, anneal_sweep=leg)
    r.update({"K": [int(k) for k in K], "leg_sweep": "1 HB + 1 OR", "t_base_ms": round(t_base, 4),
              "t_leg_ms": round(t_leg, 5), "learner_s": round(learn_s, 2), "train_mse": round(loss, 5)})
    out["annealed_learned"] = r
    # decimated exchange (paper Sec. III.A), even / odd pairs alternating
    out["decimated_dense_ladder"] = timed(make(R_dense), "decimate", steps_plain)
    out["decimated_own_ladder"] = timed(make(R0), "decimate", steps_anneal)
    # cooling / heating exchange (paper Sec. III.B), eps tuned by short acceptance runs
    # as in the paper; its quoted eps for this L is reported beside
    e = make(R_dense)
    t0 = time.perf_counter()
    eps, table = runtime.tune_coolheat_eps(e, COOLHEAT_EPS_GRID, steps=200, n_hb=w["n_hb"], n_or=w["n_or"])
    tune_s = time.perf_counter() - t0
    r = timed(e, "coolheat", steps_plain, eps=eps)
    r.update({"eps": eps, "eps_paper": COOLHEAT_EPS_PAPER.get(L), "tuner_s": round(tune_s, 2),
              "tuner_acceptance": {("%g" % k): round(v, 4) for k, v in table.items()}})
    out["coolheat_dense_ladder"] = r
    base = out["plain_dense_ladder"]
    for k in ("decimated_dense_ladder", "coolheat_dense_ladder"):
        ratio = out[k]["_acc"] / np.maximum(base["_acc"], 1e-12)
        out[k]["acceptance_vs_plain_same_ladder"] = {
            "min": round(float(ratio.min()), 3), "mean": round(float(ratio.mean()), 3),
            "max": round(float(ratio.max()), 3)}
    for v in out.values():
        if isinstance(v, dict):
            v.pop("_acc", None)
    for k in ("annealed_uniform_K", "annealed_learned", "decimated_dense_ladder", "decimated_own_ladder",
              "coolheat_dense_ladder"):
        out[k]["accepted_swaps_per_gpu_s_vs_plain"] = round(
            out[k]["accepted_swaps_per_gpu_s"] / max(base["accepted_swaps_per_gpu_s"], 1e-12), 4)
    # Round trips on these ladders take far longer than these runs (beta 1..8 spans the
    # whole low-temperature phase), so the counts above describe the approach to steady
    # state, not its rate; steady-state round-trip times per GPU-second come from the
    # paper-ladder study (--paper-ladder L).
    out["round_trips_note"] = ("transient counts: each run is short against the round-trip time of its "
                               "ladder; steady-state round-trip speed-ups are in the paper-ladder study")
    return out


def learned_workload_study(torch, hsg, steps=200, seed=0x100642470005):
    """The learned schedule at its own workload: L = 32, 16 samples x 2 chains x 10
    temperatures, beta geometric 1..8 (plain exchange accepts ~0 on this ladder), FP32.
    The network is trained on annealed exchanges of random protocols (K in 0..32, path
    shapes gamma) generated on this ensemble with the project's kernels; the schedule
    minimises the predicted GPU time per round trip from the measured cost of a step and
    of one annealing sweep of one pair.  Against the fallback (linear protocol, the same
    K for every pair, K = 4 and K = 32): acceptance per pair, GPU time per step, accepted
    exchanges per GPU-second and the round-trip cost (sum_i 1/acc_i) x (ms per step)
    from the measured values."""
    from paper_1006_4247_amd import runtime
    from paper_1006_4247_amd import schedule as sch

    L, S, C, R = 32, 16, 2, 10
    betas = hsg.geometric_betas(1.0, 8.0, R)
    K_grid = [0, 1, 2, 4, 8, 16, 32]
    K_long = 256  # beyond the schedule's range: where acceptance appears on this ladder
    leg = (1, 1)

    def make(K_max):
        # the streaming annealing legs launch 2 K_max (n_hb + n_or) half-sweeps (pairs with
        # shorter protocols idle in the later ones), so K_max is kept to what a run uses
        x = hsg.Ensemble(L, S, C, betas, seed, precision="fp32", K_max=K_max)
        x.init_couplings()
        x.init_spins()
        x.sweep(100, 1, 3)
        return x

    e = make(max(K_grid))

    def run_ms(K, lam, n):
        e.set_schedule(K, lam)
        # statistics read before the capture (host reads between warm and timed replays
        # slow the replays that follow); they then cover the 4 warm replays too
        st0 = e.swap_stats.cpu().numpy().copy()
        run = runtime.PTRun([e], 1, 3, mode="anneal", anneal_sweep=leg)
        run.capture()
        run.replay(4)
        run.synchronize()
        t0 = time.perf_counter()
        run.replay(n)
        run.synchronize()
        dt = time.perf_counter() - t0
        run.release()
        st = e.swap_stats.cpu().numpy() - st0
        acc = st[..., 1].sum(axis=(0, 1)) / np.maximum(st[..., 0].sum(axis=(0, 1)), 1)
        return dt / n * 1e3, acc, float(st[..., 1].sum()) * n / (n + 4) / dt

    t0 = time.perf_counter()
    zero = np.zeros(R - 1, np.int32)
    t_base = run_ms(zero, None, 20)[0]
    t_leg = (run_ms(np.full(R - 1, 8, np.int32), None, 20)[0] - t_base) / (8 * (R - 1) / 2.0)
    rng = np.random.default_rng(5)
    x, y, wt = sch.generate_data(e, 40, K_grid, rng, n_hb=1, n_or=3, leg=leg)
    net, loss = sch.train(x, y, wt, steps=3000)
    _, _, et = e.measure()
    ebar = et.mean(dim=(0, 1)).cpu().numpy()
    K, G, pred = sch.select_schedule_round_trips(net, betas, ebar, L, K_grid, t_base, t_leg)
    learn_s = time.perf_counter() - t0
    out = {"study": "learned-schedule", "L": L, "samples": S, "chains": C, "temperatures": R, "beta": [1.0, 8.0],
           "sweep": "1 HB + 3 OR", "leg_sweep": "1 HB + 1 OR", "steps": steps,
           "data": "synthetic (Gaussian J_xy and random unit spins from Philox, seed %#x)" % seed,
           "t_base_ms": round(t_base, 4), "t_leg_ms": round(t_leg, 5), "train_mse": round(loss, 5),
           "learner_s": round(learn_s, 2)}

    def entry(K, Gm, n=steps):
        ms, acc, aps = run_ms(K, sch.protocol(betas, K, Gm, e.K_max), n)
        return {"K": [int(k) for k in K], "ms_per_step": round(ms, 4),
                "acceptance": [round(float(a), 4) for a in acc], "acceptance_min": round(float(acc.min()), 4),
                "accepted_swaps_per_gpu_s": round(aps, 1),
                "round_trip_cost_ms": round(float(np.sum(1.0 / np.maximum(acc, 1e-3)) * ms), 2)}

    out["learned"] = dict(entry(K, G), gamma=[float(g) for g in G],
                          predicted_acceptance=[round(float(a), 4) for a in pred])
    for kf in (4, 32):
        out["fixed_linear_K%d" % kf] = entry(*sch.fixed_schedule(R, kf))
    e.check()
    e = make(K_long)
    out["fixed_linear_K%d" % K_long] = entry(*sch.fixed_schedule(R, K_long), n=max(20, steps // 4))
    e.check()
    if max(out[k]["acceptance_min"] for k in ("learned", "fixed_linear_K4", "fixed_linear_K32")) == 0.0:
        # no protocol in the schedule's range is ever accepted on this ladder: every cost
        # is set by the acceptance floor, and a speed-up would be an artefact of it
        out["note"] = ("no exchange accepted at K <= 32 on this ladder (every pair of every protocol in the "
                       "schedule's range); the learner then keeps the cheapest protocol; see the K = %d row "
                       "for the protocol length at which acceptance appears" % K_long)
    else:
        for kf in (4, 32):
            f = out["fixed_linear_K%d" % kf]
            out["learned_round_trip_speedup_vs_K%d" % kf] = round(f["round_trip_cost_ms"] /
                                                                 max(out["learned"]["round_trip_cost_ms"], 1e-9), 3)
    return out


# The paper's ladders (Sec. IV): T_i = T_max (T_min/T_max)^((i-1)/(N_T-1)), one heat-bath
# and (5/4) L overrelaxation sweeps per cycle.
PAPER_T_MIN, PAPER_T_MAX = 0.12, 0.19
PAPER_LADDERS = {16: dict(n_temps=15, n_or=20), 24: dict(n_temps=27, n_or=30), 32: dict(n_temps=43, n_or=40)}


STUDY_METHODS = ("standard", "decimation", "coolheat", "coolheat_pairs", "learned")
STUDY_DEFAULT = ("standard", "decimation", "coolheat")


def paper_ladder_study(torch, hsg, L, S, cycles, equil, seed=0x100642470010, methods=STUDY_DEFAULT, n_temps=0,
                       compact=False, split=2):
    """Standard, decimated and cooling / heating tempering (or a subset, `methods`; with
    "coolheat_pairs", cooling / heating with its parameter tuned per pair; with
    "learned", annealed exchanges whose protocols the learned schedule picks to minimise
    the predicted GPU time per round trip) on the paper's ladder for L (Sec. IV; n_temps
    > 0 replaces its N_T, as in the paper's N_T = 22 runs at L = 24), all pairs in
    ascending order every cycle (the annealed exchange alternates even and odd pairs),
    on the same S coupling sets (fresh Gaussian sets; the paper's ten are unpublished)
    with 2 chains: per coupling set the acceptance, the round-trip time t_R = cycles x
    configurations / trips (Sec. IV.B) and tau_int of the overlap susceptibility at
    T_min (window c = 4), and, with standard tempering among the methods, the per-set
    speed-ups over it averaged over the sets (Table II), with their standard errors;
    per GPU-second they are divided by the relative GPU time of a cycle, timed from the
    library's captured cycle of each method (at L <= 16 with `split` > 1 the coupling
    sets as that many parts on streams of their own, for every method alike)."""
    from paper_1006_4247_amd import analysis, runtime
    from paper_1006_4247_amd import schedule as sch

    cfg = PAPER_LADDERS[L]
    R, n_or = (n_temps or cfg["n_temps"]), cfg["n_or"]
    i = np.arange(1, R + 1)
    temps = PAPER_T_MAX * (PAPER_T_MIN / PAPER_T_MAX) ** ((i - 1) / (R - 1))
    betas = 1.0 / temps
    C = 2
    res = {}

    def steps(run, n, what, chunk=2000):
        # in chunks, with a progress line after each (long studies run for minutes)
        done = 0
        while done < n:
            k = min(chunk, n - done)
            run.step(k)
            run.synchronize()
            done += k
            print("[paper-ladder L=%d] %s %d/%d" % (L, what, done, n), file=sys.stderr, flush=True)

    def cycle_ms(e, mode, eps, n=300, **kw):
        # GPU time per cycle from the library's captured cycle
        run = runtime.PTRun([e], 1, n_or, mode=mode, eps=eps, split=split if L <= 16 else 1, **kw)
        run.capture()
        run.replay(20)
        run.synchronize()
        t0 = time.perf_counter()
        run.replay(n)
        run.synchronize()
        dt = time.perf_counter() - t0
        run.release()
        return dt / n * 1e3

    for method, mode in (("standard", "plain"), ("decimation", "decimate"), ("coolheat", "coolheat"),
                         ("coolheat_pairs", "coolheat"), ("learned", "anneal")):
        if method not in methods:
            continue
        K_grid = (0, 1, 2, 4, 8)
        e = hsg.Ensemble(L, S, C, betas, seed, precision="fp32", K_max=max(K_grid) if method == "learned" else 0)
        e.init_couplings()
        e.init_spins()
        t0 = time.perf_counter()
        eps, table, extra = 0.0, None, {}
        kw = dict(pairing=0)
        steps(runtime.PTRun([e], 1, n_or, mode="plain", pairing=0, measure=False), equil // 2,
              method + " equilibration (plain)")
        if method == "coolheat":
            eps, table = runtime.tune_coolheat_eps(e, COOLHEAT_EPS_GRID_STUDY.get(L, COOLHEAT_EPS_GRID), steps=300,
                                                   n_hb=1, n_or=n_or, pairing=0)
        elif method == "coolheat_pairs":
            eps, table = runtime.tune_coolheat_eps_pairs(e, COOLHEAT_EPS_GRID_PAIRS, steps=300, n_hb=1,
                                                         n_or=n_or, pairing=0)
        elif method == "learned":
            # legs of one heat-bath and one overrelaxation lattice sweep per annealing step
            # (any composition keeps the exchange exact; these cost a tenth of the cycle's)
            leg = (1, 1)
            kw = dict(anneal_sweep=leg)
            tl = time.perf_counter()
            e.set_schedule(np.zeros(R - 1, dtype=np.int32))
            t_base = cycle_ms(e, "anneal", 0.0, **kw)
            K0 = 4
            e.set_schedule(np.full(R - 1, K0, dtype=np.int32))
            t_leg = (cycle_ms(e, "anneal", 0.0, **kw) - t_base) / (K0 * (R - 1) / 2.0)
            rng = np.random.default_rng(7)
            x, y, wt = sch.generate_data(e, 40, K_grid, rng, n_hb=1, n_or=n_or, leg=leg)
            net, loss = sch.train(x, y, wt, steps=3000)
            kcol = np.rint(x[:, 5] * 32).astype(int)
            fit = sch.predict(net, x)
            extra_fit = {str(k): [round(float(y[kcol == k].mean()), 4), round(float(fit[kcol == k].mean()), 4)]
                         for k in K_grid if np.any(kcol == k)}
            _, _, et = e.measure()
            ebar = et.mean(dim=(0, 1)).cpu().numpy()
            K, G, pred = sch.select_schedule_round_trips(net, betas, ebar, L, K_grid, t_base, t_leg)
            e.set_schedule(K, sch.protocol(betas, K, G, e.K_max))
            extra = {"K": [int(k) for k in K], "gamma": [float(g) for g in G],
                     "predicted_acceptance": [round(float(a), 4) for a in pred], "leg_sweep": "1 HB + 1 OR",
                     "t_base_ms": round(t_base, 4), "t_leg_ms": round(t_leg, 5), "train_mse": round(loss, 5),
                     "data_vs_fit_acceptance_by_K": extra_fit,
                     "learner_s": round(time.perf_counter() - tl, 2)}
        steps(runtime.PTRun([e], 1, n_or, mode=mode, eps=eps, measure=False, **kw), equil - equil // 2,
              method + " equilibration")
        torch.cuda.synchronize()
        eq_s = time.perf_counter() - t0
        st0 = e.swap_stats.cpu().numpy().copy()
        rt0 = e.rt_trips.cpu().numpy().copy()
        run = runtime.PTRun([e], 1, n_or, mode=mode, eps=eps, series_len=cycles, **kw)
        t0 = time.perf_counter()
        steps(run, cycles, method)
        dt = time.perf_counter() - t0
        e.check()
        chi, _ = run.series(0)  # [T][S][R]
        st = e.swap_stats.cpu().numpy() - st0  # [S][C][R-1][2]
        rt = e.rt_trips.cpu().numpy() - rt0
        acc_set = st[..., 1].sum(axis=(1, 2)) / np.maximum(st[..., 0].sum(axis=(1, 2)), 1)  # [S]
        acc_pair = st[..., 1].sum(axis=(0, 1)) / np.maximum(st[..., 0].sum(axis=(0, 1)), 1)  # [R-1]
        trips = rt.sum(axis=(1, 2)).astype(np.float64)
        t_R = cycles * C * R / np.maximum(trips, 1.0)
        tau = np.array([analysis.tau_int(chi[:, s, R - 1], c=4.0)[0] for s in range(S)])
        # the paper's other two windows (Sec. IV.B), for how the speed-up depends on c
        tau_c = {c: np.array([analysis.tau_int(chi[:, s, R - 1], c=float(c))[0] for s in range(S)])
                 for c in (6, 10)}
        ms = cycle_ms(e, mode, eps, **kw)
        res[method] = dict(acc_set=acc_set, acc_pair=acc_pair, t_R=t_R, tau=tau, tau_c=tau_c, trips=trips,
                           gpu_s=dt, eq_s=eq_s, eps=eps, table=table, ms=ms, extra=extra)

    def q(a):
        a = np.asarray(a, dtype=np.float64)
        return {"mean": round(float(a.mean()), 4), "min": round(float(a.min()), 4),
                "max": round(float(a.max()), 4)}

    def me(a):
        # mean over the coupling sets and its standard error
        a = np.asarray(a, dtype=np.float64)
        return [round(float(a.mean()), 3), round(float(a.std(ddof=1) / np.sqrt(len(a))), 3)]

    out = {"study": "paper-ladder", "L": L, "coupling_sets": S, "chains": C, "temperatures": R,
           "T": [PAPER_T_MIN, PAPER_T_MAX], "sweep": "1 HB + %d OR" % n_or, "exchange": "all pairs ascending",
           "cycles": cycles, "equilibration_cycles": equil, "data": "synthetic Gaussian coupling sets from Philox",
           "cycle_timing": "captured cycle" + (", the sets as %d parts on streams of their own" % split
                                               if split > 1 and L <= 16 else ", the sets as one ensemble")}
    std = res.get("standard")
    for m, r in res.items():
        d = {"acceptance_per_set": q(r["acc_set"]), "acceptance_per_pair": q(r["acc_pair"]),
             "t_R_per_set": q(r["t_R"]), "round_trips": int(r["trips"].sum()),
             "tau_int_chi_Tmin_c4": q(r["tau"]), "gpu_s": round(r["gpu_s"], 2),
             "ms_per_cycle": round(r["ms"], 4)}
        if not compact:
            d["tau_int_chi_Tmin_c6"] = q(r["tau_c"][6])
            d["tau_int_chi_Tmin_c10"] = q(r["tau_c"][10])
            # per coupling set, in set order, so that runs of one method each on the same
            # sets (same seed) can be paired set by set
            d["sets"] = {"acceptance": [round(float(x), 5) for x in r["acc_set"]],
                         "t_R": [round(float(x), 1) for x in r["t_R"]],
                         "tau_int_chi_Tmin_c4": [round(float(x), 3) for x in r["tau"]],
                         "tau_int_chi_Tmin_c6": [round(float(x), 3) for x in r["tau_c"][6]],
                         "tau_int_chi_Tmin_c10": [round(float(x), 3) for x in r["tau_c"][10]]}
        if m in ("coolheat", "coolheat_pairs"):
            d["eps"] = r["eps"] if m == "coolheat" else [float(x) for x in r["eps"]]
            d["eps_paper"] = COOLHEAT_EPS_PAPER.get(L)
            if m == "coolheat":
                d["tuner_acceptance"] = {("%g" % k): round(v, 4) for k, v in r["table"].items()}
            else:
                d["tuner_acceptance_per_pair"] = {("%g" % k): [round(x, 4) for x in v] for k, v in r["table"].items()}
        d.update(r["extra"])
        if m != "standard" and std is not None:
            cost = r["ms"] / std["ms"]  # GPU time per cycle vs standard
            rt_ratio = std["t_R"] / r["t_R"]
            tau_ratio = std["tau"] / r["tau"]
            d["cost_per_cycle_vs_standard"] = round(cost, 3)
            d["speedup_vs_standard"] = {
                "acceptance": me(r["acc_set"] / np.maximum(std["acc_set"], 1e-12)),
                "round_trip": me(rt_ratio), "tau_int_chi": me(tau_ratio),
                # the same per GPU-second: per-cycle speed-ups over the relative cost of a cycle
                "round_trip_per_gpu_s": me(rt_ratio / cost), "tau_int_chi_per_gpu_s": me(tau_ratio / cost),
                "form": "[mean over coupling sets, standard error]"}
            if not compact:
                d["speedup_vs_standard"]["tau_int_chi_c6"] = me(std["tau_c"][6] / r["tau_c"][6])
                d["speedup_vs_standard"]["tau_int_chi_c10"] = me(std["tau_c"][10] / r["tau_c"][10])
        out[m] = d
    return out


# The uneven batch: five size classes, one geometric ladder beta 1..8 each, 424 MB of
# FP32 spins in all (more than the 256 MB MALL, so the sweeps' bytes come from HBM).
UNEVEN = dict(Ls=[8, 12, 16, 24, 32], samples=[128, 64, 32, 16, 8], temps=[8, 12, 16, 24, 32],
              seed=0x100642470004)


def uneven_study(torch, hsg, steps, warm=20):
    """Steps of the uneven batch (sweep 1 HB + 3 OR, measurement, plain exchange of all
    pairs ascending, per class) replayed from the library's captured cycle: site updates
    per ns over the batch, and the algorithmic HBM bytes of its sweeps per second
    (LDS-resident classes: the parity-1 half of every replica read and all of it written
    once per sweep, couplings once; streaming classes, one launch per half-sweep: per
    half-sweep the updated half read and written and the other half read, couplings once
    per sample; wavefront: one read and one write per lattice sweep).  Four forms: the
    library's default kernels with the classes one after another, the same with each
    class on its own stream, the streaming classes one after another beside the
    LDS-resident ones, and the autotuner's kernels and order; and, for the sweeps
    alone, one persistent launch over all classes (tuning path 5) against the classes'
    sweeps one after another."""
    import ctypes
    from paper_1006_4247_amd import _abi, runtime
    ens = runtime.uneven_batch(UNEVEN["Ls"], UNEVEN["samples"], UNEVEN["temps"], UNEVEN["seed"])
    for e in ens:
        e.init_couplings()
        e.init_spins()
    out = {"study": "uneven-batch", "chains": 2, "steps": steps,
           "data": "synthetic (Gaussian J_xy and random unit spins from Philox, seed %#x)" % UNEVEN["seed"]}
    # the streaming classes (HBM-bound) one after another on one stream, so that each has
    # the MALL to itself, and the LDS-resident classes (compute-bound) beside them on another
    grouped = [1 if e.L <= 16 else 0 for e in ens]
    for key, tun, conc in (("default_kernels_in_sequence", None, False), ("default_kernels_concurrent", None, True),
                           ("streaming_beside_resident", None, grouped), ("autotuned", "auto", "auto")):
        run = runtime.PTRun(ens, 1, 3, mode="plain", pairing=0, tunings=tun, concurrent=conc)
        run.step(warm)
        run.capture()
        run.replay(warm)
        run.synchronize()
        t0 = time.perf_counter()
        run.replay(steps)
        run.synchronize()
        dt = time.perf_counter() - t0
        run.check()
        run.release()
        upd = run.site_updates_per_step() * steps
        nbytes = 0
        classes = []
        for e, t in zip(ens, run.tunings):
            N, slots = e.N, e.n_slots
            path = (t or {}).get("path", 0) or (3 if e.L <= 16 else 2)
            if path in (1, 3, 6):  # one launch per sweep
                b = slots * (3 * (N // 2) * 4 + 3 * N * 4) + e.S * 3 * N * 4
            elif path == 4:  # one pass per lattice sweep: read all, write all
                b = 4 * (slots * 2 * 3 * N * 4 + e.S * 3 * N * 4)
            else:  # 8 half-sweeps, each reading the whole replica and writing half of it
                b = 8 * (slots * (3 * N * 4 + 3 * (N // 2) * 4) + e.S * 3 * N * 4)
            nbytes += b * steps
            classes.append({"L": e.L, "samples": e.S, "temperatures": e.R, "tuning": t or "default",
                            "spin_MB": round(slots * 3 * N * 4 / 1e6, 1)})
        gbs = nbytes / dt / 1e9
        out[key] = {"classes": classes, "concurrent": run.concurrent if run.groups is None else run.groups,
                    "spin_MB_total": round(sum(c["spin_MB"] for c in classes), 1),
                    "site_updates_per_ns": round(upd / dt / 1e9, 2), "ms_per_step": round(dt / steps * 1e3, 4),
                    "sweep_algorithmic_hbm_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    # the sweeps alone: one persistent launch over the five classes against the classes'
    # default sweep launches one after another
    for e in ens:
        e.stream = None
    descs = (_abi.HsgEnsemble * len(ens))(*[e.desc for e in ens])
    tb = _abi.HsgTuning(5, 0, 0, 0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def one_launch():
        _abi.check(_abi.lib().hsg_sweep_tuned(descs, len(ens), 1, 1, 3, ctypes.byref(tb), stream))

    def in_sequence():
        for e in ens:
            e.sweep(1, 1, 3)

    res = {}
    n = max(10, steps // 10)
    for name, fn in (("classes_in_sequence", in_sequence), ("one_persistent_launch", one_launch)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n
        res[name] = {"ms_per_sweep": round(dt * 1e3, 4),
                     "site_updates_per_ns": round(sum(e.n_slots * e.N * 4 for e in ens) / dt / 1e9, 2)}
    for e in ens:
        e.check()
    out["sweeps_one_persistent_launch_vs_in_sequence"] = res
    return out


def copy_probe(torch, mib, reps=10):
    """Plain device-to-device copy of `mib` MiB: prints the achieved bandwidth (read + write)."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        b.copy_(a)
        e1.record()
    torch.cuda.synchronize()
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    print(json.dumps({"copy_probe_bytes_per_launch": 2 * n * 4, "read_bytes": n * 4,
                      "write_bytes": n * 4, "avg_ms": float(ms.mean()),
                      "GBs": 2 * n * 4 / (ms.mean() / 1e3) / 1e9}), flush=True)


PROBE_KINDS = ("fp32_fma", "fp64_fma", "fp32_exp2", "lds_4B_reads", "lds_16B_reads")


def issue_probe(torch, reps=5):
    """Issue rates of the compute units (hsg_probe_issue): every thread runs rounds of 16
    independent operations of one kind.  Prints, per kind and launch shape, the lane
    operations (VALU kinds) or LDS bytes per second from HIP events on the launch
    stream, and the same per CU and clock at the published 2.4 GHz."""
    from paper_1006_4247_amd import _abi
    lib = _abi.lib()
    shapes = (("1 wave per SIMD", 256, 256), ("full occupancy", 2048, 1024))
    sink = torch.empty(2048 * 1024, dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    out = {"probe": "issue", "clock_GHz_assumed": CLOCK_GHZ, "n_cu": N_CU, "results": []}
    for kind, kname in enumerate(PROBE_KINDS):
        for sname, groups, threads in shapes:
            iters = 2000 if kind in (1, 2) else 4000

            def run():
                _abi.check(lib.hsg_probe_issue(kind, groups, threads, iters, ctypes.c_void_p(sink.data_ptr()),
                                               ctypes.c_void_p(stream.cuda_stream)))
            run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                run()
            e1.record(stream)
            torch.cuda.synchronize()
            s_per = e0.elapsed_time(e1) / 1e3 / reps
            lane_ops = groups * threads * iters * 16
            rec = {"kind": kname, "shape": sname, "groups": groups, "threads": threads,
                   "ms": round(s_per * 1e3, 4)}
            if kind <= 2:
                rate = lane_ops / s_per
                rec.update(T_lane_ops_per_s=round(rate / 1e12, 2),
                           lane_ops_per_cu_clock=round(rate / N_CU / (CLOCK_GHZ * 1e9), 1))
            else:
                rate = lane_ops * 4 / s_per
                rec.update(TB_per_s=round(rate / 1e12, 2),
                           bytes_per_cu_clock=round(rate / N_CU / (CLOCK_GHZ * 1e9), 1))
            out["results"].append(rec)
            phase("probe %s, %s done" % (kname, sname))
    print(json.dumps(out), flush=True)


def phase(name):
    """A progress line on stderr naming the phase that starts (so a log says where a
    run stopped)."""
    print("[bench %.1fs] %s" % (time.perf_counter() - _T0, name), file=sys.stderr, flush=True)


_T0 = time.perf_counter()


def headline(torch, hsg, w, steps, warmup, clock_warmup_s, fused_ok=True, split=2):
    """The workload's step (sweep of every replica, measurement, plain exchange of all
    pairs ascending) as the library's captured cycle (a plan: graphs of up to 16 cycles
    per launch; the samples as `split` parts on streams of their own), timed over
    exactly `steps` replays after `warmup` untimed ones; before those, the
    cycle is replayed for about `clock_warmup_s` seconds so that the chip runs at its
    steady clock.  The dominant kernel's average duration is then taken from HIP events
    around a batch of back-to-back sweep launches on the same stream."""
    from paper_1006_4247_amd import runtime
    dev = torch.device("cuda:0")
    betas = hsg.geometric_betas(w["bmin"], w["bmax"], w["R"])
    ens = hsg.Ensemble(w["L"], w["S"], w["C"], betas, w["seed"], precision=w["prec"], device=dev)
    ens.init_couplings()
    ens.init_spins()
    # unfused: the sweep kernel with one workgroup per replica (tuning path 3), then the
    # measurement pass.  The cycle runs the samples as two halves on streams of their own
    # (the plan's split: one half's exchange and launch edges overlap the other's sweep;
    # the same results bit for bit)
    run = runtime.PTRun([ens], w["n_hb"], w["n_or"], mode="plain", pairing=0,
                        tunings=None if fused_ok else [{"path": 3}], split=split)
    run.capture()
    stream = torch.cuda.current_stream(dev)
    # exchange statistics over every replay of the cycle, read before the first one: a
    # PyTorch kernel and device-to-host copy on this stream between the clock warm-up
    # and the timed replays slowed the replays that followed by about 8 % for tens of
    # steps (measured: 0.168 against 0.155 ms per step)
    stats0 = ens.swap_stats.sum(dim=(0, 1)).cpu().numpy()
    # steady clocks: replay until clock_warmup_s has passed (not counted)
    t_w = time.perf_counter()
    n_clock = 0
    while time.perf_counter() - t_w < clock_warmup_s:
        run.replay(200)
        run.synchronize()
        n_clock += 200
    run.replay(warmup)
    torch.cuda.synchronize()
    evs = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    t0 = time.perf_counter()
    evs[0].record(stream)  # replays go to this stream
    run.replay(steps)
    evs[1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    device_ms = evs[0].elapsed_time(evs[1])
    run.check()
    stats1 = ens.swap_stats.sum(dim=(0, 1)).cpu().numpy()
    acc = (stats1[:, 1] - stats0[:, 1]).astype(np.float64)
    att = (stats1[:, 0] - stats0[:, 0]).astype(np.float64)
    run.release()
    ens.stream = None  # eager calls below go to this stream (the run had given it its own)
    # the dominant kernel (the step's sweep, with the measurement where the library
    # fuses it): back-to-back launches on this stream, events around them
    name, fused = step_kernel(w, fused_ok)

    def launch():
        if fused:
            ens.sweep_measure(1, w["n_hb"], w["n_or"])
        else:
            ens.sweep(1, w["n_hb"], w["n_or"])

    n_k = max(50, min(400, int(0.05 / max(elapsed / max(steps, 1), 1e-5))))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(5):
        launch()
    ev0.record(stream)
    for _ in range(n_k):
        launch()
    ev1.record(stream)
    torch.cuda.synchronize()
    avg_launch_s = ev0.elapsed_time(ev1) / 1e3 / n_k
    ens.check()

    N = w["L"] ** 3
    slots = w["S"] * w["C"] * w["R"]
    upd_per_step = slots * N * (w["n_hb"] + w["n_or"])
    ops = algorithmic_ops_per_update(w["n_hb"], w["n_or"]) * upd_per_step
    if fused:
        ops += OPS_OVERLAP_SITE * N * w["S"] * w["R"]
    alu_achieved = ops / avg_launch_s / 1e12
    hbm_achieved = hbm_bytes_per_launch(w, measure=fused) / avg_launch_s / 1e9
    workload = [k for k, v in WORKLOADS.items() if v == w]
    valu = measured_valu_instructions(workload[0] if workload else None, name)
    roofline = {"bound": "alu", "achieved": round(alu_achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "Tops/s", "frac": round(alu_achieved / VALU_PEAK_TOPS, 4),
                "traffic": measured_traffic(workload[0], name) if workload else None,
                "kernel": "%s (one sweep of every replica%s per launch)" % (
                    name, " and the measurement" if fused else ""),
                "avg_launch_ms": round(avg_launch_s * 1e3, 5),
                "avg_launch_from": "HIP events around %d back-to-back %s launches on the run's stream" % (
                    n_k, "sweep-and-measurement" if fused else "sweep"),
                "ops_per_site_update": algorithmic_ops_per_update(w["n_hb"], w["n_or"]),
                "ops_per_launch": int(ops),
                "valu_issue_frac": (round(valu / (N_CU * WAVE_INSTR_PER_CU_CLOCK * CLOCK_GHZ * 1e9 * avg_launch_s), 4)
                                    if valu else None),
                "valu_wave_instructions_per_launch": valu,
                "hbm_algorithmic_GBs": round(hbm_achieved, 1),
                "hbm_frac": round(hbm_achieved / HBM_PEAK_GBS, 4),
                "sweep_site_updates_per_ns": round(upd_per_step / avg_launch_s / 1e9, 2)}
    return {"value": round(steps * upd_per_step / (elapsed * 1e9), 3),
            "acceptance_over": "the %d clock warm-up, %d warm-up and %d timed steps" % (n_clock, warmup, steps),
            "ms_per_step": round(elapsed * 1e3 / steps, 5),
            "timing": {"timed": "%d replays of the captured cycle (hsg_plan_run: graphs of up to 16 cycles per "
                                "launch%s)" % (steps, "; the samples as %d parts on streams of their own" % split
                                               if split > 1 else ""),
                       "device_ms_per_step": round(device_ms / max(steps, 1), 5),
                       "clock_warmup": "%d untimed replays (%.2f s) before the %d warm-up steps"
                                       % (n_clock, clock_warmup_s, warmup)},
            "roofline": roofline,
            "acceptance": [round(a / max(t, 1), 4) for a, t in zip(acc, att)],
            "accepted_swaps_per_gpu_s": round(float(acc.sum()) * steps / max(n_clock + steps + warmup, 1) / elapsed, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exchange-comparison", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the binary64 line, the uneven batch and the paper-ladder study")
    ap.add_argument("--clock-warmup", type=float, default=1.5, metavar="SECONDS",
                    help="untimed replays of the step before the counted warm-up (steady clocks)")
    ap.add_argument("--uneven-steps", type=int, default=200, help="steps of the uneven batch in the default run")
    ap.add_argument("--study-sets-default", type=int, default=64,
                    help="coupling sets of the default run's compact L = 16 paper-ladder study")
    ap.add_argument("--study-cycles-default", type=int, nargs=2, default=[3000, 12000], metavar=("EQUIL", "MEASURE"))
    ap.add_argument("--compare-steps", type=int, nargs=2, default=[20000, 4000], metavar=("PLAIN", "ANNEAL"),
                    help="steps of the plain dense-ladder run and of each annealed run")
    ap.add_argument("--paper-ladder", type=int, default=0, metavar="L",
                    help="only run the study of standard / decimated / cooling-heating tempering on "
                         "the paper's ladder for L (16, 24 or 32) and print its JSON line")
    ap.add_argument("--study-sets", type=int, default=64, help="coupling sets of the paper-ladder study")
    ap.add_argument("--study-split", type=int, default=2,
                    help="parts of the coupling sets on streams of their own in the timed cycles (every method)")
    ap.add_argument("--study-cycles", type=int, nargs=2, default=[10000, 20000], metavar=("EQUIL", "MEASURE"),
                    help="equilibration and measurement cycles of the paper-ladder study")
    ap.add_argument("--study-methods", nargs="+", choices=STUDY_METHODS, default=list(STUDY_DEFAULT),
                    help="tempering methods of the paper-ladder study")
    ap.add_argument("--study-temps", type=int, default=0, metavar="N_T",
                    help="number of temperatures of the paper-ladder study (default: the paper's for L)")
    ap.add_argument("--uneven", type=int, default=0, metavar="STEPS",
                    help="only time STEPS steps of the uneven batch (five size classes, 424 MB of "
                         "spins) and print its JSON line")
    ap.add_argument("--split", type=int, default=2,
                    help="parts of the samples the captured cycle runs on streams of their own (1 = whole)")
    ap.add_argument("--unfused", action="store_true",
                    help="headline step with the sweep kernel and the measurement as two launches "
                         "(profiles the sweep kernel as the dominant one)")
    ap.add_argument("--issue-probe", action="store_true",
                    help="issue rates of the compute units (VALU kinds, LDS reads), then exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM bandwidth probe and the "
                         "calibration of rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: every (sample, chain) is an independent Markov chain, "
              "so N GPUs would each run 1/N of the samples with no communication; run it with "
              "--gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1006_4247_amd as hsg

    if args.issue_probe:
        issue_probe(torch)
        return
    if args.copy_probe:
        copy_probe(torch, args.copy_probe)
        return
    if args.uneven:
        print(json.dumps(uneven_study(torch, hsg, args.uneven)), flush=True)
        return
    if args.paper_ladder:
        if args.paper_ladder not in PAPER_LADDERS:
            print("--paper-ladder takes L = 16, 24 or 32", file=sys.stderr)
            sys.exit(2)
        print(json.dumps(paper_ladder_study(torch, hsg, args.paper_ladder, args.study_sets,
                                            args.study_cycles[1], args.study_cycles[0],
                                            methods=tuple(args.study_methods), n_temps=args.study_temps,
                                            split=args.study_split)),
              flush=True)
        return
    w = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    phase("headline: %s" % args.workload)
    head = headline(torch, hsg, w, args.steps, args.warmup, args.clock_warmup, fused_ok=not args.unfused,
                    split=args.split)
    line = {
        "metric": "site-updates/ns & HBM roofline %; accepted swaps per GPU-s vs plain PT",
        "value": head["value"], "unit": "site-updates/ns", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": w["prec"].replace("fp", "f"),
        "data": "synthetic (Gaussian J_xy and random unit spins from Philox, seed %#x)" % w["seed"],
        "config": {"workload": args.workload, "L": w["L"], "samples": w["S"], "chains": w["C"],
                   "temperatures": w["R"], "beta": [w["bmin"], w["bmax"]], "sweep": "%d HB + %d OR" % (w["n_hb"], w["n_or"]),
                   "exchange": "all neighbour pairs, ascending, every step", "measure": "every step",
                   "step_kernels": ("sweep, then the measurement as a launch of its own" if args.unfused
                                    else "the library's choice (sweep and measurement fused where it fuses)")},
        "timing": head["timing"],
        "roofline": head["roofline"],
        "swap_acceptance_per_pair": head["acceptance"],
        "accepted_swaps_per_gpu_s": head["accepted_swaps_per_gpu_s"],  # this ladder (acceptance ~0)
    }
    if not args.no_extras:
        if w["prec"] == "fp32":
            phase("the same workload in binary64 (the paper's precision)")
            w64 = dict(w, prec="fp64")
            h64 = headline(torch, hsg, w64, max(args.steps, 200), args.warmup, 0.5)
            line["fp64_same_shape"] = {"value": h64["value"], "unit": "site-updates/ns",
                                       "ms_per_step": h64["ms_per_step"],
                                       "sweep_kernel_avg_ms": h64["roofline"]["avg_launch_ms"],
                                       "kernel": h64["roofline"]["kernel"], "steps": max(args.steps, 200)}
        # one GPU's share of the workload when it runs on N GPUs (64 / N samples each):
        # the shards exchange nothing during the run, so a GPU's share at its real
        # shape is what decides the job's rate; fewer samples per launch fill fewer CUs
        phase("one GPU's share of the workload on 2, 4 and 8 GPUs")
        shares = {}
        for n in (2, 4, 8):
            if w["S"] % n:
                continue
            s_n = w["S"] // n
            # the cycle in two halves only where each half's launch still holds 192 or
            # more workgroups (one per (sample, temperature)); at 8 x 24 the halves
            # measured 141 against 166 site-updates/ns for the whole
            sp = 2 if (s_n // 2) * w["R"] >= 192 else 1
            hn = headline(torch, hsg, dict(w, S=s_n), max(args.steps, 200), args.warmup, 0.3, split=sp)
            shares[str(n)] = {"samples": s_n, "value": hn["value"], "unit": "site-updates/ns",
                              "ms_per_step": hn["ms_per_step"], "split": sp,
                              "sweep_kernel_avg_ms": hn["roofline"]["avg_launch_ms"],
                              "steps": max(args.steps, 200)}
        line["per_gpu_share"] = shares
        phase("uneven batch (five size classes, beyond the MALL)")
        line["uneven_batch"] = uneven_study(torch, hsg, args.uneven_steps)
        phase("learned schedule at L=32 (16 x 2 x 10)")
        line["learned_schedule_L32"] = learned_workload_study(torch, hsg)
        phase("paper-ladder study L=16 (round trips per GPU-second)")
        line["paper_ladder_L16"] = paper_ladder_study(torch, hsg, 16, args.study_sets_default,
                                                      args.study_cycles_default[1], args.study_cycles_default[0],
                                                      methods=STUDY_DEFAULT + ("learned",), compact=True)
    if not args.no_exchange_comparison:
        phase("exchange comparison (dense ladder, annealed, decimated, cooling/heating)")
        line["exchange_comparison"] = exchange_comparison(torch, hsg, w, *args.compare_steps)
    if not args.no_cpu_baseline:
        phase("cpu baseline (the oracle on the host)")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    phase("done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
