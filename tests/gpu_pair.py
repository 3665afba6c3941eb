"""Helpers that set up the same ensemble on the GPU (through the C ABI) and in the
oracle, from oracle-generated initial state, and compare them.

Spin bars, each from the arithmetic of the step it bounds:
  * One call of single-kind lattice sweeps (heat-bath or overrelaxation, each the W
    then the B half-sweep; the paper's unit of a sweep, Sec. III.C), compared with the
    oracle replayed from the GPU's own state before the call on the same uniforms:
    every site within 1e-5 (FP32) / 1e-12 (FP64) per component, or, where the site's
    a-priori rounding bound (propagate_bounds) is larger, within that bound.  The
    bound follows the oracle's own trajectory: a field summed in the spin precision
    from exact inputs is off by at most gamma_6 sum_d |J_d| in 2-norm (six fused
    multiply-adds of unit vectors), plus sum_d |J_d| D(y_d) where the neighbours
    already differ by D(y_d) (observed where they are final); the site may then differ
    by as much as the oracle's own update changes when its field moves that far
    (measured on the oracle along the six axis directions and doubled), plus the
    rounding of the update itself.  So a
    site is admitted beyond the bar only with a quantified, per-site reason: a small
    or ill-conditioned field, the heat-bath frame's seam, or a neighbour that was.
  * A composite launch (1 heat-bath + n overrelaxation lattice sweeps, the workloads'
    sweep) is checked in two parts: the launch equals, bit for bit, the same step run
    as single-kind calls on the GPU; and each of those calls meets the rule above
    against the oracle from the GPU's state before it.  (Overrelaxation is a chaotic
    map: two trajectories of one composite step started together drift apart by
    2-3.5x per overrelaxation lattice sweep, so the composite is not compared with
    one long oracle trajectory.)
  * Energies: the fused FP64 energy against the oracle's energy of the GPU's own final
    configuration, within the rounding of the fused sum; against the oracle's own
    trajectory within sum_bonds |J| (|ds_x| + |ds_y|) plus that rounding.
"""
import numpy as np
import torch

import paper_1006_4247_amd as hsg
from paper_1006_4247_amd.ensemble import device_to_natural, natural_to_device
from oracle import hsgref

LATTICE_BAR = {"fp32": 1e-5, "fp64": 1e-12}
ROUND = {"fp32": 5e-6, "fp64": 1e-11}
UNIT = {"fp32": 2.0 ** -24, "fp64": 2.0 ** -53}


def make_pair(L, S, C, betas, seed, prec="fp64", K_max=0, sample_base=0, chain_base=0,
              slot_base=0, cold=False, J=None, spins=None):
    """GPU Ensemble and oracle RefEnsemble in the same state (oracle's init, uploaded)."""
    ref = hsgref.RefEnsemble(L, S, C, betas, seed, prec=prec, sample_base=sample_base,
                             chain_base=chain_base, slot_base=slot_base)
    ref.init_couplings()
    ref.init_spins(cold=cold)
    if J is not None or spins is not None:
        ref.set_state(J=J, spins=spins)
    gpu = hsg.Ensemble(L, S, C, betas, seed, precision=prec, sample_base=sample_base,
                       chain_base=chain_base, slot_base=slot_base, K_max=K_max)
    gpu.set_couplings_natural(ref.J)
    gpu.set_spins_natural(ref.spins)
    gpu.reset_labels()
    gpu.energy_from_scratch(out=gpu.energy)
    torch.cuda.synchronize()
    return gpu, ref


def snapshot(ref):
    return {"spins": ref.spins.copy(), "sweep_ctr": ref.sweep_ctr.copy()}


def _geometry(L):
    """Natural neighbour indices nbr [N][6] (order +x, -x, +y, -y, +z, -z) and parity [N]."""
    N = L ** 3
    x = np.arange(N)
    i, row = x % L, x // L
    j, k = row % L, row // L
    nbr = np.stack([((i + 1) % L) + L * row, ((i - 1) % L) + L * row,
                    i + L * (((j + 1) % L) + L * k), i + L * (((j - 1) % L) + L * k),
                    i + L * (j + L * ((k + 1) % L)), i + L * (j + L * ((k - 1) % L))], axis=1)
    return nbr, (i + j + k) & 1


def _bond_magnitudes(L, J, nbr):
    """|J| of the six bonds of every site [N][6]: the bond to +mu is stored at the site,
    the bond to -mu at the -mu neighbour."""
    a = np.empty((L ** 3, 6))
    for mu in range(3):
        a[:, 2 * mu] = np.abs(J[:, mu])
        a[:, 2 * mu + 1] = np.abs(J[nbr[:, 2 * mu + 1], mu])
    return a


def energy_bound(L, J, ds, prec):
    """Per-slot bound on |H_gpu - H_ref| from per-site spin differences ds [S][C][R][N]."""
    nbr, _ = _geometry(L)
    out = np.zeros(ds.shape[:-1])
    for mu in range(3):
        Jm = np.abs(J[:, :, mu])[:, None, None, :]
        out += np.sum(Jm * (ds + ds[..., nbr[:, 2 * mu]]), axis=-1)
    return out + ROUND[prec] * L ** 3


def _update_rounding(prec, kind, R, r1):
    """Bound on the 2-norm error of one update evaluated in the spin precision from a
    given field (the field's own error is accounted separately).
    binary32 heat-bath: c within 5.2e-7 and sin(theta) within 2e-7 (the angle
      evaluation, measured over 8.4 M (R, r) pairs spanning every regime), sin/cos of
      the azimuth within 1.3e-7 each, the frame and rotation ~12 roundings of unit-size
      values: below 3e-6.
    binary32 overrelaxation: s.S, S.S (three terms each), the 1-ulp reciprocal, the
      product and the fused multiply-subtract, on values of size <= 2: below 2e-6.
    binary64: a few ulp, except that the heat-bath's single expression
      1 - c = -log1p((1 - r) expm1(-2R))/R loses relative precision ~u/r near c = -1,
      i.e. an absolute ~u/(r R)."""
    u = UNIT[prec]
    if prec == "fp32":
        return np.full(R.shape, 3e-6 if kind == 0 else 2e-6)
    base = np.full(R.shape, 64 * u)
    if kind == 0:
        base += 16 * u / (r1 * np.maximum(R, 1e-300))
    return base


_AXES = np.concatenate([np.eye(3), -np.eye(3)])


def propagate_bounds(L, J, s0, seq, beta, seed, slot_global, t, rng32, prec, observed=None):
    """Per-site bound D [N] on the 2-norm of s_gpu - s_oracle after the half-sweeps
    `seq` [(parity, kind, hs)] (kind 0 heat-bath, 1 overrelaxation) of one replica
    started from the same configuration s0 [N][3] on both sides, and the oracle's own
    final configuration.  A site's field, summed in the spin precision from inputs that
    differ by D(y) at the neighbours, is off by at most gamma_6 sum_d |J_d| + sum_d
    |J_d| D(y_d) in 2-norm (six fused multiply-adds of unit vectors); the site may then
    differ by twice the largest change of the oracle's own update when its field moves
    that far along +-x, +-y, +-z (for a linear map the maximum over all directions
    exceeds the maximum over the axes by at most sqrt(3)), plus the rounding of the
    update itself; overrelaxation, linear and norm-preserving in s, adds the site's own
    previous difference.  With `observed` (the GPU's configuration after the call), the
    neighbours' differences are the observed ones wherever those neighbours are not
    updated again later in the call (then they are exactly the inputs' differences)."""
    nbr, par = _geometry(L)
    Jb = _bond_magnitudes(L, J, nbr)
    sum_j = Jb.sum(axis=1)
    u = UNIT[prec]
    g6 = 6 * u / (1 - 6 * u)
    s = np.ascontiguousarray(s0, dtype=np.float64).copy()
    D = np.zeros(L ** 3)
    last = {p: max([i for i, q in enumerate(seq) if q[0] == p], default=-1) for p in (0, 1)}
    done = {0: -1, 1: -1}  # index of the latest half-sweep of each parity so far
    for i, (p, kind, hs) in enumerate(seq):
        q = 1 - p
        Din = D
        if observed is not None and done[q] >= 0 and done[q] == last[q]:
            Din = D.copy()
            xq = np.nonzero(par == q)[0]
            Din[xq] = np.sqrt(((observed[xq] - s[xq]) ** 2).sum(axis=1))
        xs = np.nonzero(par == p)[0]
        S = hsgref.fields(L, J, s, p)[xs]
        eS = g6 * sum_j[xs] + (Jb[xs] * Din[nbr[xs]]).sum(axis=1)
        n = len(xs)
        pert = (S[None, :, :] + eS[None, :, None] * _AXES[:, None, :]).reshape(6 * n, 3)
        if kind == 0:
            r1, r2 = hsgref.hb_uniforms_all(L, rng32, seed, slot_global, t, hs, p)
            r1, r2 = r1[xs], r2[xs]
            base = hsgref.heatbath_many(S, beta, r1, r2)
            moved = hsgref.heatbath_many(pert, beta, np.tile(r1, 6), np.tile(r2, 6)).reshape(6, n, 3)
        else:
            r1 = np.ones(n)
            base = hsgref.overrelax_many(s[xs], S)
            moved = hsgref.overrelax_many(np.tile(s[xs], (6, 1)), pert).reshape(6, n, 3)
        dev = np.sqrt(((moved - base[None]) ** 2).sum(axis=-1)).max(axis=0)
        R = beta * np.sqrt((S ** 2).sum(axis=1))
        newD = 2.0 * dev + _update_rounding(prec, kind, R, r1)
        if kind == 1:
            newD += D[xs]  # the reflection is linear and norm-preserving in s
            if prec == "fp32":  # binary32 sweeps without heat-bath renormalise |s| to 1
                newD += np.abs(np.sqrt((s[xs] ** 2).sum(axis=1)) - 1.0)
        D[xs] = np.minimum(newD, 2.0)  # two unit vectors are at most 2 apart
        s[xs] = base
        done[p] = i
    return D, s


def call_sequence(n_hb, n_or):
    """Half-sweeps (parity, kind, hs) of one sweep of n_hb heat-bath then n_or
    overrelaxation lattice sweeps, forward order."""
    return ([(p, 0, 2 * h + p) for h in range(n_hb) for p in (0, 1)]
            + [(p, 1, 0) for _ in range(n_or) for p in (0, 1)])


def _all_slots(S, C, R):
    return [(s, c, r) for s in range(S) for c in range(C) for r in range(R)]


def gpu_snap(gpu, slots=None):
    """Host copies of the GPU state needed by the checks: spins of `slots` (natural
    layout, all slots by default), labels, counters, energies."""
    slots = slots or _all_slots(gpu.S, gpu.C, gpu.R)
    torch.cuda.synchronize()
    sp = {}
    for (s, c, r) in slots:
        sp[(s, c, r)] = device_to_natural(gpu.spins[s, c, r].detach().cpu().double().numpy(), gpu.L)
    return {"spins": sp, "temp_of_slot": gpu.temp_of_slot.cpu().numpy(),
            "sweep_ctr": gpu.sweep_ctr.cpu().numpy().view(np.uint32).copy(),
            "energy": gpu.energy.cpu().numpy(), "slots": slots}


def _restore(gpu, snap):
    """Put the spins of the snapshot's slots, the counters and energies back."""
    for (s, c, r), a in snap["spins"].items():
        gpu.spins[s, c, r].copy_(torch.from_numpy(natural_to_device(a, gpu.L)).to(gpu.spins.dtype))
    gpu.sweep_ctr.copy_(torch.from_numpy(snap["sweep_ctr"].view(np.int32)))
    gpu.energy.copy_(torch.from_numpy(snap["energy"]))
    torch.cuda.synchronize()


class ParityReport:
    """Spin differences over every checked site of a series of calls: the max, the
    1-in-10^6 quantile, the sites beyond the bar and those admitted by their bound."""

    def __init__(self, prec):
        self.prec = prec
        self.d = []
        self.sites = 0
        self.beyond = 0
        self.admitted_bound_max = 0.0
        self.n_bound_above_bar = 0

    def add(self, d, D):
        bar = LATTICE_BAR[self.prec]
        self.d.append(d)
        self.sites += d.size
        self.beyond += int(np.count_nonzero(d > bar))
        self.n_bound_above_bar += int(np.count_nonzero(D > bar))
        if np.any(d > bar):
            self.admitted_bound_max = max(self.admitted_bound_max, float(D[d > bar].max()))

    def summary(self):
        d = np.concatenate(self.d) if self.d else np.zeros(1)
        return {"sites": self.sites, "max": float(d.max()),
                "q_1e-6": float(np.quantile(d, 1.0 - 1e-6)),
                "beyond_bar": self.beyond, "bound_above_bar": self.n_bound_above_bar,
                "largest_admitting_bound": self.admitted_bound_max}


def check_lattice_call(gpu, pre, post, n_hb, n_or, J=None, report=None, what=""):
    """One GPU call of n_hb heat-bath then n_or overrelaxation lattice sweeps, from
    snapshot `pre` to snapshot `post`, against the oracle replayed slot by slot from the
    GPU's own state before the call (same counters and uniforms)."""
    prec = gpu.precision
    bar = LATTICE_BAR[prec]
    report = report or ParityReport(prec)
    J = gpu.couplings_natural() if J is None else J
    betas = gpu.betas_host
    seq = call_sequence(n_hb, n_or)
    slot_base = int(gpu.desc.slot_base)
    for key in pre["slots"]:
        s, c, r = key
        beta = betas[pre["temp_of_slot"][s, c, r]]
        g = slot_base + (s * gpu.C + c) * gpu.R + r
        t = int(pre["sweep_ctr"][s, c, r])
        D, s_ref = propagate_bounds(gpu.L, J[s], pre["spins"][key], seq, beta, gpu.seed, g, t,
                                    prec == "fp32", prec, observed=post["spins"][key])
        d = np.abs(post["spins"][key] - s_ref).max(axis=-1)
        bad = np.nonzero(d > np.maximum(bar, D))[0]
        assert len(bad) == 0, "%s slot %s: sites beyond both the bar %.0e and their bound: %s" % (
            what, key, bar, [(int(x), float(d[x]), float(D[x])) for x in bad[:8]])
        report.add(d, D)
        # the fused energy against the oracle's energy of the GPU's own configuration
        Hg = hsgref.energy(gpu.L, J[s], post["spins"][key])
        assert abs(post["energy"][s, c, r] - Hg) <= ROUND[prec] * gpu.N, (
            "%s slot %s: fused energy %.12g, oracle %.12g" % (what, key, post["energy"][s, c, r], Hg))
    assert np.array_equal(post["sweep_ctr"], pre["sweep_ctr"] + 1), what
    return report


def sweep_and_check(gpu, n_hb, n_or, tuning=None, launch=None, slots=None, what=""):
    """Run the launch under test (default gpu.sweep(1, n_hb, n_or, tuning)) and check it
    against the oracle: a single-kind call directly (check_lattice_call); a composite
    step through its replay as single-kind calls on the GPU ([n_hb heat-bath lattice
    sweeps] then n_or one-overrelaxation-sweep calls without renormalisation, the
    counter put back after each),
    which must equal the launch bit for bit, each replayed call meeting
    check_lattice_call.  Returns the ParityReport."""
    prec = gpu.precision
    J = gpu.couplings_natural()
    pre = gpu_snap(gpu, slots)
    if launch is None:
        gpu.sweep(1, n_hb, n_or, tuning=tuning)
    else:
        launch()
    post = gpu_snap(gpu, pre["slots"])
    report = ParityReport(prec)
    if n_hb == 0 or n_or == 0:
        return check_lattice_call(gpu, pre, post, n_hb, n_or, J=J, report=report, what=what)
    # the launch's own counters and energies (all slots) before the replay overwrites them
    assert np.array_equal(post["sweep_ctr"], pre["sweep_ctr"] + 1), what
    _restore(gpu, pre)
    calls = [(n_hb, 0)] + [(0, 1)] * n_or
    # the one-overrelaxation-sweep calls without the renormalisation that sweeps without
    # heat-bath apply by default (the composite step has a heat-bath and does not)
    replay_tuning = dict(tuning or {}, flags=hsg._abi.HSG_TUNE_NO_RENORM)
    for k, (h, o) in enumerate(calls):
        a = gpu_snap(gpu, pre["slots"])
        gpu.sweep(1, h, o, tuning=replay_tuning)
        b = gpu_snap(gpu, pre["slots"])
        check_lattice_call(gpu, a, b, h, o, J=J, report=report, what="%s replay call %d" % (what, k))
        gpu.sweep_ctr.copy_(torch.from_numpy(pre["sweep_ctr"].view(np.int32)))
    gpu.sweep_ctr.copy_(torch.from_numpy(post["sweep_ctr"].view(np.int32)))
    fin = gpu_snap(gpu, pre["slots"])
    for key in pre["slots"]:
        assert np.array_equal(fin["spins"][key], post["spins"][key]), (
            "%s slot %s: the launch differs from its replay as single-kind calls" % (what, key))
        s, c, r = key
        assert abs(fin["energy"][s, c, r] - post["energy"][s, c, r]) <= ROUND[prec] * gpu.N, (what, key)
    gpu.energy.copy_(torch.from_numpy(post["energy"]))  # leave the launch's own energies
    torch.cuda.synchronize()
    return report


def compare_ints(gpu, ref, what=""):
    st = gpu.host_state()
    for k in ["temp_of_slot", "slot_of_temp", "sweep_ctr", "swap_ctr", "stats", "rt_state",
              "rt_trips"]:
        assert np.array_equal(st[k], getattr(ref, k)), "%s %s differs" % (what, k)
    return st


def compare_states(gpu, ref, prec, mode="lattice", before=None, n_hb=1, n_or=0,
                   check_energy=True, what="", bar=None):
    """Integer state bit for bit; spins: mode 'lattice' -- after one call of single-kind
    lattice sweeps from the state `before` = snapshot(ref) taken before both sides ran,
    every site within the bar or its a-priori bound (propagate_bounds); mode 'bar' -- a
    plain max |ds| <= bar (callers derive it).  Energies within the bound implied by the
    spin differences."""
    st = compare_ints(gpu, ref, what)
    diff = np.abs(st["spins"] - ref.spins)
    if mode == "lattice":
        lbar = LATTICE_BAR[prec]
        if diff.max() > lbar:
            assert before is not None, "%s: max %.2e > %.1e" % (what, diff.max(), lbar)
            d = diff.max(axis=-1)
            seq = call_sequence(n_hb, n_or)
            for (s, c, r) in zip(*np.nonzero((d > lbar).any(axis=-1))):
                beta = ref.betas[ref.temp_of_slot[s, c, r]]
                g = ref.slot_base + (s * ref.C + c) * ref.R + r
                D, s_ref = propagate_bounds(ref.L, ref.J[s], before["spins"][s, c, r], seq, beta,
                                            ref.seed, g, int(before["sweep_ctr"][s, c, r]),
                                            ref.rng32, prec, observed=st["spins"][s, c, r])
                assert np.array_equal(s_ref, ref.spins[s, c, r]), "replay differs from the oracle's sweep"
                bad = np.nonzero(d[s, c, r] > np.maximum(lbar, D))[0]
                assert len(bad) == 0, "%s slot %s: sites beyond the bar and their bound: %s" % (
                    what, (s, c, r), [(int(x), float(d[s, c, r, x]), float(D[x])) for x in bad[:8]])
    else:
        assert diff.max() <= bar, "%s: max %.2e > %.1e" % (what, diff.max(), bar)
    if check_energy:
        ds = np.sqrt((diff ** 2).sum(axis=-1))
        bound = energy_bound(ref.L, ref.J, ds, prec)
        de = np.abs(st["energy"] - ref.energy)
        assert np.all(de <= bound), "%s energy differs by %.3e (bound %.3e)" % (
            what, de.max(), bound.ravel()[np.argmax(de)])
    return diff.max()


def shadow_leg(L, J, s0, path, down, n_hb, n_or, seed, slot_global, t0, rng32, rel, seed_pert=7):
    """How far two oracle trajectories of one annealing leg drift apart when one starts
    perturbed by `rel` per component: the scale that elementwise comparisons of long
    (chaotic) trajectories can be held to.  path = [l_0 = a, l_1, ..., l_K, l_K+1 = b];
    the up-leg (down = False) sweeps forward at l_1..l_K, the down-leg adjoint at
    l_K..l_1, at counters t0, t0 + 1, ...  Returns (max-abs spin difference at the end,
    its 99th percentile over all components, |W_a - W_b| with
    W = sum_k (l_k+1 - l_k) H(x_k) along the leg)."""
    rng = np.random.default_rng(seed_pert)
    a = np.ascontiguousarray(s0, dtype=np.float64).copy()
    b = a + rel * rng.standard_normal(a.shape)
    b /= np.linalg.norm(b, axis=-1, keepdims=True)
    K = len(path) - 2
    lam = list(reversed(path)) if down else list(path)
    W = [0.0, 0.0]
    for k in range(K + 1):
        for n, x in enumerate((a, b)):
            W[n] += (lam[k + 1] - lam[k]) * hsgref.energy(L, J, x)
        if k < K:
            for x in (a, b):
                hsgref.sweep(L, J, x, n_hb, n_or, lam[k + 1], seed, slot_global, t0 + k, adjoint=down,
                             rng32=rng32)
    d = np.abs(a - b)
    return float(d.max()), float(np.quantile(d, 0.99)), abs(W[0] - W[1])


def decision_log_u(ref, ch, i, n):
    """ln u of the exchange decision of pair i of chain ch at exchange counter n."""
    w = hsgref.philox([i, n, ref.chain_base + ch, 4 << 24], [ref.seed & 0xFFFFFFFF, ref.seed >> 32])
    return float(np.log(hsgref.u01_52(int(w[0]), int(w[1]))))


def anneal_and_check(gpu, ref, parity, K, lam, n_hb, n_or, what=""):
    """One annealed exchange of the pairs i = parity mod 2 on both sides, from the same
    state, compared pair by pair.  Each leg runs 2 K (n_hb + n_or) half-sweeps in one
    launch; its spin bar is that number times the drift of two oracle trajectories of
    the same leg started one update-rounding apart (shadow_leg: the growth of a
    rounding-level difference along this very protocol; each half-sweep injects at most
    that much, and an earlier injection grows at least as much as a later one), and at
    least the lattice bar, for the max and for the 99th percentile over the leg's
    components (where a rare site near the heat-bath frame's seam flips, the max
    saturates while the bulk stays close); its work bar likewise that number times the shadow's work
    difference, plus the fused sums' rounding.  A decision is compared where
    |ln u + W_up + W_dn| exceeds the two works' bars: then labels and statistics bit
    for bit, an accepted pair's states within the
    legs' bars, a rejected pair's states unchanged bit for bit.  Slots outside the
    selected pairs, counters and integer state: bit for bit.  Returns (pairs decided,
    pairs compared, largest p99 spin difference / its bar)."""
    prec = gpu.precision
    S, C, R, L = ref.S, ref.C, ref.R, ref.L
    K = np.asarray(K, dtype=np.int32)
    # both sides start from the GPU's state (an earlier call may have left them apart
    # within its bars)
    st0 = gpu.host_state()
    ref.spins[...] = st0["spins"]
    for k, v in (("temp_of_slot", "temp_of_slot"), ("slot_of_temp", "slot_of_temp"), ("sweep_ctr", "sweep_ctr"),
                 ("swap_ctr", "swap_ctr"), ("stats", "stats"), ("rt_state", "rt_state"), ("rt_trips", "rt_trips"),
                 ("energy", "energy")):
        getattr(ref, v)[...] = st0[k]
    before = ref.spins.copy()
    ctr0, sot0, n0 = ref.sweep_ctr.copy(), ref.slot_of_temp.copy(), ref.swap_ctr.copy()
    stats0, tos0 = ref.stats.copy(), ref.temp_of_slot.copy()
    gpu.set_schedule(K, lam)
    gpu.anneal_swap(parity, n_hb, n_or)
    w_ref = ref.anneal_swap(parity, K, lam, n_hb=n_hb, n_or=n_or)
    st = gpu.host_state()
    w_gpu = gpu.work.cpu().numpy()
    assert np.array_equal(st["sweep_ctr"], ref.sweep_ctr), what
    assert np.array_equal(st["swap_ctr"], ref.swap_ctr), what
    rel = {"fp32": 3e-6, "fp64": 64 * UNIT["fp64"]}[prec]
    touched = np.zeros((S, C, R), dtype=bool)
    n_dec = n_cmp = 0
    worst = 0.0
    for s in range(S):
        sumJ = np.abs(ref.J[s]).sum()
        for c in range(C):
            ch = s * C + c
            for i in range(parity, R - 1, 2):
                a, b = ref.betas[i], ref.betas[i + 1]
                Ki = int(K[i])
                if lam is None:
                    path = [a + k * (b - a) / (Ki + 1) for k in range(Ki + 2)]
                else:
                    path = [a] + [float(v) for v in lam[i][:Ki]] + [b]
                x, y = int(sot0[s, c, i]), int(sot0[s, c, i + 1])
                touched[s, c, x] = touched[s, c, y] = True
                bars, bars99, wb = [], [], []
                n_half = 2 * Ki * (n_hb + n_or)
                for leg, slot in ((0, x), (1, y)):
                    g = ref.slot_base + ch * R + slot
                    sh, sh99, shw = shadow_leg(L, ref.J[s], before[s, c, slot], path, leg == 1, n_hb, n_or,
                                               ref.seed, g, int(ctr0[s, c, slot]), prec == "fp32", rel)
                    bars.append(max(LATTICE_BAR[prec], n_half * sh))
                    bars99.append(max(LATTICE_BAR[prec], n_half * sh99))
                    wb.append(max(n_half, 1) * shw + (b - a) * ROUND[prec] * ref.N)
                for leg in (0, 1):
                    dw = abs(w_gpu[s, c, i, leg] - w_ref[s, c, i, leg])
                    assert dw <= wb[leg], "%s chain %d pair %d leg %d: |dW| %.3e > %.3e" % (
                        what, ch, i, leg, dw, wb[leg])
                n_dec += 1
                margin = decision_log_u(ref, ch, i, int(n0[s, c])) + w_ref[s, c, i, 0] + w_ref[s, c, i, 1]
                if abs(margin) <= wb[0] + wb[1]:
                    continue  # either decision is correct at this precision
                n_cmp += 1
                assert np.array_equal(st["stats"][s, c, i] - stats0[s, c, i],
                                      ref.stats[s, c, i] - stats0[s, c, i]), (what, ch, i)
                for slot in (x, y):
                    assert st["temp_of_slot"][s, c, slot] == ref.temp_of_slot[s, c, slot], (what, ch, i)
                accepted = ref.temp_of_slot[s, c, x] != tos0[s, c, x]
                for leg, slot in ((0, x), (1, y)):
                    if accepted:
                        dd = np.abs(st["spins"][s, c, slot] - ref.spins[s, c, slot])
                        d, d99 = float(dd.max()), float(np.quantile(dd, 0.99))
                        assert d <= bars[leg] and d99 <= bars99[leg], (
                            "%s chain %d pair %d leg %d: max %.3e (bar %.3e), p99 %.3e (bar %.3e)" % (
                                what, ch, i, leg, d, bars[leg], d99, bars99[leg]))
                        worst = max(worst, d99 / bars99[leg])
                    else:
                        assert np.array_equal(st["spins"][s, c, slot], before[s, c, slot]), (what, ch, i)
                        assert np.array_equal(ref.spins[s, c, slot], before[s, c, slot])
    idle = ~touched
    assert np.array_equal(st["spins"][idle], before[idle]), what
    return n_dec, n_cmp, worst
