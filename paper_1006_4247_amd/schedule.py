"""Learned annealing schedules.

A small MLP (2 hidden tanh layers of 64, FP32) is a surrogate of the annealed
exchange: from the pair's inverse temperatures, the running-mean energies per site
at both temperatures, the lattice size and a candidate protocol (K sweeps, path
shape gamma) it predicts the mean acceptance probability <min(1, exp(-W))>.  It is
trained on data the method itself generates (annealed exchanges with random
protocols; the work W of every attempt gives the target) with the project's own
forward / backward / Adam kernels, and then picks, per neighbouring pair, the
protocols that maximise the predicted number of accepted exchanges per unit of
sweep work over the whole ladder.

Exactness: a protocol never depends on the current states of the pair - the
energies fed to the network are running means of earlier segments, and the chosen
schedule is frozen for the whole next segment; every exchange is still accepted
with min[1, exp(-W)].  The plain linear schedule with a fixed K is the fallback.

Protocol family: l_k = a + (b - a) g(k / (K + 1)), k = 1..K, with
g(u) = (exp(gamma u) - 1) / (exp(gamma) - 1) (gamma = 0: linear in beta).
"""
import ctypes

import numpy as np
import torch

from . import _abi

N_FEATURES = 7
GAMMAS = (-2.0, -1.0, 0.0, 1.0, 2.0)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class MLP:
    """Device-resident MLP  x -> tanh -> tanh -> y  driven by the hsg_mlp_* kernels."""

    def __init__(self, I=N_FEATURES, H=64, O=1, seed=0, device="cuda", max_batch=65536):
        self.I, self.H, self.O = int(I), int(H), int(O)
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        r = np.random.default_rng(seed)
        sizes = [(H, I), (H,), (H, H), (H,), (O, H), (O,)]
        parts = []
        for shp in sizes:
            if len(shp) == 2:
                parts.append(r.standard_normal(shp).ravel() * np.sqrt(1.0 / shp[1]))
            else:
                parts.append(np.zeros(shp))
        p = np.concatenate(parts).astype(np.float32)
        z = dict(device=self.device)
        self.params = torch.from_numpy(p).to(**z)
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.max_batch = int(max_batch)
        self.acts = torch.zeros((self.max_batch, 4 * self.H), dtype=torch.float32, **z)
        self.y = torch.zeros((self.max_batch, self.O), dtype=torch.float32, **z)
        self.dy = torch.zeros((self.max_batch, self.O), dtype=torch.float32, **z)
        self.loss = torch.zeros((1,), dtype=torch.float64, **z)

    @property
    def n_params(self):
        return self.params.numel()

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _check_in(self, x, cols, name):
        if (x.dim() != 2 or x.shape[1] != cols or x.dtype != torch.float32 or not x.is_contiguous()
                or x.device != self.device):
            raise ValueError("%s must be a contiguous float32 [B][%d] tensor on %s (got %s %s %s)"
                             % (name, cols, self.device, tuple(x.shape), x.dtype, x.device))
        if x.shape[0] > self.max_batch:
            raise ValueError("batch larger than max_batch")

    def forward(self, x):
        """x: device float32 [B][I] -> view of y [B][O] (valid until the next call)."""
        self._check_in(x, self.I, "x")
        B = x.shape[0]
        _abi.check(_abi.lib().hsg_mlp_forward(_p(self.params), self.I, self.H, self.O, _p(x), B,
                                              _p(self.acts), _p(self.y), self._stream()))
        return self.y[:B]

    def loss_and_grad(self, x, t, w=None):
        """Forward, weighted squared error and backward; leaves the gradient in self.grad
        and the loss in self.loss (device)."""
        B = x.shape[0]
        self._check_in(t, self.O, "t")
        if t.shape[0] != B or (w is not None and (w.dim() != 1 or w.shape[0] != B or
                                                  w.dtype != torch.float32 or not w.is_contiguous())):
            raise ValueError("t must be [B][O] and w a contiguous float32 [B] (B = %d)" % B)
        self.forward(x)
        lib = _abi.lib()
        _abi.check(lib.hsg_mlp_mse_grad(_p(self.y), _p(t), _p(w), B, self.O, _p(self.dy), _p(self.loss),
                                        self._stream()))
        _abi.check(lib.hsg_mlp_backward(_p(self.params), self.I, self.H, self.O, _p(x), B, _p(self.acts),
                                        _p(self.dy), _p(self.grad), self._stream()))

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        _abi.check(_abi.lib().hsg_mlp_adam(_p(self.params), _p(self.grad), _p(self.m), _p(self.v),
                                           self.n_params, float(lr), float(b1), float(b2), float(eps),
                                           self.t, self._stream()))

    def fit(self, x, t, w=None, steps=2000, lr=3e-3, report_every=0):
        """Full-batch Adam on device tensors; returns the final loss (host float)."""
        hist = []
        for k in range(steps):
            self.loss_and_grad(x, t, w)
            self.adam_step(lr)
            if report_every and (k % report_every == 0):
                hist.append(float(self.loss.item()))
        self.loss_and_grad(x, t, w)
        return float(self.loss.item()), hist


# ---------------------------------------------------------------- protocols
def path_fraction(u, gamma):
    u = np.asarray(u, dtype=np.float64)
    if abs(gamma) < 1e-12:
        return u
    return np.expm1(gamma * u) / np.expm1(gamma)


def protocol(betas, K, gammas, K_max):
    """Interior points [R-1][K_max] of each pair's protocol (zeros past K)."""
    betas = np.asarray(betas, dtype=np.float64)
    R = len(betas)
    lam = np.zeros((R - 1, max(int(K_max), 1)))
    for i in range(R - 1):
        k = np.arange(1, int(K[i]) + 1)
        lam[i, : int(K[i])] = betas[i] + (betas[i + 1] - betas[i]) * path_fraction(k / (K[i] + 1), gammas[i])
    return lam


def features(beta_a, beta_b, e_a, e_b, L, K, gamma):
    """Normalised network inputs (beta / 8, energy per site, L / 32, K / 32, gamma / 2)."""
    cols = [np.asarray(v, dtype=np.float64) for v in (beta_a, beta_b, e_a, e_b, L, K, gamma)]
    n = max(c.size for c in cols)
    cols = [np.broadcast_to(c, (n,)) for c in cols]
    return np.stack([cols[0] / 8.0, cols[1] / 8.0, cols[2], cols[3], cols[4] / 32.0, cols[5] / 32.0,
                     cols[6] / 2.0], axis=1).astype(np.float32)


def acceptance_from_work(work, parity):
    """Mean of min(1, exp(-(W_up + W_dn))) per pair of the given parity over samples and
    chains; work [S][C][R-1][2]."""
    W = work[..., 0] + work[..., 1]
    a = np.minimum(1.0, np.exp(-np.clip(W, -50, 700)))
    m = a.reshape(-1, a.shape[-1]).mean(axis=0)
    sel = np.zeros(m.shape, dtype=bool)
    sel[parity::2] = True
    return m, sel


# ---------------------------------------------------------------- data and selection
def generate_data(ens, n_rounds, K_choices, rng, gammas=GAMMAS, sweeps_between=2, n_hb=1, n_or=3, leg=None):
    """Annealed exchanges with random protocols (chosen independently of the states) on
    `ens` (needs K_max >= max(K_choices)), sweeps of n_hb + n_or between them, legs of
    `leg` = (n_hb, n_or) sweeps (default the same).  Returns (x [n][7] float32,
    target [n], weight [n]) with one record per (pair, attempt)."""
    leg = leg or (n_hb, n_or)
    X, Y, Wt = [], [], []
    R = ens.R
    betas = ens.betas_host
    n_chains = ens.S * ens.C
    for _ in range(n_rounds):
        K = rng.choice(np.asarray(K_choices), size=R - 1).astype(np.int32)
        G = rng.choice(np.asarray(gammas), size=R - 1)
        ens.set_schedule(K, protocol(betas, K, G, ens.K_max))
        for parity in (0, 1):
            ens.sweep(sweeps_between, n_hb, n_or)
            _, _, e = ens.measure()
            ebar = e.mean(dim=(0, 1)).cpu().numpy()
            ens.anneal_swap(parity, *leg)
            acc, sel = acceptance_from_work(ens.work.cpu().numpy(), parity)
            idx = np.nonzero(sel)[0]
            X.append(features(betas[idx], betas[idx + 1], ebar[idx], ebar[idx + 1], ens.L, K[idx], G[idx]))
            Y.append(acc[idx])
            Wt.append(np.full(idx.size, float(n_chains)))
    return np.concatenate(X), np.concatenate(Y), np.concatenate(Wt)


def train(x, y, w=None, H=64, steps=3000, lr=3e-3, seed=0, device="cuda"):
    """Fit a 1-output network to (x [n][I], y [n]) on device; returns (mlp, final weighted MSE)."""
    x = np.asarray(x, dtype=np.float32)
    net = MLP(x.shape[1], H, 1, seed=seed, device=device, max_batch=max(len(x), 1))
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(net.device)
    yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32).reshape(-1, 1)).to(net.device)
    wd = None
    if w is not None:
        ww = np.asarray(w, dtype=np.float64)
        wd = torch.from_numpy((ww / ww.mean()).astype(np.float32)).to(net.device)
    loss, _ = net.fit(xd, yd, wd, steps=steps, lr=lr)
    return net, loss


def predict(net, x):
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(net.device)
    out = []
    for s in range(0, len(x), net.max_batch):
        out.append(net.forward(xd[s:s + net.max_batch]).cpu().numpy()[:, 0])
    return np.concatenate(out).astype(np.float64)


def ladder_efficiency(acc, K):
    """Accepted exchanges per replica sweep for a ladder with per-pair acceptance acc and
    protocol lengths K, pairs alternating even / odd: each step every replica sweeps once
    and half the pairs attempt an exchange, costing 2 K annealing sweeps each, so
    efficiency = (sum_i acc_i / 2) / (R + sum_i K_i)."""
    acc = np.asarray(acc, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    R = len(acc) + 1
    return (acc.sum() / 2.0) / (R + K.sum())


def select_schedule(net, betas, ebar, L, K_grid, gammas=GAMMAS, floor=0.05, iters=50):
    """Per-pair protocols (K, gamma) that maximise the predicted ladder efficiency
    (accepted exchanges per unit of sweep work, ladder_efficiency) - a fractional
    objective solved by Dinkelbach iterations: with eta the current efficiency, each
    pair independently maximises acc/2 - eta K.  Candidates are restricted to those
    predicted to reach `floor` where any does, so that no pair blocks the ladder."""
    betas = np.asarray(betas, dtype=np.float64)
    R = len(betas)
    grid = [(k, g) for k in K_grid for g in gammas]
    Ks = np.array([k for k, _ in grid], dtype=np.float64)
    Gs = np.array([g for _, g in grid], dtype=np.float64)
    A = np.zeros((R - 1, len(grid)))
    for i in range(R - 1):
        x = features(betas[i], betas[i + 1], ebar[i], ebar[i + 1], L, Ks, Gs)
        A[i] = np.clip(predict(net, x), 0.0, 1.0)
    allowed = A >= floor
    allowed[~allowed.any(axis=1)] = True
    eta = 0.0
    pick = np.zeros(R - 1, dtype=np.int64)
    for _ in range(iters):
        score = np.where(allowed, A / 2.0 - eta * Ks[None, :], -np.inf)
        # ties: the shorter protocol
        score = score - 1e-12 * Ks[None, :]
        pick = np.argmax(score, axis=1)
        new = ladder_efficiency(A[np.arange(R - 1), pick], Ks[pick])
        if abs(new - eta) < 1e-12:
            break
        eta = new
    K = Ks[pick].astype(np.int32)
    G = Gs[pick]
    return K, G, A[np.arange(R - 1), pick]


def round_trip_cost(acc, K, t_base, t_leg):
    """Wall time per round trip, up to a constant, for a ladder whose pairs accept with
    probability acc_i and anneal with K_i sweeps, pairs alternating even / odd.  A
    configuration's temperature index is a random walk that crosses pair i with
    probability acc_i / 2 per step; the commute time between the ends of such a walk
    with a uniform stationary law is proportional to sum_i 1/acc_i steps.  A step costs
    t_base (the sweep, measurement and exchange of every replica) plus t_leg per
    annealing sweep of one pair (both legs, all chains; half the pairs anneal per step):
    cost = (sum_i 1/acc_i) (t_base + t_leg sum_i K_i / 2)."""
    acc = np.maximum(np.asarray(acc, dtype=np.float64), 1e-3)
    K = np.asarray(K, dtype=np.float64)
    return np.sum(1.0 / acc) * (t_base + t_leg * K.sum() / 2.0)


def select_schedule_round_trips(net, betas, ebar, L, K_grid, t_base, t_leg, gammas=GAMMAS, sweeps=20):
    """Per-pair protocols (K, gamma) minimising the predicted wall time per round trip
    (round_trip_cost; K = 0 is the plain exchange of Eq. (1), acceptance min(1, e^{d beta
    d H}) predicted by the same network), by coordinate descent over the pairs from the
    plain exchange everywhere.  t_base and t_leg come from timing the method on the
    device (seconds per step and per annealing sweep of one pair)."""
    betas = np.asarray(betas, dtype=np.float64)
    R = len(betas)
    grid = [(k, g) for k in K_grid for g in (gammas if k > 0 else (0.0,))]
    Ks = np.array([k for k, _ in grid], dtype=np.float64)
    Gs = np.array([g for _, g in grid], dtype=np.float64)
    A = np.zeros((R - 1, len(grid)))
    for i in range(R - 1):
        x = features(betas[i], betas[i + 1], ebar[i], ebar[i + 1], L, Ks, Gs)
        A[i] = np.clip(predict(net, x), 1e-3, 1.0)
    pick = np.array([int(np.argmin(Ks + np.abs(Gs))) for _ in range(R - 1)])  # K = 0 first
    for _ in range(sweeps):
        changed = False
        for i in range(R - 1):
            inv = np.sum(1.0 / A[np.arange(R - 1), pick]) - 1.0 / A[i, pick[i]]
            ksum = Ks[pick].sum() - Ks[pick[i]]
            cost = (inv + 1.0 / A[i]) * (t_base + t_leg * (ksum + Ks) / 2.0)
            best = int(np.argmin(cost + 1e-12 * Ks))
            if best != pick[i]:
                pick[i] = best
                changed = True
        if not changed:
            break
    return Ks[pick].astype(np.int32), Gs[pick], A[np.arange(R - 1), pick]


def fixed_schedule(R, K_fix):
    """The fallback: linear protocol with the same K for every pair."""
    return np.full(R - 1, int(K_fix), dtype=np.int32), np.zeros(R - 1)
