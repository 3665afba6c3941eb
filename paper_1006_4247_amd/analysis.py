"""Host-side analysis of parallel-tempering runs: the figures of merit of the paper's
Sec. IV (acceptance rates, round-trip times, integrated autocorrelation times) and
blocked / jackknife error estimates (Sec. IV.B blocks the data into sub-ensembles).

Plain numpy on small arrays read back from the device; nothing here is on the hot path.
"""
import numpy as np


def block_means(x, n_blocks):
    """Means of n_blocks contiguous blocks along axis 0 (the tail that does not fill a
    block is dropped)."""
    x = np.asarray(x, dtype=np.float64)
    n = (x.shape[0] // n_blocks) * n_blocks
    if n == 0:
        raise ValueError("need at least n_blocks samples")
    return x[:n].reshape((n_blocks, n // n_blocks) + x.shape[1:]).mean(axis=1)


def jackknife(x, n_blocks=20, f=None):
    """Jackknife estimate and error of f(mean) over n_blocks blocks along axis 0.

    f maps a mean (array over the trailing axes) to the quantity of interest; the
    default is the mean itself.  Returns (estimate, error)."""
    b = block_means(x, n_blocks)
    f = f or (lambda m: m)
    total = b.mean(axis=0)
    loo = np.array([f((total * n_blocks - b[i]) / (n_blocks - 1)) for i in range(n_blocks)])
    est = f(total)
    err = np.sqrt((n_blocks - 1) / n_blocks * np.sum((loo - loo.mean(axis=0)) ** 2, axis=0))
    return est, err


def autocorrelation(x, t_max):
    """Normalised autocorrelation rho(t), t = 0..t_max, of the series x (Sec. IV.B):
    rho(t) = <(O_i - <O>)(O_{i+t} - <O>)> / <(O - <O>)^2>, averaged over the n - t
    available pairs (computed with a zero-padded FFT)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    t_max = min(t_max, n - 1)
    d = x - x.mean()
    var = np.mean(d * d)
    if var == 0.0:
        return np.concatenate([[1.0], np.zeros(t_max)])
    m = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(d, m)
    acov = np.fft.irfft(f * np.conj(f), m)[: t_max + 1] / (n - np.arange(t_max + 1))
    return acov / var


def tau_int(x, c=4.0, t_cap=None):
    """Integrated autocorrelation time tau = 1/2 + sum_{t=1}^{t_f} rho(t) with the window
    chosen self-consistently as the smallest t_f >= c tau(t_f) (Sec. IV.B; the paper
    uses c = 4, 6, 10).  Returns (tau, t_f)."""
    x = np.asarray(x, dtype=np.float64)
    t_cap = t_cap or max(1, len(x) // 4)
    rho = autocorrelation(x, t_cap)
    tau = 0.5
    for t in range(1, t_cap + 1):
        tau += rho[t]
        if t >= c * tau:
            return tau, t
    return tau, t_cap


def acceptance(stats):
    """Per-pair acceptance from swap statistics [..., R-1, 2] (attempts, accepts),
    summed over the leading axes."""
    s = np.asarray(stats).reshape(-1, np.asarray(stats).shape[-2], 2).sum(axis=0)
    return s[:, 1] / np.maximum(s[:, 0], 1)


def round_trip_time(rt_trips, n_steps):
    """t_R = (steps x configurations) / round trips (Sec. IV.B), per chain and overall.

    rt_trips: [..., R] completed trips per configuration.  Returns (overall, per_chain)
    with inf where no trip completed."""
    t = np.asarray(rt_trips, dtype=np.float64)
    R = t.shape[-1]
    per_chain = t.reshape(-1, R).sum(axis=1)
    with np.errstate(divide="ignore"):
        pc = np.where(per_chain > 0, n_steps * R / np.maximum(per_chain, 1), np.inf)
        total = t.sum()
        overall = n_steps * t.reshape(-1, R).size / total if total > 0 else np.inf
    return overall, pc


def paper_energy(e):
    """The paper's internal energy E = (1/L^3) sum J s.s (Sec. II) = -H/N."""
    return -np.asarray(e)
