"""Small statistics helpers for the statistical pins (test-side only)."""
import numpy as np


def block_mean_err(x, n_blocks=20):
    """Mean and its standard error from n_blocks contiguous blocks (first axis is time)."""
    x = np.asarray(x, dtype=np.float64)
    n = (x.shape[0] // n_blocks) * n_blocks
    b = x[:n].reshape((n_blocks, n // n_blocks) + x.shape[1:]).mean(axis=1)
    return b.mean(axis=0), b.std(axis=0, ddof=1) / np.sqrt(n_blocks)


def block_var_err(x, n_blocks=20):
    """Variance and its standard error by jackknife over blocks."""
    x = np.asarray(x, dtype=np.float64)
    n = (x.shape[0] // n_blocks) * n_blocks
    blocks = x[:n].reshape(n_blocks, n // n_blocks)
    full = x[:n].var()
    jk = np.array([np.delete(blocks, i, axis=0).ravel().var() for i in range(n_blocks)])
    err = np.sqrt((n_blocks - 1) / n_blocks * np.sum((jk - jk.mean()) ** 2))
    return full, err


def jackknife_mean_err(x, n_blocks=20):
    """Mean of a time series and its block-jackknife error: the n_blocks leave-one-block-out
    means m_k give err^2 = (n-1)/n sum_k (m_k - mean(m))^2."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x) // n_blocks * n_blocks
    b = x[:n].reshape(n_blocks, -1).mean(axis=1)
    loo = (b.sum() - b) / (n_blocks - 1)
    err = np.sqrt((n_blocks - 1) / n_blocks * np.sum((loo - loo.mean()) ** 2))
    return float(b.mean()), float(err)
