"""Closed forms that pin the oracle, derived from the model of the paper (Sec. I Eq. (2),
Sec. III.A Eq. (HI) and Sec. III.C), independent of the oracle's code.

Open-chain forest: with only the non-wrapping x-bonds present, every bond variable
u_b = s_x . s_{x+1} is independent with density proportional to exp(beta J_b u) on
[-1, 1] (the relative orientation of two O(3) spins has a uniform cosine).  Hence
  <u_b> = Lang(beta J_b),   Lang(a) = coth a - 1/a,
  Var(u_b) = 1/a^2 - 1/sinh^2 a,
  <s_x . s_y> = product of Lang over the bonds of the path (0 on different chains),
  ln Z(beta) = sum_b ln(sinh(beta J_b)/(beta J_b)) + const (cf. Eq. (HI)).
"""
import numpy as np


def langevin(a):
    a = np.asarray(a, dtype=np.float64)
    out = np.empty_like(a)
    small = np.abs(a) < 1e-3
    out[small] = a[small] / 3.0 - a[small] ** 3 / 45.0
    b = a[~small]
    out[~small] = 1.0 / np.tanh(b) - 1.0 / b
    return out


def langevin_var(a):
    a = np.asarray(a, dtype=np.float64)
    out = np.empty_like(a)
    small = np.abs(a) < 1e-2
    out[small] = 1.0 / 3.0 - a[small] ** 2 / 15.0
    b = a[~small]
    # 1/sinh(b)^2 = 4 e^{-2b} / (1 - e^{-2b})^2, without overflow
    out[~small] = 1.0 / b ** 2 - 4.0 * np.exp(-2.0 * np.abs(b)) / np.expm1(-2.0 * np.abs(b)) ** 2
    return out


def log_sinhc(a):
    """ln(sinh(a)/a), stable for all a."""
    a = np.abs(np.asarray(a, dtype=np.float64))
    out = np.empty_like(a)
    small = a < 1e-4
    out[small] = a[small] ** 2 / 6.0
    b = a[~small]
    out[~small] = b + np.log1p(-np.exp(-2.0 * b)) - np.log(2.0 * b)
    return out


def forest_bonds(L, J):
    """List of (x, y, J) for the nonzero bonds of a forest coupling array J [N][3]."""
    N = L ** 3
    out = []
    for x in range(N):
        if J[x, 0] != 0.0:
            i = x % L
            y = x - i + (i + 1) % L
            out.append((x, y, J[x, 0]))
    return out


def forest_mean_H(beta, Jb):
    return -np.sum(Jb * langevin(beta * Jb))


def forest_var_H(beta, Jb):
    return np.sum(Jb ** 2 * langevin_var(beta * Jb))


def forest_log_Z(beta, Jb):
    return np.sum(log_sinhc(beta * Jb))


def forest_chi(L, J, beta):
    """<chi> = (1/N) sum_{x,y} <s_x.s_y>^2 for two independent replicas on the forest."""
    N = L ** 3
    lam = np.zeros((N, 3))
    lam[:, 0] = langevin(beta * J[:, 0])
    total = 0.0
    for row in range(L * L):
        base = row * L
        # correlation along the open chain base .. base+L-1 (bond i joins i and i+1)
        c = np.ones((L, L))
        for a in range(L):
            prod = 1.0
            for b in range(a + 1, L):
                prod *= lam[base + b - 1, 0]
                c[a, b] = c[b, a] = prod
        total += np.sum(c ** 2)
    return total / N


def hb_cdf(c, R):
    """Distribution function of c = s'.S/|S| under density ~ exp(R c) on [-1, 1]."""
    c = np.asarray(c, dtype=np.float64)
    if R == 0.0:
        return (1.0 + c) / 2.0
    # (e^{Rc} - e^{-R}) / (e^{R} - e^{-R}) written without overflow
    return np.exp(R * (c - 1.0)) * (-np.expm1(-R * (1.0 + c))) / (-np.expm1(-2.0 * R))
