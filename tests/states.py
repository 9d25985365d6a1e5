"""Random physical states and metrics for pointwise tests (test-side helpers, no method arithmetic)."""
import numpy as np


def random_metric(rng, curved=True, amp=0.2):
    """(alpha, beta^x..z, gxx, gxy, gxz, gyy, gyz, gzz) with a positive-definite spatial metric."""
    if not curved:
        return np.array([1.0, 0, 0, 0, 1.0, 0, 0, 1.0, 0, 1.0])
    alpha = rng.uniform(0.5, 1.5)
    beta = rng.uniform(-0.3, 0.3, 3)
    M = rng.uniform(-amp, amp, (3, 3))
    g = np.eye(3) + 0.5 * (M + M.T)
    return np.array([alpha, *beta, g[0, 0], g[0, 1], g[0, 2], g[1, 1], g[1, 2], g[2, 2]])


def gmat(m10):
    return np.array([[m10[4], m10[5], m10[6]], [m10[5], m10[7], m10[8]], [m10[6], m10[8], m10[9]]])


def random_prim(rng, m10, vmax=0.9, rho=(0.1, 1.5), p=(0.1, 1.0), log=False):
    g = gmat(m10)
    if log:
        r = 10 ** rng.uniform(np.log10(rho[0]), np.log10(rho[1]))
        pp = 10 ** rng.uniform(np.log10(p[0]), np.log10(p[1]))
    else:
        r = rng.uniform(*rho)
        pp = rng.uniform(*p)
    d = rng.normal(size=3)
    norm = np.sqrt(d @ g @ d)
    v = d / norm * rng.uniform(0.0, vmax)
    return np.array([r, pp, *v])


def random_Bt(rng, m10, bmax=1.0):
    g = gmat(m10)
    sqrtg = np.sqrt(np.linalg.det(g))
    return sqrtg * rng.uniform(-bmax, bmax, 3)
