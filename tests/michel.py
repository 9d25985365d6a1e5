"""Michel's stationary spherical accretion onto a Schwarzschild black hole, in Kerr-Schild coordinates, as
Valencia primitives (test helper, independent of the oracle and of the HIP path).

An isentropic ideal gas (p = K rho^G) falls radially.  Rest-mass conservation makes rho u r^2 constant
(u = -u^r), and the Bernoulli integral of the stationary flow makes h^2 (1 - 2M/r + u^2) constant, with
h = 1 + G/(G-1) K rho^(G-1).  The transonic solution passes the sonic radius r_c, where u_c^2 = M/(2 r_c) and
the sound speed obeys a_c^2 = u_c^2 / (1 - 3 u_c^2); it is subsonic outside r_c and supersonic inside.  At
every r, rho is the root of the Bernoulli function on that branch.

Kerr-Schild coordinates keep r and the radial direction l = x / r: lapse alpha = 1/sqrt(1 + 2M/r), shift
beta^i = (2M/r) alpha^2 l^i, gamma_ij = delta_ij + (2M/r) l_i l_j, and for the static metric
K_ij = (2 M alpha / r^2) (delta_ij - (2 + M/r) l_i l_j).  The fluid's u^t follows from u.u = -1 with
g_tt = -(1 - 2M/r), g_tr = 2M/r, g_rr = 1 + 2M/r; then W = alpha u^t and v^i = u^i / W + beta^i / alpha.
"""
import math

import numpy as np
from scipy.optimize import brentq, minimize_scalar


class Michel:
    def __init__(self, M=1.0, rc=5.0, rho_c=1.0, G=4.0 / 3.0):
        self.M, self.rc, self.G = float(M), float(rc), float(G)
        uc2 = M / (2.0 * rc)
        ac2 = uc2 / (1.0 - 3.0 * uc2)
        n_c = ac2 / (1.0 - ac2 / (G - 1.0))  # G K rho_c^(G-1) from the sound speed
        self.K = n_c / (G * rho_c ** (G - 1.0))
        self.C1 = rho_c * math.sqrt(uc2) * rc * rc
        hc = self.h(rho_c)
        self.C2 = hc * hc * (1.0 - 2.0 * M / rc + uc2)
        self.rho_c, self.uc = rho_c, math.sqrt(uc2)

    def h(self, rho):
        G = self.G
        return 1.0 + G / (G - 1.0) * self.K * rho ** (G - 1.0)

    def sound2(self, rho):
        G = self.G
        n = G * self.K * rho ** (G - 1.0)
        return n / (1.0 + n / (G - 1.0))

    def bernoulli(self, rho, r):
        u = self.C1 / (rho * r * r)
        return self.h(rho) ** 2 * (1.0 - 2.0 * self.M / r + u * u) - self.C2

    def at(self, r):
        """(rho, u) on the transonic branch at radius r (u = -u^r > 0)."""
        f = lambda lr: self.bernoulli(math.exp(lr), r)
        lo, hi = math.log(self.rho_c) - 30.0, math.log(self.rho_c) + 30.0
        m = minimize_scalar(f, bounds=(lo, hi), method="bounded", options={"xatol": 1e-14})
        lm = m.x
        if f(lm) >= 0.0:  # at the sonic radius (within rounding) the two roots meet
            rho = math.exp(lm)
        elif r > self.rc:  # subsonic: the denser root
            rho = math.exp(brentq(f, lm, hi, xtol=1e-15, rtol=1e-15, maxiter=500))
        else:
            rho = math.exp(brentq(f, lo, lm, xtol=1e-15, rtol=1e-15, maxiter=500))
        return rho, self.C1 / (rho * r * r)

    def primitives(self, x, y, z):
        """(rho, p, v^x, v^y, v^z) at a point (Kerr-Schild coordinates, M at the origin)."""
        M = self.M
        r = math.sqrt(x * x + y * y + z * z)
        l = (x / r, y / r, z / r)
        rho, u = self.at(r)
        ur = -u
        gtt, gtr, grr = -(1.0 - 2.0 * M / r), 2.0 * M / r, 1.0 + 2.0 * M / r
        # gtt ut^2 + 2 gtr ut ur + grr ur^2 + 1 = 0, future-directed root
        a, b, c = gtt, 2.0 * gtr * ur, grr * ur * ur + 1.0
        disc = math.sqrt(b * b - 4.0 * a * c)
        ut = max((-b + disc) / (2.0 * a), (-b - disc) / (2.0 * a))
        alpha = 1.0 / math.sqrt(1.0 + 2.0 * M / r)
        W = alpha * ut
        beta_r = 2.0 * M / r * alpha * alpha
        v = [ur * l[i] / W + beta_r * l[i] / alpha for i in range(3)]
        return np.array([rho, self.K * rho ** self.G, v[0], v[1], v[2]])


class MichelField:
    """Vectorized primitives of a Michel flow over a radial range, from its exact profile tabulated on a
    fine radial grid (rho(r) by a cubic spline in log rho; the rest follows in closed form)."""

    def __init__(self, flow, r_min, r_max, npts=4001):
        from scipy.interpolate import CubicSpline
        self.flow = flow
        rr = np.linspace(r_min, r_max, npts)
        self.spline = CubicSpline(rr, np.log([flow.at(r)[0] for r in rr]))

    def __call__(self, x, y, z):
        f = self.flow
        M, G = f.M, f.G
        r = np.sqrt(x * x + y * y + z * z)
        rho = np.exp(self.spline(r))
        ur = -f.C1 / (rho * r * r)
        a = -(1.0 - 2.0 * M / r)
        b = 2.0 * (2.0 * M / r) * ur
        c = (1.0 + 2.0 * M / r) * ur * ur + 1.0
        disc = np.sqrt(b * b - 4.0 * a * c)
        ut = np.maximum((-b + disc) / (2.0 * a), (-b - disc) / (2.0 * a))
        alpha = 1.0 / np.sqrt(1.0 + 2.0 * M / r)
        W = alpha * ut
        beta_r = 2.0 * M / r * alpha * alpha
        v = [(ur / W + beta_r / alpha) * q / r for q in (x, y, z)]
        return np.stack([rho, f.K * rho ** G, v[0], v[1], v[2]])
