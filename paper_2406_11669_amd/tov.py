"""A static polytropic star (Tolman-Oppenheimer-Volkoff) in isotropic coordinates, as a fixed 3+1 metric and
hydrostatic primitives.  Initial data only: the oracle and the HIP path both receive its metric and
primitives as inputs, and neither uses this module.

Polytrope p = K rho^G with the ideal-gas energy density e = rho + p / (G - 1).  In the Schwarzschild radius
r the structure follows dm/dr = 4 pi r^2 e, dp/dr = -(e + p)(m + 4 pi r^3 p) / (r (r - 2m)) and the lapse
alpha = exp(nu) with dnu/dr = (m + 4 pi r^3 p) / (r (r - 2m)), out to the surface p = 0 (radius R, mass M).
The isotropic radius rb obeys d ln rb / dr = 1 / (r sqrt(1 - 2m/r)), fixed by matching the exterior
rb = (r - M + sqrt(r^2 - 2 M r)) / 2 at R, where nu(R) = ln(1 - 2M/R) / 2 fixes nu too.  The spatial metric is
conformally flat, gamma_ij = psi^4 delta_ij with psi^4 = (r / rb)^2; outside the star psi = 1 + M / (2 rb)
and alpha = (1 - M / (2 rb)) / (1 + M / (2 rb)).  The shift and the extrinsic curvature vanish.
"""
import math

import numpy as np
from scipy.integrate import solve_ivp
from scipy.interpolate import CubicSpline


class TOV:
    def __init__(self, K=100.0, G=2.0, rho_c=1.28e-3):
        self.K, self.G, self.rho_c = float(K), float(G), float(rho_c)

        def rho_of(p):
            return (max(p, 0.0) / K) ** (1.0 / G)

        def rhs(r, y):
            m, p, nu, lrb = y
            rho = rho_of(p)
            e = rho + max(p, 0.0) / (G - 1.0)
            f = (m + 4.0 * math.pi * r ** 3 * max(p, 0.0)) / (r * (r - 2.0 * m))
            return [4.0 * math.pi * r * r * e, -(e + max(p, 0.0)) * f, f, 1.0 / (r * math.sqrt(1.0 - 2.0 * m / r))]

        surface = lambda r, y: y[1] - 1e-14 * K * rho_c ** G
        surface.terminal = True
        r0 = 1e-6
        p_c = K * rho_c ** G
        e_c = rho_c + p_c / (G - 1.0)
        y0 = [4.0 / 3.0 * math.pi * r0 ** 3 * e_c, p_c, 0.0, math.log(r0)]
        sol = solve_ivp(rhs, (r0, 100.0), y0, events=surface, rtol=1e-12, atol=1e-16, dense_output=True,
                        max_step=0.01)
        R = float(sol.t_events[0][0])
        M = float(sol.y_events[0][0][0])
        self.R, self.M = R, M
        rbR = 0.5 * (R - M + math.sqrt(R * R - 2.0 * M * R))
        rr = np.linspace(r0, R, 20001)
        ys = sol.sol(rr)
        lrb = ys[3] - ys[3][-1] + math.log(rbR)
        nu = ys[2] - ys[2][-1] + 0.5 * math.log(1.0 - 2.0 * M / R)
        rb = np.exp(lrb)
        self.rbR = rbR
        # interior profiles as functions of the isotropic radius
        self._p = CubicSpline(rb, np.maximum(ys[1], 0.0))
        self._alpha = CubicSpline(rb, np.exp(nu))
        self._psi4 = CubicSpline(rb, (rr / rb) ** 2)

    def fields(self, x, y, z, rho_atm):
        """(alpha, psi^4, rho, p) at the points (arrays); rho = rho_atm outside the star, p = K rho^G."""
        M, G, K = self.M, self.G, self.K
        rb = np.sqrt(x * x + y * y + z * z)
        inside = rb < self.rbR
        rc = np.clip(rb, 0.0, self.rbR)
        h = M / (2.0 * np.maximum(rb, self.rbR))  # used outside the star only
        alpha = np.where(inside, self._alpha(rc), (1.0 - h) / (1.0 + h))
        psi4 = np.where(inside, self._psi4(rc), (1.0 + h) ** 4)
        p_in = np.maximum(self._p(rc), 0.0)
        rho = np.where(inside, np.maximum((p_in / K) ** (1.0 / G), rho_atm), rho_atm)
        return alpha, psi4, rho, K * rho ** G
