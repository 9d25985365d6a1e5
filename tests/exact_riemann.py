"""Exact solution of the one-dimensional special-relativistic Riemann problem for an ideal gas with no magnetic
field and no tangential velocity (test helper, independent of the oracle and of the HIP path).

With B = 0, a flat metric (alpha = 1, beta = 0, gamma_ij = delta_ij) and velocities along x only, the evolved
system of Sec. 2.2 reduces to special-relativistic hydrodynamics in one dimension, whose Riemann problem has
a closed-form solution up to one scalar root: a left wave, a contact and a right wave separate the two
initial states; each wave is a shock or a rarefaction according to whether the middle pressure lies above or
below the pressure ahead of it.  The pieces follow from the mathematics, written out here:

* Rarefaction.  Along the characteristics that cross a fan, dp/(rho h c) = -+ dv/(1 - v^2); for an isentropic
  ideal gas the left side integrates to (1/sqrt(G-1)) ln((sqrt(G-1) + c)/(sqrt(G-1) - c)), so
  atanh(v) +- (1/sqrt(G-1)) ln((sqrt(G-1) + c)/(sqrt(G-1) - c)) is constant across a left (+) or right (-)
  fan, with p/rho^G constant.  Inside the fan, x/t equals the characteristic speed (v -+ c)/(1 -+ v c).
* Shock.  The jump conditions for rest mass, momentum and energy give the Taub adiabat
  h_b^2 - h_a^2 = (h_b/rho_b + h_a/rho_a)(p_b - p_a) (a quadratic in h_b for an ideal gas), the invariant mass
  flux j^2 = -(p_b - p_a)/(h_b/rho_b - h_a/rho_a), the shock speed
  V = (rho_a^2 W_a^2 v_a +- |j| sqrt(j^2 + rho_a^2)) / (rho_a^2 W_a^2 + j^2), and the velocity behind it from
  the momentum jump (solved here directly from [S v + p] = V [S], which the tests check against all three
  jump conditions).

h = 1 + G/(G-1) p/rho, c^2 = G p/(rho h), W = 1/sqrt(1 - v^2).  The middle pressure is the root of
v_left(p) - v_right(p), bracketed and found by Brent's method.
"""
import math

import numpy as np
from scipy.optimize import brentq


def enthalpy(rho, p, G):
    return 1.0 + G / (G - 1.0) * p / rho


def sound_speed(rho, p, G):
    return math.sqrt(G * p / (rho * enthalpy(rho, p, G)))


def conserved(rho, p, v, G):
    """(D, S, tau) of special-relativistic hydrodynamics in one dimension."""
    W2 = 1.0 / (1.0 - v * v)
    h = enthalpy(rho, p, G)
    D = rho * math.sqrt(W2)
    S = rho * h * W2 * v
    return np.array([D, S, rho * h * W2 - p - D])


def flux(rho, p, v, G):
    D, S, tau = conserved(rho, p, v, G)
    return np.array([D * v, S * v + p, S - D * v])


def _fan_log(c, G):
    a = math.sqrt(G - 1.0)
    return math.log((a + c) / (a - c)) / a


def rarefaction(state, p, G, sign):
    """State behind a rarefaction into `state` = (rho, p, v) that lowers the pressure to p.
    sign = +1 for the left fan, -1 for the right fan."""
    rho_a, p_a, v_a = state
    rho = rho_a * (p / p_a) ** (1.0 / G)
    inv = math.atanh(v_a) + sign * _fan_log(sound_speed(rho_a, p_a, G), G)
    v = math.tanh(inv - sign * _fan_log(sound_speed(rho, p, G), G))
    return rho, v


def shock(state, p, G, sign):
    """(rho_b, v_b, V) behind a shock into `state` = (rho, p, v) that raises the pressure to p; V is the shock
    speed.  sign = -1 for the left (left-moving) shock, +1 for the right shock."""
    rho_a, p_a, v_a = state
    h_a = enthalpy(rho_a, p_a, G)
    dp = p - p_a
    # Taub adiabat with h_b/rho_b = h_b (G-1)(h_b - 1)/(G p): (1-k) h_b^2 + k h_b - C = 0
    k = (G - 1.0) * dp / (G * p)
    C = h_a * h_a + h_a * dp / rho_a
    h_b = (-k + math.sqrt(k * k + 4.0 * (1.0 - k) * C)) / (2.0 * (1.0 - k))
    rho_b = G * p / ((G - 1.0) * (h_b - 1.0))
    j2 = -dp / (h_b / rho_b - h_a / rho_a)
    W2a = 1.0 / (1.0 - v_a * v_a)
    V = (rho_a * rho_a * W2a * v_a + sign * math.sqrt(j2) * math.sqrt(j2 + rho_a * rho_a)) / (rho_a * rho_a * W2a + j2)
    # momentum and rest-mass jumps: S_b (v_b - V) + p_b = S_a (v_a - V) + p_a with D_b (v_b - V) = D_a (v_a - V);
    # with m = D_a (v_a - V) (the rest-mass flux through the shock), S_b (v_b - V) = m h_b W_b v_b.
    Da = rho_a / math.sqrt(1.0 - v_a * v_a)
    m = Da * (v_a - V)
    Sa = rho_a * h_a * W2a * v_a
    rhs = Sa * (v_a - V) + p_a - p  # = m h_b W_b v_b
    u = rhs / (m * h_b)  # W_b v_b
    v_b = u / math.sqrt(1.0 + u * u)
    return rho_b, v_b, V


def wave(state, p, G, sign):
    """Density and velocity behind the wave that takes `state` to pressure p (sign -1 left, +1 right)."""
    if p > state[1]:
        rho, v, _ = shock(state, p, G, sign)
    else:
        rho, v = rarefaction(state, p, G, -sign)
    return rho, v


class Solution:
    """The exact solution for left/right states (rho, p, v) with the interface at x0 at t = 0."""

    def __init__(self, left, right, G, x0=0.5):
        self.L = tuple(float(v) for v in left)
        self.R = tuple(float(v) for v in right)
        self.G = float(G)
        self.x0 = float(x0)
        f = lambda p: wave(self.L, p, G, -1)[1] - wave(self.R, p, G, +1)[1]
        lo, hi = 1e-12 * min(self.L[1], self.R[1]), 10.0 * max(self.L[1], self.R[1])
        while f(hi) > 0.0:
            hi *= 10.0
        self.p = brentq(f, lo, hi, xtol=1e-15 * hi, rtol=1e-15, maxiter=500)
        self.rhoL, self.v = wave(self.L, self.p, G, -1)
        self.rhoR, vR = wave(self.R, self.p, G, +1)
        self.v_mismatch = abs(self.v - vR)
        self.left_shock = self.p > self.L[1]
        self.right_shock = self.p > self.R[1]

    def _fan_state(self, state, xi, sign):
        """Point inside a fan (sign +1 left fan, -1 right fan) whose characteristic speed is xi."""
        G = self.G
        pa = state[1]
        pm = self.p

        def speed(p):
            rho, v = rarefaction(state, p, G, sign)
            c = sound_speed(rho, p, G)
            return (v - sign * c) / (1.0 - sign * v * c) - xi

        p = brentq(speed, pm, pa, xtol=1e-15 * pa, rtol=1e-15, maxiter=500)
        rho, v = rarefaction(state, p, G, sign)
        return rho, p, v

    def wave_speeds(self):
        """(left wave's leading and trailing speeds, contact speed, right wave's trailing and leading speeds)."""
        G = self.G
        if self.left_shock:
            lh = lt = shock(self.L, self.p, G, -1)[2]
        else:
            cL = sound_speed(self.L[0], self.L[1], G)
            cs = sound_speed(self.rhoL, self.p, G)
            lh = (self.L[2] - cL) / (1.0 - self.L[2] * cL)
            lt = (self.v - cs) / (1.0 - self.v * cs)
        if self.right_shock:
            rh = rt = shock(self.R, self.p, G, +1)[2]
        else:
            cR = sound_speed(self.R[0], self.R[1], G)
            cs = sound_speed(self.rhoR, self.p, G)
            rh = (self.R[2] + cR) / (1.0 + self.R[2] * cR)
            rt = (self.v + cs) / (1.0 + self.v * cs)
        return lh, lt, self.v, rt, rh

    def sample(self, x, t):
        """(rho, p, v) at the points x and time t > 0."""
        lh, lt, vc, rt, rh = self.wave_speeds()
        out = np.empty((3, len(x)))
        for i, xv in enumerate(np.asarray(x, dtype=np.float64)):
            xi = (xv - self.x0) / t
            if xi < lh:
                s = self.L
            elif xi < lt:
                s = self._fan_state(self.L, xi, +1)
            elif xi < vc:
                s = (self.rhoL, self.p, self.v)
            elif xi < rt:
                s = (self.rhoR, self.p, self.v)
            elif xi < rh:
                s = self._fan_state(self.R, xi, -1)
            else:
                s = self.R
            out[:, i] = s
        return out


# ---- a transverse field --------------------------------------------------------------------------------------
#
# Flow along x with a field B^t across it (no normal field, no tangential velocity).  The induction equation
# gives B^t the flux B^t v, like the rest mass, so B^t / D = k is carried with the fluid and is continuous
# across shocks: k is constant on each side of the contact.  With B.v = 0, b^0 = 0 and b^2 = (B^t / W)^2 =
# k^2 rho^2, the system is that of a fluid with total pressure P = p + k^2 rho^2 / 2, total enthalpy density
# w = rho + G/(G-1) p + k^2 rho^2 and sound speed c^2 = (G p + k^2 rho^2) / w (the fast speed across the
# field).  Its Riemann problem is solved with the same pieces as above, now numerically: the Taub adiabat in
# the total quantities (h = w / rho) for rho behind a shock, the isentrope p / rho^G = const with the
# invariant atanh(v) +- int c drho / rho (by quadrature) across a fan, and the middle total pressure by
# Brent's method.  With k = 0 it reduces to the closed forms above (checked by the tests).

def totals(rho, p, k, G):
    """(P, w, c): total pressure, total enthalpy density and fast speed for b^2 = k^2 rho^2."""
    b2 = (k * rho) ** 2
    w = rho + G / (G - 1.0) * p + b2
    return p + 0.5 * b2, w, math.sqrt((G * p + b2) / w)


def conserved_t(rho, p, v, k, G):
    """(D, S, tau, B^t) of flow along x with the transverse field B^t = k D."""
    W = 1.0 / math.sqrt(1.0 - v * v)
    P, w, _ = totals(rho, p, k, G)
    D = rho * W
    return np.array([D, w * W * W * v, w * W * W - P - D, k * D])


def flux_t(rho, p, v, k, G):
    D, S, tau, B = conserved_t(rho, p, v, k, G)
    P = totals(rho, p, k, G)[0]
    return np.array([D * v, S * v + P, (tau + P) * v, B * v])


def _fan_integral(rho, rho_a, K, k, G):
    """int_rho^rho_a c(r) / r dr along the isentrope p = K r^G."""
    from scipy.integrate import quad
    f = lambda r: totals(r, K * r ** G, k, G)[2] / r
    val, _ = quad(f, rho, rho_a, epsabs=0.0, epsrel=1e-13, limit=200)
    return val


def _isentrope_rho(state, k, G, P):
    """Density on the isentrope through `state` = (rho, p, v) where the total pressure is P (below state's)."""
    rho_a, p_a, _ = state
    K = p_a / rho_a ** G
    f = lambda r: K * r ** G + 0.5 * (k * r) ** 2 - P
    if f(rho_a) <= 0.0:  # P at (or within rounding of) the state's own
        return rho_a
    return brentq(f, 1e-300, rho_a, xtol=1e-16 * rho_a, rtol=1e-15, maxiter=500)


def rarefaction_t(state, k, G, P, sign):
    """(rho, p, v) behind a fan into `state` that lowers the total pressure to P (sign +1 left, -1 right)."""
    rho_a, p_a, v_a = state
    K = p_a / rho_a ** G
    rho = _isentrope_rho(state, k, G, P)
    v = math.tanh(math.atanh(v_a) + sign * _fan_integral(rho, rho_a, K, k, G))
    return rho, K * rho ** G, v


def shock_t(state, k, G, P, sign):
    """(rho, p, v, V) behind a shock into `state` that raises the total pressure to P (sign -1 left, +1 right)."""
    rho_a, p_a, v_a = state
    Pa, wa, _ = totals(rho_a, p_a, k, G)
    ha = wa / rho_a
    dP = P - Pa

    def taub(r):
        p = P - 0.5 * (k * r) ** 2
        h = totals(r, p, k, G)[1] / r
        return h * h - ha * ha - (h / r + ha / rho_a) * dP

    hi = math.sqrt(2.0 * P) / abs(k) * (1.0 - 1e-12) if k != 0.0 else 1e6 * rho_a
    grid = rho_a * (hi / rho_a) ** np.linspace(1e-12, 1.0, 4001)
    vals = [taub(r) for r in grid]
    i = next(i for i in range(len(grid) - 1) if vals[i] * vals[i + 1] <= 0.0)
    rho = brentq(taub, grid[i], grid[i + 1], xtol=1e-16 * grid[i], rtol=1e-15, maxiter=500)
    p = P - 0.5 * (k * rho) ** 2
    h = totals(rho, p, k, G)[1] / rho
    j2 = -dP / (h / rho - ha / rho_a)
    W2a = 1.0 / (1.0 - v_a * v_a)
    V = (rho_a * rho_a * W2a * v_a + sign * math.sqrt(j2) * math.sqrt(j2 + rho_a * rho_a)) / (rho_a * rho_a * W2a + j2)
    m = rho_a / math.sqrt(1.0 - v_a * v_a) * (v_a - V)
    Sa = wa * W2a * v_a
    u = (Sa * (v_a - V) + Pa - P) / (m * h)  # W_b v_b
    return rho, p, u / math.sqrt(1.0 + u * u), V


class TransverseSolution:
    """Exact solution for left/right states (rho, p, v, B^t) with the interface at x0 at t = 0."""

    def __init__(self, left, right, G, x0=0.5):
        self.G = float(G)
        self.x0 = float(x0)
        self.L = tuple(float(v) for v in left[:3])
        self.R = tuple(float(v) for v in right[:3])
        self.kL = float(left[3]) * math.sqrt(1.0 - self.L[2] ** 2) / self.L[0]
        self.kR = float(right[3]) * math.sqrt(1.0 - self.R[2] ** 2) / self.R[0]
        self.PL = totals(*self.L[:2], self.kL, G)[0]
        self.PR = totals(*self.R[:2], self.kR, G)[0]

        def behind(state, k, Pa, P, sign):
            if P > Pa:
                return shock_t(state, k, G, P, sign)[:3]
            return rarefaction_t(state, k, G, P, -sign)

        self.behind = behind
        f = lambda P: behind(self.L, self.kL, self.PL, P, -1)[2] - behind(self.R, self.kR, self.PR, P, +1)[2]
        lo, hi = 1e-10 * min(self.PL, self.PR), 10.0 * max(self.PL, self.PR)
        while f(hi) > 0.0:
            hi *= 10.0
        self.P = brentq(f, lo, hi, xtol=1e-15 * hi, rtol=1e-15, maxiter=500)
        self.starL = behind(self.L, self.kL, self.PL, self.P, -1)
        self.starR = behind(self.R, self.kR, self.PR, self.P, +1)
        self.v = self.starL[2]
        self.v_mismatch = abs(self.starL[2] - self.starR[2])
        self.left_shock = self.P > self.PL
        self.right_shock = self.P > self.PR

    def wave_speeds(self):
        G = self.G
        if self.left_shock:
            lh = lt = shock_t(self.L, self.kL, G, self.P, -1)[3]
        else:
            c0, c1 = totals(*self.L[:2], self.kL, G)[2], totals(*self.starL[:2], self.kL, G)[2]
            lh = (self.L[2] - c0) / (1.0 - self.L[2] * c0)
            lt = (self.v - c1) / (1.0 - self.v * c1)
        if self.right_shock:
            rh = rt = shock_t(self.R, self.kR, G, self.P, +1)[3]
        else:
            c0, c1 = totals(*self.R[:2], self.kR, G)[2], totals(*self.starR[:2], self.kR, G)[2]
            rh = (self.R[2] + c0) / (1.0 + self.R[2] * c0)
            rt = (self.v + c1) / (1.0 + self.v * c1)
        return lh, lt, self.v, rt, rh

    def _fan(self, state, k, xi, sign):
        G = self.G
        Pa = totals(*state[:2], k, G)[0]

        def speed(P):
            rho, p, v = rarefaction_t(state, k, G, P, sign)
            c = totals(rho, p, k, G)[2]
            return (v - sign * c) / (1.0 - sign * v * c) - xi

        P = brentq(speed, self.P, Pa, xtol=1e-15 * Pa, rtol=1e-15, maxiter=500)
        return rarefaction_t(state, k, G, P, sign)

    def sample(self, x, t):
        """(rho, p, v, B^t) at the points x and time t > 0."""
        lh, lt, vc, rt, rh = self.wave_speeds()
        out = np.empty((4, len(x)))
        for i, xv in enumerate(np.asarray(x, dtype=np.float64)):
            xi = (xv - self.x0) / t
            if xi < lh:
                s, k = self.L, self.kL
            elif xi < lt:
                s, k = self._fan(self.L, self.kL, xi, +1), self.kL
            elif xi < vc:
                s, k = self.starL, self.kL
            elif xi < rt:
                s, k = self.starR, self.kR
            elif xi < rh:
                s, k = self._fan(self.R, self.kR, xi, -1), self.kR
            else:
                s, k = self.R, self.kR
            out[:3, i] = s
            out[3, i] = k * s[0] / math.sqrt(1.0 - s[2] ** 2)
        return out
