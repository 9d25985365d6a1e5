"""Pins of the oracle's forward-mode derivative of the differentiation workload's loss.

The loss is (sum over owned cells of rho^2 dV)^(1/2) after whole RK steps from the initial primitives; its
directional derivative along (dv, dGamma) is computed by running the plain implementation on dual numbers.
Pinned against the definition of the derivative (central differences of the plain FP64 run), against the
value of the plain run, and against linearity in the direction."""
import math

import numpy as np
import pytest

from paper_2406_11669_amd import workloads as W


def _loss_plain(orc, w, prim0, gamma, nsteps):
    L = w.layout
    p = dict(w.params, gamma=gamma)
    cons = orc.prim2con(L, p, w.metric, w.A, prim0)
    orc.fill_ghosts(L, cons, w.bc_cell)
    state = w.state(cons)
    prim = prim0.copy()
    orc.run(L, p, w.metric, w.curv, state, prim, w.dt, nsteps, w.rk, w.bc_cell, w.bc_A, A_shift=w.A_shift)
    c = state[0:5].copy()
    orc.c2p(L, p, w.metric, state[5:8], c, prim)
    dV = L.dx[0] * L.dx[1] * L.dx[2]
    return math.sqrt(math.fsum((L.owned(prim[0]) ** 2 * dV).ravel()))


def _direction(w, seed):
    rng = np.random.default_rng(seed)
    L = w.layout
    d = L.zeros(5)
    L.owned(d)[2:5] = rng.normal(size=(3,) + L.owned(d).shape[1:])
    dg = rng.normal()
    nrm = math.sqrt(float(np.sum(d ** 2)) + dg * dg)
    d /= nrm
    L.periodic_wrap(d)
    return d, dg / nrm


def _jvp(orc, w, prim0, d, dg, nsteps):
    return orc.loss_jvp(w.layout, w.params, w.metric, w.curv, prim0, w.A, w.psi, w.dt, nsteps, w.rk, w.bc_cell,
                        w.bc_A, dprim0=d, dgamma=dg, A_shift=w.A_shift)


def test_jvp_value_equals_plain_run(orc):
    w = W.periodic_riemann_box(seed=31, n=8, nsteps=2, v_amp=0.05)
    loss, jvp, stats = _jvp(orc, w, w.prim, None, 0.0, 2)
    assert jvp == 0.0
    ref = _loss_plain(orc, w, w.prim, w.params["gamma"], 2)
    assert abs(loss - ref) <= 1e-14 * ref  # summation order only


def _smooth_direction(w, phase):
    L = w.layout
    d = L.zeros(5)
    x, y, z = L.coords("centre")
    d[2] = np.broadcast_to(np.sin(2 * np.pi * y + phase) * np.cos(2 * np.pi * z), L.shape3)
    d[3] = np.broadcast_to(np.cos(2 * np.pi * x + 0.3 + phase), L.shape3)
    d[4] = np.broadcast_to(0.5 * np.sin(2 * np.pi * (x + y) - phase), L.shape3)
    return d


@pytest.mark.parametrize("phase,dg", [(0.0, 0.0), (1.1, 0.3)])
def test_jvp_matches_central_differences(orc, phase, dg):
    """At a generic point (smooth seeded velocity) and along a smooth direction, the dual-number JVP equals the
    central difference quotient of the plain run (h = 1e-6) to the quotient's own error.  (At the Riemann
    problem's rest state every cell sits on a limiter tie and the loss is not differentiable in v.)"""
    w = W.periodic_riemann_box(seed=32, n=8, nsteps=2, v_amp=0.05)
    d = _smooth_direction(w, phase)
    loss, jvp, _ = _jvp(orc, w, w.prim, d, dg, 2)
    g0 = w.params["gamma"]
    h = 1e-6
    lp = _loss_plain(orc, w, w.prim + h * d, g0 + h * dg, 2)
    lm = _loss_plain(orc, w, w.prim - h * d, g0 - h * dg, 2)
    fd = (lp - lm) / (2 * h)
    assert abs(fd - jvp) <= 1e-5 * abs(jvp), (fd, jvp)


def test_jvp_gamma_only_matches_differences(orc):
    w = W.periodic_riemann_box(seed=33, n=6, nsteps=1, v_amp=0.05)
    loss, jvp, _ = _jvp(orc, w, w.prim, None, 1.0, 1)
    g0 = w.params["gamma"]
    h = 1e-5
    fd = (_loss_plain(orc, w, w.prim, g0 + h, 1) - _loss_plain(orc, w, w.prim, g0 - h, 1)) / (2 * h)
    assert abs(fd - jvp) <= 1e-6 * abs(jvp) + 1e-10 * loss, (fd, jvp)


def test_jvp_linear_in_direction(orc):
    w = W.periodic_riemann_box(seed=34, n=6, nsteps=1, v_amp=0.05)
    d1, g1 = _direction(w, 5)
    d2, g2 = _direction(w, 6)
    _, j1, _ = _jvp(orc, w, w.prim, d1, g1, 1)
    _, j2, _ = _jvp(orc, w, w.prim, d2, g2, 1)
    _, j12, _ = _jvp(orc, w, w.prim, 2.0 * d1 - 3.0 * d2, 2.0 * g1 - 3.0 * g2, 1)
    assert abs(j12 - (2.0 * j1 - 3.0 * j2)) <= 1e-12 * (abs(2 * j1) + abs(3 * j2))
