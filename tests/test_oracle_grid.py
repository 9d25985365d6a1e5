"""Grid-level pins of the oracle: invariants, special cases and convergence of the full right-hand side and
time step (Secs. 2.2-3.4, 3.12; Alfven-wave set-up of Sec. 4)."""
import math

import numpy as np
import pytest

from paper_2406_11669_amd import workloads as W
from paper_2406_11669_amd.workloads import Layout, default_params
from tests.states import gmat

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _const_metric(L, m10):
    m = L.zeros(10)
    for c in range(10):
        m[c] = m10[c]
    return m


def _uniform_setup(n=8, seed=0, vel=(0.3, -0.2, 0.1), B=(0.375, -0.25, 0.625), ng=3):
    """Uniform fluid and field in a constant non-trivial metric; dx = 1/16 and dyadic B make the edge potential
    and its differences exact, so the face field is bitwise uniform."""
    rng = np.random.default_rng(seed)
    L = Layout((n, n, n), ng, dx=(1 / 16, 1 / 16, 1 / 16))
    m10 = np.array([0.875, 0.125, -0.0625, 0.25, 1.25, 0.125, -0.0625, 1.125, 0.0625, 0.9375])
    metric = _const_metric(L, m10)
    prim = L.zeros(5)
    prim[0], prim[1] = 0.7, 0.4
    for d in range(3):
        prim[2 + d] = vel[d]
    A = L.zeros(3)
    # B-tilde = curl A with A = (0, Bz x, Bx y - By x)
    xy, _, _ = L.coords("yedge")
    A[1] = np.broadcast_to(B[2] * xy, L.shape3)
    xz, yz, _ = L.coords("zedge")
    A[2] = np.broadcast_to(B[0] * yz - B[1] * xz, L.shape3)
    return L, m10, metric, prim, A, np.array(B)


@pytest.mark.parametrize("recon,riemann,ct", [("minmod", "hlle", "fct"), ("ppm", "hlle", "fct"),
                                              ("wenoz", "hlle", "fct"), ("mp5", "hlle", "fct"), ("ppm", "lxf", "fct"),
                                              ("ppm", "hlle", "uct"), ("mp5", "lxf", "uct")])
def test_uniform_state_constant_metric(orc, recon, riemann, ct):
    """Uniform (rho, p, v, B) in a constant metric: hydro right-hand side bitwise 0; dA/dt = vt x Btilde
    (the edge field of a uniform state, E = -vt x Btilde, by flux CT and by upwind CT alike: the upwind
    velocities and the reconstructed fields are the uniform ones, and the jump terms vanish) to round-off;
    dPsi/dt = -alpha sqrt(gamma) gamma^jk d_j A_k - xi alpha Psi."""
    L, m10, metric, prim, A, Bt = _uniform_setup(ng=4 if ct == "uct" else 3)
    P = default_params(gamma=5.0 / 3.0, recon=recon, riemann=riemann, ct=ct)
    psi = L.zeros(1) + 0.25
    dt = 0.01
    out, red, nfix = orc.rhs(L, P, metric, L.zeros(6), prim, A, psi, dt)
    assert nfix == 0
    assert np.all(L.owned(out[0:5]) == 0.0)
    vt = m10[0] * prim[2:5, 0, 0, 0] - m10[1:4]
    E = np.cross(vt, Bt)
    dA = np.zeros((3, 3))  # dA[j, k] = d_j A_k
    dA[0, 1] = Bt[2]
    dA[1, 2] = Bt[0]
    dA[0, 2] = -Bt[1]
    # -d_i G_A = d_i (beta^j A_j) for uniform Psi and constant metric
    gauge = dA @ m10[1:4]
    for a in range(3):
        np.testing.assert_allclose(L.owned(out[5 + a]), E[a] + gauge[a] + 0 * L.owned(out[5 + a]), rtol=0,
                                   atol=1e-13)
    g = gmat(m10)
    gi = np.linalg.inv(g)
    ref = -m10[0] * np.sqrt(np.linalg.det(g)) * np.sum(gi * dA) - P["xi"] / dt * m10[0] * 0.25
    np.testing.assert_allclose(L.owned(out[8]), ref + 0 * L.owned(out[8]), rtol=1e-13)
    assert red[1] == 0.0


def _at_rest_curved(n, recon="ppm"):
    L = Layout((n, n, n), 3)
    metric, curv, _ = W.curved_metric(L, seed=5, alpha0=1.0, alpha_amp=0.0, beta_amp=0.0, gamma_amp=0.1)
    prim = L.zeros(5)
    prim[0] = 1.0
    prim[1] = 0.5
    return L, metric, curv, prim


def test_at_rest_curved_static_metric(orc):
    """Fluid at rest with uniform pressure, no field, alpha = 1, beta = 0 and a curved static gamma: the D and tau
    right-hand sides vanish exactly; the momentum residual (flux of sqrt(gamma) p against the source
    p d sqrt(gamma)) vanishes at second order or better with resolution."""
    errs = []
    for n in (16, 32, 64):
        L, metric, curv, prim = _at_rest_curved(n)
        P = default_params(gamma=2.0, recon="ppm")
        out, red, _ = orc.rhs(L, P, metric, curv, prim, L.zeros(3), L.zeros(1), 0.01)
        assert np.all(L.owned(out[0]) == 0.0) and np.all(L.owned(out[4]) == 0.0)
        errs.append(np.max(np.abs(L.owned(out[1:4]))))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert order[-1] >= 1.9 and order[-1] > order[0], (errs, order)


def _init_state(orc, w):
    cons = orc.prim2con(w.layout, w.params, w.metric, w.A, w.prim)
    orc.fill_ghosts(w.layout, cons, w.bc_cell)
    return w.state(cons)


@pytest.mark.parametrize("recon,riemann,ct", [("ppm", "hlle", "fct"), ("wenoz", "hlle", "fct"),
                                              ("mp5", "hlle", "fct"), ("ppm", "lxf", "fct"), ("ppm", "hlle", "uct")])
def test_conservation_and_divB_curved_periodic(orc, recon, riemann, ct):
    """Periodic block in a curved metric: sum of D-tilde is constant to round-off (the flux form telescopes) and
    the discrete divergence of the face field stays at round-off under constrained transport."""
    w = W.curved_block(seed=3, n=10, recon=recon, nsteps=2, ng=4 if ct == "uct" else 3)
    w.params["riemann"] = riemann
    w.params["ct"] = ct
    L = w.layout
    state = _init_state(orc, w)
    prim = w.prim.copy()
    D0 = math.fsum(L.owned(state[0]).ravel())
    flags, stats, red = orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, w.nsteps, w.rk, w.bc_cell,
                                w.bc_A)
    D1 = math.fsum(L.owned(state[0]).ravel())
    assert abs(D1 - D0) <= 1e-13 * abs(D0)
    Bf = orc.face_B(L, state[5:8])
    assert red[1] <= 1e-12 * np.max(np.abs(Bf)) / min(L.dx)
    assert stats[3] == 0 and stats[2] == 0


def test_flat_periodic_conserves_momentum_and_energy(orc):
    w = W.curved_block(seed=4, n=8, recon="ppm", nsteps=2)
    L = w.layout
    w.metric = W.flat_metric(L)
    w.curv = L.zeros(6)
    state = _init_state(orc, w)
    prim = w.prim.copy()
    s0 = [math.fsum(L.owned(state[c]).ravel()) for c in range(5)]
    orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, w.nsteps, w.rk, w.bc_cell, w.bc_A)
    s1 = [math.fsum(L.owned(state[c]).ravel()) for c in range(5)]
    scale = max(abs(v) for v in s0)
    for c in range(5):
        assert abs(s1[c] - s0[c]) <= 1e-13 * scale, (c, s0[c], s1[c])


@pytest.mark.parametrize("rk", [2, 4])
def test_psi_damping_follows_rk_amplification(orc, rk):
    """No field, uniform Psi, constant lapse: dPsi/dt = -xi alpha Psi, so after n steps Psi equals R(z)^n Psi0
    with z = -xi alpha dt and R the stability polynomial of the RK tableau (Heun: 1 + z + z^2/2; classical RK4:
    1 + z + z^2/2 + z^3/6 + z^4/24) -- a pin of the tableaux."""
    L = Layout((4, 4, 4), 3)
    m10 = np.array([0.8, 0, 0, 0, 1.0, 0, 0, 1.0, 0, 1.0])
    metric = _const_metric(L, m10)
    prim = L.zeros(5)
    prim[0], prim[1] = 1.0, 0.3
    P = default_params(gamma=5.0 / 3.0)
    cons = orc.prim2con(L, P, metric, L.zeros(3), prim)
    orc.fill_ghosts(L, cons, ["periodic"] * 3)
    state = L.zeros(9)
    state[0:5] = cons
    state[8] = 0.7
    dt = 0.01
    nsteps = 3
    orc.run(L, P, metric, L.zeros(6), state, prim, dt, nsteps, rk, ["periodic"] * 3, ["periodic"] * 3)
    z = -P["xi"] / dt * 0.8 * dt
    R = 1 + z + z * z / 2 + ((z ** 3 / 6 + z ** 4 / 24) if rk == 4 else 0)
    np.testing.assert_allclose(L.owned(state[8]), 0.7 * R ** nsteps, rtol=1e-13)


def _entropy_wave(orc, N, recon, metric10, t_final=0.25):
    L = Layout((N, 2, 2), 3, dx=(1.0 / N, 1.0 / N, 1.0 / N))
    metric = _const_metric(L, metric10)
    prim = L.zeros(5)
    xc, _, _ = L.coords("centre")
    prim[0] = np.broadcast_to(1.0 + 0.2 * np.sin(2 * np.pi * xc), L.shape3)
    prim[1] = 1.0
    prim[2] = 0.3
    prim[3] = 0.1
    B = (0.5, 0.3, -0.2)
    A = L.zeros(3)
    xy, _, _ = L.coords("yedge")
    A[1] = np.broadcast_to(B[2] * xy, L.shape3)
    xz, yz, _ = L.coords("zedge")
    A[2] = np.broadcast_to(B[0] * yz - B[1] * xz, L.shape3)
    P = default_params(gamma=5.0 / 3.0, recon=recon)
    cons = orc.prim2con(L, P, metric, A, prim)
    bc_cell = ["periodic"] * 3
    bc_A = ["linear"] * 3
    orc.fill_ghosts(L, cons, bc_cell)
    state = L.zeros(9)
    state[0:5] = cons
    state[5:8] = A
    dt = 0.25 / N
    nsteps = int(round(t_final / dt))
    orc.run(L, P, metric, L.zeros(6), state, prim, dt, nsteps, 2, bc_cell, bc_A)
    speed = metric10[0] * 0.3 - metric10[1]
    ex = 1.0 + 0.2 * np.sin(2 * np.pi * (xc - speed * nsteps * dt))
    return np.mean(np.abs(L.owned(prim[0]) - L.owned(np.broadcast_to(ex, L.shape3))))


@pytest.mark.parametrize("recon,min_order", [("minmod", 1.8), ("ppm", 2.0), ("mp5", 1.9)])
@pytest.mark.parametrize("curved", [False, True])
def test_entropy_wave_convergence(orc, recon, min_order, curved):
    """A smooth entropy wave (uniform p, v, B) translates exactly with coordinate speed alpha v^x - beta^x;
    the L1 error converges at second order (flat and constant non-trivial metric).  The RK2 time error caps
    the observed order at 2, also for fifth-order MP5 (measured 1.94, 1.99)."""
    m10 = np.array([1.0, 0, 0, 0, 1.0, 0, 0, 1.0, 0, 1.0])
    if curved:
        m10 = np.array([0.9, 0.05, -0.02, 0.01, 1.0, 0.0, 0.0, 1.1, 0.05, 0.95])
    errs = [_entropy_wave(orc, N, recon, m10) for N in (32, 64, 128)]
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert order[-1] >= min_order, (errs, order)


def alfven_speed(rho, p, gamma, B0, eta):
    """Propagation speed of the exact circularly polarized Alfven wave of relativistic MHD (amplitude eta of
    the transverse field against the normal field B0): with w = rho h + B0^2 (1 + eta^2),
    vA^2 = (2 B0^2 / w) / (1 + sqrt(1 - (2 eta B0^2 / w)^2)).  The wave translates rigidly at vA, with
    v^y,z = -vA B^y,z / B0."""
    w = rho + gamma / (gamma - 1.0) * p + B0 * B0 * (1.0 + eta * eta)
    a = 2.0 * B0 * B0 / w
    return math.sqrt(a / (1.0 + math.sqrt(1.0 - (eta * a) ** 2)))


def alfven_errors(orc, w, prim, state):
    """L2 errors of B^y (y faces, at the cells' x) and of v^y against the exact wave translated by vA t."""
    L = w.layout
    n = L.n[0]
    t, A0, vA, Bx = (w.info[k] for k in ("t_end", "A0", "vA", "Bx"))
    k = 2.0 * np.pi
    x = (np.arange(n) + 0.5) / n - 0.5
    By = L.owned(orc.face_B(L, state[5:8])[1])[0, 0, :]
    vy = L.owned(prim[3])[0, 0, :]
    ph = np.cos(k * (x - vA * t))
    return np.sqrt(np.mean((By - A0 * Bx * ph) ** 2)), np.sqrt(np.mean((vy + vA * A0 * ph) ** 2))


def run_alfven(orc, n, recon="minmod", lib_=None):
    w = W.alfven_wave(n=n, recon=recon)
    L = w.layout
    cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
    orc.fill_ghosts(L, cons, w.bc_cell)
    state = w.state(cons)
    prim = w.prim.copy()
    orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, w.nsteps, w.rk, w.bc_cell, w.bc_A,
            A_shift=w.A_shift, lib_=lib_)
    return w, prim, state


def test_alfven_wave_converges_to_exact(orc):
    """The Alfven-wave test of Sec. 4 (rho = 1, p = 0.5 -- the printed 'rho = 0.5' read as p --, A0 = 1,
    B^x = 1, Gamma = 5/3, MINMOD, HLLE, RK2, CFL 0.2, periodic): for these values the exact circularly
    polarized wave travels at exactly the printed vA = 0.5, so after one period (t = 2) the solution is the
    initial data again.  The L2 errors of B^y and v^y against it fall at second order, as the paper reports
    (order >= 1.75 from 16 to 32 and from 32 to 64 cells; 1.83-1.99 measured)."""
    assert abs(alfven_speed(1.0, 0.5, 5.0 / 3.0, 1.0, 1.0) - 0.5) <= 1e-15
    lib = orc.lib_omp()[0]
    errs = [alfven_errors(orc, *run_alfven(orc, n, lib_=lib)) for n in (16, 32, 64)]
    print("L2 (B^y, v^y):", errs)
    for a, b in zip(errs[:-1], errs[1:]):
        assert math.log2(a[0] / b[0]) >= 1.75 and math.log2(a[1] / b[1]) >= 1.75


def test_riemann_block_smoke(orc):
    """The seeded magnetized Riemann-problem block runs without c2p failures and keeps positivity (no exact
    magnetized solver exists here; the unmagnetized tubes are pinned to the exact solution in
    test_oracle_exact_riemann.py)."""
    w = W.riemann_block(seed=7, n=12, nsteps=4)
    L = w.layout
    state = _init_state(orc, w)
    prim = w.prim.copy()
    flags, stats, red = orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, w.nsteps, w.rk, w.bc_cell,
                                w.bc_A)
    assert stats[0] == 0 and stats[3] == 0
    assert np.all(L.owned(prim[0]) > 0) and np.all(L.owned(prim[1]) > 0)
    assert red[0] <= 1.0 and red[1] <= 1e-12 * 8 / min(L.dx)


def test_periodic_riemann_box_potential_and_conservation(orc):
    """Periodic Riemann box: the potential with a constant offset per wrap reproduces the piecewise-constant face
    field exactly (ghosts included, after the offset fill), and a periodic run conserves D, S and tau to
    round-off while div B stays at round-off (the offset fill carries the mean field's net flux)."""
    w = W.periodic_riemann_box(seed=9, n=8, nsteps=2)
    L = w.layout
    A = w.A.copy()
    A_owned = L.owned(A).copy()
    orc.fill_ghosts_shift(L, A, w.A_shift)
    assert np.array_equal(L.owned(A), A_owned)
    assert np.max(np.abs(A - w.A)) <= 1e-14 * np.max(np.abs(w.A))
    Bf = orc.face_B(L, A)
    i = info = w.info
    x, _, _ = L.coords("centre")
    left = np.broadcast_to(np.mod(x, 1.0) < 0.5, L.shape3)
    g = L.ng
    core = (slice(1, None), slice(g - 2, g + L.n[2] + 2), slice(g - 2, g + L.n[1] + 2), slice(g - 2, g + L.n[0] + 2))
    expect = np.stack([np.full(L.shape3, info["Bx"]), np.where(left, i["ByL"], i["ByR"]),
                       np.where(left, i["BzL"], i["BzR"])])
    assert np.max(np.abs(Bf[core] - expect[core])) <= 1e-13
    state = _init_state(orc, w)
    prim = w.prim.copy()
    s0 = [math.fsum(L.owned(state[c]).ravel()) for c in range(5)]
    flags, stats, red = orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, w.nsteps, w.rk, w.bc_cell,
                                w.bc_A, A_shift=w.A_shift)
    s1 = [math.fsum(L.owned(state[c]).ravel()) for c in range(5)]
    scale = max(abs(v) for v in s0)
    for c in range(5):
        assert abs(s1[c] - s0[c]) <= 1e-13 * scale, (c, s0[c], s1[c])
    assert stats[3] == 0 and red[1] <= 1e-12 * 8 / min(L.dx)


def test_uct_and_fct_agree_to_second_order(orc):
    """Upwind CT (eq. eq3.20) and flux CT are two discretizations of the same edge field: on smooth data (the
    curved periodic workload refined at fixed physical fields) their dA/dt differ by a residual that falls at
    second order or better."""
    diffs = []
    for n in (12, 24, 48):
        w = W.curved_block(seed=4, n=n, recon="ppm", nsteps=1, ng=4)
        L = w.layout
        outs = []
        for ct in ("fct", "uct"):
            P = dict(w.params, ct=ct)
            out, _, _ = orc.rhs(L, P, w.metric, w.curv, w.prim, w.A, w.psi, w.dt)
            outs.append(out)
        assert np.array_equal(L.owned(outs[0][0:5]), L.owned(outs[1][0:5]))  # hydro unaffected
        diffs.append(np.max(np.abs(L.owned(outs[0][5:8]) - L.owned(outs[1][5:8]))))
    order = np.log2(np.array(diffs[:-1]) / np.array(diffs[1:]))
    assert order[-1] >= 1.8, (diffs, order)
