"""The HIP path on Michel accretion onto a Schwarzschild black hole in Kerr-Schild coordinates (the exact
stationary flow of tests/michel.py on [3, 6] x [0.5, 3.5] x [0.5, 3.5], M = 1, sonic radius 5, Gamma = 4/3):
right-hand side and evolution against the oracle, and second-order convergence to the exact flow at sizes
the oracle would take minutes for."""
import math

import numpy as np
import pytest

from paper_2406_11669_amd import workloads as W
from tests.michel import Michel, MichelField
from tests.parity import assert_fields_close
from tests.test_oracle_michel import Q_STRONG, SCHEMES, _all_rhs_errors, michel_interior_errors, scheme_block

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]
STATE_NAMES = ["D", "Sx", "Sy", "Sz", "tau", "Ax", "Ay", "Az", "Psi"]
PRIM_NAMES = ["rho", "p", "vx", "vy", "vz"]


@pytest.fixture(scope="module")
def ax():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_11669_amd import asterx
    asterx.lib()
    return asterx


@pytest.fixture(scope="module")
def field():
    return MichelField(Michel(), 2.0, 10.0)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _gpu_rhs(ax, w):
    import torch
    L = w.layout
    out = torch.zeros((9,) + L.shape3, dtype=torch.float64, device="cuda")
    red = torch.zeros(2, dtype=torch.float64, device="cuda")
    ws = torch.empty(ax.workspace_size(L) // 8, dtype=torch.float64, device="cuda")
    ax.rhs(L, w.params, _dev(w.metric), _dev(w.curv), _dev(w.prim), _dev(w.A), _dev(w.psi), w.dt, out, red, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _truncation(w, out, cons):
    L = w.layout
    r, c = L.owned(out[0:5]), L.owned(cons)
    return np.array([np.mean(np.abs(r[q])) / np.max(np.abs(c[q])) for q in range(5)])


def test_michel_rhs_matches_oracle(ax, orc, field):
    """The right-hand side at the exact data on 24^3 against the oracle's.  On a stationary solution it is
    the small remainder (truncation error, about 1e-5 of the conserved variables) of flux differences and
    sources of order |U| / dx that cancel, so the two sides' rounding is measured against that scale:
    |gpu - oracle| <= 1e-13 max|D| / dx in every hydrodynamic component (against its own small magnitude
    the same rounding reads up to 8e-10)."""
    w = W.kerr_schild_block(n=24, prim_fn=field, recon="ppm")
    L = w.layout
    print("case michel rhs 24", flush=True)
    g = _gpu_rhs(ax, w)
    ref, _, _ = orc.rhs(L, w.params, w.metric, w.curv, w.prim, w.A, w.psi, w.dt)
    cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
    scale = np.max(np.abs(L.owned(cons[0]))) / L.dx[0]
    d = np.abs(L.owned(g[0:5]) - L.owned(ref[0:5])).reshape(5, -1).max(axis=1) / scale
    print("  max |gpu - oracle| / (max|D| / dx):", d)
    assert np.all(d <= 1e-13)
    assert np.all(L.owned(g[5:9]) == 0.0) and np.all(L.owned(ref[5:9]) == 0.0)


def test_michel_rhs_truncation_second_order(ax, orc, field):
    """The right-hand side at the exact stationary data falls by 3.6x or more per halving of dx in every
    hydrodynamic component, from 32 to 64 to 128 cells per side."""
    prev = None
    for n in (32, 64, 128):
        w = W.kerr_schild_block(n=n, prim_fn=field, recon="ppm")
        print("case michel rhs", n, flush=True)
        out = _gpu_rhs(ax, w)
        cons = orc.prim2con(w.layout, w.params, w.metric, w.A, w.prim)
        e = _truncation(w, out, cons)
        print("  L1 rhs / scale", e)
        if prev is not None:
            assert np.all(prev >= 3.6 * e)
        prev = e


def _evolve(ax, w, T):
    import torch
    nsteps = int(math.ceil(T / w.dt - 1e-9))
    w.dt = T / nsteps
    blk = ax.Block(w)
    blk.run(nsteps)
    torch.cuda.synchronize()
    return blk.prim.cpu().numpy(), blk.state.cpu().numpy(), blk.stats.cpu().numpy(), nsteps


def _interior_errors(w, prim, margin):
    L = w.layout
    n = L.n[0]
    own, ex = L.owned(prim), L.owned(w.prim)
    xc = (np.arange(n) + 0.5) * L.dx[0]
    inner = (xc > margin) & (xc < w.info["extent"] - margin)
    sel = np.ix_(inner, inner, inner)
    return np.array([np.mean(np.abs(own[q][sel] - ex[q][sel])) / np.max(np.abs(ex[q])) for q in range(5)])


def test_michel_evolution_matches_oracle(ax, orc, field):
    """RK2 to t = 0.5 M on 24^3 (ghosts extrapolated linearly): state and primitives within 1e-10 of the
    oracle's."""
    w = W.kerr_schild_block(n=24, prim_fn=field, recon="ppm", rk=2)
    print("case michel evolution 24", flush=True)
    pg, sg, st, nsteps = _evolve(ax, w, 0.5)
    L = w.layout
    cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
    orc.fill_ghosts(L, cons, w.bc_cell)
    state = w.state(cons)
    prim = w.prim.copy()
    flags, stats, red = orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, nsteps, w.rk, w.bc_cell, w.bc_A)
    assert_fields_close(sg, state, 1e-10, L.owned, STATE_NAMES)
    assert_fields_close(pg, prim, 1e-10, L.owned, PRIM_NAMES)
    assert st[3] == 0 and stats[3] == 0


def test_michel_evolution_stays_exact_second_order(ax, field):
    """RK2 to t = 0.5 M at 48, 96 and 192 cells per side: inside the cube shrunk by 0.75 M per face the
    primitives stay at the exact flow, L1 errors falling by 3.2x or more per doubling."""
    prev = None
    for n in (48, 96, 192):
        w = W.kerr_schild_block(n=n, prim_fn=field, recon="ppm", rk=2)
        print("case michel evolution", n, flush=True)
        pg, sg, st, nsteps = _evolve(ax, w, 0.5)
        assert st[0] == 0 and st[3] == 0
        e = _interior_errors(w, pg, 0.75)
        print("  interior L1 / scale", e)
        if prev is not None:
            assert np.all(prev >= 3.2 * e)
        prev = e


@pytest.mark.parametrize("scheme", SCHEMES)
def test_magnetized_michel_rhs_matches_oracle(ax, orc, field, scheme):
    """The monopole-field flow (|B| about 1) on 24^3, every reconstruction, Riemann solver and edge-field
    scheme: the right-hand side against the oracle's, measured against the scale of the terms that cancel
    (max|D| / dx for the hydrodynamic components, max|A| / dx for the potential and Psi): within 1e-13."""
    w = scheme_block(24, field, scheme, monopole=Q_STRONG)
    L = w.layout
    print("case magnetized michel rhs 24", scheme, flush=True)
    g = _gpu_rhs(ax, w)
    ref, red, _ = orc.rhs(L, w.params, w.metric, w.curv, w.prim, w.A, w.psi, w.dt)
    cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
    sD = np.max(np.abs(L.owned(cons[0]))) / L.dx[0]
    sA = np.max(np.abs(L.owned(w.A))) / L.dx[0]
    d = np.abs(L.owned(g) - L.owned(ref)).reshape(9, -1).max(axis=1) / np.array([sD] * 5 + [sA] * 4)
    print("  max |gpu - oracle| / scale:", d)
    assert np.all(d <= 1e-13)


@pytest.mark.parametrize("scheme", ["ppm+hlle+fct", "mp5+lxf+uct"])
def test_magnetized_michel_rhs_truncation_second_order(ax, orc, field, scheme):
    """The monopole-field flow: the right-hand side at the exact data falls by 3.6x or more per halving in all
    nine components from 32 to 64 to 128 cells per side."""
    prev = None
    for n in (32, 64, 128):
        w = scheme_block(n, field, scheme, monopole=Q_STRONG)
        print("case magnetized michel rhs", scheme, n, flush=True)
        out = _gpu_rhs(ax, w)
        cons = orc.prim2con(w.layout, w.params, w.metric, w.A, w.prim)
        e = _all_rhs_errors(w, out, cons)
        print("  L1 rhs / scale", e)
        if prev is not None:
            assert np.all(prev >= 3.6 * e)
        prev = e


def test_magnetized_michel_evolution_matches_oracle(ax, orc, field):
    """The monopole-field flow, RK2 to t = 0.5 M on 24^3: state and primitives within 1e-10 of the oracle's."""
    w = W.kerr_schild_block(n=24, prim_fn=field, recon="ppm", rk=2, monopole=Q_STRONG)
    print("case magnetized michel evolution 24", flush=True)
    pg, sg, st, nsteps = _evolve(ax, w, 0.5)
    L = w.layout
    cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
    orc.fill_ghosts(L, cons, w.bc_cell)
    state = w.state(cons)
    prim = w.prim.copy()
    flags, stats, red = orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, nsteps, w.rk, w.bc_cell, w.bc_A)
    assert_fields_close(sg, state, 1e-10, L.owned, STATE_NAMES)
    assert_fields_close(pg, prim, 1e-10, L.owned, PRIM_NAMES)
    assert st[3] == 0 and stats[3] == 0


def test_magnetized_michel_evolution_stays_exact_second_order(ax, orc, field):
    """The monopole-field flow, RK2 to t = 0.5 M at 48, 96 and 192 cells per side: inside the cube shrunk by
    0.75 M per face the primitives and the face field stay at the exact flow, L1 errors falling by 3.2x or
    more per doubling."""
    prev = None
    for n in (48, 96, 192):
        w = W.kerr_schild_block(n=n, prim_fn=field, recon="ppm", rk=2, monopole=Q_STRONG)
        print("case magnetized michel evolution", n, flush=True)
        pg, sg, st, nsteps = _evolve(ax, w, 0.5)
        assert st[0] == 0 and st[3] == 0
        e = michel_interior_errors(orc, w, pg, sg)
        print("  interior L1 / scale (rho, p, v, B)", e)
        if prev is not None:
            assert np.all(prev >= 3.2 * e)
        prev = e
