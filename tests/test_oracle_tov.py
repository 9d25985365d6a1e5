"""The oracle against a static star: a TOV polytrope (K = 100, Gamma = 2, central density 1.28e-3; M = 1.400,
Schwarzschild radius 9.586, isotropic radius 8.125; paper_2406_11669_amd/tov.py) in its own fixed isotropic metric (the
Cowling set-up of the paper's TOV test, Sec. 4), on the octant [0, 10]^3.  Hydrostatic equilibrium makes the
right-hand side vanish, so its discrete value at the exact data is truncation error: the momentum
components, a pressure gradient balanced by the lapse's and conformal factor's derivatives, fall at second
order inside the star; D and tau, which vanish for a fluid at rest except for the Riemann solver's
dissipation of reconstruction jumps, fall at nearly second order in L1 (their largest values, at the
central maximum that PPM flattens, at first order)."""
import numpy as np
import pytest

from paper_2406_11669_amd import workloads as W
from paper_2406_11669_amd.tov import TOV

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.fixture(scope="module")
def star():
    return TOV()


def test_tov_structure(star):
    """The standard star's mass and radii; lapse and conformal factor continuous at the surface with the
    exterior Schwarzschild solution in isotropic coordinates."""
    assert abs(star.M - 1.40016) <= 1e-4 and abs(star.R - 9.5856) <= 1e-3 and abs(star.rbR - 8.1251) <= 1e-3
    rb = np.array([star.rbR * (1 - 1e-9), star.rbR * (1 + 1e-9)])
    a, p4, rho, p = star.fields(rb, 0.0 * rb, 0.0 * rb, 1e-10)
    assert abs(a[0] - a[1]) <= 1e-7 and abs(p4[0] - p4[1]) <= 1e-7


def interior_rhs(star, w, out, cons, frac=0.8):
    """L1 over the cells inside frac R of |rhs| for D, S_x, S_y, S_z, tau, over max|D|."""
    L = w.layout
    n = L.n[0]
    xc = (np.arange(n) + 0.5) * L.dx[0] + np.array(w.info["origin"])[:, None]
    R = np.sqrt(xc[2][:, None, None] ** 2 + xc[1][None, :, None] ** 2 + xc[0][None, None, :] ** 2)
    inner = R < frac * star.rbR
    r = L.owned(out)
    s = np.max(np.abs(L.owned(cons[0])))
    return np.array([np.mean(np.abs(r[q][inner])) for q in range(5)]) / s


def test_tov_rhs_truncation(orc, star):
    """At 20, 40 and 80 cells per side (spacing 0.5 to 0.125): inside 0.8 R the L1 of the momentum right-hand
    side falls by 3.6x or more per halving (4.0x measured), of D and tau by 3.2x or more (3.45-3.73x); no face
    fell back."""
    prev = None
    for n in (20, 40, 80):
        w = W.static_star_block(n=n, star_fn=star.fields, recon="ppm")
        L = w.layout
        out, red, nfix = orc.rhs(L, w.params, w.metric, w.curv, w.prim, w.A, w.psi, w.dt)
        cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
        e = interior_rhs(star, w, out, cons)
        print(n, "interior L1 rhs / max D", e)
        assert nfix == 0
        if prev is not None:
            assert np.all(prev[1:4] >= 3.6 * e[1:4]) and prev[0] >= 3.2 * e[0] and prev[4] >= 3.2 * e[4]
        prev = e


def test_setup_a_star_field(orc):
    """The Setup A workload's field: divergence-free to round-off under the discrete curl, confined to the
    star (zero on every face outside the isotropic radius), and largest at about 1e14 G (the scaling uses
    centred differences, the curl the staggered ones: within 20%)."""
    w = W.magnetized_star_block(n=32)
    L = w.layout
    Bf = orc.face_B(L, w.A)
    g = L.ng
    own = Bf[:, g:g + 32, g:g + 32, g:g + 32]
    div = (np.diff(Bf[0], axis=2)[g:g + 32, g:g + 32, g:g + 32] + np.diff(Bf[1], axis=1)[g:g + 32, g:g + 32, g:g + 32]
           + np.diff(Bf[2], axis=0)[g:g + 32, g:g + 32, g:g + 32])
    assert np.max(np.abs(div)) <= 1e-12 * np.max(np.abs(own))
    x, y, z = L.coords("centre")
    r = np.sqrt((x - 20.0) ** 2 + (y - 20.0) ** 2 + (z - 20.0) ** 2)[g:g + 32, g:g + 32, g:g + 32]
    outside = r > 8.125 + 2.0
    assert np.all(own[:, outside] == 0.0)
    psi6 = L.owned(w.metric[4]) ** 1.5
    bmax = np.max(np.sqrt(np.sum(own ** 2, axis=0)) / psi6) * 8.351e19
    assert 0.8e14 <= bmax <= 1.2e14, bmax
