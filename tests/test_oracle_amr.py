"""Pins of the oracle's factor-2 inter-level operators (prolongation at refinement boundaries, Sec. 3.9 and the AMR
tests of Sec. 4; restriction): conservation (restriction undoes prolongation), polynomial exactness per staggering,
no new extrema at a step (the linear fallback), and Stokes consistency of the potential's prolongation."""
import numpy as np
import pytest

from paper_2406_11669_amd.workloads import Layout

NC, NF, NG = 8, 8, 3   # the fine block covers coarse cells [C0, C0 + NF/2)
C0 = (2, 3, 1)


def _grids():
    coarse = Layout((NC, NC, NC), NG, dx=(0.1, 0.1, 0.1))
    fine = Layout((NF, NF, NF), NG, dx=(0.05, 0.05, 0.05))
    return coarse, fine


def _fine_box(fine):
    """Fine points prolonged here: the owned cells plus two ghost layers (their coarse stencils stay inside the
    coarse block's stored points)."""
    return (-2, -2, -2), tuple(fine.n[a] + 1 for a in range(3))


def _coarse_cover(fine):
    """Coarse cells whose 8 children are all inside _fine_box."""
    lo = tuple(C0[a] - 1 for a in range(3))
    hi = tuple(C0[a] + fine.n[a] // 2 for a in range(3))
    return lo, hi


def _ix(L, lo, hi):
    g = L.ng
    return tuple(slice(g + lo[a], g + hi[a] + 1) for a in (2, 1, 0))


def _coords_cell(L):
    return L.coords("centre")


def _cell_avg(F, L, stag):
    """Cell averages (cell-centred directions) and point values (vertex-centred directions) of a separable
    polynomial F = (fx, Fx, fy, Fy, fz, Fz) (point function and antiderivative per axis)."""
    out = 1.0
    xs = L.coords("vertex")
    for a in range(3):
        f, Fa = F[2 * a], F[2 * a + 1]
        v = xs[a]
        h = L.dx[a]
        out = out * (f(v) if stag[a] else (Fa(v + h) - Fa(v)) / h)
    return np.broadcast_to(out, L.shape3).copy()


@pytest.mark.parametrize("stag", ["cell", "vertex", "xedge", "zedge"])
def test_restriction_undoes_prolongation(orc, stag):
    """restrict(prolong(u)) = u on the covered coarse points: the children's mean (cell directions) and the
    coincident fine point (vertex directions) return the coarse value, also where the fallback acts."""
    coarse, fine = _grids()
    rng = np.random.default_rng(11)
    cf = rng.normal(size=(2,) + coarse.shape3)
    ff = np.zeros((2,) + fine.shape3)
    lo, hi = _fine_box(fine)
    orc.prolong(coarse, fine, C0, stag, cf, ff, lo, hi)
    back = np.zeros_like(cf)
    clo, chi = _coarse_cover(fine)
    orc.restrict(coarse, fine, C0, stag, ff, back, clo, chi)
    sl = (slice(None),) + _ix(coarse, clo, chi)
    np.testing.assert_allclose(back[sl], cf[sl], rtol=0, atol=1e-14)


@pytest.mark.parametrize("stag", ["cell", "vertex", "xedge", "yedge"])
def test_prolongation_exact_on_polynomials(orc, stag):
    """Quadratic in cell-centred directions (conservative, cell averages) and cubic in vertex-centred ones (point
    values): the prolonged fine data are the fine averages/values of the same polynomial; a monotone polynomial
    never triggers the fallback."""
    from oracle.oracle import STAG
    s = STAG[stag]
    coarse, fine = _grids()
    px = (lambda x: 1.0 + 0.4 * x + 0.3 * x ** 2, lambda x: x + 0.2 * x ** 2 + 0.1 * x ** 3)
    cx = (lambda x: 2.0 + 0.5 * x - 0.2 * x ** 2 + 0.1 * x ** 3, None)
    F = []
    for a in range(3):
        F += list(cx if s[a] else px)
    cf = _cell_avg(F, coarse, s)[None]
    ff = np.zeros((1,) + fine.shape3)
    lo, hi = _fine_box(fine)
    orc.prolong(coarse, fine, C0, s, cf, ff, lo, hi)
    # the fine grid in coarse coordinates: shift by C0 coarse cells
    shifted = []
    for a in range(3):
        f_, Fa = F[2 * a], F[2 * a + 1]
        off = C0[a] * coarse.dx[a]
        shifted += [lambda x, f_=f_, off=off: f_(x + off), None if Fa is None else (lambda x, Fa=Fa, off=off: Fa(x + off))]
    ref = _cell_avg(shifted, fine, s)
    sl = _ix(fine, lo, hi)
    np.testing.assert_allclose(ff[0][sl], ref[sl], rtol=1e-13, atol=1e-13)


def test_prolongation_step_has_no_new_extrema(orc):
    """A unit step in x (cell field): the third-order children overshoot next to the jump, so those coarse cells fall
    back to limited linear children; every fine value stays in [0, 1] and the means stay the coarse values."""
    coarse, fine = _grids()
    xc, _, _ = coarse.coords("centre")
    cf = np.broadcast_to((xc > (C0[0] + 2) * coarse.dx[0]).astype(float), coarse.shape3).copy()[None]
    ff = np.zeros((1,) + fine.shape3)
    lo, hi = _fine_box(fine)
    orc.prolong(coarse, fine, C0, "cell", cf, ff, lo, hi)
    vals = ff[0][_ix(fine, lo, hi)]
    # without the fallback the children beside the jump would be -1/8 and 9/8
    assert vals.min() >= 0.0 and vals.max() <= 1.0
    back = np.zeros_like(cf)
    clo, chi = _coarse_cover(fine)
    orc.restrict(coarse, fine, C0, "cell", ff, back, clo, chi)
    sl = (slice(None),) + _ix(coarse, clo, chi)
    np.testing.assert_allclose(back[sl], cf[sl], atol=1e-15)


def test_potential_prolongation_keeps_coarse_face_fluxes(orc):
    """The prolonged potential keeps each coarse edge's line integral (restriction undoes it along edges), so by
    Stokes the fine face fields (curl of the fine potential) averaged over the 4 fine faces of a coarse face equal
    the coarse face field."""
    coarse, fine = _grids()
    rng = np.random.default_rng(12)
    Ac = rng.normal(size=(3,) + coarse.shape3)
    Af = np.zeros((3,) + fine.shape3)
    lo, hi = _fine_box(fine)
    for c, stag in enumerate(["xedge", "yedge", "zedge"]):
        orc.prolong(coarse, fine, C0, stag, Ac[c:c + 1], Af[c:c + 1], lo, hi)
    Bc = orc.face_B(coarse, Ac)
    Bf = orc.face_B(fine, Af)
    g, gf = coarse.ng, fine.ng
    for (ci, cj, ck) in [(C0[0], C0[1], C0[2]), (C0[0] + 1, C0[1] + 2, C0[2] + 3), (C0[0] + 3, C0[1] + 1, C0[2])]:
        fi, fj, fk = 2 * (ci - C0[0]), 2 * (cj - C0[1]), 2 * (ck - C0[2])
        # x-face at coarse (ci - 1/2, cj, ck): fine x-faces at fi with (fj..fj+1, fk..fk+1)
        fx = np.mean([Bf[0, gf + fk + b, gf + fj + a, gf + fi] for a in (0, 1) for b in (0, 1)])
        fy = np.mean([Bf[1, gf + fk + b, gf + fj, gf + fi + a] for a in (0, 1) for b in (0, 1)])
        fz = np.mean([Bf[2, gf + fk, gf + fj + b, gf + fi + a] for a in (0, 1) for b in (0, 1)])
        np.testing.assert_allclose([fx, fy, fz], [Bc[0, g + ck, g + cj, g + ci], Bc[1, g + ck, g + cj, g + ci],
                                                  Bc[2, g + ck, g + cj, g + ci]], rtol=1e-12, atol=1e-12)
