"""Pins of three oracle parts that the grid-level invariants do not reach: the maximum characteristic speed
over the faces of owned cells (the Courant number behind the time steps of Sec. 4), the Runge-Kutta stage
combination, and the operation-counting scalar behind every FLOP figure."""
import numpy as np
import pytest

from paper_2406_11669_amd.workloads import Layout, default_params
from tests.states import gmat

FLAT = np.array([1.0, 0, 0, 0, 1.0, 0, 0, 1.0, 0, 1.0])
# a constant non-trivial metric with dyadic entries (its interpolations to faces and centres are exact)
CURVED = np.array([0.875, 0.125, -0.0625, 0.25, 1.25, 0.125, -0.0625, 1.125, 0.0625, 0.9375])


def _uniform(m10, rho, p, vel, B, n=6, ng=3, fast_corner=None):
    """Uniform fluid and densitized field B~ in a constant metric (dx = 1/16, dyadic B: the face field is bitwise
    uniform).  fast_corner: primitives planted in the ghost cells with j < 0 and k < 0, which only faces outside the
    owned range read (x faces at j = -1, k = -1 and the y and z faces of the ghost rows)."""
    L = Layout((n, n, n), ng, dx=(1 / 16, 1 / 16, 1 / 16))
    metric = L.zeros(10)
    for c in range(10):
        metric[c] = m10[c]
    prim = L.zeros(5)
    prim[0], prim[1] = rho, p
    for d in range(3):
        prim[2 + d] = vel[d]
    if fast_corner is not None:
        for c in range(5):
            prim[c, :ng, :ng, :] = fast_corner[c]
    A = L.zeros(3)
    xy, _, _ = L.coords("yedge")
    A[1] = np.broadcast_to(B[2] * xy, L.shape3)
    xz, yz, _ = L.coords("zedge")
    A[2] = np.broadcast_to(B[0] * yz - B[1] * xz, L.shape3)
    return L, metric, prim, A


def _sound(gam, rho, p):
    """cs^2 and rho h of an ideal gas."""
    rhoh = rho + gam / (gam - 1.0) * p
    return gam * p / rhoh, rhoh


def _banyuls(m10, gam, rho, p, v, d):
    """Unmagnetized characteristic speeds along d in a general 3+1 metric (Banyuls et al. 1997), closed form."""
    g = gmat(m10)
    gi = np.linalg.inv(g)
    cs2, _ = _sound(gam, rho, p)
    v = np.asarray(v, dtype=float)
    v2 = v @ g @ v
    root = np.sqrt((1 - v2) * (gi[d, d] * (1 - v2 * cs2) - v[d] ** 2 * (1 - cs2)))
    a = m10[0] / (1 - v2 * cs2)
    return a * (v[d] * (1 - cs2) - np.sqrt(cs2) * root) - m10[1 + d], \
        a * (v[d] * (1 - cs2) + np.sqrt(cs2) * root) - m10[1 + d]


def _red(orc, L, metric, prim, A, gam, recon):
    P = default_params(gamma=gam, recon=recon)
    out, red, nfix = orc.rhs(L, P, metric, L.zeros(6), prim, A, L.zeros(1), 0.01)
    assert nfix == 0
    return red


FAST = [0.7, 0.4, 0.85, 0.0, 0.0]


@pytest.mark.parametrize("recon", ["minmod", "ppm"])
def test_max_speed_unmagnetized_curved(orc, recon):
    """B = 0, uniform flow in a constant curved metric with shift: red[0] is the largest of lambda_+ and -lambda_-
    over the three directions (the HLLE speeds c_max, c_min are max(0, lambda_+) and max(0, -lambda_-)).  The
    ghost corner flows at 0.85 along x: counting a face outside the owned range would raise the maximum."""
    gam, rho, p, v = 5.0 / 3.0, 0.7, 0.4, (0.3, -0.2, 0.1)
    L, metric, prim, A = _uniform(CURVED, rho, p, v, (0.0, 0.0, 0.0), fast_corner=FAST)
    red = _red(orc, L, metric, prim, A, gam, recon)
    ref = max(max(lp, -lm, 0.0) for lm, lp in (_banyuls(CURVED, gam, rho, p, v, d) for d in range(3)))
    assert abs(red[0] - ref) <= 1e-13 * ref, (red[0], ref)
    assert red[1] == 0.0


def test_max_speed_at_rest_perpendicular_field(orc):
    """At rest in flat space with B~ along z: the x and y fronts run at the fast speed
    w^2 = cs^2 + cA^2 - cs^2 cA^2 (cA^2 = B^2/(rho h + B^2)), the z front at max(cs, cA) <= w."""
    gam, rho, p = 2.0, 0.7, 0.4
    B = (0.0, 0.0, 0.75)
    L, metric, prim, A = _uniform(FLAT, rho, p, (0, 0, 0), B, fast_corner=FAST)
    red = _red(orc, L, metric, prim, A, gam, "ppm")
    cs2, rhoh = _sound(gam, rho, p)
    cA2 = B[2] ** 2 / (rhoh + B[2] ** 2)
    ref = np.sqrt(cs2 + cA2 - cs2 * cA2)
    assert abs(red[0] - ref) <= 1e-13, (red[0], ref)


def test_max_speed_boost_along_field_counts_the_left_going_front(orc):
    """Flat space, flow at vx = -0.6 along a field along x: the left-going front moves at -(0.6 + c)/(1 + 0.6 c)
    with c = max(cs, cA) the rest-frame fast speed along the field (relativistic velocity addition); its magnitude
    is the maximum.  A reduction over c_max alone would miss it (the right-going front is (c - 0.6)/(1 - 0.6 c))."""
    gam, rho, p, vx = 5.0 / 3.0, 0.7, 0.4, -0.6
    B = (0.5, 0.0, 0.0)
    L, metric, prim, A = _uniform(FLAT, rho, p, (vx, 0, 0), B, fast_corner=FAST)
    red = _red(orc, L, metric, prim, A, gam, "minmod")
    cs2, rhoh = _sound(gam, rho, p)
    c = np.sqrt(max(cs2, B[0] ** 2 / (rhoh + B[0] ** 2)))
    ref = (-vx + c) / (1 - vx * c)
    assert abs(red[0] - ref) <= 1e-12, (red[0], ref)
    assert ref > (c + vx) / (1 + vx * c)


def test_max_speed_lapse_and_shift(orc):
    """At rest, no field, gamma = delta, constant lapse and shift: lambda_+- = +-alpha cs - beta^d, so the maximum is
    alpha cs + max_d |beta^d|."""
    gam, rho, p = 5.0 / 3.0, 0.7, 0.4
    m10 = np.array([0.75, 0.125, -0.25, 0.0625, 1.0, 0, 0, 1.0, 0, 1.0])
    L, metric, prim, A = _uniform(m10, rho, p, (0, 0, 0), (0, 0, 0), fast_corner=FAST)
    red = _red(orc, L, metric, prim, A, gam, "ppm")
    cs2, _ = _sound(gam, rho, p)
    ref = 0.75 * np.sqrt(cs2) + 0.25
    assert abs(red[0] - ref) <= 1e-13, (red[0], ref)


# ---- Runge-Kutta stage combination ------------------------------------------------------------------------

def test_rk_combine_hand_evaluated(orc):
    """out = sum a_m u_m + b dt L on owned points of all 9 fields, ghosts untouched.  Dyadic values make the
    result exact: field f has u_0 = 4 (f + 1), u_1 = 2, u_2 = 8, L = 16, with a = (1/4, 1/2, 1/8) and
    b dt = 1/16, so out = (f + 1) + 1 + 1 + 1 = f + 4."""
    L = Layout((5, 4, 3), 3)
    u0, u1, u2, rhs = L.zeros(9), L.zeros(9) + 2.0, L.zeros(9) + 8.0, L.zeros(9) + 16.0
    for f in range(9):
        u0[f] = 4.0 * (f + 1)
    out = L.zeros(9) - 7.0
    orc.rk_stage(L, [0.25, 0.5, 0.125], [u0, u1, u2], 1.0 / 16.0, rhs, out)
    own = np.zeros(L.shape3, dtype=bool)
    L.owned(own)[...] = True
    for f in range(9):
        assert np.all(out[f][own] == f + 4.0), f
        assert np.all(out[f][~own] == -7.0), f


@pytest.mark.parametrize("rk", [2, 4])
def test_rk_combine_stability_polynomial(orc, rk):
    """The tableaux composed of stage combinations integrate y' = lambda y with the amplification factor
    1 + z + z^2/2 (Heun) and 1 + z + z^2/2 + z^3/6 + z^4/24 (classical RK4), z = lambda dt."""
    L = Layout((4, 3, 2), 3)
    rng = np.random.default_rng(3)
    y0 = L.zeros(9)
    L.owned(y0)[...] = rng.uniform(0.5, 2.0, L.owned(y0).shape)
    lam, dt = -1.7, 0.3
    z = lam * dt

    def comb(a, us, bdt, r):
        out = L.zeros(9)
        orc.rk_stage(L, a, us, bdt, r, out)
        return out

    if rk == 2:
        k1 = lam * y0
        y1 = comb([1.0], [y0], dt, k1)
        y = comb([0.5, 0.5], [y0, y1], 0.5 * dt, lam * y1)
        amp = 1 + z + z * z / 2
    else:
        k1 = lam * y0
        y2 = comb([1.0], [y0], 0.5 * dt, k1)
        k2 = lam * y2
        y3 = comb([1.0], [y0], 0.5 * dt, k2)
        k3 = lam * y3
        y4 = comb([1.0], [y0], dt, k3)
        k4 = lam * y4
        acc = comb([1.0, dt / 6, dt / 3, dt / 3], [y0, k1, k2, k3], dt / 6, k4)
        y = acc
        amp = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    np.testing.assert_allclose(L.owned(y), amp * L.owned(y0), rtol=1e-14, atol=0)


# ---- operation-counting scalar ----------------------------------------------------------------------------

def test_counter_building_blocks_hand_counted(orc):
    """Each +, -, *, /, sqrt and pow counts one operation; negation, fabs and comparisons none.  Hand counts:
    Lagrange value (-1, 9, 9, -1)/16: 4 products + 3 sums = 7; midpoint derivative (27 (f2 - f1) - (f3 - f0))/(24 dx):
    3 differences, 1 product, 1 quotient = 5; face value (4 x 4 points): 4 column values + 1 row value = 35;
    centre value: 16 + 4 + 1 Lagrange values = 147; centre value and three derivatives: 16 x (7 + 5) in z,
    4 x (7 + 5 + 7) in y, 7 + 5 + 7 + 7 in x = 294; face field (curl of A): 2 differences, 2 quotients, 1 difference
    = 5; centre field: 3 x (2 face fields + a sum and a halving) = 36; 3+1 geometry: 9 cofactors x 3, determinant
    5, inverse 9, sqrt 1, lowered shift 3 x 6 = 60; the mixed probe expression: 8."""
    c = orc.count_probe()
    assert c == dict(lag_value=7, lag_deriv=5, face_interp=35, centre_value=147, centre_interp=294, face_B=5,
                     centre_B=36, make_geom=60, mixed_expression=8), c


def test_counter_grid_phases_decompose(orc):
    """Grid counts are sums of their parts with no hidden work.  Centre field: 36 operations per cell of the
    (n + 2 ng)^3 box.  Recovery: per owned cell, 10 metric values (147 each), the centre field (36), the geometry
    (60) and the point recovery itself (counted on the same inputs; uniform data converge identically in every
    cell): no metric derivatives, which the recovery does not use.  Faces and cells: a uniform state does the same
    work at every face and cell, so the counts are exact multiples of 3 (n + 1)^3 faces (flux CT covers the
    transverse range [-1, n - 1]) and of n^3 cells, with the same per-face and per-cell figures at two sizes."""
    gam, rho, p, v, B = 5.0 / 3.0, 0.7, 0.4, (0.3, -0.2, 0.1), (0.375, -0.25, 0.625)
    per = {}
    for n in (4, 6):
        L, metric, prim, A = _uniform(CURVED, rho, p, v, B, n=n)
        P = default_params(gamma=gam, recon="ppm")
        cnt = orc.count_ops(L, P, metric, L.zeros(6), prim, A, L.zeros(1), 0.01)
        assert cnt["centre_B"] == 36 * (n + 6) ** 3
        cons = orc.prim2con(L, P, metric, A, prim)
        cell = (slice(None), 3, 3, 3)
        Bt = np.array(B)
        ops, it = orc.count_c2p_point(P, CURVED, cons[cell], Bt, prim[cell])
        assert it >= 1
        assert cnt["c2p"] == n ** 3 * (10 * 147 + 36 + 60 + ops), (cnt["c2p"], ops)
        nfaces = 3 * (n + 1) ** 3
        assert cnt["faces"] % nfaces == 0 and cnt["cells"] % n ** 3 == 0
        per[n] = (cnt["faces"] // nfaces, cnt["cells"] // n ** 3)
    assert per[4] == per[6], per
    # a face interpolates 10 metric components (35 each), forms its geometry and normal field at least
    assert per[4][0] > 10 * 35 + 60 + 5


def test_near_tie_counter_sees_constructed_ties(orc):
    """The limiter near-tie counter: a PPM cell whose right-face value differs from the cell value only in its
    last bits is counted as a near tie of the extremum test; uniform data (exact equalities) and well separated
    data are not."""
    import numpy as np
    from paper_2406_11669_amd.workloads import default_params
    P = default_params(recon="ppm")
    orc.tie_counts()
    orc.recon_1d(P, "ppm", np.ones(12))
    dec, near = orc.tie_counts()
    assert dec > 0 and near == 0
    orc.recon_1d(P, "ppm", np.linspace(0.0, 1.0, 12) ** 2)
    assert orc.tie_counts()[1] == 0
    # a monotone ramp whose next value repeats the centre up to one ulp: the right face lands within
    # rounding of the centre value
    a = np.array([0.0, 0.25, 0.5, 0.75, 1.0, 1.0 + 2.0 ** -51, 1.0 + 2.0 ** -50, 1.5, 2.0, 2.5, 3.0, 3.5])
    orc.recon_1d(P, "ppm", a)
    assert orc.tie_counts()[1] > 0
