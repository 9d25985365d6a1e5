"""Pins of the oracle's stencils: reconstruction (Sec. 3.3), vertex interpolation (Sec. 3.2), the staggered
curl (Secs. 2.3, 3.1) and the geometric sources (Sec. 2.2, eq. grmhdsrc) against brute force."""
import itertools

import numpy as np
import pytest

from paper_2406_11669_amd.workloads import Layout, default_params
from tests.states import gmat, random_Bt, random_metric, random_prim

P = default_params()


# ---------------------------------------------------------------- reconstruction


@pytest.mark.parametrize("kind", ["minmod", "ppm", "wenoz", "mp5"])
def test_recon_constants_exact(orc, kind):
    a = np.full(20, 0.37)
    aL, aR = orc.recon_1d(P, kind, a)
    assert np.all(aL[2:-2] == 0.37) and np.all(aR[2:-2] == 0.37)


@pytest.mark.parametrize("kind", ["minmod", "ppm", "wenoz", "mp5"])
def test_recon_linear_exact(orc, kind):
    """Linear data are reproduced at the faces by every scheme."""
    x = np.arange(30, dtype=float)
    a = 0.3 + 0.7 * x
    aL, aR = orc.recon_1d(P, kind, a)
    np.testing.assert_allclose(aL[2:-2], 0.3 + 0.7 * (x[2:-2] - 0.5), rtol=0, atol=1e-12)
    np.testing.assert_allclose(aR[2:-2], 0.3 + 0.7 * (x[2:-2] + 0.5), rtol=0, atol=1e-12)


def test_ppm_interpolant_exact_on_cubic_averages(orc):
    """Without limiting, the PPM face value 7/12 (a_i + a_i+1) - 1/12 (a_i-1 + a_i+2) is exact for cell
    averages of a cubic; on a smooth monotone cubic the limiters stay inactive."""
    x = np.linspace(1.0, 2.0, 41)  # faces
    F = lambda t: 0.2 * t ** 4 / 4 + 0.1 * t ** 3 / 3 + t ** 2 / 2 + t  # antiderivative of a monotone cubic
    f = lambda t: 0.2 * t ** 3 + 0.1 * t ** 2 + t + 1
    a = (F(x[1:]) - F(x[:-1])) / (x[1] - x[0])
    aL, aR = orc.recon_1d(P, "ppm", a)
    np.testing.assert_allclose(aR[2:-2], f(x[3:-2]), rtol=1e-12)
    np.testing.assert_allclose(aL[2:-2], f(x[2:-3]), rtol=1e-12)


@pytest.mark.parametrize("kind", ["minmod", "ppm"])
def test_recon_no_new_extrema(orc, kind):
    """TVD/monotonicity: face values lie between the neighbouring cell values."""
    rng = np.random.default_rng(30)
    for _ in range(50):
        a = rng.normal(size=40) * rng.uniform(0.1, 10)
        aL, aR = orc.recon_1d(P, kind, a)
        for c in range(2, 38):
            lo = min(a[c - 1], a[c], a[c + 1]) - 1e-14
            hi = max(a[c - 1], a[c], a[c + 1]) + 1e-14
            assert lo <= aL[c] <= hi and lo <= aR[c] <= hi


@pytest.mark.parametrize("kind", ["minmod", "ppm", "wenoz", "mp5"])
def test_recon_mirror_symmetry(orc, kind):
    """Reversing the data swaps left and right face values bitwise."""
    rng = np.random.default_rng(31)
    a = rng.normal(size=40)
    aL, aR = orc.recon_1d(P, kind, a)
    bL, bR = orc.recon_1d(P, kind, a[::-1].copy())
    np.testing.assert_array_equal(aL[2:-2], bR[::-1][2:-2])
    np.testing.assert_array_equal(aR[2:-2], bL[::-1][2:-2])


def test_wenoz_fifth_order_on_smooth_averages(orc):
    """WENO-Z face values from exact cell averages of a smooth function converge at fifth order."""
    errs = []
    for n in (20, 40, 80):
        x = np.linspace(0, 1, n + 1)
        h = x[1] - x[0]
        a = -(np.cos(2 * np.pi * x[1:]) - np.cos(2 * np.pi * x[:-1])) / (2 * np.pi * h) + 2.0
        aL, aR = orc.recon_1d(P, "wenoz", a)
        ex = np.sin(2 * np.pi * x[3:-2]) + 2.0
        errs.append(np.max(np.abs(aR[2:-2] - ex)))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(order > 4.5), (errs, order)


def test_mp5_exact_on_quartic_averages(orc):
    """The MP5 interpolant (2, -13, 47, 27, -3)/60 is exact for cell averages of a quartic, and on a smooth
    monotone quartic the monotonicity test leaves it untouched."""
    x = np.linspace(1.0, 2.0, 41)  # faces
    F = lambda t: 0.05 * t ** 5 / 5 + 0.2 * t ** 4 / 4 + 0.1 * t ** 3 / 3 + t ** 2 / 2 + t
    f = lambda t: 0.05 * t ** 4 + 0.2 * t ** 3 + 0.1 * t ** 2 + t + 1
    a = (F(x[1:]) - F(x[:-1])) / (x[1] - x[0])
    aL, aR = orc.recon_1d(P, "mp5", a)
    np.testing.assert_allclose(aR[2:-2], f(x[3:-2]), rtol=1e-12)
    np.testing.assert_allclose(aL[2:-2], f(x[2:-3]), rtol=1e-12)


@pytest.mark.parametrize("data,left,right", [
    # isolated maximum: interpolant 47/60 at the right face; the curvature measures have mixed signs, so the
    # accuracy-preserving interval collapses to [1, 1] and both faces take the cell value
    ((0.0, 0.0, 1.0, 0.0, 0.0), 1.0, 1.0),
    # last cell before a unit step: interpolant 24/60, limited to 0 (no overshoot)
    ((0.0, 0.0, 0.0, 1.0, 1.0), 0.0, 0.0),
    # first cell after the step: interpolants 71/60 (right) and 36/60 (left), both limited to 1
    ((0.0, 0.0, 1.0, 1.0, 1.0), 1.0, 1.0),
    # linear data: the interpolant (0 - 13 + 94 + 81 - 12)/60 = 2.5 passes the monotonicity test
    ((0.0, 1.0, 2.0, 3.0, 4.0), 1.5, 2.5),
])
def test_mp5_worked_examples(orc, data, left, right):
    """Face values of the middle cell worked out by hand from the MP5 definition (Suresh & Huynh 1997, alpha =
    4): an extremum is flattened, a step stays sharp, linear data pass."""
    aL, aR = orc.recon_1d(P, "mp5", np.array(data))
    assert aL[2] == left and aR[2] == right


def test_mp5_affine_invariance(orc):
    """MP5 commutes with a -> s a + t for s of either sign (a sign error in a limiter breaks this)."""
    rng = np.random.default_rng(33)
    for _ in range(20):
        a = rng.normal(size=30) * rng.uniform(0.1, 3.0)
        aL, aR = orc.recon_1d(P, "mp5", a)
        for s_, t_ in ((2.0, 0.5), (-0.5, 3.0)):
            bL, bR = orc.recon_1d(P, "mp5", s_ * a + t_)
            np.testing.assert_allclose(bL[2:-2], s_ * aL[2:-2] + t_, rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(bR[2:-2], s_ * aR[2:-2] + t_, rtol=1e-12, atol=1e-12)


def test_mp5_fifth_order_on_smooth_averages(orc):
    """MP5 face values from exact cell averages of a smooth periodic function (with extrema) converge at fifth
    order: the curvature-based bounds keep the limiter from clipping smooth extrema."""
    errs = []
    for n in (20, 40, 80):
        x = np.linspace(0, 1, n + 1)
        h = x[1] - x[0]
        a = -(np.cos(2 * np.pi * x[1:]) - np.cos(2 * np.pi * x[:-1])) / (2 * np.pi * h) + 2.0
        aL, aR = orc.recon_1d(P, "mp5", a)
        ex = np.sin(2 * np.pi * x[3:-2]) + 2.0
        errs.append(np.max(np.abs(aR[2:-2] - ex)))
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(order > 4.5), (errs, order)


# ---------------------------------------------------------------- vertex -> centre / face interpolation


def _poly_field(L, coef, where="vertex"):
    x, y, z = L.coords(where)
    out = np.zeros(L.shape3)
    for (a, b, c), k in coef.items():
        out = out + k * x ** a * y ** b * z ** c
    return out


def _poly_deriv(coef, d):
    out = {}
    for (a, b, c), k in coef.items():
        e = [a, b, c]
        if e[d] == 0:
            continue
        kk = k * e[d]
        e[d] -= 1
        out[tuple(e)] = out.get(tuple(e), 0.0) + kk
    return out


def test_metric_interpolation_exact_on_tricubics(orc):
    """Fourth-order Lagrange interpolation (Sec. 3.2) and its midpoint derivative are exact on tensor-product
    cubics, at cell centres and at faces."""
    rng = np.random.default_rng(32)
    L = Layout((5, 6, 7), 3, dx=(0.11, 0.13, 0.17))
    metric = L.zeros(10)
    coefs = []
    for c in range(10):
        coef = {e: rng.uniform(-1, 1) for e in itertools.product(range(4), repeat=3) if rng.uniform() < 0.3}
        coefs.append(coef)
        metric[c] = _poly_field(L, coef)
    out = orc.centre_metric(L, metric)
    for c in range(10):
        ref = L.owned(_poly_field(L, coefs[c], "centre"))
        np.testing.assert_allclose(L.owned(out[c]), ref, rtol=0, atol=1e-12 * (1 + np.abs(ref).max()))
        for d in range(3):
            dref = L.owned(_poly_field(L, _poly_deriv(coefs[c], d), "centre"))
            np.testing.assert_allclose(L.owned(out[10 * (d + 1) + c]), dref, rtol=0,
                                       atol=1e-11 * (1 + np.abs(dref).max()))
    # faces: the x-face sits at vertex x and centre y, z
    for d, where_off in enumerate([(0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0)]):
        fi = orc.face_interp(L, metric[3], d)
        x = (np.arange(L.ld[0]) - L.ng + where_off[0]) * L.dx[0]
        y = (np.arange(L.ld[1]) - L.ng + where_off[1]) * L.dx[1]
        z = (np.arange(L.ld[2]) - L.ng + where_off[2]) * L.dx[2]
        ref = sum(k * x[None, None, :] ** a * y[None, :, None] ** b * z[:, None, None] ** cc
                  for (a, b, cc), k in coefs[3].items())
        np.testing.assert_allclose(L.owned(fi), L.owned(ref + 0 * fi), rtol=0, atol=1e-12)


def test_metric_interpolation_fourth_order(orc):
    errs = []
    for n in (8, 16, 32):
        L = Layout((n, n, n), 3)
        metric = L.zeros(10)
        x, y, z = L.coords("vertex")
        metric[0] = np.broadcast_to(np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y + 0.3) * np.sin(2 * np.pi * z + 1),
                                    L.shape3)
        out = orc.centre_metric(L, metric)
        x, y, z = L.coords("centre")
        ex = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y + 0.3) * np.sin(2 * np.pi * z + 1)
        dex = 2 * np.pi * np.cos(2 * np.pi * x) * np.cos(2 * np.pi * y + 0.3) * np.sin(2 * np.pi * z + 1)
        errs.append((np.max(np.abs(L.owned(out[0] - ex))), np.max(np.abs(L.owned(out[10] - dex)))))
    e = np.array(errs)
    order = np.log2(e[:-1] / e[1:])
    assert np.all(order > 3.8), (e, order)


# ---------------------------------------------------------------- staggered curl


def test_face_field_divergence_free(orc):
    """The face field is the curl of the edge potential, so its discrete divergence vanishes to round-off."""
    rng = np.random.default_rng(33)
    L = Layout((6, 7, 8), 3, dx=(0.1, 0.2, 0.3))
    A = rng.normal(size=(3,) + L.shape3)
    Bf = orc.face_B(L, A)
    g = L.ng
    sl = lambda a, b, c: (slice(g + c, g + c + L.n[2]), slice(g + b, g + b + L.n[1]), slice(g + a, g + a + L.n[0]))
    div = ((Bf[0][sl(1, 0, 0)] - Bf[0][sl(0, 0, 0)]) / L.dx[0] + (Bf[1][sl(0, 1, 0)] - Bf[1][sl(0, 0, 0)]) / L.dx[1]
           + (Bf[2][sl(0, 0, 1)] - Bf[2][sl(0, 0, 0)]) / L.dx[2])
    assert np.max(np.abs(div)) <= 1e-13 * np.max(np.abs(Bf))


def test_curl_sign_magnetic_loop(orc):
    """Sec. 4 (magnetic loop): A_z = A0 (R - r) inside the loop gives B^x = -A0 y/r, B^y = A0 x/r; the
    discrete curl reproduces that orientation (right-handed Levi-Civita symbol)."""
    n = 32
    L = Layout((n, n, 2), 3, dx=(2.0 / n, 2.0 / n, 0.1))
    A = L.zeros(3)
    x, y, z = L.coords("zedge")
    x = x - 1.0
    y = y - 1.0
    r = np.sqrt(x ** 2 + y ** 2)
    A[2] = np.broadcast_to(np.maximum(0.0, 1e-3 * (0.6 - r)), L.shape3)
    Bf = orc.face_B(L, A)
    xf, yf, _ = L.coords("centre")  # x-face: vertex x, centre y
    xv = (np.arange(L.ld[0]) - L.ng) * L.dx[0] - 1.0
    yc = (np.arange(L.ld[1]) - L.ng + 0.5) * L.dx[1] - 1.0
    X, Y = np.meshgrid(xv, yc, indexing="xy")
    R = np.sqrt(X ** 2 + Y ** 2)
    mask = (R > 0.15) & (R < 0.45)
    bx = Bf[0][L.ng][mask]
    ref = -1e-3 * Y[mask] / R[mask]
    np.testing.assert_allclose(bx, ref, rtol=0, atol=2e-5)


# ---------------------------------------------------------------- sources vs brute force


def _metric_at(m0, grad, x):
    """Metric components linear in x: m(x) = m0 + grad . x (grad: [3][10])."""
    return m0 + grad.T @ x


def _g4(m):
    a, b = m[0], m[1:4]
    g = gmat(m)
    bl = g @ b
    G = np.zeros((4, 4), dtype=np.result_type(m))
    G[0, 0] = -a * a + b @ bl
    G[0, 1:] = G[1:, 0] = bl
    G[1:, 1:] = g
    return G


def test_sources_match_christoffel_brute_force(orc):
    """S_j = T^{mu nu}(d_mu g_{nu j} - Gamma^d_{nu mu} g_{d j}) and
    S_tau = alpha (T^{mu 0} d_mu ln alpha - T^{mu nu} Gamma^0_{nu mu}) (eq. grmhdsrc) evaluated with
    Christoffel symbols of a numerically differentiated static 4-metric; K_ij = (D_i beta_j + D_j beta_i)/(2 alpha)
    for a static metric.  Both times alpha sqrt(gamma)."""
    rng = np.random.default_rng(34)
    for _ in range(50):
        gam = rng.uniform(1.3, 2.0)
        m0 = random_metric(rng)
        grad = rng.uniform(-0.5, 0.5, (3, 10))
        pr = random_prim(rng, m0, vmax=0.8)
        Bt = random_Bt(rng, m0, 1.5)
        h = 1e-30
        dg4 = np.zeros((4, 4, 4))  # [rho, mu, nu], d_t = 0; complex-step derivative, exact to round-off
        for j in range(3):
            e = np.zeros(3, dtype=complex)
            e[j] = 1j * h
            dg4[j + 1] = np.imag(_g4(_metric_at(m0.astype(complex), grad, e))) / h
        g4 = _g4(m0)
        gi4 = np.linalg.inv(g4)
        Gam = 0.5 * (np.einsum("ds,msn->dmn", gi4, dg4) + np.einsum("ds,nsm->dmn", gi4, dg4)
                     - np.einsum("ds,smn->dmn", gi4, dg4))
        T = orc.pt_tmunu(m0, pr, Bt, gam)
        alpha = m0[0]
        dlna = np.zeros(4)
        dlna[1:] = grad[:, 0] / alpha
        Sj = np.array([np.einsum("mn,mn->", T, dg4[:, :, j + 1]) - np.einsum("mn,dnm,d->", T, Gam, g4[:, j + 1])
                       for j in range(3)])
        Stau = alpha * (T[:, 0] @ dlna - np.einsum("mn,nm->", T, Gam[0]))
        # K for the static metric, written with the 3-covariant derivative
        g3 = gmat(m0)
        dg3 = np.stack([gmat(grad[k]) for k in range(3)])  # d_k gamma_ij (linear field)
        gi3 = np.linalg.inv(g3)
        G3 = 0.5 * (np.einsum("kl,ilj->kij", gi3, dg3) + np.einsum("kl,jli->kij", gi3, dg3)
                    - np.einsum("kl,lij->kij", gi3, dg3))
        beta = m0[1:4]
        dbeta = grad[:, 1:4]  # [i, a] = d_i beta^a
        bl = g3 @ beta
        dbl = np.einsum("ija,a->ij", dg3, beta) + np.einsum("ja,ia->ij", g3, dbeta)
        Db = dbl - np.einsum("kij,k->ij", G3, bl)
        K = (Db + Db.T) / (2 * alpha)
        K6 = [K[0, 0], K[0, 1], K[0, 2], K[1, 1], K[1, 2], K[2, 2]]
        src = orc.pt_sources(m0, grad.reshape(-1), K6, pr, Bt, gam)
        sg = np.sqrt(np.linalg.det(g3))
        ref = alpha * sg * np.array([0.0, *Sj, Stau])
        scale = alpha * sg * np.max(np.abs(T)) * np.max(np.abs(grad))
        np.testing.assert_allclose(src, ref, rtol=0, atol=1e-12 * scale)


def test_sources_flat_vanish(orc):
    rng = np.random.default_rng(35)
    m = random_metric(rng, curved=False)
    for _ in range(20):
        pr = random_prim(rng, m)
        src = orc.pt_sources(m, np.zeros(30), np.zeros(6), pr, rng.uniform(-1, 1, 3), 5.0 / 3.0)
        assert np.all(src == 0.0)
