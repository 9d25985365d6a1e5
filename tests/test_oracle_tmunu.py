"""Pins of the oracle's vertex stress-energy tensor T_{mu nu} (Sec. 3.1 storage at vertices; eq. tmunu): its normal
projections are the conserved energy and momentum densities of prim->cons, the rest-frame closed form, and the
8-cell vertex average on linear data."""
import numpy as np

from paper_2406_11669_amd.workloads import Layout, default_params
from tests.states import gmat
from tests.test_oracle_grid import _const_metric, _uniform_setup

IDX = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]


def _full(T10):
    T = np.zeros((4, 4))
    for c, (a, b) in enumerate(IDX):
        T[a, b] = T[b, a] = T10[c]
    return T


def _g4(m10):
    g = gmat(m10)
    alpha, beta = m10[0], m10[1:4]
    bl = g @ beta
    g4 = np.zeros((4, 4))
    g4[0, 0] = -alpha ** 2 + beta @ bl
    g4[0, 1:] = g4[1:, 0] = bl
    g4[1:, 1:] = g
    return g4


def test_tmunu_uniform_state_normal_projections(orc):
    """Uniform state in a constant metric: every vertex carries the same T_{mu nu}, whose projections on the normal
    n^mu = (1, -beta^i)/alpha are E = (tau + D)/sqrt(gamma) and S_i = S~_i/sqrt(gamma) of prim->cons."""
    L, m10, metric, prim, A, Bt = _uniform_setup()
    P = default_params(gamma=5.0 / 3.0)
    T = orc.tmunu(L, P, metric, prim, A)
    g = L.ng
    n = L.n[0]
    blk = T[:, g:g + n + 1, g:g + n + 1, g:g + n + 1].reshape(10, -1)
    assert np.all(blk == blk[:, :1])
    Tl = _full(blk[:, 0])
    nu = np.concatenate([[1.0], -m10[1:4]]) / m10[0]
    cons = orc.pt_prim2con(m10, prim[:, 0, 0, 0], Bt, 5.0 / 3.0)
    sg = np.sqrt(np.linalg.det(gmat(m10)))
    np.testing.assert_allclose(nu @ Tl @ nu, (cons[4] + cons[0]) / sg, rtol=1e-13)
    np.testing.assert_allclose(-(nu @ Tl)[1:], cons[1:4] / sg, rtol=1e-12, atol=1e-14)


def test_tmunu_rest_frame_flat(orc):
    """Fluid at rest in flat space with a uniform field: T_00 = rho (1 + eps) + B^2/2, T_0i = 0,
    T_ij = (p + B^2/2) delta_ij - B_i B_j."""
    B = np.array([0.375, -0.25, 0.625])
    L, _, _, prim, A, _ = _uniform_setup(vel=(0.0, 0.0, 0.0), B=tuple(B))
    m10 = np.array([1.0, 0, 0, 0, 1.0, 0, 0, 1.0, 0, 1.0])
    metric = _const_metric(L, m10)
    gam = 5.0 / 3.0
    T = orc.tmunu(L, default_params(gamma=gam), metric, prim, A)
    Tl = _full(T[:, L.ng + 2, L.ng + 3, L.ng + 1])
    rho, p = prim[0, 0, 0, 0], prim[1, 0, 0, 0]
    eps = p / ((gam - 1.0) * rho)
    B2 = B @ B
    np.testing.assert_allclose(Tl[0, 0], rho * (1 + eps) + 0.5 * B2, rtol=1e-14)
    np.testing.assert_allclose(Tl[0, 1:], 0.0, atol=1e-15)
    np.testing.assert_allclose(Tl[1:, 1:], (p + 0.5 * B2) * np.eye(3) - np.outer(B, B), rtol=1e-14, atol=1e-15)


def test_tmunu_vertex_average_exact_on_linear_fields(orc):
    """Primitives linear in space (uniform field, constant curved metric): the mean of the 8 cells around a vertex is
    the value at the vertex, so T_{mu nu} there equals the tensor of the exact vertex state (T^{mu nu} of the oracle's
    point routine, lowered here with the 4-metric)."""
    L, m10, metric, prim, A, Bt = _uniform_setup(vel=(0.1, -0.05, 0.2))
    xc, yc, zc = L.coords("centre")
    lin = lambda c0, cx, cy, cz, X, Y, Z: c0 + cx * X + cy * Y + cz * Z
    prim[0] = lin(0.7, 0.3, -0.2, 0.1, xc, yc, zc)
    prim[1] = lin(0.4, -0.1, 0.2, 0.15, xc, yc, zc)
    prim[2] = lin(0.1, 0.05, 0.02, -0.03, xc, yc, zc)
    gam = 5.0 / 3.0
    T = orc.tmunu(L, default_params(gamma=gam), metric, prim, A)
    xv, yv, zv = L.coords("vertex")
    g4 = _g4(m10)
    rng = np.random.default_rng(1)
    for _ in range(10):
        i, j, k = (L.ng + int(rng.integers(0, L.n[a] + 1)) for a in range(3))
        X, Y, Z = xv[0, 0, i], yv[0, j, 0], zv[k, 0, 0]
        pv = np.array([lin(0.7, 0.3, -0.2, 0.1, X, Y, Z), lin(0.4, -0.1, 0.2, 0.15, X, Y, Z),
                       lin(0.1, 0.05, 0.02, -0.03, X, Y, Z), prim[3, 0, 0, 0], prim[4, 0, 0, 0]])
        Tu = orc.pt_tmunu(m10, pv, Bt, gam)
        np.testing.assert_allclose(_full(T[:, k, j, i]), g4 @ Tu @ g4, rtol=1e-12, atol=1e-14)
