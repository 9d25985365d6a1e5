"""Pins of the oracle's pointwise physics against closed forms, identities and brute force.

Each test states what fixes the expected value: a printed identity of the paper,
a textbook special case, or a brute-force evaluation written independently here.
"""
import numpy as np
import pytest

from tests.states import gmat, random_Bt, random_metric, random_prim

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _aux(m10, prim, Bt, gam):
    """Independent numpy construction of W, v_i, B^i, B_i, z for identity checks."""
    g = gmat(m10)
    sg = np.sqrt(np.linalg.det(g))
    v = prim[2:]
    vl = g @ v
    v2 = v @ vl
    W = 1.0 / np.sqrt(1.0 - v2)
    B = Bt / sg
    Bl = g @ B
    rho, p = prim[0], prim[1]
    eps = p / ((gam - 1.0) * rho)
    h = 1.0 + eps + p / rho
    return dict(g=g, sg=sg, v=v, vl=vl, v2=v2, W=W, B=B, Bl=Bl, B2=B @ Bl, Bv=B @ vl, rho=rho, p=p, h=h,
                z=rho * h * W * W, eps=eps)


# ---------------------------------------------------------------- EOS


def test_eos_closed_forms(orc):
    """Ideal gas (Sec. 3.7): p = (Gamma-1) rho eps and h = 1 + eps + p/rho = 1 + Gamma eps."""
    rng = np.random.default_rng(1)
    for _ in range(50):
        gam = rng.uniform(1.2, 2.0)
        m = random_metric(rng)
        pr = random_prim(rng, m)
        f = orc.pt_fluid(m, pr, np.zeros(3), gam)
        assert abs((gam - 1) * pr[0] * f["eps"] - pr[1]) <= 1e-14 * pr[1]
        assert abs(f["h"] - (1 + gam * f["eps"])) <= 1e-14 * f["h"]


# ---------------------------------------------------------------- prim -> cons


def test_prim2con_equals_second_printed_form(orc):
    """Sec. 3.5 rewrites S_i as (z + B^2) v_i - (B^j v_j) B_i; tau follows likewise.

    The oracle evaluates the conserved-variable definitions with b^mu; the
    printed rewrite with z = rho h W^2 must agree to round-off."""
    rng = np.random.default_rng(2)
    for _ in range(200):
        gam = rng.uniform(1.3, 2.0)
        m = random_metric(rng)
        pr = random_prim(rng, m, vmax=0.95)
        Bt = random_Bt(rng, m, 2.0)
        a = _aux(m, pr, Bt, gam)
        cons = orc.pt_prim2con(m, pr, Bt, gam)
        D = a["rho"] * a["W"]
        S = (a["z"] + a["B2"]) * a["vl"] - a["Bv"] * a["Bl"]
        tau = a["z"] + a["B2"] - a["p"] - a["B2"] / (2 * a["W"] ** 2) - a["Bv"] ** 2 / 2 - D
        ref = a["sg"] * np.array([D, *S, tau])
        scale = np.max(np.abs(ref)) + a["sg"] * (a["z"] + a["B2"])
        np.testing.assert_allclose(cons, ref, rtol=0, atol=1e-13 * scale)


def test_prim2con_srmhd_limit(orc):
    """Flat metric, B = 0: D = rho W, S = rho h W^2 v, tau = rho h W^2 - p - D (special relativity)."""
    rng = np.random.default_rng(3)
    m = random_metric(rng, curved=False)
    for _ in range(50):
        pr = random_prim(rng, m)
        a = _aux(m, pr, np.zeros(3), 5.0 / 3.0)
        cons = orc.pt_prim2con(m, pr, np.zeros(3), 5.0 / 3.0)
        ref = [a["rho"] * a["W"], *(a["rho"] * a["h"] * a["W"] ** 2 * a["v"]),
               a["rho"] * a["h"] * a["W"] ** 2 - a["p"] - a["rho"] * a["W"]]
        np.testing.assert_allclose(cons, ref, rtol=1e-14, atol=1e-15)


def test_tmunu_normal_projections(orc):
    """T^{mu nu} n_mu n_nu = tau + D and -n_mu T^mu_i = S_i (Sec. 3.5), n_mu = (-alpha, 0, 0, 0)."""
    rng = np.random.default_rng(4)
    for _ in range(100):
        gam = rng.uniform(1.3, 2.0)
        m = random_metric(rng)
        pr = random_prim(rng, m)
        Bt = random_Bt(rng, m)
        T = orc.pt_tmunu(m, pr, Bt, gam)
        cons = orc.pt_prim2con(m, pr, Bt, gam)
        g = gmat(m)
        sg = np.sqrt(np.linalg.det(g))
        alpha, beta = m[0], m[1:4]
        beta_l = g @ beta
        g4 = np.zeros((4, 4))
        g4[0, 0] = -alpha ** 2 + beta @ beta_l
        g4[0, 1:] = g4[1:, 0] = beta_l
        g4[1:, 1:] = g
        E = alpha ** 2 * T[0, 0]
        Si = alpha * (g4[1:, :] @ T[0, :])
        scale = np.max(np.abs(cons)) / sg
        assert abs(E - (cons[4] + cons[0]) / sg) <= 1e-13 * scale
        np.testing.assert_allclose(Si, cons[1:4] / sg, rtol=0, atol=1e-13 * scale)


# ---------------------------------------------------------------- fluxes


def test_flux_srmhd_limit(orc):
    """Flat metric: the fluxes equal the special-relativistic MHD fluxes written here from their flat form."""
    rng = np.random.default_rng(5)
    m = random_metric(rng, curved=False)
    for _ in range(100):
        gam = rng.uniform(1.3, 2.0)
        pr = random_prim(rng, m, vmax=0.95)
        B = rng.uniform(-2, 2, 3)
        rho, p, v = pr[0], pr[1], pr[2:]
        W = 1 / np.sqrt(1 - v @ v)
        h = 1 + gam / (gam - 1) * p / rho
        Bv = B @ v
        b0 = W * Bv
        b = B / W + b0 * v
        b2 = B @ B / W ** 2 + Bv ** 2
        D = rho * W
        S = (rho * h + b2) * W ** 2 * v - b0 * b
        tau = (rho * h + b2) * W ** 2 - (p + b2 / 2) - b0 ** 2 - D
        for d in range(3):
            U, F = orc.pt_flux(m, pr, B, gam, d)
            ref = np.zeros(7)
            ref[0] = D * v[d]
            ref[1:4] = S * v[d] - b * B[d] / W
            ref[1 + d] += p + b2 / 2
            ref[4] = tau * v[d] + (p + b2 / 2) * v[d] - b0 * B[d] / W
            t1, t2 = (d + 1) % 3, (d + 2) % 3
            ref[5] = B[t1] * v[d] - B[d] * v[t1]
            ref[6] = B[t2] * v[d] - B[d] * v[t2]
            scale = np.max(np.abs(ref)) + p + b2
            np.testing.assert_allclose(F, ref, rtol=0, atol=1e-13 * scale)
            np.testing.assert_allclose(U[:5], [D, *S, tau], rtol=0, atol=1e-13 * scale)


def test_flux_constant_metric_is_transformed_flat(orc):
    """Lapse and shift enter as F = alpha sqrt(gamma) (...) with vt = alpha v - beta: for alpha, beta
    constant and gamma = identity, F(alpha, beta) = alpha F_flat - beta^d U_flat for D, S, tau."""
    rng = np.random.default_rng(6)
    for _ in range(50):
        gam = 5.0 / 3.0
        flat = random_metric(rng, curved=False)
        m = flat.copy()
        m[0] = rng.uniform(0.5, 1.5)
        m[1:4] = rng.uniform(-0.3, 0.3, 3)
        pr = random_prim(rng, flat)
        B = rng.uniform(-1, 1, 3)
        for d in range(3):
            Uf, Ff = orc.pt_flux(flat, pr, B, gam, d)
            U, F = orc.pt_flux(m, pr, B, gam, d)
            np.testing.assert_allclose(U, Uf, rtol=1e-14, atol=1e-15)
            ref = m[0] * Ff - m[1 + d] * Uf
            # induction fluxes: vt^d B^k - vt^k B^d
            vt = m[0] * pr[2:] - m[1:4]
            t1, t2 = (d + 1) % 3, (d + 2) % 3
            ref[5] = B[t1] * vt[d] - B[d] * vt[t1]
            ref[6] = B[t2] * vt[d] - B[d] * vt[t2]
            np.testing.assert_allclose(F, ref, rtol=0, atol=1e-13 * (np.max(np.abs(ref)) + 1))


# ---------------------------------------------------------------- characteristic speeds


def _cs2(gam, rho, p):
    h = 1 + gam / (gam - 1) * p / rho
    return gam * p / (rho * h), rho * h


def test_speeds_unmagnetized_general_metric(orc):
    """B = 0: the GR hydro eigenvalues (Banyuls et al. 1997), a textbook closed form,
    lambda = alpha/(1 - v^2 cs^2) {v^i (1 - cs^2) +- cs sqrt[(1-v^2)(gamma^ii (1 - v^2 cs^2) - v^i v^i (1 - cs^2))]} - beta^i."""
    rng = np.random.default_rng(7)
    for _ in range(300):
        gam = rng.uniform(1.3, 2.0)
        m = random_metric(rng)
        pr = random_prim(rng, m, vmax=0.95)
        g = gmat(m)
        gi = np.linalg.inv(g)
        cs2, _ = _cs2(gam, pr[0], pr[1])
        v = pr[2:]
        v2 = v @ g @ v
        for d in range(3):
            root = np.sqrt((1 - v2) * (gi[d, d] * (1 - v2 * cs2) - v[d] ** 2 * (1 - cs2)))
            lp = m[0] / (1 - v2 * cs2) * (v[d] * (1 - cs2) + np.sqrt(cs2) * root) - m[1 + d]
            lm = m[0] / (1 - v2 * cs2) * (v[d] * (1 - cs2) - np.sqrt(cs2) * root) - m[1 + d]
            out = orc.pt_speeds(m, pr, np.zeros(3), gam, d)
            assert abs(out[1] - lp) <= 1e-12 * (1 + abs(lp)), (out, lp)
            assert abs(out[0] - lm) <= 1e-12 * (1 + abs(lm)), (out, lm)


def test_speeds_at_rest_magnetized(orc):
    """At rest, flat: B perpendicular to the direction gives lambda^2 = cs^2 + cA^2 - cs^2 cA^2;
    B parallel gives the larger of cs and cA (cA^2 = b^2/(rho h + b^2))."""
    rng = np.random.default_rng(8)
    m = random_metric(rng, curved=False)
    for _ in range(200):
        gam = rng.uniform(1.3, 2.0)
        pr = np.array([rng.uniform(0.1, 2), rng.uniform(0.05, 2), 0, 0, 0])
        cs2, rhoh = _cs2(gam, pr[0], pr[1])
        bmag = rng.uniform(0.05, 3.0)
        cA2 = bmag ** 2 / (rhoh + bmag ** 2)
        w2 = cs2 + cA2 - cs2 * cA2
        Bperp = np.array([0.0, bmag * np.cos(0.3), bmag * np.sin(0.3)])
        out = orc.pt_speeds(m, pr, Bperp, gam, 0)
        assert abs(out[1] - np.sqrt(w2)) <= 1e-12 and abs(out[0] + np.sqrt(w2)) <= 1e-12
        Bpar = np.array([bmag, 0.0, 0.0])
        out = orc.pt_speeds(m, pr, Bpar, gam, 0)
        fast = np.sqrt(max(cs2, cA2))
        # a double root when cs = cA converges only linearly: looser there
        tol = 1e-12 if abs(cs2 - cA2) > 1e-3 else 1e-7
        assert abs(out[1] - fast) <= tol and abs(out[0] + fast) <= tol, (out, fast, cs2, cA2)


def test_speeds_boost_velocity_addition(orc):
    """Flow and field both along x: lab speeds are the relativistic sums (v +- c)/(1 +- v c) of the
    rest-frame fast speed c = max(cs, cA)."""
    rng = np.random.default_rng(9)
    m = random_metric(rng, curved=False)
    for _ in range(200):
        gam = rng.uniform(1.3, 2.0)
        rho, p = rng.uniform(0.1, 2), rng.uniform(0.05, 2)
        vx = rng.uniform(-0.95, 0.95)
        cs2, rhoh = _cs2(gam, rho, p)
        bmag = rng.uniform(0.0, 3.0)
        # a boost along the field leaves it unchanged: comoving b^2 = B^2
        cA2 = bmag ** 2 / (rhoh + bmag ** 2)
        c = np.sqrt(max(cs2, cA2))
        if abs(cs2 - cA2) < 1e-3:
            continue
        out = orc.pt_speeds(m, [rho, p, vx, 0, 0], [bmag, 0, 0], gam, 0)
        assert abs(out[1] - (vx + c) / (1 + vx * c)) <= 1e-12
        assert abs(out[0] - (vx - c) / (1 - vx * c)) <= 1e-12


def _rot_to_x(k):
    """Rotation matrix R with R k_hat = e_x."""
    kh = k / np.linalg.norm(k)
    ex = np.array([1.0, 0, 0])
    vv = np.cross(kh, ex)
    s = np.linalg.norm(vv)
    c = kh @ ex
    if s < 1e-14:
        return np.eye(3) if c > 0 else np.diag([-1.0, -1.0, 1.0])
    vx = np.array([[0, -vv[2], vv[1]], [vv[2], 0, -vv[0]], [-vv[1], vv[0], 0]])
    return np.eye(3) + vx + vx @ vx * ((1 - c) / s ** 2)


def test_speeds_constant_metric_is_flat_space(orc):
    """A constant (alpha, beta, gamma) is flat space in other coordinates: with gamma' = M^T M,
    v' = M^-1 v, B' = M^-1 B, the speed along x'^d is alpha |k| lambda_flat(R v, R B) - beta^d,
    where k = M^-T e_d and R rotates k onto e_x (fast speeds along the front normal)."""
    rng = np.random.default_rng(10)
    flat = random_metric(rng, curved=False)
    for _ in range(200):
        gam = rng.uniform(1.3, 2.0)
        M = np.eye(3) + rng.uniform(-0.25, 0.25, (3, 3))
        g = M.T @ M
        alpha = rng.uniform(0.5, 1.5)
        beta = rng.uniform(-0.3, 0.3, 3)
        m = np.array([alpha, *beta, g[0, 0], g[0, 1], g[0, 2], g[1, 1], g[1, 2], g[2, 2]])
        rho, p = rng.uniform(0.1, 2), rng.uniform(0.05, 2)
        vc = rng.normal(size=3)
        vc *= rng.uniform(0, 0.9) / np.linalg.norm(vc)
        Bc = rng.uniform(-1.5, 1.5, 3)
        Mi = np.linalg.inv(M)
        vp, Bp = Mi @ vc, Mi @ Bc
        Btp = np.sqrt(np.linalg.det(g)) * Bp
        for d in range(3):
            k = Mi.T[:, d]
            R = _rot_to_x(k)
            ref = orc.pt_speeds(flat, [rho, p, *(R @ vc)], R @ Bc, gam, 0)
            out = orc.pt_speeds(m, [rho, p, *vp], Btp, gam, d)
            kn = np.linalg.norm(k)
            exp_p = alpha * kn * ref[1] - beta[d]
            exp_m = alpha * kn * ref[0] - beta[d]
            assert abs(out[1] - exp_p) <= 1e-10 and abs(out[0] - exp_m) <= 1e-10, (out, exp_p, exp_m)


def test_quartic_roots_match_polynomial_roots(orc):
    """The Newton outer roots equal the extreme real roots of the same quartic found by numpy.roots."""
    rng = np.random.default_rng(11)
    for _ in range(300):
        gam = rng.uniform(1.3, 2.0)
        m = random_metric(rng)
        pr = random_prim(rng, m, vmax=0.9)
        Bt = random_Bt(rng, m, 2.0)
        d = int(rng.integers(0, 3))
        out = orc.pt_speeds(m, pr, Bt, gam, d)
        xs = np.linspace(-1.0, 1.0, 5)
        q = orc.pt_quartic_eval(m, pr, Bt, gam, d, xs)
        coef = np.polyfit(xs, q, 4)
        r = np.roots(coef)
        rr = np.real(r[np.abs(np.imag(r)) < 1e-6 * (1 + np.abs(r))])
        assert rr.size >= 2
        assert abs(out[1] - rr.max()) <= 1e-7 and abs(out[0] - rr.min()) <= 1e-7, (out, r)
        # evaluation at the roots vanishes relative to the polynomial's scale
        qs = orc.pt_quartic_eval(m, pr, Bt, gam, d, out[:2])
        assert np.all(np.abs(qs) <= 1e-10 * np.max(np.abs(q)))


def test_bound_encloses_quartic(orc):
    """The isotropic bound w^2 = cs^2 + cA^2 - cs^2 cA^2 is never inside the fast speeds."""
    rng = np.random.default_rng(12)
    for _ in range(3000):
        gam = rng.uniform(1.1, 2.0)
        m = random_metric(rng)
        pr = random_prim(rng, m, vmax=0.99, rho=(1e-3, 10), p=(1e-3, 10), log=True)
        Bt = random_Bt(rng, m, 10 ** rng.uniform(-2, 1))
        d = int(rng.integers(0, 3))
        c = orc.pt_speeds(m, pr, Bt, gam, d)
        assert c[3] >= c[1] - 1e-12 * (1 + abs(c[1])) and c[2] <= c[0] + 1e-12 * (1 + abs(c[0])), c


# ---------------------------------------------------------------- HLLE


def test_hlle_consistency_and_upwinding(orc):
    """F(U, U) = F(U); c_min = 0 gives the left flux; c_max = 0 gives the right flux."""
    rng = np.random.default_rng(13)
    for _ in range(100):
        U, F = rng.normal(size=7), rng.normal(size=7)
        U2, F2 = rng.normal(size=7), rng.normal(size=7)
        np.testing.assert_allclose(orc.pt_hlle(U, F, -0.3, 0.5, U, F, -0.2, 0.7), F, rtol=1e-14, atol=1e-15)
        out = orc.pt_hlle(U, F, 0.1, 0.5, U2, F2, 0.2, 0.7)  # all speeds positive -> left flux
        np.testing.assert_allclose(out, F, rtol=1e-14, atol=1e-15)
        out = orc.pt_hlle(U, F, -0.5, -0.1, U2, F2, -0.7, -0.2)  # all negative -> right flux
        np.testing.assert_allclose(out, F2, rtol=1e-14, atol=1e-15)
        # generic case: the printed formula
        cmax, cmin = 0.7, 0.4
        ref = (cmin * F2 + cmax * F - cmax * cmin * (U2 - U)) / (cmax + cmin)
        np.testing.assert_allclose(orc.pt_hlle(U, F, -0.4, 0.7, U2, F2, -0.1, 0.2), ref, rtol=1e-13, atol=1e-14)


def test_lxf_consistency_and_relation_to_hlle(orc):
    """Lax-Friedrichs (eq. LxFfluxes): F(U, U) = F(U); with c_max = c_min it coincides with HLLE (both reduce to
    (F_l + F_r - c (U_r - U_l)) / 2); otherwise it uses the larger of the two speeds on both sides."""
    rng = np.random.default_rng(14)
    for _ in range(100):
        U, F = rng.normal(size=7), rng.normal(size=7)
        U2, F2 = rng.normal(size=7), rng.normal(size=7)
        np.testing.assert_allclose(orc.pt_lxf(U, F, -0.3, 0.5, U, F, -0.2, 0.7), F, rtol=1e-14, atol=1e-15)
        # symmetric speeds: c_max = max(0.4, 0.6) = 0.6 = c_min = -min(-0.6, -0.2)
        np.testing.assert_allclose(orc.pt_lxf(U, F, -0.6, 0.4, U2, F2, -0.2, 0.6),
                                   orc.pt_hlle(U, F, -0.6, 0.4, U2, F2, -0.2, 0.6), rtol=1e-13, atol=1e-14)
        # c_max = 0.7 > c_min = 0.1: the same as with symmetric speeds +-0.7
        np.testing.assert_allclose(orc.pt_lxf(U, F, -0.1, 0.7, U2, F2, 0.05, 0.2),
                                   orc.pt_hlle(U, F, -0.7, 0.7, U2, F2, -0.7, 0.7), rtol=1e-13, atol=1e-14)
        # supersonic flow: unlike HLLE, LxF does not reduce to the upwind flux
        assert np.max(np.abs(orc.pt_lxf(U, F, 0.1, 0.5, U2, F2, 0.2, 0.7) - F)) > 1e-3


def test_lxf_equals_hlle_for_resting_flat_states(orc):
    """Flat metric, v = 0 on both sides (different rho, p, B): the fast speeds are symmetric about zero on each
    side, so c_max = c_min and the LxF face flux equals the HLLE one."""
    rng = np.random.default_rng(15)
    m10 = np.array([1.0, 0, 0, 0, 1.0, 0, 0, 1.0, 0, 1.0])
    for _ in range(20):
        sides = []
        Bn = rng.uniform(-1, 1)
        for _s in range(2):
            prim = np.array([rng.uniform(0.1, 1.0), rng.uniform(0.1, 1.0), 0.0, 0.0, 0.0])
            Bt = np.array([Bn, rng.uniform(-1, 1), rng.uniform(-1, 1)])
            U, F = orc.pt_flux(m10, prim, Bt, 5.0 / 3.0, 0)
            cm, cp = orc.pt_speeds(m10, prim, Bt, 5.0 / 3.0, 0)[:2]
            sides.append((U, F, cm, cp))
        (UL, FL, cmL, cpL), (UR, FR, cmR, cpR) = sides
        np.testing.assert_allclose(cmL, -cpL, rtol=1e-13)
        np.testing.assert_allclose(orc.pt_lxf(UL, FL, cmL, cpL, UR, FR, cmR, cpR),
                                   orc.pt_hlle(UL, FL, cmL, cpL, UR, FR, cmR, cpR), rtol=1e-12, atol=1e-14)
