"""Pins of the oracle's conservative-to-primitive recovery (Sec. 3.5) and atmosphere (Sec. 3.6)."""
import numpy as np
import pytest

from paper_2406_11669_amd.workloads import default_params
from tests.states import gmat, random_Bt, random_metric, random_prim

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _truth(m, pr, Bt, gam):
    g = gmat(m)
    v = pr[2:]
    v2 = v @ g @ v
    W = 1 / np.sqrt(1 - v2)
    h = 1 + gam / (gam - 1) * pr[1] / pr[0]
    return pr[0] * h * W * W, v2


def test_noble_residuals_vanish_at_true_state(orc):
    """Both equations (Noble2D momentum, Noble2D energy) hold at z = rho h W^2, w = v^2 of the state that
    generated the conserved variables."""
    rng = np.random.default_rng(20)
    for _ in range(200):
        gam = rng.uniform(1.3, 2.0)
        m = random_metric(rng)
        pr = random_prim(rng, m, vmax=0.95)
        Bt = random_Bt(rng, m, 2.0)
        cons = orc.pt_prim2con(m, pr, Bt, gam)
        z, w = _truth(m, pr, Bt, gam)
        R, J = orc.pt_noble_residual(m, cons, Bt, gam, z, w)
        sg = np.sqrt(np.linalg.det(gmat(m)))
        B2 = (Bt / sg) @ gmat(m) @ (Bt / sg)
        assert abs(R[0]) <= 1e-12 * (B2 + z) ** 2
        assert abs(R[1]) <= 1e-12 * (z + B2 + cons[4] / sg + cons[0] / sg)


def test_noble_jacobian_matches_finite_differences(orc):
    rng = np.random.default_rng(21)
    for _ in range(100):
        gam = rng.uniform(1.3, 2.0)
        m = random_metric(rng)
        pr = random_prim(rng, m, vmax=0.9)
        Bt = random_Bt(rng, m, 2.0)
        cons = orc.pt_prim2con(m, pr, Bt, gam)
        z, w = _truth(m, pr, Bt, gam)
        z *= rng.uniform(0.8, 1.2)
        w *= rng.uniform(0.8, 1.0)
        _, J = orc.pt_noble_residual(m, cons, Bt, gam, z, w)
        hz, hw = 1e-6 * z, 1e-7
        Rzp, _ = orc.pt_noble_residual(m, cons, Bt, gam, z + hz, w)
        Rzm, _ = orc.pt_noble_residual(m, cons, Bt, gam, z - hz, w)
        Rwp, _ = orc.pt_noble_residual(m, cons, Bt, gam, z, w + hw)
        Rwm, _ = orc.pt_noble_residual(m, cons, Bt, gam, z, w - hw)
        Jfd = np.stack([(Rzp - Rzm) / (2 * hz), (Rwp - Rwm) / (2 * hw)], axis=1)
        np.testing.assert_allclose(J, Jfd, rtol=1e-5, atol=1e-6 * np.max(np.abs(J)))


@pytest.mark.parametrize("gam", [5.0 / 3.0, 2.0])
@pytest.mark.parametrize("warm", [True, False])
def test_round_trip_workload_ranges(orc, gam, warm):
    """prim -> cons -> prim to 1e-12 relative over the state ranges of the benchmark workloads
    (rho in [0.1, 1.5], p in [0.1, 1], |v| <= 0.45, |B| <= 1.8), warm and cold started."""
    rng = np.random.default_rng(22 if warm else 23)
    P = default_params(gamma=gam)
    for _ in range(500):
        m = random_metric(rng, amp=0.1)
        pr = random_prim(rng, m, vmax=0.45, rho=(0.1, 1.5), p=(0.1, 1.0))
        Bt = random_Bt(rng, m, 1.0)
        cons = orc.pt_prim2con(m, pr, Bt, gam)
        if warm:
            prev = pr * (1 + rng.uniform(-0.05, 0.05, 5))
        else:
            prev = np.zeros(5)  # unusable: cold start
        out, fl, it, _ = orc.pt_c2p(P, m, cons, Bt, prev)
        assert fl == 0, fl
        vmag = np.sqrt(pr[2:] @ gmat(m) @ pr[2:])
        assert abs(out[0] - pr[0]) <= 1e-12 * pr[0]
        assert abs(out[1] - pr[1]) <= 1e-12 * pr[1]
        assert np.max(np.abs(out[2:] - pr[2:])) <= 1e-12 * max(vmag, 1e-3)


def test_round_trip_wide_range_report(orc):
    """Over a wide range (W up to 10, sigma up to 10, p/rho down to 1e-3) the round trip is limited by the
    cancellation tau ~ p; the error must stay below 1e-12 times the condition estimate (tau + D)/p."""
    rng = np.random.default_rng(24)
    P = default_params(gamma=4.0 / 3.0)
    worst = 0.0
    for _ in range(300):
        m = random_metric(rng, amp=0.1)
        W = rng.uniform(1, 10)
        vmag = np.sqrt(1 - 1 / W ** 2)
        rho = 10 ** rng.uniform(-8, 0)
        p = rho * 10 ** rng.uniform(-3, 1)
        g = gmat(m)
        d = rng.normal(size=3)
        v = d / np.sqrt(d @ g @ d) * vmag
        pr = np.array([rho, p, *v])
        Bt = random_Bt(rng, m, np.sqrt(rho) * 10 ** rng.uniform(-1.5, 0.5))
        cons = orc.pt_prim2con(m, pr, Bt, P["gamma"])
        out, fl, it, _ = orc.pt_c2p(dict(P, rho_atm=1e-30), m, cons, Bt, pr * 1.01)
        if fl & 8:
            continue
        cond = (cons[4] + cons[0]) / (np.sqrt(np.linalg.det(g)) * p)
        err = abs(out[1] - p) / p / max(cond, 1.0)
        worst = max(worst, err)
    assert worst <= 1e-11, worst


def test_c2p_special_cases(orc):
    """v = 0 gives S = 0 and a recovered velocity of exactly 0; B = 0 gives the pure-hydro inversion;
    Noble and Palenzuela agree where both converge; the true x = h W lies inside the printed bracket."""
    rng = np.random.default_rng(25)
    P = default_params(gamma=5.0 / 3.0)
    for _ in range(200):
        m = random_metric(rng)
        pr = random_prim(rng, m, vmax=0.9)
        Bt = random_Bt(rng, m, 1.5)
        # v = 0
        p0 = pr.copy()
        p0[2:] = 0
        cons = orc.pt_prim2con(m, p0, Bt, P["gamma"])
        assert np.all(cons[1:4] == 0)
        out, fl, _, _ = orc.pt_c2p(P, m, cons, Bt, p0 * 1.02)
        assert fl == 0 and np.all(out[2:] == 0.0)
        # Noble only vs Palenzuela only
        cons = orc.pt_prim2con(m, pr, Bt, P["gamma"])
        a, fa, _, _ = orc.pt_c2p(dict(P, c2p_method=1), m, cons, Bt, pr * 1.01)
        b, fb, _, _ = orc.pt_c2p(dict(P, c2p_method=2), m, cons, Bt, np.zeros(5))
        assert fa == 0 and fb == 0, (fa, fb)
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.max(np.abs(pr)))
        # bracket
        g = gmat(m)
        W = 1 / np.sqrt(1 - pr[2:] @ g @ pr[2:])
        h = 1 + P["gamma"] / (P["gamma"] - 1) * pr[1] / pr[0]
        f, br = orc.pt_palen(m, cons, Bt, P["gamma"], P["wmax"], [h * W])
        assert br[0] < h * W < br[1]
        assert abs(f[0]) <= 1e-12 * h * W  # the master function vanishes at the true x
        # B = 0
        cons = orc.pt_prim2con(m, pr, np.zeros(3), P["gamma"])
        out, fl, _, _ = orc.pt_c2p(P, m, cons, np.zeros(3), pr * 0.98)
        assert fl == 0
        np.testing.assert_allclose(out, pr, rtol=1e-12, atol=1e-12)


def test_atmosphere_reset(orc):
    """D < sqrt(gamma) rho_atm: rho = rho_atm, p = K rho_atm^Gamma, v = 0, conserved variables recomputed from
    these primitives with the field kept -- bitwise what prim -> cons gives for that state (Sec. 3.6)."""
    rng = np.random.default_rng(26)
    P = default_params(gamma=2.0, rho_atm=1e-6, k_atm=1.0)
    for _ in range(50):
        m = random_metric(rng)
        pr = random_prim(rng, m, vmax=0.5, rho=(1e-9, 5e-7), p=(1e-12, 1e-9))
        Bt = random_Bt(rng, m, 1e-3)
        cons = orc.pt_prim2con(m, pr, Bt, P["gamma"])
        out, fl, _, cons_after = orc.pt_c2p(P, m, cons, Bt, pr)
        assert fl & 4
        atm = np.array([1e-6, 1e-12, 0, 0, 0])
        assert np.all(out == atm)
        assert np.all(cons_after == orc.pt_prim2con(m, atm, Bt, P["gamma"]))


def test_failure_injection(orc):
    """Corrupted conserved states take the documented paths: NaN -> atmosphere with the NaN flag; a state with
    S^2 > (tau + D)^2 (no physical solution) -> both solvers fail -> atmosphere with the hard-fail flag."""
    rng = np.random.default_rng(27)
    P = default_params(gamma=5.0 / 3.0, rho_atm=1e-8)
    m = random_metric(rng)
    pr = random_prim(rng, m, vmax=0.4)
    Bt = random_Bt(rng, m, 0.5)
    cons = orc.pt_prim2con(m, pr, Bt, P["gamma"])
    bad = cons.copy()
    bad[2] = np.nan
    out, fl, _, after = orc.pt_c2p(P, m, bad, Bt, pr)
    assert fl & 16 and fl & 4 and np.all(np.isfinite(out)) and np.all(np.isfinite(after))
    bad = cons.copy()
    bad[1:4] *= 50.0  # momentum far beyond the energy
    out, fl, _, after = orc.pt_c2p(P, m, bad, Bt, pr)
    assert fl & 8 and fl & 4 and fl & 1, fl
    assert out[0] == 1e-8 and np.all(out[2:] == 0)
    bad = cons.copy()
    bad[4] = -abs(bad[4])  # negative energy
    out, fl, _, after = orc.pt_c2p(P, m, bad, Bt, pr)
    assert fl & 4 and np.all(np.isfinite(out))


@pytest.mark.parametrize("gam", [4.0 / 3.0, 5.0 / 3.0, 2.0])
def test_no_solution_bound(orc, gam):
    """Without a field and with Gamma <= 2, E^2 - S^2 - D^2 = W^2 rho^2 (2 eps + eps^2 (1 - (Gamma-1)^2)) + p^2 > 0
    for every physical state (checked here on sampled ones, nearly cold included), so S^2 < tau (tau + 2D) and
    tau > 0; beyond that bound the recovery takes the failure branch (atmosphere, Noble-failed and hard-fail
    flags), and just inside it the nearly cold states still recover to 1e-9."""
    rng = np.random.default_rng(31)
    P = default_params(gamma=gam, rho_atm=1e-12)
    zero = np.zeros(3)
    for _ in range(200):
        m = random_metric(rng)
        g = gmat(m)
        sq = np.sqrt(np.linalg.det(g))
        pr = random_prim(rng, m, vmax=0.95, rho=(1e-3, 1.0), p=(1e-9, 1e-1), log=True)
        cons = orc.pt_prim2con(m, pr, zero, gam) / sq
        D, S, tau = cons[0], cons[1:4], cons[4]
        S2 = S @ np.linalg.inv(g) @ S
        assert tau > 0 and S2 < tau * (tau + 2 * D)
        out, fl, _, _ = orc.pt_c2p(P, m, cons * sq, zero, pr)
        assert not fl & 8
        assert np.allclose(out, pr, rtol=1e-9, atol=1e-12)
        bad = cons.copy()
        bad[1:4] *= np.sqrt(tau * (tau + 2 * D) / S2) * rng.uniform(1.0 + 1e-8, 3.0) if S2 > 0 else 1.0
        out, fl, _, after = orc.pt_c2p(P, m, bad * sq, zero, pr)
        if S2 > 0:
            assert fl & 8 and fl & 4 and fl & 1, fl
            assert out[0] == P["rho_atm"] and np.all(out[2:] == 0)
