"""The HIP path on unmagnetized shock tubes: parity with the oracle after a whole run, and convergence to the
exact solution of the relativistic Riemann problem at resolutions the oracle would take minutes for (the
B = 0, flat-space special case of Sec. 2.2 in one dimension; exact solver in tests/exact_riemann.py).

Tolerance of the whole-run parity: 2e-9 on O(1) primitives after 280 steps through a shock, a contact and a
rarefaction.  Limiter decisions taken within rounding of their switching point may go either way on the two
sides, and the difference of one such decision is carried by the flow; MINMOD and MP5 stay within 1e-14,
PPM and WENO-Z (whose flattening and smoothness weights switch on more points) within 4e-10."""
import numpy as np
import pytest

from paper_2406_11669_amd import workloads as W
from tests.test_oracle_exact_riemann import (BLAST1, FRAMES, MODERATE, _oracle_tube, _oracle_tube_state,
                                             frame_exact, l1_errors, plateau_errors, tube_profile,
                                             transverse_errors, transverse_field)

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def ax():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_11669_amd import asterx
    asterx.lib()
    return asterx


def _gpu_tube(ax, w, with_state=False):
    import torch
    blk = ax.Block(w)
    blk.run(w.nsteps)
    torch.cuda.synchronize()
    out = (blk.prim.cpu().numpy(), blk.stats.cpu().numpy())
    return out + (blk.state.cpu().numpy(),) if with_state else out


@pytest.mark.parametrize("recon", ["minmod", "ppm", "wenoz", "mp5"])
def test_shock_tube_matches_oracle(ax, orc, recon):
    """The moderate tube at 200 cells to t = 0.35 (280 RK2 steps): primitives within 2e-9 of the oracle's, no
    recovery failure on either side."""
    w = W.shock_tube(*MODERATE, n=200, recon=recon, t_end=0.35)
    print("case shock tube 200", recon, flush=True)
    pg, st = _gpu_tube(ax, w)
    pc, stc, _ = _oracle_tube(orc, w)
    d = np.abs(w.layout.owned(pg) - w.layout.owned(pc)).reshape(5, -1).max(axis=1)
    print("  max |gpu - oracle| per primitive:", d)
    assert np.all(d <= 2e-9)
    assert st[3] == 0 and stc[3] == 0


def test_shock_tube_converges_to_exact(ax):
    """The moderate tube with PPM at 400, 800, 1600 and 3200 cells: the summed L1 error of (rho, p, v) falls by
    at least 1.6x per doubling (first order) and the middle states stay within 3e-4 of the exact ones."""
    prev = None
    for n in (400, 800, 1600, 3200):
        w = W.shock_tube(*MODERATE, n=n, recon="ppm", t_end=0.35)
        print("case shock tube", n, flush=True)
        pg, st = _gpu_tube(ax, w)
        assert st[3] == 0
        e, S, x, got = l1_errors(w, pg)
        pl = plateau_errors(S, x, got, 0.35)
        print("  L1", e, "middle states", pl)
        assert pl <= 3e-4
        if prev is not None:
            assert prev >= 1.6 * np.sum(e)
        prev = np.sum(e)


def test_blast_wave_converges_to_exact(ax):
    """The first blast wave (pressure ratio 1.3e7) with PPM at 1600 and 3200 cells: L1 falls by at least 1.6x,
    and at 3200 cells both middle states, the dense shell (146 cells wide) included, are within 4e-3."""
    scale = np.array([10.0, 40.0 / 3.0, 1.0])
    errs = []
    for n in (1600, 3200):
        w = W.shock_tube(*BLAST1, n=n, recon="ppm", t_end=0.4)
        print("case blast wave", n, flush=True)
        pg, st = _gpu_tube(ax, w)
        assert st[3] == 0
        e, S, x, got = l1_errors(w, pg)
        errs.append(np.sum(e / scale))
        print("  L1", e)
    assert errs[0] >= 1.6 * errs[1]
    assert plateau_errors(S, x, got, 0.4) <= 4e-3


@pytest.mark.parametrize("recon", ["ppm", "mp5"])
def test_normal_field_tube_matches_oracle(ax, orc, recon):
    """The moderate tube with a uniform field Bn = 1.5 along it (Alfven speed above the sound speed) at 200
    cells, 280 steps: primitives within 2e-9 of the oracle's."""
    w = W.shock_tube(*MODERATE, n=200, recon=recon, t_end=0.35, Bn=1.5)
    print("case normal-field tube 200", recon, flush=True)
    pg, st = _gpu_tube(ax, w)
    pc, stc, _ = _oracle_tube(orc, w)
    d = np.abs(w.layout.owned(pg) - w.layout.owned(pc)).reshape(5, -1).max(axis=1)
    print("  max |gpu - oracle| per primitive:", d)
    assert np.all(d <= 2e-9)
    assert st[3] == 0 and stc[3] == 0


def test_normal_field_tube_converges_to_exact(ax):
    """Bn = 1.5 along the moderate tube with PPM at 800, 1600 and 3200 cells: the field drops out of the flow,
    so the primitives converge to the hydrodynamic exact solution, at first order, with middle states
    within 5e-4."""
    prev = None
    for n in (800, 1600, 3200):
        w = W.shock_tube(*MODERATE, n=n, recon="ppm", t_end=0.35, Bn=1.5)
        print("case normal-field tube", n, flush=True)
        pg, st = _gpu_tube(ax, w)
        assert st[3] == 0
        e, S, x, got = l1_errors(w, pg)
        pl = plateau_errors(S, x, got, 0.35)
        print("  L1", e, "middle states", pl)
        assert pl <= 5e-4
        if prev is not None:
            assert prev >= 1.6 * np.sum(e)
        prev = np.sum(e)


@pytest.mark.parametrize("recon,ct", [("ppm", "fct"), ("mp5", "fct"), ("ppm", "uct")])
def test_transverse_field_tube_matches_oracle(ax, orc, recon, ct):
    """The moderate tube with a transverse field changing sign at the contact (1.0 | -0.3), 200 cells, 280
    steps (flux CT; upwind CT with PPM): primitives within 2e-9 of the oracle's, the field within 5e-9 (a difference quotient of the
    potential over dx = 1/200, so the potential's differences count 200-fold; 1.6e-9 measured with PPM)."""
    w = W.shock_tube(*MODERATE, n=200, recon=recon, t_end=0.35, Bt=(1.0, -0.3), ng=4 if ct == "uct" else 3)
    w.params["ct"] = ct
    print("case transverse-field tube 200", recon, ct, flush=True)
    pg, st, sg = _gpu_tube(ax, w, with_state=True)
    pc, sc, stc, _ = _oracle_tube_state(orc, w)
    d = np.abs(w.layout.owned(pg) - w.layout.owned(pc)).reshape(5, -1).max(axis=1)
    dB = np.max(np.abs(transverse_field(w, sg) - transverse_field(w, sc)))
    print("  max |gpu - oracle| per primitive:", d, "field:", dB)
    assert np.all(d <= 2e-9) and dB <= 5e-9
    assert st[3] == 0 and stc[3] == 0


@pytest.mark.parametrize("Bt", [(1.0, -0.3), (2.0, 0.1)])
def test_transverse_field_tube_converges_to_exact(ax, Bt):
    """Transverse-field tubes with PPM at 800, 1600 and 3200 cells: rho, p, v and B^t converge to the exact
    solution at first order (normalized L1 falls by at least 1.6x per doubling), with middle states within
    1e-3."""
    prev = None
    for n in (800, 1600, 3200):
        w = W.shock_tube(*MODERATE, n=n, recon="ppm", t_end=0.35, Bt=Bt)
        print("case transverse-field tube", Bt, n, flush=True)
        pg, st, sg = _gpu_tube(ax, w, with_state=True)
        assert st[3] == 0
        e, mid, scale = transverse_errors(w, pg, sg)
        print("  L1", e, "middle states", mid)
        assert np.all(mid <= 1e-3)
        if prev is not None:
            assert prev >= 1.6 * np.sum(e / scale)
        prev = np.sum(e / scale)


def test_moving_frame_tube_matches_oracle(ax, orc):
    """The moderate tube in the frame (lapse 0.8, shift 0.3, g_aa 1.44), PPM, 200 cells, 280 steps:
    primitives within 2e-9 of the oracle's."""
    w = W.shock_tube(*MODERATE, n=200, recon="ppm", t_end=0.35, frame=FRAMES[0])
    print("case moving-frame tube 200", flush=True)
    pg, st = _gpu_tube(ax, w)
    pc, stc, _ = _oracle_tube(orc, w)
    d = np.abs(w.layout.owned(pg) - w.layout.owned(pc)).reshape(5, -1).max(axis=1)
    print("  max |gpu - oracle| per primitive:", d)
    assert np.all(d <= 2e-9)
    assert st[3] == 0 and stc[3] == 0


@pytest.mark.parametrize("frame", FRAMES)
def test_moving_frame_tube_converges_to_exact(ax, frame):
    """Tubes in constant frames with PPM at 800, 1600 and 3200 cells: L1 falls by at least 1.6x per doubling
    against the exact solution carried over to the code's coordinates, and is below 1e-3 per primitive at
    3200 cells."""
    prev = None
    for n in (800, 1600, 3200):
        w = W.shock_tube(*MODERATE, n=n, recon="ppm", t_end=0.35, frame=frame)
        print("case moving-frame tube", frame, n, flush=True)
        pg, st = _gpu_tube(ax, w)
        assert st[3] == 0
        x, got = tube_profile(w, pg)
        ex, _ = frame_exact(w, x)
        e = np.mean(np.abs(got - ex), axis=1)
        print("  L1", e)
        if prev is not None:
            assert prev >= 1.6 * np.sum(e)
        prev = np.sum(e)
    assert np.all(e <= 1e-3)


def _gpu_alfven(ax, w):
    import torch
    blk = ax.Block(w)
    blk.run(w.nsteps)
    torch.cuda.synchronize()
    return blk.prim.cpu().numpy(), blk.state.cpu().numpy()


def test_alfven_wave_matches_oracle(ax, orc):
    """The Alfven-wave test of Sec. 4 (MINMOD, RK2, CFL 0.2) on 32 cells for one period (320 steps): state
    and primitives within 1e-10 of the oracle's."""
    from tests.test_oracle_grid import run_alfven
    w = W.alfven_wave(n=32)
    print("case alfven 32", flush=True)
    pg, sg = _gpu_alfven(ax, w)
    _, pc, sc = run_alfven(orc, 32)
    L = w.layout
    d = np.abs(L.owned(sg) - L.owned(sc)).reshape(9, -1).max(axis=1)
    dp = np.abs(L.owned(pg) - L.owned(pc)).reshape(5, -1).max(axis=1)
    print("  max |gpu - oracle| state", d, "primitives", dp)
    assert np.all(d <= 1e-10) and np.all(dp <= 1e-10)


@pytest.mark.parametrize("recon", ["minmod", "ppm"])
def test_alfven_wave_converges_to_exact(ax, orc, recon):
    """The Alfven wave for one period at 64, 128, 256 and 512 cells: the L2 errors of B^y and v^y against the
    exact wave fall at second order (order >= 1.75 per doubling)."""
    from tests.test_oracle_grid import alfven_errors
    prev = None
    for n in (64, 128, 256, 512):
        w = W.alfven_wave(n=n, recon=recon)
        print("case alfven", recon, n, flush=True)
        pg, sg = _gpu_alfven(ax, w)
        e = alfven_errors(orc, w, pg, sg)
        print("  L2 (B^y, v^y)", e)
        if prev is not None:
            assert np.log2(prev[0] / e[0]) >= 1.75 and np.log2(prev[1] / e[1]) >= 1.75
        prev = e


@pytest.mark.parametrize("recon,ct", [("minmod", "fct"), ("ppm", "uct")])
def test_loop_advection_matches_oracle(ax, orc, recon, ct):
    """The loop advection test of Sec. 4 on 32 x 32 cells to t = 0.3 (39 RK4 steps): state within 1e-10 of
    the oracle's (per field, against the field's largest value)."""
    from tests.parity import assert_fields_close
    from tests.test_oracle_loop import run_loop
    w = W.loop_advection(n=32, recon=recon, ng=4 if ct == "uct" else 3, t_end=0.3)
    w.params["ct"] = ct
    print("case loop 32", recon, ct, flush=True)
    pg, sg = _gpu_alfven(ax, w)
    _, sc, pc, stc, _ = run_loop(orc, 32, recon, ct)
    e = assert_fields_close(sg, sc, 1e-10, w.layout.owned)
    print("  max error per field", e)


@pytest.mark.parametrize("recon,ct", [("minmod", "fct"), ("ppm", "uct")])
def test_loop_advection_converges_to_exact(ax, recon, ct):
    """The loop to t = 1.2 at 64, 128, 256 and 512 cells per side: the L1 error of the face field against the
    translated loop falls by 1.45x or more per doubling, and the magnetic energy kept rises toward 1."""
    from tests.test_oracle_loop import loop_errors
    prev = None
    for n in (64, 128, 256, 512):
        w = W.loop_advection(n=n, recon=recon, ng=4 if ct == "uct" else 3, t_end=1.2)
        w.params["ct"] = ct
        print("case loop", recon, ct, n, flush=True)
        pg, sg = _gpu_alfven(ax, w)
        e, kept = loop_errors(w, sg[5:8])
        print("  L1 (B^x, B^y) / A_loop", e, "energy kept", kept)
        if prev is not None:
            assert np.all(prev[0] >= 1.45 * e) and prev[1] < kept < 1.0
        prev = (e, kept)
