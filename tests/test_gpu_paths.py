"""GPU parity of the paths and configurations that the basic parity tests leave idle: the 1-D Brent fallback of the
recovery (Sec. 3.5), the first-order fallback of unphysical face states, the algebraic gauge and the bounded
speeds, the 128^3 curved workload at full size (PPM and WENO-Z, a whole RK4 step), ten RK4 steps of a curved
block, and the batched patches in their stated mix of sides.

Tolerances as elsewhere: 1e-12 per stage, 1e-10 after several steps (cancellation-aware scale); flags and
counters bit-exact."""
import numpy as np
import pytest

from paper_2406_11669_amd import workloads as W
from tests.parity import assert_fields_close, cell_relative_errors, field_errors

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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    return t.detach().cpu().numpy()


# ---- the recovery's Brent fallback ---------------------------------------------------------------------------

@pytest.mark.parametrize("method,maxit,expect_flags", [(2, 50, 0), (0, 1, 3), (0, 2, 3), (1, 1, 13)])
def test_c2p_grid_fallback_paths(ax, orc, method, maxit, expect_flags):
    """Palenzuela's 1-D scheme with Brent's method deciding every cell: alone (method 2), behind a Noble iteration
    capped at one or two steps (method 0: flags noble-fail | fallback), and the capped Noble iteration alone
    (method 1: hard failure and atmosphere).  Flags and counters bit-exact, primitives within 1e-12."""
    import torch
    w = W.curved_block(seed=12, n=(70, 9, 7), recon="ppm", rho_atm=1e-6)
    L = w.layout
    P = dict(w.params, c2p_method=method, c2p_maxit=maxit)
    cons = orc.prim2con(L, P, w.metric, w.A, w.prim)
    guess = w.prim * (1.0 + np.random.default_rng(12).uniform(-0.02, 0.02, w.prim.shape))
    print("case c2p fallback method=%d maxit=%d" % (method, maxit), flush=True)
    c_ref, p_ref = cons.copy(), guess.copy()
    fl_ref, st_ref = orc.c2p(L, P, w.metric, w.A, c_ref, p_ref)
    assert np.all(L.owned(fl_ref) == expect_flags)
    c_g, p_g = _dev(cons), _dev(guess)
    flags = torch.zeros(L.shape3, dtype=torch.uint8, device="cuda")
    stats = torch.zeros(6, dtype=torch.int64, device="cuda")
    ax.c2p(L, P, _dev(w.metric), _dev(w.A), c_g, p_g, flags, stats)
    torch.cuda.synchronize()
    assert np.array_equal(L.owned(_host(flags)), L.owned(fl_ref))
    st = _host(stats).astype(np.uint64)
    assert np.array_equal(st, st_ref), (st, st_ref)
    assert_fields_close(_host(p_g), p_ref, 1e-12, L.owned, PRIM_NAMES)
    assert_fields_close(_host(c_g), c_ref, 1e-13, L.owned, PRIM_NAMES)


@pytest.mark.parametrize("method,maxit", [(2, 50), (0, 1)])
def test_c2p_points_fallback_paths(ax, orc, method, maxit):
    """The Brent fallback on 500 independent states of the learned guess's training ranges (W up to 10,
    magnetisation up to 10, p/rho down to 1e-3): flags equal the oracle's, primitives within 1e-12 of
    cancellation-aware scales (rho; p + tau, since p comes from the energy; velocities ~ 1)."""
    import torch
    from paper_2406_11669_amd import learned as Lr
    s = W.c2p_states(12, 500)
    d = Lr.device_states(s)
    cons, _ = Lr.conserved(d)
    P = dict(Lr.C2P_PARAMS, c2p_method=method, c2p_maxit=maxit)
    prim = torch.empty((5, 500), dtype=torch.float64, device="cuda")
    flags = torch.empty(500, dtype=torch.uint8, device="cuda")
    iters = torch.empty(500, dtype=torch.int32, device="cuda")
    print("case c2p points fallback method=%d maxit=%d" % (method, maxit), flush=True)
    ax.c2p_points(P, d["gam"], d["metric"], d["Bt"], cons, prim, flags=flags, iters=iters)
    torch.cuda.synchronize()
    c_host = cons.cpu().numpy()
    pg, fg = prim.cpu().numpy(), flags.cpu().numpy()
    nfb = 0
    for i in range(500):
        p = dict(P, gamma=float(s["gam"][i]))
        pr, fl, it, _ = orc.pt_c2p(p, s["metric"][:, i], c_host[:, i], s["Bt"][:, i], np.zeros(5))
        assert fl == fg[i], (i, fl, fg[i])
        if fl & 8:
            continue  # both sides reset to the atmosphere; compared through the flags
        nfb += 1
        sc = np.array([pr[0], pr[1] + abs(c_host[4, i]), 1.0, 1.0, 1.0])
        assert np.max(np.abs(pg[:, i] - pr) / sc) <= 1e-12, (i, pg[:, i], pr)
    assert nfb >= 450


# ---- unphysical face states, gauge and speed options -----------------------------------------------------------

def _rhs_both(ax, orc, w):
    import torch
    L = w.layout
    ref, red_ref, nfix = orc.rhs(L, w.params, w.metric, w.curv, w.prim, w.A, w.psi, w.dt)
    out = torch.zeros((9,) + L.shape3, dtype=torch.float64, device="cuda")
    red = torch.zeros(2, dtype=torch.float64, device="cuda")
    ws = torch.empty(ax.workspace_size(L) // 8, dtype=torch.float64, device="cuda")
    ax.rhs(L, w.params, _dev(w.metric), _dev(w.curv), _dev(w.prim), _dev(w.A), _dev(w.psi), w.dt, out, red, ws)
    torch.cuda.synchronize()
    return _host(out), ref, _host(red), red_ref, nfix


def _rough_pressure(w, pmin=1e-3, seed=2):
    """Every cell has its own pressure, log-uniform in [pmin, 1]: WENO-Z and MP5 (neither preserves positivity on
    such data) reconstruct p <= 0 at thousands of faces, with the smooth velocities of the workload (|v| <= 0.45)."""
    L = w.layout
    rng = np.random.default_rng(seed)
    w.prim[1] = 10.0 ** rng.uniform(np.log10(pmin), 0.0, L.shape3)
    return w


@pytest.mark.parametrize("recon", ["wenoz", "mp5"])
def test_rhs_parity_face_fallback_pressure(ax, orc, recon):
    """Faces whose reconstructed state is unphysical (here p <= 0) take the adjacent cell's values on that side
    (first order): the oracle takes that branch at many faces, and the GPU right-hand side agrees within 1e-12."""
    w = _rough_pressure(W.curved_block(seed=5, n=(40, 10, 9), recon=recon))
    print("case rhs face fallback (pressure)", recon, flush=True)
    g, c, red, red_ref, nfix = _rhs_both(ax, orc, w)
    assert nfix >= 100, nfix
    assert_fields_close(g, c, 1e-12, w.layout.owned, STATE_NAMES)
    assert abs(red[0] - red_ref[0]) <= 1e-12 * red_ref[0]


def _face_w2_max(orc, L, prim, params, recon):
    """Largest W^2 = 1/(1 - v^2) over the physical face states of a flat-metric block: each velocity component
    reconstructed along each direction by the oracle's 1-D reconstruction (both sides of every face)."""
    w2 = 1.0
    for d in range(3):
        comps = []
        for c in range(3):
            a = np.moveaxis(prim[2 + c], 2 - d, -1)
            lo, hi = np.full(a.shape, np.nan), np.full(a.shape, np.nan)
            for idx in np.ndindex(a.shape[:-1]):
                lo[idx], hi[idx] = orc.recon_1d(params, recon, np.ascontiguousarray(a[idx]))
            comps.append((lo, hi))
        for side in (0, 1):
            v2 = sum(comps[c][side] ** 2 for c in range(3))
            v2 = v2[np.isfinite(v2) & (v2 < 1.0)]
            w2 = max(w2, float(1.0 / (1.0 - v2.max())))
    return w2


@pytest.mark.parametrize("recon", ["minmod", "ppm"])
def test_rhs_parity_face_fallback_velocity(ax, orc, recon):
    """MINMOD and PPM keep every reconstructed component within its neighbours' range, so only v^2 >= 1 (the
    components reconstructed separately) triggers the fallback: flat space, every cell at speed 0.9 in its own random
    direction.  The physical face states then come arbitrarily close to v^2 = 1, where a few-ulp difference in v^2
    between the two implementations (FMA contraction and Newton-refined reciprocals on the GPU, correctly rounded
    operations in the oracle) is magnified by W^2 = 1/(1 - v^2) in the face fluxes: W changes by dv^2 W^2 / 2 in
    relative terms, and v^2 = sum v_i^2 of three reconstructed components, each up to two roundings apart, can
    differ by ~8 ulp.  The tolerance is max(1e-12, 32 eps W^2_max), eps = 2^-53 (8 ulp of v^2 times W^2 / 2, with a
    factor 4 for face fluxes above the right-hand side's scale), W^2_max measured over the face states of this
    block."""
    w = W.riemann_block(seed=5, n=(24, 10, 9), recon=recon)
    L = w.layout
    rng = np.random.default_rng(1)
    d = rng.normal(size=(3,) + L.shape3)
    d /= np.sqrt(np.sum(d * d, axis=0))
    w.prim[0], w.prim[1], w.prim[2:5] = 0.5, 0.5, 0.9 * d
    w2 = _face_w2_max(orc, L, w.prim, w.params, recon)
    tol = max(1e-12, 32.0 * 2.0 ** -53 * w2)
    print("case rhs face fallback (velocity)", recon, "W^2 max %.3g tol %.3g" % (w2, tol), flush=True)
    g, c, red, red_ref, nfix = _rhs_both(ax, orc, w)
    assert nfix >= 100, nfix
    e = assert_fields_close(g, c, tol, L.owned, STATE_NAMES)
    print("  max error %.3g" % e.max(), flush=True)


@pytest.mark.parametrize("opt", [dict(gauge="algebraic"), dict(speeds="bound"),
                                 dict(gauge="algebraic", speeds="bound", recon="wenoz")])
def test_rhs_and_steps_parity_options(ax, orc, opt):
    """The algebraic gauge (dA/dt = -E, no Psi evolution) and the quadratic bound on the characteristic speeds:
    one right-hand side within 1e-12 and two RK4 steps within 1e-10 of the oracle."""
    recon = opt.get("recon", "ppm")
    w = W.curved_block(seed=15, n=(13, 11, 9), recon=recon, nsteps=2)
    w.params.update({k: v for k, v in opt.items() if k != "recon"})
    w.psi = w.layout.zeros(1) + 0.01 * np.random.default_rng(3).normal(size=(1,) + w.layout.shape3)
    w.layout.periodic_wrap(w.psi)
    print("case options", opt, flush=True)
    g, c, red, red_ref, _ = _rhs_both(ax, orc, w)
    assert_fields_close(g, c, 1e-12, w.layout.owned, STATE_NAMES)
    assert abs(red[0] - red_ref[0]) <= 1e-12 * red_ref[0]
    blk, state, prim = _run_both(ax, orc, w, 2)
    assert_fields_close(_host(blk.state), state, 1e-10, w.layout.owned, STATE_NAMES)
    assert_fields_close(_host(blk.prim), prim, 1e-10, w.layout.owned, PRIM_NAMES)


# ---- whole steps -------------------------------------------------------------------------------------------

def _run_both(ax, orc, w, nsteps):
    import torch
    L = w.layout
    blk = ax.Block(w)
    blk.run(nsteps)
    torch.cuda.synchronize()
    cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
    orc.fill_ghosts(L, cons, w.bc_cell)
    state = w.state(cons)
    prim = w.prim.copy()
    orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, nsteps, w.rk, w.bc_cell, w.bc_A, A_shift=w.A_shift)
    return blk, state, prim


@pytest.mark.parametrize("recon", ["ppm", "wenoz"])
def test_curved32_ten_rk4_steps(ax, orc, recon):
    """Ten RK4 steps of a 32^3 periodic block in the curved static metric: state and primitives within 1e-10."""
    w = W.curved_block(seed=24, n=32, recon=recon, nsteps=10)
    print("case curved32 10 steps", recon, flush=True)
    blk, state, prim = _run_both(ax, orc, w, 10)
    e = assert_fields_close(_host(blk.state), state, 1e-10, w.layout.owned, STATE_NAMES)
    assert_fields_close(_host(blk.prim), prim, 1e-10, w.layout.owned, PRIM_NAMES)
    print("  max state error %.2e" % e.max(), flush=True)
    _check_cell_relative(_host(blk.state), state, w.layout.owned)


def _check_cell_relative(gpu, ref, owned):
    """Per-cell relative errors beside the normalised ones: asserted for the conserved density and energy (bounded
    away from zero in these workloads), printed for every field."""
    cr = cell_relative_errors(gpu, ref, owned)
    print("  per-cell relative (max, fraction of cells below 1e-6 of the field's max): " +
          ", ".join("%s %.1e (%.0e)" % (n, r, x) for n, (r, x) in zip(STATE_NAMES, cr)), flush=True)
    for f in (0, 4):
        assert cr[f][1] == 0.0 and cr[f][0] <= 1e-10, (STATE_NAMES[f], cr[f])


@pytest.mark.parametrize("recon", ["ppm", "mp5"])
def test_unmagnetized_curved_rk4_steps(ax, orc, recon):
    """B = 0 (A = 0): pure hydrodynamics in the curved metric -- the recovery without field terms, and the
    dispersion quartic whose inner roots collapse to the double root a^2 = 0 (only the outer, fast roots are
    sought).  Three RK4 steps of a 24 x 20 x 16 block: state and primitives within 1e-10 of the oracle; the
    potential and Psi stay exactly zero (E = 0 and no gauge source) and so does the div B maximum."""
    w = W.curved_block(seed=7, n=(24, 20, 16), recon=recon, nsteps=3)
    w.A[...] = 0.0
    print("case unmagnetized curved 3 RK4 steps", recon, flush=True)
    blk, state, prim = _run_both(ax, orc, w, 3)
    L = w.layout
    g = _host(blk.state)
    e = assert_fields_close(g, state, 1e-10, L.owned, STATE_NAMES)
    assert_fields_close(_host(blk.prim), prim, 1e-10, L.owned, PRIM_NAMES)
    assert np.all(L.owned(g)[5:9] == 0.0) and np.all(L.owned(state)[5:9] == 0.0)
    assert float(_host(blk.red)[1]) == 0.0
    print("  max state error %.2e" % e.max(), flush=True)
    _check_cell_relative(g, state, L.owned)


@pytest.mark.parametrize("recon", ["ppm", "wenoz"])
def test_full_size_curved128_rk4_steps(ax, orc, recon):
    """The 128^3 curved workload at full size, stepped as the benchmark steps it: c2p and the right-hand side of
    the first stage within 1e-12, and whole RK4 steps within 1e-10 at every owned cell: ten with PPM, five
    (the workload's own step count) with WENO-Z, whose oracle steps take twice as long (the oracle's steps on
    its OpenMP build, bitwise the serial one)."""
    import torch
    w = W.curved_block(seed=0, n=128, recon=recon, nsteps=1)
    L = w.layout
    print("case full-size 128 RK4 step", recon, flush=True)
    blk = ax.Block(w)
    blk.eval_rhs(blk.state, blk.k)
    torch.cuda.synchronize()
    k_gpu, p_gpu = _host(blk.k), _host(blk.prim)
    cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
    prim = w.prim.copy()
    orc.c2p(L, w.params, w.metric, w.A, cons, prim)
    orc.fill_ghosts(L, prim, w.bc_cell)
    assert_fields_close(p_gpu, prim, 1e-12, L.owned, PRIM_NAMES)
    orc.tie_counts()
    ref, red_ref, _ = orc.rhs(L, w.params, w.metric, w.curv, prim, w.A, w.psi, w.dt)
    dec, near = orc.tie_counts()
    e1 = assert_fields_close(k_gpu, ref, 1e-12, L.owned, STATE_NAMES)
    print("  first-stage right-hand side: max error %.2e; PPM constraint decisions %d, near ties %d" % (
        float(e1.max()), dec, near), flush=True)
    del ref, k_gpu
    nsteps = 10 if recon == "ppm" else 5
    step = ax.Block(w)
    step.run(nsteps)
    torch.cuda.synchronize()
    cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
    orc.fill_ghosts(L, cons, w.bc_cell)
    state = w.state(cons)
    prim = w.prim.copy()
    lib_omp, threads = orc.lib_omp()
    orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, nsteps, w.rk, w.bc_cell, w.bc_A, lib_=lib_omp)
    e = assert_fields_close(_host(step.state), state, 1e-10, L.owned, STATE_NAMES)
    assert_fields_close(_host(step.prim), prim, 1e-10, L.owned, PRIM_NAMES)
    print("  %d RK4 steps (oracle on %d threads): max state error %.2e" % (nsteps, threads, e.max()), flush=True)
    _check_cell_relative(_host(step.state), state, L.owned)


# ---- batched patches in the stated mix ----------------------------------------------------------------------

def _batch_vs_loop_and_oracle(ax, orc, wls, nsteps, tuning, sampled, lib_=None):
    import torch
    bt = ax.Batch(wls, tuning=tuning)
    bt.run(nsteps)
    # the per-patch launch loop runs the batch's kernel bodies (sources in the cell kernel)
    blocks = [ax.Block(w, src_in_c2p=False) for w in wls]
    for _ in range(nsteps):
        for b in blocks:
            b.step()
    torch.cuda.synchronize()
    for p, b in enumerate(blocks):
        assert torch.equal(bt.unpack(bt.state, p), b.state), p
        assert torch.equal(bt.unpack(bt.prim, p), b.prim), p
    worst = 0.0
    for p in sampled:
        w = wls[p]
        L = w.layout
        cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
        orc.fill_ghosts(L, cons, w.bc_cell)
        state = w.state(cons)
        prim = w.prim.copy()
        orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, nsteps, w.rk, w.bc_cell, w.bc_A, lib_=lib_)
        e = assert_fields_close(bt.unpack(bt.state, p).cpu().numpy(), state, 1e-10, L.owned, STATE_NAMES)
        worst = max(worst, float(e.max()))
    return worst


def _sample_by_side(wls, per_side):
    by = {}
    for q, w in enumerate(wls):
        by.setdefault(w.layout.n[0], []).append(q)
    return by, [q for s in sorted(by) for q in by[s][:per_side]]


def test_batch_stated_mix_ten_steps(ax, orc):
    """32 patches drawn from sides {16, 24, 32, 48} on 3 levels (every side present), MINMOD, RK2, 10 steps:
    the persistent batch equals the per-patch launch loop bit for bit, and two sampled patches of each side
    match the oracle within 1e-10."""
    wls = W.patch_set(seed=8, npatches=32, sides=(16, 24, 32, 48), levels=3, nsteps=10)
    by, sampled = _sample_by_side(wls, 2)
    assert sorted(by) == [16, 24, 32, 48]
    print("case batch stated mix", {s: len(v) for s, v in by.items()}, flush=True)
    worst = _batch_vs_loop_and_oracle(ax, orc, wls, 10, (4, 1), sampled)
    print("  sampled patches max error %.2e" % worst, flush=True)


def test_batch_stated_configuration_512_patches(ax, orc):
    """The batched workload as stated: 512 patches of sides drawn from {16, 24, 32, 48} on 3 levels, MINMOD,
    HLLE, RK2, 10 steps, autotuned schedule of the benchmark (8 workgroups per CU, order as given): the
    persistent batch equals the per-patch launch loop bit for bit on every patch, and 32 sampled patches
    (8 of each side) match the oracle (its OpenMP build, bitwise the serial one) within 1e-10."""
    wls = W.patch_set(seed=0, npatches=512, sides=(16, 24, 32, 48), levels=3, nsteps=10)
    by, sampled = _sample_by_side(wls, 8)
    assert sorted(by) == [16, 24, 32, 48] and len(sampled) == 32
    print("case batch stated configuration", {s: len(v) for s, v in by.items()}, flush=True)
    lib_omp, threads = orc.lib_omp()
    worst = _batch_vs_loop_and_oracle(ax, orc, wls, 10, (8, 0), sampled, lib_=lib_omp)
    print("  32 sampled patches (oracle on %d threads) max error %.2e" % (threads, worst), flush=True)


@pytest.mark.parametrize("recon", ["ppm", "wenoz"])
def test_batch_wide_patches_one_workgroup_per_cu(ax, orc, recon):
    """Patches of sides 32 and 48 (face rows 32 wide and wider: the wavefront-row metric path and the x-face
    remainder tiles), one workgroup per CU so that each walks many items across patches: bit for bit equal to the
    per-patch loop, and one patch of each side within 1e-10 of the oracle."""
    wls = W.patch_set(seed=9, npatches=6, sides=(32, 48), levels=2, nsteps=2, recon=recon)
    by, sampled = _sample_by_side(wls, 1)
    assert sorted(by) == [32, 48]
    print("case batch wide patches", recon, flush=True)
    _batch_vs_loop_and_oracle(ax, orc, wls, 2, (1, 0), sampled)
