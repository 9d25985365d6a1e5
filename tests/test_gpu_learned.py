"""GPU: point prim->cons and c2p against the CPU oracle, the network's forward and backward kernels against the
CPU reference network (oracle/mlp_ref.py), one Adam step, and what a briefly trained network gains over the
plain start of the recovery on held-out states."""
import numpy as np
import pytest

from paper_2406_11669_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_11669_amd import asterx, learned
    asterx.lib()
    return learned


def _stdz(rng):
    return dict(in_shift=rng.normal(size=8) * 0.3, in_scale=rng.uniform(0.5, 2.0, 8),
                out_shift=rng.normal(size=2), out_scale=rng.uniform(0.5, 2.0, 2))


def test_prim2con_points_vs_oracle(L, orc):
    import torch
    s = W.c2p_states(11, 777)
    d = L.device_states(s)
    cons, tgt = L.conserved(d, with_targets=True)
    torch.cuda.synchronize()
    c = cons.cpu().numpy()
    for i in range(0, 777, 5):
        ref = orc.pt_prim2con(s["metric"][:, i], s["prim"][:, i], s["Bt"][:, i], s["gam"][i])
        assert np.max(np.abs(c[:, i] - ref)) <= 1e-13 * np.max(np.abs(ref)), i
        f = orc.pt_fluid(s["metric"][:, i], s["prim"][:, i], s["Bt"][:, i], s["gam"][i])
        t = tgt[:, i].cpu().numpy()
        assert abs(t[0] - np.log(f["W"])) <= 1e-13 and abs(t[1] - np.log(f["h"] * f["W"])) <= 1e-12


@pytest.mark.parametrize("warm", [False, True])
def test_c2p_points_vs_oracle(L, orc, warm):
    """Plain point c2p (cold or warm start) against the oracle's: flags and iteration counts equal, primitives
    within 1e-12 relative (the training ranges reach W = 10 and sigma = 10)."""
    import torch
    from paper_2406_11669_amd import asterx as ax
    s = W.c2p_states(12, 500)
    d = L.device_states(s)
    cons, _ = L.conserved(d)
    rng = np.random.default_rng(3)
    guess = s["prim"] * (1.0 + 1e-3 * rng.uniform(-1, 1, s["prim"].shape)) if warm else np.zeros_like(s["prim"])
    prim = torch.empty((5, 500), dtype=torch.float64, device="cuda")
    flags = torch.empty(500, dtype=torch.uint8, device="cuda")
    iters = torch.empty(500, dtype=torch.int32, device="cuda")
    c_host = cons.cpu().numpy()
    ax.c2p_points(L.C2P_PARAMS, d["gam"], d["metric"], d["Bt"], cons, prim,
                  guess=L._dev(guess) if warm else None, flags=flags, iters=iters)
    torch.cuda.synchronize()
    pg, fg, ig = prim.cpu().numpy(), flags.cpu().numpy(), iters.cpu().numpy()
    for i in range(500):
        p = dict(L.C2P_PARAMS, gamma=float(s["gam"][i]))
        pr, fl, it, _ = orc.pt_c2p(p, s["metric"][:, i], c_host[:, i], s["Bt"][:, i], guess[:, i])
        # flags equal; the Newton stopping test may fall one iteration apart at the tolerance boundary
        assert fl == fg[i] and abs(it - ig[i]) <= 1, (i, fl, fg[i], it, ig[i])
        # cancellation-aware scales: rho, p + tau (p is recovered from the energy), velocities ~ 1
        sc = np.array([pr[0], pr[1] + abs(c_host[4, i]), 1.0, 1.0, 1.0])
        assert np.max(np.abs(pg[:, i] - pr) / sc) <= 1e-12, (i, pg[:, i], pr)


def _net(L, seed):
    import torch
    from oracle import mlp_ref as M
    rng = np.random.default_rng(seed)
    p = M.init_params(seed)
    p[512:576] = rng.normal(size=64) * 0.2      # non-zero biases exercise the bias paths
    p[4672:4736] = rng.normal(size=64) * 0.2
    p[4864:4866] = rng.normal(size=2) * 0.2
    return p, torch.from_numpy(p).cuda(), _stdz(rng)


def test_mlp_forward_vs_reference(L):
    """Forward on the matrix cores against the reference network with the same bfloat16 roundings (ragged n)."""
    import torch
    from oracle import mlp_ref as M
    from paper_2406_11669_amd import asterx as ax
    p, pt, st = _net(L, 5)
    rng = np.random.default_rng(6)
    n = 1000
    feat = rng.normal(size=(8, n)).astype(np.float32)
    out = torch.empty((2, n), dtype=torch.float32, device="cuda")
    ax.mlp_forward(ax.make_mlp(pt, st), torch.from_numpy(feat).cuda(), out)
    torch.cuda.synchronize()
    ref, _ = M.forward(p, feat, {k: np.asarray(v, np.float32) for k, v in st.items()})
    g = out.cpu().numpy()
    err = np.abs(g - ref)
    scale = np.max(np.abs(ref))
    # bfloat16 operands: one rounding decided differently (FP32 accumulation order) moves an output by at most a
    # few parts in 1e3 of one term; most outputs agree to FP32 rounding
    assert np.max(err) <= 2e-3 * scale, np.max(err)
    assert np.median(err) <= 1e-5 * scale, np.median(err)


def test_mlp_gradient_vs_reference(L):
    import torch
    from oracle import mlp_ref as M
    from paper_2406_11669_amd import asterx as ax
    p, pt, st = _net(L, 7)
    rng = np.random.default_rng(8)
    n = 999
    feat = rng.normal(size=(8, n)).astype(np.float32)
    tgt = rng.normal(size=(2, n)).astype(np.float32)
    grad = torch.empty(ax.MLP_NPARAMS + 1, dtype=torch.float32, device="cuda")
    ws = torch.empty(ax.mlp_grad_workspace_size(n) // 4 + 1, dtype=torch.float32, device="cuda")
    ax.mlp_grad(ax.make_mlp(pt, st), torch.from_numpy(feat).cuda(), torch.from_numpy(tgt).cuda(), grad, ws)
    torch.cuda.synchronize()
    g = grad.cpu().numpy()
    loss, gref = M.loss_grad(p, feat, tgt, {k: np.asarray(v, np.float32) for k, v in st.items()})
    assert abs(g[-1] - loss) <= 1e-4 * loss
    sl = {"W1": slice(0, 512), "b1": slice(512, 576), "W2": slice(576, 4672), "b2": slice(4672, 4736),
          "W3": slice(4736, 4864), "b3": slice(4864, 4866)}
    for name, s in sl.items():
        a, b = g[:-1][s], gref[s]
        scale = np.max(np.abs(b))
        print("  %s: max err %.3e  median err %.3e  scale %.3e" % (name, np.max(np.abs(a - b)),
                                                                  np.median(np.abs(a - b)), scale), flush=True)
        assert np.max(np.abs(a - b)) <= 2e-2 * scale, name
        assert np.median(np.abs(a - b)) <= 2e-3 * scale, name
    # deterministic: a second evaluation is bitwise identical
    grad2 = torch.empty_like(grad)
    ax.mlp_grad(ax.make_mlp(pt, st), torch.from_numpy(feat).cuda(), torch.from_numpy(tgt).cuda(), grad2, ws)
    assert torch.equal(grad, grad2)


def test_network_exact_on_dyadic_network(L):
    """On a network whose every rounded value is exactly representable (tests/mlp_exact.py: small dyadic weights,
    inputs and targets, 1024 samples), the matrix-core forward and gradient equal the plain float64 network bit
    for bit -- a pin that does not restate the kernel's rounding points.  Forward and gradient kernels both."""
    import torch
    from oracle import mlp_ref as M
    from paper_2406_11669_amd import asterx as ax
    from tests import mlp_exact as X
    p, st, feat, off = X.network(3)
    n = feat.shape[1]
    pt = torch.from_numpy(p).cuda()
    mlp = ax.make_mlp(pt, st)
    out = torch.empty((2, n), dtype=torch.float32, device="cuda")
    ax.mlp_forward(mlp, torch.from_numpy(feat).cuda(), out)
    ref, _ = M.forward(p, feat, st, precise=True)
    tgt = (ref - off).astype(np.float32)
    grad = torch.empty(ax.MLP_NPARAMS + 1, dtype=torch.float32, device="cuda")
    ws = torch.empty(ax.mlp_grad_workspace_size(n) // 4 + 1, dtype=torch.float32, device="cuda")
    ax.mlp_grad(mlp, torch.from_numpy(feat).cuda(), torch.from_numpy(tgt).cuda(), grad, ws)
    torch.cuda.synchronize()
    loss, gref = M.loss_grad(p, feat, tgt, st, precise=True)
    g = grad.cpu().numpy().astype(np.float64)
    print("  forward mismatches %d of %d, gradient mismatches %d of %d, loss %.9g vs %.9g" % (
        int(np.sum(out.cpu().numpy().astype(np.float64) != ref)), ref.size, int(np.sum(g[:-1] != gref)), gref.size,
        g[-1], loss), flush=True)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)
    assert np.array_equal(g[:-1], np.asarray(gref, np.float64)) and g[-1] == loss


def test_adam_step_vs_reference(L):
    import torch
    from oracle import mlp_ref as M
    from paper_2406_11669_amd import asterx as ax
    rng = np.random.default_rng(9)
    p = rng.normal(size=ax.MLP_NPARAMS).astype(np.float32)
    g = rng.normal(size=ax.MLP_NPARAMS + 1).astype(np.float32)
    m = rng.normal(size=ax.MLP_NPARAMS).astype(np.float32) * 0.1
    v = np.abs(rng.normal(size=ax.MLP_NPARAMS)).astype(np.float32) * 0.1
    pt, gt, mt, vt = (torch.from_numpy(x.copy()).cuda() for x in (p, g, m, v))
    ax.mlp_adam(pt, gt, mt, vt, 1e-3, 0.9, 0.999, 1e-8, 3)
    torch.cuda.synchronize()
    pr, mr, vr = M.adam(p, g[:-1], m, v, 1e-3, 0.9, 0.999, 1e-8, 3)
    assert np.allclose(pt.cpu().numpy(), pr, rtol=1e-6, atol=1e-7)
    assert np.allclose(mt.cpu().numpy(), mr, rtol=1e-6, atol=1e-8)


@pytest.fixture(scope="module")
def trained(L):
    """A network trained briefly (2e6 states, 10 epochs) by the library's own kernels."""
    import torch
    from paper_2406_11669_amd import asterx as ax
    feat, tgt = L.training_set(2_000_000, seed=21)
    st = L.standardization(feat, tgt)
    # loss of the untrained network (same seeded initial parameters) on the first batch of states
    grad = torch.zeros(ax.MLP_NPARAMS + 1, dtype=torch.float32, device="cuda")
    ws = torch.empty(ax.mlp_grad_workspace_size(16384) // 4 + 1, dtype=torch.float32, device="cuda")
    mlp0 = ax.make_mlp(torch.from_numpy(L.init_params(3)).cuda(), st)
    ax.mlp_grad(mlp0, feat[:, :16384].contiguous(), tgt[:, :16384].contiguous(), grad, ws)
    loss0 = float(grad[ax.MLP_NPARAMS].item())
    params, losses = L.train(feat, tgt, st, epochs=10, batch=16384, seed=3)
    return params, st, [loss0] + losses


def test_trained_guess_cuts_newton_iterations(L, trained):
    """The trained network seeds Noble's iteration on held-out states: every state is recovered, to the same
    primitives as the plain cold start, in fewer iterations on average."""
    import torch
    from paper_2406_11669_amd import asterx as ax
    params, st, losses = trained
    print("untrained loss %.4g, epoch losses %s" % (losses[0], ["%.4g" % x for x in losses[1:]]), flush=True)
    assert losses[-1] < 0.5 * losses[0], losses
    mlp = ax.make_mlp(params, st)
    d = L.device_states(W.c2p_states(22, 20_000))
    res = L.evaluate(d, mlp, seed=1)
    print(res, flush=True)
    cold, learned = res["cold"], res["learned"]
    assert cold["hard_fail_frac"] == 0.0 and learned["hard_fail_frac"] == 0.0
    assert learned["iters_mean"] < cold["iters_mean"]
    assert learned["rho_rel_diff_vs_cold_max"] <= 1e-12 and learned["p_diff_vs_cold_max"] <= 1e-12


@pytest.mark.parametrize("cold_planes", [0, 3])
def test_grid_c2p_learned_matches_plain(L, trained, orc, cold_planes):
    """asterx_c2p_learned on a curved block recovers the same primitives as the oracle's c2p within 1e-12
    (cancellation-aware), with the same flags apart from bit 32: with warm starts everywhere (as inside a step:
    the network is not consulted), and with the previous primitives zeroed on some z planes (no warm start
    there: the wavefronts holding those cells evaluate the network, the oracle starts cold)."""
    import torch
    from paper_2406_11669_amd import asterx as ax
    from tests.parity import assert_fields_close
    params, st, _ = trained
    w = W.curved_block(seed=12, n=(20, 13, 11), recon="ppm", rho_atm=1e-6)
    Lg = w.layout
    cons = orc.prim2con(Lg, w.params, w.metric, w.A, w.prim)
    rng = np.random.default_rng(4)
    guess = w.prim * (1.0 + rng.uniform(-0.02, 0.02, w.prim.shape))
    for k in range(cold_planes):
        guess[:, Lg.ng + 2 + 3 * k] = 0.0
    c_ref, p_ref = cons.copy(), guess.copy()
    fl_ref, _ = orc.c2p(Lg, w.params, w.metric, w.A, c_ref, p_ref)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    c_g, p_g = dev(cons), dev(guess)
    flags = torch.zeros(Lg.shape3, dtype=torch.uint8, device="cuda")
    stats = torch.zeros(6, dtype=torch.int64, device="cuda")
    ax.c2p(Lg, w.params, dev(w.metric), dev(w.A), c_g, p_g, flags, stats, mlp=ax.make_mlp(params, st))
    torch.cuda.synchronize()
    fg = Lg.owned(flags.cpu().numpy()).astype(np.int32)
    assert np.array_equal(fg & ~32, Lg.owned(fl_ref).astype(np.int32))
    assert_fields_close(p_g.cpu().numpy(), p_ref, 1e-12, Lg.owned, ["rho", "p", "vx", "vy", "vz"])


@pytest.mark.parametrize("cold_planes", [0, 2])
def test_block_steps_with_learned_guess_vs_oracle(L, trained, orc, cold_planes):
    """A curved block stepped with the learned guess in every stage's recovery (the recovery-with-sources kernel
    that contains the network): two RK4 steps within 1e-10 of the oracle's steps; with the previous primitives
    of some z planes zeroed before the first stage (no warm start there: those wavefronts evaluate the network,
    the oracle starts cold)."""
    import torch
    from paper_2406_11669_amd import asterx as ax
    from tests.parity import assert_fields_close
    params, st, _ = trained
    w = W.curved_block(seed=31, n=(24, 13, 11), recon="ppm", nsteps=2)
    Lg = w.layout
    blk = ax.Block(w)
    assert blk.src_in_c2p
    blk.mlp = ax.make_mlp(params, st)
    prim0 = w.prim.copy()
    for k in range(cold_planes):
        prim0[:, Lg.ng + 3 + 4 * k] = 0.0
        blk.prim[:, Lg.ng + 3 + 4 * k] = 0.0
    blk.run(2)
    torch.cuda.synchronize()
    cons = orc.prim2con(Lg, w.params, w.metric, w.A, w.prim)
    orc.fill_ghosts(Lg, cons, w.bc_cell)
    state = w.state(cons)
    orc.run(Lg, w.params, w.metric, w.curv, state, prim0, w.dt, 2, w.rk, w.bc_cell, w.bc_A)
    names = ["D", "Sx", "Sy", "Sz", "tau", "Ax", "Ay", "Az", "Psi"]
    e = assert_fields_close(blk.state.cpu().numpy(), state, 1e-10, Lg.owned, names)
    print("  learned-guess steps, %d cold planes: max error %.2e" % (cold_planes, float(e.max())), flush=True)
