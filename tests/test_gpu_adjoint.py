"""GPU adjoint of whole RK steps (through the C ABI and the torch.autograd.Function wrappers) against the CPU
oracle's forward-mode derivative of the same loss: <grad, d> versus the oracle's dual-number JVP along d."""
import numpy as np
import pytest

from paper_2406_11669_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def adj():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_11669_amd import adjoint, asterx
    asterx.lib()
    return adjoint


def _grad(adj, w, nsteps):
    import torch
    runner = adj.Runner(w)
    prim = torch.from_numpy(w.prim.copy()).cuda().requires_grad_(True)
    gam = torch.tensor(w.params["gamma"], dtype=torch.float64, device="cuda", requires_grad=True)
    loss = adj.density_loss_run(runner, prim, gam, nsteps)
    loss.backward()
    torch.cuda.synchronize()
    g = prim.grad.detach().cpu().numpy()
    return float(loss.item()), g, float(gam.grad.item()), runner


def _check_dirs(orc, w, nsteps, loss, g, gg, dirs, tol):
    L = w.layout
    for d, dg in dirs:
        lo, jvp, _ = orc.loss_jvp(L, w.params, w.metric, w.curv, w.prim, w.A, w.psi, w.dt, nsteps, w.rk, w.bc_cell,
                                  w.bc_A, dprim0=d, dgamma=dg, A_shift=w.A_shift)
        assert abs(lo - loss) <= 1e-12 * lo, (lo, loss)
        terms = L.owned(g)[2:5] * L.owned(d)[2:5]
        mine = float(np.sum(terms)) + gg * dg
        scale = float(np.sum(np.abs(terms))) + abs(gg * dg)
        print("  jvp oracle %.15e  adjoint %.15e  scale %.3e" % (jvp, mine, scale), flush=True)
        assert abs(mine - jvp) <= tol * scale, (mine, jvp, scale)


def test_adjoint_periodic_riemann_vs_oracle_jvp(adj, orc):
    """Periodic Riemann box (offset potential fill), PPM, RK2, 2 steps on 12^3 at a generic point (smooth seeded
    velocity): random directions in (v, Gamma), Gamma alone, velocity alone."""
    w = W.periodic_riemann_box(seed=41, n=12, nsteps=2, v_amp=0.1)
    print("case adjoint periodic_riemann12", flush=True)
    loss, g, gg, _ = _grad(adj, w, 2)
    dirs = [W.gradient_direction(w.layout, 1), (w.layout.zeros(5), 1.0), W.gradient_direction(w.layout, 2, False)]
    _check_dirs(orc, w, 2, loss, g, gg, dirs, 1e-10)


@pytest.mark.parametrize("recon", ["minmod", "ppm", "wenoz"])
def test_adjoint_curved_rk4_vs_oracle_jvp(adj, orc, recon):
    """Periodic block in a curved static metric (lapse, shift, curvature sources active), RK4, one step."""
    w = W.curved_block(seed=42, n=(12, 10, 9), recon=recon, nsteps=1, vmax=0.3)
    print("case adjoint curved", recon, flush=True)
    loss, g, gg, _ = _grad(adj, w, 1)
    dirs = [W.gradient_direction(w.layout, 3), (w.layout.zeros(5), 1.0)]
    _check_dirs(orc, w, 1, loss, g, gg, dirs, 1e-10)


def test_adjoint_forward_equals_plain_driver(adj):
    """The differentiable forward is the plain driver's sequence of calls: the loss agrees bitwise with the
    forward-only evaluation used by the finite differences."""
    import torch
    w = W.periodic_riemann_box(seed=43, n=12, nsteps=2, v_amp=0.1)
    loss, g, gg, runner = _grad(adj, w, 2)
    prim = torch.from_numpy(w.prim.copy()).cuda()
    assert adj.density_loss_value(runner, prim, w.params["gamma"], 2) == loss
    assert np.all(np.isfinite(g)) and np.isfinite(gg)
