"""asterx_rhs_rk_noalloc (the library-held workspace, for callers that cannot allocate) against asterx_rhs_rk with a
caller-provided workspace: the same kernels on the same inputs, so stage outputs and reductions must agree bit for
bit, call after call on one device (the array keeps the previous call's contents), each call smaller than the one
before it, from the largest block the library's workspace holds down to a small ragged one."""
import numpy as np
import pytest

from paper_2406_11669_amd import workloads as W

pytestmark = pytest.mark.gpu


def _stage_both(ax, torch, shape, seed, recon):
    w = W.curved_block(seed=seed, n=shape, recon=recon, nsteps=1, rk=4)
    print("case rhs_rk_noalloc", shape, recon, "workspace bytes", ax.workspace_size(w.layout), flush=True)
    assert ax.workspace_size(w.layout) <= ax.NOALLOC_WS_BYTES
    blk = ax.Block(w)
    blk.recover(blk.state)
    U, dt = blk.state, blk.dt
    res = []
    for noalloc in (False, True):
        t1, t2 = torch.zeros_like(U), torch.zeros_like(U)
        red = torch.zeros(2, dtype=torch.float64, device=U.device)
        outs = [([1.0], [U], 0.5 * dt, t1), ([1.0], [U], dt / 6.0, t2)]
        if noalloc:
            ax.rhs_rk_noalloc(blk.L, blk.params, blk.metric, blk.curv, blk.prim, U[5:8], U[8:9], dt, outs, red)
        else:
            ax.rhs_rk(blk.L, blk.params, blk.metric, blk.curv, blk.prim, U[5:8], U[8:9], dt, outs, red, blk.ws)
        res.append((t1, t2, red))
    torch.cuda.synchronize()
    (a1, a2, ra), (b1, b2, rb) = res
    assert torch.equal(a1, b1) and torch.equal(a2, b2)
    assert torch.equal(ra, rb)
    owned = w.layout.owned
    # the stage outputs moved away from the state on owned points (the call did its work)
    assert np.max(np.abs(owned(a1[0].cpu().numpy()) - owned(U[0].cpu().numpy()))) > 0.0


def test_noalloc_matches_workspace_entry_point_calls_in_a_row():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_11669_amd import asterx as ax
    ax.lib()
    # 52^3 with 3 ghost layers is the largest cube the 64 MiB array holds; then smaller blocks on the same array
    _stage_both(ax, torch, (52, 52, 52), 41, "ppm")
    _stage_both(ax, torch, (24, 13, 11), 42, "wenoz")
    _stage_both(ax, torch, (12, 9, 8), 43, "ppm")
