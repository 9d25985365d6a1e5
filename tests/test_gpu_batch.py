"""Batched persistent launches over AMR-like patches: bitwise equal to the per-patch launch loop for every
schedule, stable under HIP-graph replay, and within tolerance of the oracle on sampled patches."""
import numpy as np
import pytest

from paper_2406_11669_amd import workloads as W
from tests.parity import assert_fields_close

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]


@pytest.fixture(scope="module")
def ax():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_11669_amd import asterx
    asterx.lib()
    return asterx


def _patches(n=10, nsteps=2, recon="minmod"):
    return W.patch_set(seed=3, npatches=n, sides=(16, 24), levels=3, nsteps=nsteps, recon=recon)


def _per_patch(ax, wls, nsteps):
    # the per-patch launch loop runs the batch's kernel bodies (sources in the cell kernel)
    blocks = [ax.Block(w, src_in_c2p=False) for w in wls]
    for _ in range(nsteps):
        for b in blocks:
            b.step()
    return blocks


def test_batch_fused_equals_stored_per_patch_loop(ax):
    """The batch with right-hand sides combined into the stage outputs (asterx_batch_rhs_rk) against per-patch
    blocks that store the right-hand side and combine with asterx_rk_stage: bitwise equal."""
    import torch
    wls = _patches(recon="ppm")
    print("case batch fused vs stored loop", flush=True)
    bt = ax.Batch(wls, tuning=(4, 1))
    bt.run(2)
    blocks = [ax.Block(w, fused=False) for w in wls]
    for _ in range(2):
        for b in blocks:
            b.step()
    torch.cuda.synchronize()
    for p, b in enumerate(blocks):
        assert torch.equal(bt.unpack(bt.state, p), b.state), p
        assert torch.equal(bt.unpack(bt.prim, p), b.prim), p


@pytest.mark.parametrize("tuning", [(1, 0), (4, 1), (8, 2)])
def test_batch_bitwise_equals_per_patch_loop(ax, tuning):
    import torch
    wls = _patches()
    print("case batch vs loop", tuning, flush=True)
    bt = ax.Batch(wls, tuning=tuning)
    bt.run(2)
    blocks = _per_patch(ax, wls, 2)
    torch.cuda.synchronize()
    for p, b in enumerate(blocks):
        assert torch.equal(bt.unpack(bt.state, p), b.state), p
        assert torch.equal(bt.unpack(bt.prim, p), b.prim), p


@pytest.mark.parametrize("recon", ["ppm", "wenoz"])
def test_batch_bitwise_equals_per_patch_loop_recon(ax, recon):
    """PPM and WENO-Z patches: the persistent face launches (including the LDS-staged stencils, whose
    workgroups move from item to item) equal the per-patch loop bitwise."""
    import torch
    wls = _patches(n=8, recon=recon)
    print("case batch vs loop", recon, flush=True)
    bt = ax.Batch(wls, tuning=(1, 2))
    bt.run(2)
    blocks = _per_patch(ax, wls, 2)
    torch.cuda.synchronize()
    for p, b in enumerate(blocks):
        assert torch.equal(bt.unpack(bt.state, p), b.state), p
        assert torch.equal(bt.unpack(bt.prim, p), b.prim), p


def test_batch_graph_replays_match_eager(ax):
    import torch
    wls = _patches(n=6, nsteps=3)
    eager = ax.Batch(wls)
    graphed = ax.Batch(wls)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        graphed.step()  # step 1, eager, on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graphed.step()
    eager.step()
    for rep in range(2):  # steps 2 and 3
        g.replay()
        torch.cuda.synchronize()
        eager.step()
        torch.cuda.synchronize()
        assert torch.equal(graphed.state, eager.state), rep
        x = eager.state.sum().item()  # interleaved eager work between replays
        assert np.isfinite(x)


def test_batch_sampled_patches_vs_oracle(ax, orc):
    import torch
    wls = _patches(n=8, nsteps=2)
    bt = ax.Batch(wls)
    bt.run(2)
    torch.cuda.synchronize()
    for p in (0, 3, 7):
        w = wls[p]
        L = w.layout
        cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
        orc.fill_ghosts(L, cons, w.bc_cell)
        state = w.state(cons)
        prim = w.prim.copy()
        orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, 2, 2, w.bc_cell, w.bc_A)
        assert_fields_close(bt.unpack(bt.state, p).cpu().numpy(), state, 1e-10, L.owned)
