"""GPU: the factor-2 inter-level operators (asterx_prolong, asterx_restrict) against the oracle's, element by
element, for every staggering, on rough data (the fallback acts) and smooth data."""
import numpy as np
import pytest

from paper_2406_11669_amd.workloads import Layout

pytestmark = [pytest.mark.gpu]

C0 = (2, 3, 1)


@pytest.fixture(scope="module")
def ax():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_11669_amd import asterx
    asterx.lib()
    return asterx


def _grids(nf=(10, 8, 6)):
    coarse = Layout((10, 9, 8), 3, dx=(0.1, 0.1, 0.1))
    fine = Layout(nf, 3, dx=(0.05, 0.05, 0.05))
    return coarse, fine


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("stag", ["cell", "vertex", "xedge", "yedge", "zedge"])
@pytest.mark.parametrize("rough", [True, False])
def test_prolong_restrict_vs_oracle(ax, orc, stag, rough):
    import torch
    coarse, fine = _grids()
    rng = np.random.default_rng(40)
    if rough:
        cf = rng.normal(size=(2,) + coarse.shape3)
    else:
        x, y, z = coarse.coords("centre")
        cf = np.stack([np.broadcast_to(1.0 + 0.3 * x + 0.2 * y * y - 0.1 * z + 0.05 * x * y * z, coarse.shape3)] * 2)
        cf = cf.copy()
        cf[1] *= 2.0
    lo, hi = (-2, -2, -2), (fine.n[0] + 1, fine.n[1] + 1, fine.n[2] + 1)
    print("case prolong", stag, rough, flush=True)
    ref = np.zeros((2,) + fine.shape3)
    orc.prolong(coarse, fine, C0, stag, cf, ref, lo, hi)
    out = torch.zeros((2,) + fine.shape3, dtype=torch.float64, device="cuda")
    ax.prolong(coarse, fine, C0, stag, _dev(cf), out, lo, hi)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    clo = tuple(C0[a] - 1 for a in range(3))
    chi = tuple(C0[a] + fine.n[a] // 2 for a in range(3))
    rref = np.zeros_like(cf)
    orc.restrict(coarse, fine, C0, stag, ref, rref, clo, chi)
    rout = torch.zeros((2,) + coarse.shape3, dtype=torch.float64, device="cuda")
    ax.restrict(coarse, fine, C0, stag, out, rout, clo, chi)
    torch.cuda.synchronize()
    assert np.max(np.abs(rout.cpu().numpy() - rref)) <= 1e-13 * np.max(np.abs(rref))


def test_inter_level_rejects_out_of_range_boxes(ax):
    import torch
    coarse, fine = _grids()
    cf = torch.zeros((1,) + coarse.shape3, dtype=torch.float64, device="cuda")
    ff = torch.zeros((1,) + fine.shape3, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="source grid"):
        ax.prolong(coarse, fine, (9, 3, 1), "cell", cf, ff, (0, 0, 0), (9, 7, 5))
    with pytest.raises(RuntimeError, match="target grid"):
        ax.prolong(coarse, fine, C0, "cell", cf, ff, (-4, 0, 0), (3, 3, 3))
    torch.cuda.synchronize()
