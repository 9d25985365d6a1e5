"""The C-ABI library loads on a machine without a GPU, exports every entry point declared in include/asterx.h,
matches the header's struct layouts, and rejects bad arguments on the host before any launch."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "asterx.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|size_t|const char\*)\s+(asterx_[a-z0-9_]+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2406_11669_amd import asterx
    if not os.path.exists(asterx.LIB):
        from paper_2406_11669_amd import build
        build.build()
    return asterx.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "asterx_rhs" in names and "asterx_c2p" in names and "asterx_rk_stage" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header(tmp_path):
    from paper_2406_11669_amd import asterx
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "asterx.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(asterx_grid), '
                   'offsetof(asterx_grid, dx), sizeof(asterx_params), offsetof(asterx_params, c2p_maxit), '
                   'offsetof(asterx_params, c2p_method), sizeof(asterx_c2p_stats), '
                   'offsetof(asterx_params, weno_q), offsetof(asterx_params, riemann));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert vals == [ctypes.sizeof(asterx.Grid), asterx.Grid.dx.offset, ctypes.sizeof(asterx.Params),
                    asterx.Params.c2p_maxit.offset, asterx.Params.c2p_method.offset, 48,
                    asterx.Params.weno_q.offset, asterx.Params.riemann.offset]


def test_host_side_argument_validation(lib):
    from paper_2406_11669_amd import asterx
    from paper_2406_11669_amd.workloads import Layout, default_params
    L = Layout((8, 8, 8), 3)
    g = asterx.make_grid(L)
    p = asterx.make_params(default_params(recon="ppm"))
    dummy = ctypes.c_void_p(16)
    # too few ghost layers for PPM
    g2 = asterx.make_grid(Layout((8, 8, 8), 2))
    rc = lib.asterx_rhs(ctypes.byref(g2), ctypes.byref(p), dummy, dummy, dummy, dummy, dummy, 0.01, dummy, None,
                        dummy, 1 << 40, None)
    assert rc == -1 and b"ghost" in lib.asterx_last_error()
    # upwind CT needs four ghost layers
    p.ct = 1
    rc = lib.asterx_rhs(ctypes.byref(g), ctypes.byref(p), dummy, dummy, dummy, dummy, dummy, 0.01, dummy, None,
                        dummy, 1 << 40, None)
    assert rc == -1 and b"ng >= 4" in lib.asterx_last_error()
    p.ct = 0
    # workspace too small
    rc = lib.asterx_rhs(ctypes.byref(g), ctypes.byref(p), dummy, dummy, dummy, dummy, dummy, 0.01, dummy, None,
                        dummy, 8, None)
    assert rc == -1 and b"workspace" in lib.asterx_last_error()
    # bad gamma
    p.gamma = 1.0
    rc = lib.asterx_c2p(ctypes.byref(g), ctypes.byref(p), dummy, dummy, dummy, dummy, None, None, None)
    assert rc == -1 and b"gamma" in lib.asterx_last_error()
    # ld too small
    g.ld[1] = 10
    rc = lib.asterx_fill_ghosts(ctypes.byref(g), dummy, 1, (ctypes.c_int32 * 3)(0, 0, 0), None)
    assert rc == -1 and b"ld" in lib.asterx_last_error()
    # a field of 2^29 points or more: byte offsets within a field would not fit 32 bits
    g3 = asterx.make_grid(Layout((8, 8, 8), 3))
    g3.ld[0], g3.ld[1], g3.ld[2] = 1024, 1024, 512
    rc = lib.asterx_fill_ghosts(ctypes.byref(g3), dummy, 1, (ctypes.c_int32 * 3)(0, 0, 0), None)
    assert rc == -1 and b"2^29" in lib.asterx_last_error()
    g3.ld[2] = 511  # passes the size check, then stops at nf = 0 before any launch
    rc = lib.asterx_fill_ghosts(ctypes.byref(g3), dummy, 0, (ctypes.c_int32 * 3)(0, 0, 0), None)
    assert rc == -1 and b"bad arguments" in lib.asterx_last_error()
    assert lib.asterx_rhs_workspace_size(ctypes.byref(asterx.make_grid(L))) == 37 * 8 * L.npts


def test_rk_out_layout_and_fused_stage_validation(lib, tmp_path):
    """asterx_rk_out matches its ctypes mirror; asterx_rhs_rk refuses bad output sets before any launch (the
    pointers below are never dereferenced)."""
    from paper_2406_11669_amd import asterx
    from paper_2406_11669_amd.workloads import Layout, default_params
    src = tmp_path / "rkout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "asterx.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(asterx_rk_out), '
                   'offsetof(asterx_rk_out, a), offsetof(asterx_rk_out, u), offsetof(asterx_rk_out, b_dt), '
                   'offsetof(asterx_rk_out, out));return 0;}\n')
    exe = tmp_path / "rkout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    R = asterx.RKOut
    assert [int(v) for v in subprocess.check_output([str(exe)]).split()] == [
        ctypes.sizeof(R), R.a.offset, R.u.offset, R.b_dt.offset, R.out.offset]
    L = Layout((8, 8, 8), 3)
    g = asterx.make_grid(L)
    p = asterx.make_params(default_params(recon="ppm"))
    span = 9 * 8 * L.npts
    wsb = lib.asterx_rhs_workspace_size(ctypes.byref(g))
    base = 1 << 40
    ptr = lambda k: ctypes.c_void_p(base + k * (1 << 32))   # disjoint fake device addresses
    metric, curv, prim, ws = ptr(1), ptr(2), ptr(3), ptr(4)
    U, T1, T2 = base + 5 * (1 << 32), base + 6 * (1 << 32), base + 7 * (1 << 32)
    A, psi = ctypes.c_void_p(U + 5 * 8 * L.npts), ctypes.c_void_p(U + 8 * 8 * L.npts)

    def call(outs, nout=None):
        arr = (asterx.RKOut * max(1, len(outs)))()
        for k, (a, us, out) in enumerate(outs):
            arr[k].nterms = len(a)
            for m in range(len(a)):
                arr[k].a[m] = a[m]
                arr[k].u[m] = us[m]
            arr[k].b_dt = 0.1
            arr[k].out = out
        n = len(outs) if nout is None else nout
        return lib.asterx_rhs_rk(ctypes.byref(g), ctypes.byref(p), metric, curv, prim, A, psi, 0.01, n, arr, None,
                                 ws, wsb, None)

    assert call([], nout=0) == -1 and b"nout" in lib.asterx_last_error()
    assert call([([1.0, 1.0, 1.0][:2], [U, U], T1)], nout=3) == -1
    assert call([([1.0], [U], U)]) == -1 and b"overlaps an input" in lib.asterx_last_error()
    assert call([([1.0], [T1 + 8], T1)]) == -1 and b"partially" in lib.asterx_last_error()
    assert call([([1.0], [U], T1), ([1.0], [U], T1 + span - 8)]) == -1 and b"outputs overlap" in lib.asterx_last_error()
    assert call([([1.0], [U], T1), ([1.0], [T1], T2)]) == -1 and b"other output reads" in lib.asterx_last_error()
    bad = (asterx.RKOut * 1)()
    bad[0].nterms = 3
    bad[0].out = T1
    assert lib.asterx_rhs_rk(ctypes.byref(g), ctypes.byref(p), metric, curv, prim, A, psi, 0.01, 1, bad, None, ws,
                             wsb, None) == -1 and b"bad output" in lib.asterx_last_error()


def test_inter_level_validation_on_host(lib):
    """asterx_prolong / asterx_restrict refuse boxes whose stencils leave the stored points, before any launch."""
    from paper_2406_11669_amd import asterx
    from paper_2406_11669_amd.workloads import Layout
    gc = asterx.make_grid(Layout((10, 9, 8), 3))
    gf = asterx.make_grid(Layout((10, 8, 6), 3))
    i3 = lambda *v: (ctypes.c_int32 * 3)(*v)
    dummy = ctypes.c_void_p(16)
    # fine box reaching past the coarse grid's last stored cell
    rc = lib.asterx_prolong(ctypes.byref(gc), ctypes.byref(gf), i3(9, 3, 1), i3(0, 0, 0), 1, dummy, dummy,
                            i3(0, 0, 0), i3(9, 7, 5), None)
    assert rc == -1 and b"source grid" in lib.asterx_last_error()
    rc = lib.asterx_restrict(ctypes.byref(gc), ctypes.byref(gf), i3(2, 3, 1), i3(0, 0, 0), 1, dummy, dummy,
                             i3(0, 0, 0), i3(9, 8, 7), None)
    assert rc == -1 and b"source grid" in lib.asterx_last_error()
    rc = lib.asterx_prolong(ctypes.byref(gc), ctypes.byref(gf), i3(2, 3, 1), i3(2, 0, 0), 1, dummy, dummy,
                            i3(0, 0, 0), i3(1, 1, 1), None)
    assert rc == -1 and b"stag" in lib.asterx_last_error()


def test_oracle_ghost_fill_matches_definitions(orc):
    import numpy as np
    from paper_2406_11669_amd.workloads import Layout
    L = Layout((2, 5, 4), 3)
    rng = np.random.default_rng(0)
    a = rng.normal(size=(1,) + L.shape3)
    ref = a.copy()
    L.periodic_wrap(ref)
    b = a.copy()
    orc.fill_ghosts(L, b, ["periodic"] * 3)
    ext = L.n[0] + 2 * L.ng + 1
    assert np.array_equal(b[..., :ext], ref[..., :ext])
    c = a.copy()
    orc.fill_ghosts(L, c, ["linear"] * 3)
    o = L.owned(c)[0]
    g = L.ng
    # linear extrapolation along z below the block, at an owned (i, j)
    k0, k1 = c[0, g, g + 1, g + 1], c[0, g + 1, g + 1, g + 1]
    assert np.isclose(c[0, g - 2, g + 1, g + 1], k0 - 2 * (k1 - k0), rtol=1e-14)


def test_extension_entry_points_validate_on_host(lib):
    """Adjoint, point, network and batch entry points reject bad arguments before any launch, and empty point
    sets are a no-op (nothing is touched)."""
    from paper_2406_11669_amd import asterx
    from paper_2406_11669_amd.workloads import Layout, default_params
    L = Layout((8, 8, 8), 3)
    g = asterx.make_grid(L)
    p = asterx.make_params(default_params(recon="ppm"))
    dummy = ctypes.c_void_p(16)
    # adjoint: workspace too small; periodic blocks need n > ng
    rc = lib.asterx_rhs_adjoint(ctypes.byref(g), ctypes.byref(p), dummy, dummy, dummy, dummy, dummy, dummy, 0.01,
                                dummy, dummy, dummy, dummy, dummy, dummy, 8, None)
    assert rc == -1 and b"workspace" in lib.asterx_last_error()
    g3 = asterx.make_grid(Layout((3, 8, 8), 3))
    rc = lib.asterx_c2p_adjoint(ctypes.byref(g3), ctypes.byref(p), dummy, dummy, dummy, dummy, dummy, dummy, dummy,
                                dummy, dummy, 1 << 40, None)
    assert rc == -1 and b"n > ng" in lib.asterx_last_error()
    assert lib.asterx_adjoint_workspace_size(ctypes.byref(g)) >= 52 * 8 * L.npts
    # points: negative n, NULL arrays; n = 0 is a no-op
    assert lib.asterx_prim2con_points(-1, None, 5.0 / 3.0, dummy, dummy, dummy, dummy, None, None) == -1
    assert lib.asterx_prim2con_points(4, None, 5.0 / 3.0, dummy, dummy, None, dummy, None, None) == -1
    assert lib.asterx_prim2con_points(0, None, 5.0 / 3.0, dummy, dummy, dummy, dummy, None, None) == 0
    assert lib.asterx_c2p_points(ctypes.byref(p), 0, None, dummy, dummy, dummy, None, None, dummy, None, None, None,
                                 None) == 0
    assert lib.asterx_prim2con_points(4, None, 1.0, dummy, dummy, dummy, dummy, None, None) == -1  # Gamma <= 1
    # network: zero scale rejected; workspace sizing and too-small workspace
    m = asterx.MLP()
    m.params = 16
    for k in range(8):
        m.in_scale[k] = 1.0
    m.out_scale[0] = 1.0
    m.out_scale[1] = 0.0
    assert lib.asterx_mlp_forward(ctypes.byref(m), 10, dummy, dummy, None) == -1
    assert b"scale" in lib.asterx_last_error()
    m.out_scale[1] = 1.0
    assert lib.asterx_mlp_forward(ctypes.byref(m), 0, dummy, dummy, None) == 0
    assert lib.asterx_mlp_grad_workspace_size(65) == 2 * (asterx.MLP_NPARAMS + 1) * 4
    assert lib.asterx_mlp_grad(ctypes.byref(m), 65, dummy, dummy, dummy, dummy, 8, None) == -1
    assert lib.asterx_mlp_adam(dummy, dummy, dummy, dummy, 1e-3, 0.9, 0.999, 1e-8, 0, None) == -1  # step >= 1
    assert lib.asterx_c2p_learned(ctypes.byref(g), ctypes.byref(p), dummy, dummy, dummy, dummy, None, None, None,
                                  None) == -1
    # batch: at least one patch, sane ghosts
    h = ctypes.c_void_p()
    assert lib.asterx_batch_create(0, None, None, ctypes.byref(h)) == -1


def test_noalloc_refuses_grids_beyond_its_workspace_on_host(lib):
    """asterx_rhs_rk_noalloc refuses a block whose workspace exceeds the library-held 64 MiB (53^3 cells with 3 ghost
    layers) before touching any device (the pointers are never dereferenced)."""
    from paper_2406_11669_amd import asterx
    from paper_2406_11669_amd.workloads import Layout, default_params
    p = asterx.make_params(default_params(recon="ppm"))
    for n, fits in (((52, 52, 52), True), ((53, 53, 53), False)):
        g = asterx.make_grid(Layout(n, 3))
        assert (lib.asterx_rhs_workspace_size(ctypes.byref(g)) <= asterx.NOALLOC_WS_BYTES) == fits
    g = asterx.make_grid(Layout((53, 53, 53), 3))
    dummy = ctypes.c_void_p(1 << 40)
    outs = (asterx.RKOut * 1)()
    rc = lib.asterx_rhs_rk_noalloc(ctypes.byref(g), ctypes.byref(p), dummy, dummy, dummy, dummy, dummy, 0.01, 1, outs,
                                   None, None)
    assert rc == -1 and b"64 MiB" in lib.asterx_last_error()


def test_ghost_boxes_partition_the_ghost_points():
    """The six boxes of a refined patch's ghost zones cover every ghost point of each staggering exactly once and
    no owned point: the ghost points are ng layers around the owned box [0, n - 1]^3, one more on the upper side
    of a vertex-centred axis (its point n)."""
    import numpy as np
    from paper_2406_11669_amd.amr import ghost_boxes
    from paper_2406_11669_amd.workloads import Layout
    L = Layout((10, 7, 6), 3)
    for stag in [(0, 0, 0), (1, 1, 1), (0, 1, 1), (1, 0, 1), (1, 1, 0)]:
        count = np.zeros(L.shape3, dtype=int)
        for lo, hi in ghost_boxes(L, stag):
            count[lo[2] + L.ng:hi[2] + L.ng + 1, lo[1] + L.ng:hi[1] + L.ng + 1, lo[0] + L.ng:hi[0] + L.ng + 1] += 1
        idx = [np.arange(L.ld[d]) - L.ng for d in range(3)]
        own1 = [(i >= 0) & (i <= L.n[d] - 1) for d, i in enumerate(idx)]
        # within ng layers of the owned range (vertex axes: of [0, n])
        inr = [(i >= -L.ng) & (i <= L.n[d] - 1 + stag[d] + L.ng) for d, i in enumerate(idx)]
        assert all(int(np.sum(o)) == L.n[d] for d, o in enumerate(own1))
        assert all(int(np.sum(r)) == L.n[d] + 2 * L.ng + stag[d] for d, r in enumerate(inr))
        own = [(i >= 0) & (i <= L.n[d] - 1) for d, i in enumerate(idx)]
        inside = inr[2][:, None, None] & inr[1][None, :, None] & inr[0][None, None, :]
        owned = own[2][:, None, None] & own[1][None, :, None] & own[0][None, None, :]
        assert np.array_equal(count, (inside & ~owned).astype(int)), stag


def test_recovery_with_sources_validation_on_host(lib):
    """asterx_c2p_src and asterx_rhs_rk_src refuse bad arguments before any launch (the pointers are never
    dereferenced): NULL arrays, too few ghost layers, a stage output overlapping the sources buffer."""
    from paper_2406_11669_amd import asterx
    from paper_2406_11669_amd.workloads import Layout, default_params
    L = Layout((8, 8, 8), 3)
    g = asterx.make_grid(L)
    p = asterx.make_params(default_params(recon="ppm"))
    base = 1 << 40
    ptr = lambda k: ctypes.c_void_p(base + k * (1 << 32))
    metric, curv, A, cons, prim, src, ws = (ptr(k) for k in range(1, 8))
    rc = lib.asterx_c2p_src(ctypes.byref(g), ctypes.byref(p), metric, curv, A, cons, prim, None, None, None, None, None)
    assert rc == -1 and b"NULL" in lib.asterx_last_error()
    g1 = asterx.make_grid(Layout((8, 8, 8), 1))
    rc = lib.asterx_c2p_src(ctypes.byref(g1), ctypes.byref(p), metric, curv, A, cons, prim, None, None, None, src, None)
    assert rc == -1
    wsb = lib.asterx_rhs_workspace_size(ctypes.byref(g))
    U = base + 9 * (1 << 32)
    outs = (asterx.RKOut * 1)()
    outs[0].nterms = 1
    outs[0].a[0] = 1.0
    outs[0].u[0] = U
    outs[0].b_dt = 0.1
    outs[0].out = src.value + 8  # inside the sources buffer
    psi = ctypes.c_void_p(U + 8 * 8 * L.npts)
    rc = lib.asterx_rhs_rk_src(ctypes.byref(g), ctypes.byref(p), metric, prim, A, psi, src, 0.01, 1, outs, None, ws,
                               wsb, None)
    assert rc == -1 and b"overlaps an input" in lib.asterx_last_error()
    rc = lib.asterx_rhs_rk_src(ctypes.byref(g), ctypes.byref(p), metric, prim, A, psi, None, 0.01, 1, outs, None, ws,
                               wsb, None)
    assert rc == -1 and b"NULL" in lib.asterx_last_error()
