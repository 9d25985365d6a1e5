"""Python binding of libasterx.so (C ABI in include/asterx.h): argument marshalling only.

Every step of the right-hand side runs in the HIP kernels of the library.  torch is used
for device memory (float64 CUDA tensors of shape (nfields, ld[2], ld[1], ld[0])) and for
the current HIP stream.  There is no CPU fallback: if the library is not built, loading
fails with an error.
"""
import ctypes
import os

import numpy as np
import torch

from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libasterx.so")

RECON = {"minmod": 0, "ppm": 1, "wenoz": 2, "mp5": 3}
RIEMANN = {"hlle": 0, "lxf": 1}
CT = {"fct": 0, "uct": 1}
GAUGE = {"lorenz": 0, "algebraic": 1}
SPEEDS = {"quartic": 0, "bound": 1}
BC = {"periodic": 0, "copy": 1, "linear": 2}
FLAG_NOBLE_FAIL, FLAG_FALLBACK, FLAG_ATMOSPHERE, FLAG_HARD_FAIL, FLAG_NAN_IN = 1, 2, 4, 8, 16


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ng", ctypes.c_int32), ("ld", ctypes.c_int32 * 3),
                ("pad_", ctypes.c_int32), ("dx", ctypes.c_double * 3)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("order", ctypes.c_int32)]


class MLP(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("in_shift", ctypes.c_float * 8), ("in_scale", ctypes.c_float * 8),
                ("out_shift", ctypes.c_float * 2), ("out_scale", ctypes.c_float * 2)]


MLP_NPARAMS = 4866


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("rho_atm", ctypes.c_double), ("k_atm", ctypes.c_double),
                ("xi", ctypes.c_double), ("c2p_tol", ctypes.c_double), ("wmax", ctypes.c_double),
                ("weno_eps", ctypes.c_double), ("weno_q", ctypes.c_double),
                ("c2p_maxit", ctypes.c_int32), ("brent_maxit", ctypes.c_int32), ("recon", ctypes.c_int32),
                ("gauge", ctypes.c_int32), ("speeds", ctypes.c_int32), ("c2p_method", ctypes.c_int32),
                ("riemann", ctypes.c_int32), ("ct", ctypes.c_int32)]


class RKOut(ctypes.Structure):
    """asterx_rk_out: out = sum_m a[m] u[m] + b_dt rhs (nterms = 1 or 2)."""
    _fields_ = [("nterms", ctypes.c_int32), ("a", ctypes.c_double * 2), ("u", ctypes.c_void_p * 2),
                ("b_dt", ctypes.c_double), ("out", ctypes.c_void_p)]


def make_rk_outs(outs):
    """outs: [(a list, u list of tensors, b_dt, out tensor)] -> host asterx_rk_out array."""
    arr = (RKOut * len(outs))()
    for k, (a, us, b_dt, out) in enumerate(outs):
        assert 1 <= len(a) == len(us) <= 2
        for u in list(us) + [out]:
            assert u.is_cuda and u.is_contiguous() and u.dtype == torch.float64
        arr[k].nterms = len(a)
        for m in range(len(a)):
            arr[k].a[m] = float(a[m])
            arr[k].u[m] = us[m].data_ptr()
        arr[k].b_dt = float(b_dt)
        arr[k].out = out.data_ptr()
    return arr


_lib = None

EXPORTS = ["asterx_version", "asterx_last_error", "asterx_rhs_workspace_size", "asterx_prim2con", "asterx_c2p",
           "asterx_fill_ghosts", "asterx_fill_ghosts_shift", "asterx_rhs", "asterx_rk_stage", "asterx_zero", "asterx_timing_enable",
           "asterx_timing_read", "asterx_timing_reset", "asterx_timing_name", "asterx_batch_create",
           "asterx_batch_destroy", "asterx_batch_points", "asterx_batch_offset", "asterx_batch_workspace_size",
           "asterx_batch_prim2con", "asterx_batch_c2p", "asterx_batch_fill_ghosts", "asterx_batch_rhs",
           "asterx_batch_rk_stage", "asterx_adjoint_workspace_size", "asterx_rhs_adjoint", "asterx_c2p_adjoint",
           "asterx_prim2con_adjoint", "asterx_prim2con_points", "asterx_mlp_features", "asterx_mlp_forward",
           "asterx_mlp_grad_workspace_size", "asterx_mlp_grad", "asterx_mlp_adam", "asterx_c2p_points",
           "asterx_c2p_learned", "asterx_rhs_rk", "asterx_batch_rhs_rk", "asterx_tmunu", "asterx_prolong",
           "asterx_restrict", "asterx_rhs_rk_noalloc", "asterx_c2p_src", "asterx_rhs_rk_src"]


def lib():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError("libasterx.so is not built: run `python -m paper_2406_11669_amd.build` "
                               "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB)
        L.asterx_last_error.restype = ctypes.c_char_p
        L.asterx_rhs_workspace_size.restype = ctypes.c_size_t
        L.asterx_rhs_workspace_size.argtypes = [ctypes.c_void_p]
        vp = ctypes.c_void_p
        L.asterx_prim2con.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.asterx_c2p.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.asterx_fill_ghosts.argtypes = [vp, vp, ctypes.c_int32, vp, vp]
        L.asterx_fill_ghosts_shift.argtypes = [vp, vp, ctypes.c_int32, vp, vp]
        L.asterx_rhs.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, vp, vp, vp, ctypes.c_size_t, vp]
        L.asterx_rk_stage.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_double, vp, vp, vp]
        L.asterx_tmunu.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.asterx_prolong.argtypes = [vp, vp, vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp]
        L.asterx_restrict.argtypes = [vp, vp, vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp]
        L.asterx_rhs_rk.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp, vp, vp,
                                    ctypes.c_size_t, vp]
        L.asterx_c2p_src.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.asterx_rhs_rk_src.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp, vp, vp,
                                        ctypes.c_size_t, vp]
        L.asterx_rhs_rk_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp, vp,
                                            vp]
        L.asterx_batch_rhs_rk.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp, vp, vp,
                                          ctypes.c_size_t, vp]
        L.asterx_zero.argtypes = [vp, ctypes.c_int64, vp]
        L.asterx_timing_enable.argtypes = [ctypes.c_int32]
        L.asterx_timing_read.argtypes = [vp, vp, ctypes.c_int32]
        L.asterx_timing_name.restype = ctypes.c_char_p
        L.asterx_timing_name.argtypes = [ctypes.c_int32]
        L.asterx_batch_create.argtypes = [ctypes.c_int32, vp, vp, vp]
        L.asterx_batch_destroy.argtypes = [vp]
        L.asterx_batch_points.restype = ctypes.c_int64
        L.asterx_batch_points.argtypes = [vp]
        L.asterx_batch_offset.restype = ctypes.c_int64
        L.asterx_batch_offset.argtypes = [vp, ctypes.c_int32]
        L.asterx_batch_workspace_size.restype = ctypes.c_size_t
        L.asterx_batch_workspace_size.argtypes = [vp]
        L.asterx_batch_prim2con.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.asterx_batch_c2p.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.asterx_batch_fill_ghosts.argtypes = [vp, vp, ctypes.c_int32, vp, vp]
        L.asterx_batch_rhs.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, vp, vp, vp, ctypes.c_size_t,
                                       vp]
        L.asterx_batch_rk_stage.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_double, vp, vp, vp]
        i64 = ctypes.c_int64
        L.asterx_prim2con_points.argtypes = [i64, vp, ctypes.c_double, vp, vp, vp, vp, vp, vp]
        L.asterx_mlp_features.argtypes = [i64, vp, ctypes.c_double, vp, vp, vp, vp, vp]
        L.asterx_mlp_forward.argtypes = [vp, i64, vp, vp, vp]
        L.asterx_mlp_grad_workspace_size.restype = ctypes.c_size_t
        L.asterx_mlp_grad_workspace_size.argtypes = [i64]
        L.asterx_mlp_grad.argtypes = [vp, i64, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.asterx_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_int32, vp]
        L.asterx_c2p_points.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.asterx_c2p_learned.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.asterx_adjoint_workspace_size.restype = ctypes.c_size_t
        L.asterx_adjoint_workspace_size.argtypes = [vp]
        L.asterx_rhs_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp, vp, vp,
                                         ctypes.c_size_t, vp]
        L.asterx_c2p_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.asterx_prim2con_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise RuntimeError("asterx error %d: %s" % (rc, lib().asterx_last_error().decode()))


def make_grid(layout):
    g = Grid()
    for d in range(3):
        g.n[d] = int(layout.n[d])
        g.ld[d] = int(layout.ld[d])
        g.dx[d] = float(layout.dx[d])
    g.ng = int(layout.ng)
    return g


def make_params(p):
    P = Params()
    for k in ("gamma", "rho_atm", "k_atm", "xi", "c2p_tol", "wmax", "weno_eps", "weno_q"):
        setattr(P, k, float(p[k]))
    P.c2p_maxit = int(p["c2p_maxit"])
    P.brent_maxit = int(p["brent_maxit"])
    P.recon = RECON[p["recon"]] if isinstance(p["recon"], str) else int(p["recon"])
    P.gauge = GAUGE[p["gauge"]] if isinstance(p["gauge"], str) else int(p["gauge"])
    P.speeds = SPEEDS[p["speeds"]] if isinstance(p["speeds"], str) else int(p["speeds"])
    P.c2p_method = int(p.get("c2p_method", 0))
    r = p.get("riemann", "hlle")
    P.riemann = RIEMANN[r] if isinstance(r, str) else int(r)
    c = p.get("ct", "fct")
    P.ct = CT[c] if isinstance(c, str) else int(c)
    return P


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _f64(t):
    assert t.dtype == torch.float64, t.dtype
    return t


# ---- thin wrappers of the C entry points ------------------------------------------------------------------

def workspace_size(layout):
    return lib().asterx_rhs_workspace_size(ctypes.byref(make_grid(layout)))


def prim2con(layout, params, metric, A, prim, cons, stream=None):
    _check(lib().asterx_prim2con(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                                 _ptr(_f64(metric)), _ptr(_f64(A)), _ptr(_f64(prim)), _ptr(_f64(cons)),
                                 _stream(stream)))


def c2p(layout, params, metric, A, cons, prim, flags=None, stats=None, stream=None, mlp=None):
    """asterx_c2p, or asterx_c2p_learned when an asterx_mlp (make_mlp) is given."""
    if mlp is not None:
        _check(lib().asterx_c2p_learned(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                                        _ptr(_f64(metric)), _ptr(_f64(A)), _ptr(_f64(cons)), _ptr(_f64(prim)),
                                        _ptr(flags), _ptr(stats), ctypes.byref(mlp), _stream(stream)))
        return
    _check(lib().asterx_c2p(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                            _ptr(_f64(metric)), _ptr(_f64(A)), _ptr(_f64(cons)), _ptr(_f64(prim)), _ptr(flags),
                            _ptr(stats), _stream(stream)))


def c2p_src(layout, params, metric, curv, A, cons, prim, src, flags=None, stats=None, stream=None, mlp=None):
    """asterx_c2p_src: the recovery (learned guess when an asterx_mlp is given), the geometric sources of the
    recovered state (densitized) and the x-face metric, into src (SRC_FIELDS fields)."""
    _check(lib().asterx_c2p_src(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                                _ptr(_f64(metric)), _ptr(_f64(curv)), _ptr(_f64(A)), _ptr(_f64(cons)),
                                _ptr(_f64(prim)), _ptr(flags), _ptr(stats),
                                ctypes.byref(mlp) if mlp is not None else None, _ptr(_f64(src)), _stream(stream)))


def fill_ghosts_shift(layout, f, shift, stream=None):
    """Periodic ghost fill of f (nf <= 3 fields) plus shift[q, d] per period of wrap along axis d."""
    nf = f.shape[0] if f.dim() == 4 else 1
    sh = (ctypes.c_double * (3 * nf))(*np.asarray(shift, dtype=np.float64)[:nf].ravel().tolist())
    _check(lib().asterx_fill_ghosts_shift(ctypes.byref(make_grid(layout)), _ptr(_f64(f)), nf, sh, _stream(stream)))


def fill_ghosts(layout, f, kinds, stream=None):
    karr = (ctypes.c_int32 * 3)(*[BC[k] if isinstance(k, str) else int(k) for k in kinds])
    nf = f.shape[0] if f.dim() == 4 else 1
    _check(lib().asterx_fill_ghosts(ctypes.byref(make_grid(layout)), _ptr(_f64(f)), nf, karr, _stream(stream)))


def rhs(layout, params, metric, curv, prim, A, psi, dt_max, out, red, workspace, stream=None):
    _check(lib().asterx_rhs(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                            _ptr(_f64(metric)), _ptr(_f64(curv)), _ptr(_f64(prim)), _ptr(_f64(A)),
                            _ptr(_f64(psi)), float(dt_max), _ptr(_f64(out)), _ptr(red), _ptr(workspace),
                            workspace.numel() * workspace.element_size(), _stream(stream)))


def rk_stage(layout, a, us, b_dt, rhs_t, out, stream=None):
    n = len(a)
    arr_a = (ctypes.c_double * n)(*[float(x) for x in a])
    arr_u = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
    for u in us:
        assert u.is_cuda and u.is_contiguous() and u.dtype == torch.float64
    _check(lib().asterx_rk_stage(ctypes.byref(make_grid(layout)), n, arr_a, arr_u, float(b_dt), _ptr(_f64(rhs_t)),
                                 _ptr(_f64(out)), _stream(stream)))


def tmunu(layout, params, metric, prim, A, out, stream=None):
    """T_{mu nu} at the vertices [0, n]^3 into out (10 fields), asterx_tmunu."""
    _check(lib().asterx_tmunu(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                              _ptr(_f64(metric)), _ptr(_f64(prim)), _ptr(_f64(A)), _ptr(_f64(out)), _stream(stream)))


STAG = {"cell": (0, 0, 0), "vertex": (1, 1, 1), "xedge": (0, 1, 1), "yedge": (1, 0, 1), "zedge": (1, 1, 0)}


def _i3(v):
    return (ctypes.c_int32 * 3)(*[int(x) for x in v])


def prolong(coarse, fine, c0, stag, cf, ff, lo, hi, stream=None):
    """Fine points [lo, hi] of ff (nf fields) from cf (asterx_prolong); stag a name of STAG or per-axis 0/1."""
    stag = STAG[stag] if isinstance(stag, str) else stag
    _check(lib().asterx_prolong(ctypes.byref(make_grid(coarse)), ctypes.byref(make_grid(fine)), _i3(c0), _i3(stag),
                                cf.shape[0], _ptr(_f64(cf)), _ptr(_f64(ff)), _i3(lo), _i3(hi), _stream(stream)))


def restrict(coarse, fine, c0, stag, ff, cf, lo, hi, stream=None):
    """Coarse points [lo, hi] of cf from ff (asterx_restrict)."""
    stag = STAG[stag] if isinstance(stag, str) else stag
    _check(lib().asterx_restrict(ctypes.byref(make_grid(coarse)), ctypes.byref(make_grid(fine)), _i3(c0), _i3(stag),
                                 ff.shape[0], _ptr(_f64(ff)), _ptr(_f64(cf)), _i3(lo), _i3(hi), _stream(stream)))


def rhs_rk(layout, params, metric, curv, prim, A, psi, dt_max, outs, red, workspace, stream=None):
    """Right-hand side combined straight into RK stage outputs (asterx_rhs_rk); outs as make_rk_outs."""
    arr = make_rk_outs(outs)
    _check(lib().asterx_rhs_rk(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                               _ptr(_f64(metric)), _ptr(_f64(curv)), _ptr(_f64(prim)), _ptr(_f64(A)),
                               _ptr(_f64(psi)), float(dt_max), len(outs), arr, _ptr(red), _ptr(workspace),
                               workspace.numel() * workspace.element_size(), _stream(stream)))


NOALLOC_WS_BYTES = 64 << 20  # ASTERX_NOALLOC_WS_BYTES
SRC_FIELDS = 14  # ASTERX_SRC_FIELDS: sources (4) and x-face metric (10) handed from asterx_c2p_src to asterx_rhs_rk_src


def rhs_rk_src(layout, params, metric, prim, A, psi, src, dt_max, outs, red, workspace, stream=None):
    """asterx_rhs_rk_src: asterx_rhs_rk with the sources written by asterx_c2p_src."""
    arr = make_rk_outs(outs)
    _check(lib().asterx_rhs_rk_src(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                                   _ptr(_f64(metric)), _ptr(_f64(prim)), _ptr(_f64(A)), _ptr(_f64(psi)),
                                   _ptr(_f64(src)), float(dt_max), len(outs), arr, _ptr(red), _ptr(workspace),
                                   workspace.numel() * workspace.element_size(), _stream(stream)))


def rhs_rk_noalloc(layout, params, metric, curv, prim, A, psi, dt_max, outs, red, stream=None):
    """asterx_rhs_rk with the library-held workspace (asterx_rhs_rk_noalloc): no device allocation."""
    arr = make_rk_outs(outs)
    _check(lib().asterx_rhs_rk_noalloc(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                                       _ptr(_f64(metric)), _ptr(_f64(curv)), _ptr(_f64(prim)), _ptr(_f64(A)),
                                       _ptr(_f64(psi)), float(dt_max), len(outs), arr, _ptr(red), _stream(stream)))


def adjoint_workspace_size(layout):
    return lib().asterx_adjoint_workspace_size(ctypes.byref(make_grid(layout)))


def _ws(workspace):
    return _ptr(workspace), workspace.numel() * workspace.element_size()


def rhs_adjoint(layout, params, metric, curv, cons, prim_guess, A, psi, dt_max, rhs_bar, cons_bar, A_bar, psi_bar,
                gamma_bar, workspace, stream=None):
    """Adds the transposed Jacobian of (cons, A, psi) -> rhs(fill(c2p(cons, A)), A, psi) applied to rhs_bar."""
    w, nb = _ws(workspace)
    _check(lib().asterx_rhs_adjoint(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                                    _ptr(_f64(metric)), _ptr(_f64(curv)), _ptr(_f64(cons)), _ptr(_f64(prim_guess)),
                                    _ptr(_f64(A)), _ptr(_f64(psi)), float(dt_max), _ptr(_f64(rhs_bar)),
                                    _ptr(_f64(cons_bar)), _ptr(_f64(A_bar)), _ptr(_f64(psi_bar)),
                                    _ptr(_f64(gamma_bar)), w, nb, _stream(stream)))


def c2p_adjoint(layout, params, metric, cons, prim_guess, A, prim_bar, cons_bar, A_bar, gamma_bar, workspace,
                stream=None):
    w, nb = _ws(workspace)
    _check(lib().asterx_c2p_adjoint(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                                    _ptr(_f64(metric)), _ptr(_f64(cons)), _ptr(_f64(prim_guess)), _ptr(_f64(A)),
                                    _ptr(_f64(prim_bar)), _ptr(_f64(cons_bar)), _ptr(_f64(A_bar)),
                                    _ptr(_f64(gamma_bar)), w, nb, _stream(stream)))


def prim2con_adjoint(layout, params, metric, A, prim, cons_bar, prim_bar, A_bar, gamma_bar, workspace, stream=None):
    w, nb = _ws(workspace)
    _check(lib().asterx_prim2con_adjoint(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                                         _ptr(_f64(metric)), _ptr(_f64(A)), _ptr(_f64(prim)), _ptr(_f64(cons_bar)),
                                         _ptr(_f64(prim_bar)), _ptr(_f64(A_bar)), _ptr(_f64(gamma_bar)), w, nb,
                                         _stream(stream)))


# ---- independent points and the learned c2p guess -----------------------------------------------------------

def make_mlp(params, stdz):
    """asterx_mlp from a device float32 parameter tensor and the standardisation constants (dict of arrays)."""
    assert params.is_cuda and params.dtype == torch.float32 and params.numel() == MLP_NPARAMS
    m = MLP()
    m.params = params.data_ptr()
    for k in ("in_shift", "in_scale", "out_shift", "out_scale"):
        arr = getattr(m, k)
        vals = np.asarray(stdz[k], dtype=np.float64)
        for i in range(len(arr)):
            arr[i] = float(vals[i])
    return m


def _gp(gam):
    """(per-point pointer, scalar) for an adiabatic index given as a tensor of n values or a float."""
    if torch.is_tensor(gam):
        return _ptr(_f64(gam)), 0.0
    return None, float(gam)


def prim2con_points(gam, metric, Bt, prim, cons, target=None, stream=None):
    n = prim.shape[1]
    gp, gs = _gp(gam)
    _check(lib().asterx_prim2con_points(n, gp, gs, _ptr(_f64(metric)), _ptr(_f64(Bt)), _ptr(_f64(prim)),
                                        _ptr(_f64(cons)), _ptr(target), _stream(stream)))


def mlp_features(gam, metric, Bt, cons, feat, stream=None):
    n = cons.shape[1]
    gp, gs = _gp(gam)
    _check(lib().asterx_mlp_features(n, gp, gs, _ptr(_f64(metric)), _ptr(_f64(Bt)), _ptr(_f64(cons)), _ptr(feat),
                                     _stream(stream)))


def mlp_forward(mlp, feat, out, stream=None):
    _check(lib().asterx_mlp_forward(ctypes.byref(mlp), feat.shape[1], _ptr(feat), _ptr(out), _stream(stream)))


def mlp_grad_workspace_size(n):
    return lib().asterx_mlp_grad_workspace_size(n)


def mlp_grad(mlp, feat, target, grad, workspace, stream=None):
    _check(lib().asterx_mlp_grad(ctypes.byref(mlp), feat.shape[1], _ptr(feat), _ptr(target), _ptr(grad),
                                 _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream)))


def mlp_adam(params, grad, m, v, lr, beta1, beta2, eps, step, stream=None):
    _check(lib().asterx_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), float(lr), float(beta1), float(beta2),
                                 float(eps), int(step), _stream(stream)))


def c2p_points(params, gam, metric, Bt, cons, prim, guess=None, mlp=None, flags=None, iters=None, stats=None,
               stream=None):
    n = cons.shape[1]
    gp, _ = _gp(gam)
    p = make_params(params if gp is not None else dict(params, gamma=float(gam)))
    _check(lib().asterx_c2p_points(ctypes.byref(p), n, gp, _ptr(_f64(metric)), _ptr(_f64(Bt)), _ptr(_f64(cons)),
                                   _ptr(guess), None if mlp is None else ctypes.byref(mlp), _ptr(_f64(prim)),
                                   _ptr(flags), _ptr(iters), _ptr(stats), _stream(stream)))


def zero(buf, stream=None):
    _check(lib().asterx_zero(_ptr(buf), buf.numel(), _stream(stream)))


def timing_enable(on=True):
    lib().asterx_timing_enable(1 if on else 0)


def timing_reset():
    lib().asterx_timing_reset()


def timing_read():
    """{kernel name: (total ms, launches)} accumulated since the last reset (waits for the events)."""
    n = lib().asterx_timing_read(None, None, 0)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_longlong * n)()
    lib().asterx_timing_read(ms, cnt, n)
    return {lib().asterx_timing_name(k).decode(): (ms[k], cnt[k]) for k in range(n)}


# ---- a block advanced by whole RK steps (Sec. 3.12 workflow) ------------------------------------------------

class Block:
    """Device state of one block and the RK driver over the C ABI.

    Per stage: c2p (resets atmosphere cells of the stage input in place) -> ghost fill of
    the primitives -> right-hand side -> RK combine -> ghost fill of the new state.
    RK2 is Heun's method, RK4 the classical scheme (accumulator form).  With fused=True (the
    default) the right-hand side goes straight into the stage outputs (asterx_rhs_rk; RK4
    alternates two stage buffers so that no output is the state being evaluated); fused=False
    stores it and combines with asterx_rk_stage.  In the fused form the geometric sources are
    evaluated by the recovery kernel (asterx_c2p_src + asterx_rhs_rk_src) unless src_in_c2p is
    False (asterx_c2p + asterx_rhs_rk).  All give bitwise equal states."""

    def __init__(self, wl, device="cuda", fused=True, metric_fn=None, src_in_c2p=True):
        self.fused = fused
        self.src_in_c2p = fused and src_in_c2p
        # a time-dependent spacetime: metric_fn(t) -> (metric, curv) device tensors shaped like the
        # workload's, evaluated at every stage time (RK4: t, t + dt/2, t + dt/2, t + dt; RK2: t, t + dt)
        self.metric_fn = metric_fn
        self.t = 0.0
        self.wl = wl
        self.L = wl.layout
        self.params = wl.params
        dev = torch.device(device)
        t = lambda a: torch.from_numpy(a).to(dev)
        self.metric = t(wl.metric)
        self.curv = t(wl.curv)
        self.prim = t(wl.prim.copy())
        shape = (9,) + self.L.shape3
        self.state = torch.zeros(shape, dtype=torch.float64, device=dev)
        self.state[5:8] = t(wl.A)
        self.state[8] = t(wl.psi[0])
        self.tmp = torch.zeros_like(self.state)
        self.acc = torch.zeros_like(self.state)
        self.k = torch.zeros_like(self.state)
        self.tmp2 = torch.zeros_like(self.state) if fused and wl.rk == 4 else None
        self.ws = torch.empty(workspace_size(self.L) // 8, dtype=torch.float64, device=dev)
        self.src = torch.zeros((SRC_FIELDS,) + self.L.shape3, dtype=torch.float64, device=dev) if self.src_in_c2p else None
        self.red = torch.zeros(2, dtype=torch.float64, device=dev)
        self.stats = torch.zeros(6, dtype=torch.int64, device=dev)
        self.flags = torch.zeros(self.L.shape3, dtype=torch.uint8, device=dev)
        self.dt = wl.dt
        self.mlp = None  # an asterx_mlp (make_mlp) switches every stage's c2p to the learned guess
        prim2con(self.L, self.params, self.metric, self.state[5:8], self.prim, self.state[0:5])
        fill_ghosts(self.L, self.state[0:5], wl.bc_cell)

    def fill_state(self, U):
        if self.wl.A_shift is None and tuple(self.wl.bc_A) == tuple(self.wl.bc_cell):
            fill_ghosts(self.L, U, self.wl.bc_cell)  # all nine fields alike: one launch per axis
            return
        fill_ghosts(self.L, U[0:5], self.wl.bc_cell)
        if self.wl.A_shift is not None:
            fill_ghosts_shift(self.L, U[5:8], self.wl.A_shift)
        else:
            fill_ghosts(self.L, U[5:8], self.wl.bc_A)
        fill_ghosts(self.L, U[8:9], self.wl.bc_cell)

    def at_time(self, t):
        """Switch to the metric of time t when the spacetime is time dependent."""
        if self.metric_fn is not None:
            self.metric, self.curv = self.metric_fn(t)

    def recover(self, U):
        """c2p on U (in place for atmosphere cells) and the primitives' ghosts."""
        c2p(self.L, self.params, self.metric, U[5:8], U[0:5], self.prim, self.flags, self.stats, mlp=self.mlp)
        fill_ghosts(self.L, self.prim, self.wl.bc_cell)

    def eval_rhs(self, U, out):
        """c2p on U (in place for atmosphere cells), primitive ghosts, right-hand side into out."""
        self.recover(U)
        rhs(self.L, self.params, self.metric, self.curv, self.prim, U[5:8], U[8:9], self.dt, out, self.red,
            self.ws)

    def stage(self, U, outs):
        """c2p on U, then its right-hand side combined into outs = [(a, us, b_dt, out)]."""
        if self.src_in_c2p:
            c2p_src(self.L, self.params, self.metric, self.curv, U[5:8], U[0:5], self.prim, self.src, self.flags,
                    self.stats, mlp=self.mlp)
            fill_ghosts(self.L, self.prim, self.wl.bc_cell)
            rhs_rk_src(self.L, self.params, self.metric, self.prim, U[5:8], U[8:9], self.src, self.dt, outs,
                       self.red, self.ws)
            return
        self.recover(U)
        rhs_rk(self.L, self.params, self.metric, self.curv, self.prim, U[5:8], U[8:9], self.dt, outs, self.red,
               self.ws)

    def step(self):
        if self.fused:
            self._step_fused()
        else:
            self._step_stored()
        self.t += self.dt

    def _step_fused(self):
        dt, t = self.dt, self.t
        U0 = self.state
        if self.wl.rk == 2:
            U1 = self.tmp
            self.at_time(t)
            self.stage(U0, [([1.0], [U0], dt, U1)])
            self.fill_state(U1)
            self.at_time(t + dt)
            self.stage(U1, [([0.5, 0.5], [U0, U1], 0.5 * dt, U0)])
            self.fill_state(U0)
        else:
            Ua, Ub, acc = self.tmp, self.tmp2, self.acc
            self.at_time(t)
            self.stage(U0, [([1.0], [U0], dt / 6.0, acc), ([1.0], [U0], 0.5 * dt, Ua)])
            self.fill_state(Ua)
            self.at_time(t + 0.5 * dt)
            self.stage(Ua, [([1.0], [acc], dt / 3.0, acc), ([1.0], [U0], 0.5 * dt, Ub)])
            self.fill_state(Ub)
            self.stage(Ub, [([1.0], [acc], dt / 3.0, acc), ([1.0], [U0], dt, Ua)])
            self.fill_state(Ua)
            self.at_time(t + dt)
            self.stage(Ua, [([1.0], [acc], dt / 6.0, U0)])
            self.fill_state(U0)

    def _step_stored(self):
        dt, t = self.dt, self.t
        U0, K = self.state, self.k
        if self.wl.rk == 2:
            U1 = self.tmp
            self.at_time(t)
            self.eval_rhs(U0, K)
            rk_stage(self.L, [1.0], [U0], dt, K, U1)
            self.fill_state(U1)
            self.at_time(t + dt)
            self.eval_rhs(U1, K)
            rk_stage(self.L, [0.5, 0.5], [U0, U1], 0.5 * dt, K, U0)
            self.fill_state(U0)
        else:
            Ut, acc = self.tmp, self.acc
            self.at_time(t)
            self.eval_rhs(U0, K)
            rk_stage(self.L, [1.0], [U0], 0.5 * dt, K, Ut)
            rk_stage(self.L, [1.0], [U0], dt / 6.0, K, acc)
            self.fill_state(Ut)
            self.at_time(t + 0.5 * dt)
            self.eval_rhs(Ut, K)
            rk_stage(self.L, [1.0], [acc], dt / 3.0, K, acc)
            rk_stage(self.L, [1.0], [U0], 0.5 * dt, K, Ut)
            self.fill_state(Ut)
            self.eval_rhs(Ut, K)
            rk_stage(self.L, [1.0], [acc], dt / 3.0, K, acc)
            rk_stage(self.L, [1.0], [U0], dt, K, Ut)
            self.fill_state(Ut)
            self.at_time(t + dt)
            self.eval_rhs(Ut, K)
            rk_stage(self.L, [1.0], [acc], dt / 6.0, K, U0)
            self.fill_state(U0)

    def run(self, nsteps):
        for _ in range(nsteps):
            self.step()

    @property
    def stages_per_step(self):
        return 2 if self.wl.rk == 2 else 4


# ---- batches of patches (one persistent launch per phase for all patches) -----------------------------------

class Batch:
    """A set of patches advanced together through the asterx_batch_* entry points.

    Arrays are field-major pools of shape (nfields, points) with points = sum of the patches' padded
    sizes; patch p's field f is the slice [f, off[p] : off[p] + npts_p], laid out like a single block."""

    def __init__(self, workloads, tuning=(4, 1), device="cuda", fused=True):
        self.fused = fused
        self.wls = list(workloads)
        n = len(self.wls)
        grids = (Grid * n)(*[make_grid(w.layout) for w in self.wls])
        tun = BatchTuning(int(tuning[0]), int(tuning[1]))
        h = ctypes.c_void_p()
        _check(lib().asterx_batch_create(n, grids, ctypes.byref(tun), ctypes.byref(h)))
        self.h = h
        self.tuning = tuning
        self.ntot = lib().asterx_batch_points(h)
        self.off = [lib().asterx_batch_offset(h, p) for p in range(n)]
        w0 = self.wls[0]
        self.params = w0.params
        self.bc_cell, self.bc_A = w0.bc_cell, w0.bc_A
        self.dt = w0.dt
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        self.metric = self._pack([w.metric for w in self.wls], 10, dev)
        self.curv = self._pack([w.curv for w in self.wls], 6, dev)
        self.prim = self._pack([w.prim for w in self.wls], 5, dev)
        self.state = torch.zeros((9, self.ntot), **f64)
        self.state[5:8] = self._pack([w.A for w in self.wls], 3, dev)
        self.state[8:9] = self._pack([w.psi for w in self.wls], 1, dev)
        self.tmp = torch.zeros_like(self.state)
        self.k = torch.zeros_like(self.state)
        self.ws = torch.empty(lib().asterx_batch_workspace_size(h) // 8, **f64)
        self.red = torch.zeros(2, **f64)
        self.stats = torch.zeros(6, dtype=torch.int64, device=dev)
        self.flags = torch.zeros(self.ntot, dtype=torch.uint8, device=dev)
        self._call("asterx_batch_prim2con", self._P(), _ptr(self.metric), _ptr(self.state[5:8]), _ptr(self.prim),
                   _ptr(self.state[0:5]), _stream(None))
        self.fill(self.state[0:5], self.bc_cell)

    def _pack(self, arrays, nf, dev):
        import numpy as np
        out = np.zeros((nf, self.ntot))
        for a, o in zip(arrays, self.off):
            out[:, o:o + a[0].size] = a.reshape(nf, -1)
        return torch.from_numpy(out).to(dev)

    def unpack(self, pool, p):
        """Patch p's view of a pool as (nf, ld2, ld1, ld0)."""
        L = self.wls[p].layout
        o = self.off[p]
        return pool[:, o:o + L.npts].reshape((pool.shape[0],) + L.shape3)

    def _P(self):
        return ctypes.byref(make_params(self.params))

    def _call(self, name, *args):
        _check(getattr(lib(), name)(self.h, *args))

    def fill(self, f, kinds):
        karr = (ctypes.c_int32 * 3)(*[BC[k] if isinstance(k, str) else int(k) for k in kinds])
        self._call("asterx_batch_fill_ghosts", _ptr(f), f.shape[0], karr, _stream(None))

    def fill_state(self, U):
        self.fill(U[0:5], self.bc_cell)
        self.fill(U[5:8], self.bc_A)
        self.fill(U[8:9], self.bc_cell)

    def rk(self, a, us, b_dt, rhs_t, out):
        n = len(a)
        arr_a = (ctypes.c_double * n)(*[float(x) for x in a])
        arr_u = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
        self._call("asterx_batch_rk_stage", n, arr_a, arr_u, float(b_dt), _ptr(rhs_t), _ptr(out), _stream(None))

    def recover(self, U):
        self._call("asterx_batch_c2p", self._P(), _ptr(self.metric), _ptr(U[5:8]), _ptr(U[0:5]), _ptr(self.prim),
                   _ptr(self.flags), _ptr(self.stats), _stream(None))
        self.fill(self.prim, self.bc_cell)

    def eval_rhs(self, U, out):
        self.recover(U)
        self._call("asterx_batch_rhs", self._P(), _ptr(self.metric), _ptr(self.curv), _ptr(self.prim), _ptr(U[5:8]),
                   _ptr(U[8:9]), float(self.dt), _ptr(out), _ptr(self.red), _ptr(self.ws),
                   self.ws.numel() * 8, _stream(None))

    def stage(self, U, outs):
        self.recover(U)
        arr = make_rk_outs(outs)
        self._call("asterx_batch_rhs_rk", self._P(), _ptr(self.metric), _ptr(self.curv), _ptr(self.prim),
                   _ptr(U[5:8]), _ptr(U[8:9]), float(self.dt), len(outs), arr, _ptr(self.red), _ptr(self.ws),
                   self.ws.numel() * 8, _stream(None))

    def step(self):
        """One Heun (RK2) step of every patch (right-hand sides combined straight into the stage outputs)."""
        if not self.fused:
            return self._step_stored()
        U0, U1, dt = self.state, self.tmp, self.dt
        self.stage(U0, [([1.0], [U0], dt, U1)])
        self.fill_state(U1)
        self.stage(U1, [([0.5, 0.5], [U0, U1], 0.5 * dt, U0)])
        self.fill_state(U0)

    def _step_stored(self):
        U0, U1, K, dt = self.state, self.tmp, self.k, self.dt
        self.eval_rhs(U0, K)
        self.rk([1.0], [U0], dt, K, U1)
        self.fill_state(U1)
        self.eval_rhs(U1, K)
        self.rk([0.5, 0.5], [U0, U1], 0.5 * dt, K, U0)
        self.fill_state(U0)

    def run(self, nsteps):
        for _ in range(nsteps):
            self.step()

    @property
    def interior_cells(self):
        return sum(w.layout.n[0] * w.layout.n[1] * w.layout.n[2] for w in self.wls)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().asterx_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass
