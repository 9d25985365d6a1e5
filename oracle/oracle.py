"""ctypes binding of the serial FP64 CPU oracle (asterx_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU library never imports this module
and this module never imports the GPU library.

Arrays follow the padded index space of the oracle: numpy float64 arrays of
shape (nfields, ld[2], ld[1], ld[0]), C-contiguous; index (i, j, k) of the
paper's grid sits at [f, k + ng, j + ng, i + ng].
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "asterx_oracle.cpp")
LIB = os.path.join(HERE, "_build", "liboracle.so")
LIB_OMP = os.path.join(HERE, "_build", "liboracle_omp.so")

_c_double_p = ctypes.POINTER(ctypes.c_double)


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ng", ctypes.c_int32), ("ld", ctypes.c_int32 * 3),
                ("pad_", ctypes.c_int32), ("dx", ctypes.c_double * 3)]


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("rho_atm", ctypes.c_double), ("k_atm", ctypes.c_double),
                ("xi", ctypes.c_double), ("c2p_tol", ctypes.c_double), ("wmax", ctypes.c_double),
                ("weno_eps", ctypes.c_double), ("weno_q", ctypes.c_double),
                ("c2p_maxit", ctypes.c_int32), ("brent_maxit", ctypes.c_int32), ("recon", ctypes.c_int32),
                ("gauge", ctypes.c_int32), ("speeds", ctypes.c_int32), ("c2p_method", ctypes.c_int32),
                ("riemann", ctypes.c_int32), ("ct", ctypes.c_int32)]


RECON = {"minmod": 0, "ppm": 1, "wenoz": 2, "mp5": 3}
RIEMANN = {"hlle": 0, "lxf": 1}
CT = {"fct": 0, "uct": 1}
BC = {"periodic": 0, "copy": 1, "linear": 2}


FLAGS = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force=True, openmp=False):
    """Compile the oracle with g++ (FP64, no FP contraction, no fast-math): serial, or with -fopenmp (the
    all-core CPU baseline; bitwise the same results)."""
    out = LIB_OMP if openmp else LIB
    os.makedirs(os.path.dirname(out), exist_ok=True)
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    tmp = out + ".tmp"
    subprocess.check_call(FLAGS + (["-fopenmp"] if openmp else []) + ["-o", tmp, SRC])
    os.replace(tmp, out)
    return out


_lib = None
_lib_omp = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = ctypes.CDLL(LIB)
    return _lib


def lib_omp(threads=None):
    """The OpenMP build (loaded once); threads: number of OpenMP threads (default: all).  Returns (lib, threads)."""
    global _lib_omp
    if _lib_omp is None:
        build(force=False, openmp=True)
        _lib_omp = ctypes.CDLL(LIB_OMP)
    return _lib_omp, int(_lib_omp.orc_set_threads(ctypes.c_int(int(threads or 0))))


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(_c_double_p)


def make_grid(layout):
    g = Grid()
    for d in range(3):
        g.n[d] = int(layout.n[d])
        g.ld[d] = int(layout.ld[d])
        g.dx[d] = float(layout.dx[d])
    g.ng = int(layout.ng)
    return g


def make_params(p):
    """p: dict of method parameters (see paper_2406_11669_amd.workloads.default_params)."""
    P = Params()
    P.gamma = p["gamma"]
    P.rho_atm = p["rho_atm"]
    P.k_atm = p["k_atm"]
    P.xi = p["xi"]
    P.c2p_tol = p["c2p_tol"]
    P.wmax = p["wmax"]
    P.weno_eps = p["weno_eps"]
    P.weno_q = p["weno_q"]
    P.c2p_maxit = p["c2p_maxit"]
    P.brent_maxit = p["brent_maxit"]
    P.recon = RECON[p["recon"]] if isinstance(p["recon"], str) else p["recon"]
    P.gauge = {"lorenz": 0, "algebraic": 1}[p["gauge"]] if isinstance(p["gauge"], str) else p["gauge"]
    P.speeds = {"quartic": 0, "bound": 1}[p["speeds"]] if isinstance(p["speeds"], str) else p["speeds"]
    P.c2p_method = p.get("c2p_method", 0)
    r = p.get("riemann", "hlle")
    P.riemann = RIEMANN[r] if isinstance(r, str) else r
    c = p.get("ct", "fct")
    P.ct = CT[c] if isinstance(c, str) else c
    return P


def _check_ct(layout, params):
    """Upwind CT reconstructs face values three faces beyond the edge, whose face metric reaches the
    fourth vertex layer: it needs ng >= 4."""
    if params.get("ct", "fct") in ("uct", 1) and layout.ng < 4:
        raise ValueError("upwind CT needs ng >= 4")


def prim2con(layout, params, metric, A, prim):
    cons = np.zeros((5,) + layout.shape3, dtype=np.float64)
    lib().orc_prim2con(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)), _p(metric), _p(A),
                       _p(prim), _p(cons))
    return cons


def c2p(layout, params, metric, A, cons, prim):
    """In place: cons (atmosphere reset) and prim (warm start in, result out).  Returns (flags, stats)."""
    flags = np.zeros(layout.shape3, dtype=np.uint8)
    stats = np.zeros(6, dtype=np.uint64)
    lib().orc_c2p(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)), _p(metric), _p(A), _p(cons),
                  _p(prim), flags.ctypes.data_as(ctypes.c_void_p), stats.ctypes.data_as(ctypes.c_void_p))
    return flags, stats


def fill_ghosts_shift(layout, f, shift):
    """Periodic fill of f (nf <= 3 fields) with shift[q, d] added per period of wrap along axis d."""
    nf = f.shape[0] if f.ndim == 4 else 1
    sh = np.ascontiguousarray(np.asarray(shift, dtype=np.float64)[:nf])
    lib().orc_fill_ghosts_shift(ctypes.byref(make_grid(layout)), _p(f), ctypes.c_int(nf), _p(sh))


def _bc_kinds(layout, kinds):
    """Boundary kinds as integers; linear extrapolation needs two owned points along its axis."""
    kinds = [BC[k] if isinstance(k, str) else k for k in kinds]
    for a in range(3):
        if kinds[a] == BC["linear"] and layout.n[a] < 2:
            raise ValueError("linear ghost extrapolation needs n >= 2 along axis %d" % a)
    return (ctypes.c_int * 3)(*kinds)


def fill_ghosts(layout, f, kinds):
    karr = _bc_kinds(layout, kinds)
    nf = f.shape[0] if f.ndim == 4 else 1
    lib().orc_fill_ghosts(ctypes.byref(make_grid(layout)), _p(f), ctypes.c_int(nf), karr)


def tmunu(layout, params, metric, prim, A):
    """T_{mu nu} at the vertices [0, n]^3 (10 fields: 00, 0x, 0y, 0z, xx, xy, xz, yy, yz, zz)."""
    out = np.zeros((10,) + layout.shape3, dtype=np.float64)
    lib().orc_tmunu(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)), _p(metric), _p(prim),
                    _p(A), _p(out))
    return out


STAG = {"cell": (0, 0, 0), "vertex": (1, 1, 1), "xedge": (0, 1, 1), "yedge": (1, 0, 1), "zedge": (1, 1, 0)}


def _i3(v):
    return (ctypes.c_int * 3)(*[int(x) for x in v])


def prolong(coarse, fine, c0, stag, cf, ff, lo, hi):
    """Fill fine points [lo, hi] (fine indices, inclusive) of ff (nf fields) from cf; fine vertex 0 on coarse vertex
    c0; stag: per-axis 0 cell / 1 vertex, or a name of STAG."""
    stag = STAG[stag] if isinstance(stag, str) else stag
    nf = cf.shape[0]
    lib().orc_prolong(ctypes.byref(make_grid(coarse)), ctypes.byref(make_grid(fine)), _i3(c0), _i3(stag),
                      ctypes.c_int(nf), _p(cf), _p(ff), _i3(lo), _i3(hi))


def restrict(coarse, fine, c0, stag, ff, cf, lo, hi):
    """Fill coarse points [lo, hi] (coarse indices) of cf from ff."""
    stag = STAG[stag] if isinstance(stag, str) else stag
    nf = ff.shape[0]
    lib().orc_restrict(ctypes.byref(make_grid(coarse)), ctypes.byref(make_grid(fine)), _i3(c0), _i3(stag),
                       ctypes.c_int(nf), _p(ff), _p(cf), _i3(lo), _i3(hi))


def rhs(layout, params, metric, curv, prim, A, psi, dt_max):
    _check_ct(layout, params)
    out = np.zeros((9,) + layout.shape3, dtype=np.float64)
    red = np.zeros(2, dtype=np.float64)
    nfix = ctypes.c_longlong(0)
    lib().orc_rhs(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)), _p(metric), _p(curv),
                  _p(prim), _p(A), _p(psi), ctypes.c_double(dt_max), _p(out), _p(red), ctypes.byref(nfix))
    return out, red, nfix.value


def tie_counts(reset=True):
    """PPM monotonicity-constraint decisions of the serial oracle since the last reset: (all, near ties: sides
    that differ but agree to 1e-12 of their magnitude, where another valid rounding order can take the other,
    discontinuous branch)."""
    out = np.zeros(2, dtype=np.uint64)
    lib().orc_tie_counts(out.ctypes.data_as(ctypes.c_void_p), ctypes.c_int(1 if reset else 0))
    return int(out[0]), int(out[1])


def rk_stage(layout, a, us, b_dt, rhs_arr, out):
    n = len(a)
    arr_a = (ctypes.c_double * n)(*a)
    ptrs = (_c_double_p * n)(*[_p(u) for u in us])
    lib().orc_rk_stage(ctypes.byref(make_grid(layout)), ctypes.c_int(n), arr_a, ptrs, ctypes.c_double(b_dt),
                       _p(rhs_arr), _p(out))


def run(layout, params, metric, curv, state, prim, dt, nsteps, rk, bc_cell, bc_A, A_shift=None, lib_=None):
    """Advance state (9 fields) and prim in place by nsteps.  Returns (flags, stats, redmax).
    A_shift (3x3, optional): periodic fill of A with A_shift[q, d] added per period along axis d.
    lib_: the library to run (default: the serial build; lib_omp()[0] for the OpenMP build)."""
    _check_ct(layout, params)
    flags = np.zeros(layout.shape3, dtype=np.uint8)
    stats = np.zeros(6, dtype=np.uint64)
    redmax = np.zeros(2, dtype=np.float64)
    bcc = _bc_kinds(layout, bc_cell)
    bca = _bc_kinds(layout, bc_A)
    sh = None if A_shift is None else np.ascontiguousarray(A_shift, dtype=np.float64)
    (lib_ or lib()).orc_run(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)), _p(metric),
                            _p(curv), _p(state), _p(prim), ctypes.c_double(dt), ctypes.c_int(nsteps),
                            ctypes.c_int(rk), bcc, bca, flags.ctypes.data_as(ctypes.c_void_p),
                            stats.ctypes.data_as(ctypes.c_void_p), _p(redmax), None if sh is None else _p(sh))
    return flags, stats, redmax


def count_ops(layout, params, metric, curv, prim, A, psi, dt_max):
    """Algorithmic FP64 operation counts of one right-hand side and one c2p on this block:
    dict(centre_B, faces, cells, ct, c2p) in operations (each +, -, *, /, sqrt, pow counts one)."""
    _check_ct(layout, params)
    out = np.zeros(5, dtype=np.uint64)
    lib().orc_count_ops(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)), _p(metric), _p(curv),
                        _p(prim), _p(A), _p(psi), ctypes.c_double(dt_max), out.ctypes.data_as(ctypes.c_void_p))
    return dict(zip(["centre_B", "faces", "cells", "ct", "c2p"], [int(v) for v in out]))


def count_probe():
    """Operation counts of single building blocks on the counting scalar: dict(lag_value, lag_deriv,
    face_interp, centre_value, centre_interp, face_B, centre_B, make_geom, mixed_expression)."""
    out = np.zeros(9, dtype=np.uint64)
    lib().orc_count_probe(out.ctypes.data_as(ctypes.c_void_p))
    return dict(zip(["lag_value", "lag_deriv", "face_interp", "centre_value", "centre_interp", "face_B", "centre_B",
                     "make_geom", "mixed_expression"], [int(v) for v in out]))


def count_c2p_point(params, m10, cons5, Bt3, prev5):
    """Operations of one point recovery on the counting scalar.  Returns (ops, iterations)."""
    it = ctypes.c_int(0)
    f = lib().orc_count_c2p_point
    f.restype = ctypes.c_ulonglong
    ops = f(ctypes.byref(make_params(params)), _p(_v(m10, 10)), _p(_v(cons5, 5)), _p(_v(Bt3, 3)), _p(_v(prev5, 5)),
            ctypes.byref(it))
    return int(ops), it.value


def face_B(layout, A):
    out = np.zeros((3,) + layout.shape3, dtype=np.float64)
    lib().orc_face_B(ctypes.byref(make_grid(layout)), _p(A), _p(out))
    return out


def centre_metric(layout, metric):
    out = np.zeros((40,) + layout.shape3, dtype=np.float64)
    lib().orc_centre_metric(ctypes.byref(make_grid(layout)), _p(metric), _p(out))
    return out


def face_interp(layout, f, d):
    out = np.zeros(layout.shape3, dtype=np.float64)
    lib().orc_face_interp(ctypes.byref(make_grid(layout)), _p(np.ascontiguousarray(f)), ctypes.c_int(d), _p(out))
    return out


# ---- pointwise helpers -------------------------------------------------------------------------------------

def _v(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def pt_prim2con(m10, prim5, Bt3, gam):
    out = np.zeros(5)
    lib().orc_pt_prim2con(_p(_v(m10, 10)), _p(_v(prim5, 5)), _p(_v(Bt3, 3)), ctypes.c_double(gam), _p(out))
    return out


def pt_fluid(m10, prim5, Bt3, gam):
    out = np.zeros(13)
    lib().orc_pt_fluid(_p(_v(m10, 10)), _p(_v(prim5, 5)), _p(_v(Bt3, 3)), ctypes.c_double(gam), _p(out))
    keys = ["W", "b0", "bx", "by", "bz", "bsq", "u0", "ux", "uy", "uz", "h", "eps", "v2"]
    return dict(zip(keys, out))


def pt_flux(m10, prim5, Bt3, gam, d):
    U = np.zeros(7)
    F = np.zeros(7)
    lib().orc_pt_flux(_p(_v(m10, 10)), _p(_v(prim5, 5)), _p(_v(Bt3, 3)), ctypes.c_double(gam), ctypes.c_int(d),
                      _p(U), _p(F))
    return U, F


def pt_speeds(m10, prim5, Bt3, gam, d):
    """(c-, c+, bound-, bound+)"""
    out = np.zeros(4)
    lib().orc_pt_speeds(_p(_v(m10, 10)), _p(_v(prim5, 5)), _p(_v(Bt3, 3)), ctypes.c_double(gam), ctypes.c_int(d),
                        _p(out))
    return out


def pt_quartic_eval(m10, prim5, Bt3, gam, d, lam):
    lam = _v(lam)
    q = np.zeros(lam.size)
    lib().orc_pt_quartic_eval(_p(_v(m10, 10)), _p(_v(prim5, 5)), _p(_v(Bt3, 3)), ctypes.c_double(gam),
                              ctypes.c_int(d), ctypes.c_int(lam.size), _p(lam), _p(q))
    return q


def pt_hlle(UL, FL, cmL, cpL, UR, FR, cmR, cpR):
    out = np.zeros(7)
    lib().orc_pt_hlle(_p(_v(UL, 7)), _p(_v(FL, 7)), ctypes.c_double(cmL), ctypes.c_double(cpL), _p(_v(UR, 7)),
                      _p(_v(FR, 7)), ctypes.c_double(cmR), ctypes.c_double(cpR), _p(out))
    return out


def pt_lxf(UL, FL, cmL, cpL, UR, FR, cmR, cpR):
    out = np.zeros(7)
    lib().orc_pt_lxf(_p(_v(UL, 7)), _p(_v(FL, 7)), ctypes.c_double(cmL), ctypes.c_double(cpL), _p(_v(UR, 7)),
                     _p(_v(FR, 7)), ctypes.c_double(cmR), ctypes.c_double(cpR), _p(out))
    return out


def recon_1d(params, kind, a):
    a = _v(a)
    aL = np.full(a.size, np.nan)
    aR = np.full(a.size, np.nan)
    k = RECON[kind] if isinstance(kind, str) else kind
    lib().orc_recon_1d(ctypes.byref(make_params(params)), ctypes.c_int(k), ctypes.c_int(a.size), _p(a), _p(aL),
                       _p(aR))
    return aL, aR


def pt_c2p(params, m10, cons5, Bt3, prev5):
    """Returns (prim5, flags, iters, cons5_after)."""
    cons = _v(cons5, 5).copy()
    prim = np.zeros(5)
    it = ctypes.c_int(0)
    fl = lib().orc_pt_c2p(ctypes.byref(make_params(params)), _p(_v(m10, 10)), _p(cons), _p(_v(Bt3, 3)),
                          _p(_v(prev5, 5)), _p(prim), ctypes.byref(it))
    return prim, fl, it.value, cons


def pt_noble_residual(m10, cons5, Bt3, gam, z, w):
    R = np.zeros(2)
    J = np.zeros(4)
    lib().orc_pt_noble_residual(_p(_v(m10, 10)), _p(_v(cons5, 5)), _p(_v(Bt3, 3)), ctypes.c_double(gam),
                                ctypes.c_double(z), ctypes.c_double(w), _p(R), _p(J))
    return R, J.reshape(2, 2)


def pt_palen(m10, cons5, Bt3, gam, wmax, x):
    x = _v(x)
    f = np.zeros(x.size)
    br = np.zeros(2)
    lib().orc_pt_palen(_p(_v(m10, 10)), _p(_v(cons5, 5)), _p(_v(Bt3, 3)), ctypes.c_double(gam),
                       ctypes.c_double(wmax), ctypes.c_int(x.size), _p(x), _p(f), _p(br))
    return f, br


def pt_sources(m10, dm30, K6, prim5, Bt3, gam):
    out = np.zeros(5)
    lib().orc_pt_sources(_p(_v(m10, 10)), _p(_v(dm30, 30)), _p(_v(K6, 6)), _p(_v(prim5, 5)), _p(_v(Bt3, 3)),
                         ctypes.c_double(gam), _p(out))
    return out


def pt_tmunu(m10, prim5, Bt3, gam):
    out = np.zeros(16)
    lib().orc_pt_tmunu(_p(_v(m10, 10)), _p(_v(prim5, 5)), _p(_v(Bt3, 3)), ctypes.c_double(gam), _p(out))
    return out.reshape(4, 4)


def loss_jvp(layout, params, metric, curv, prim0, A0, psi0, dt, nsteps, rk, bc_cell, bc_A, dprim0=None, dgamma=0.0,
             A_shift=None):
    """Loss (sum over owned cells of rho^2 dV)^(1/2) after nsteps from prim0, and its directional derivative
    along (dprim0, dgamma), by forward-mode dual numbers through the whole run.  Returns (loss, jvp, stats)."""
    _check_ct(layout, params)
    out = np.zeros(2, dtype=np.float64)
    stats = np.zeros(6, dtype=np.uint64)
    bcc = _bc_kinds(layout, bc_cell)
    bca = _bc_kinds(layout, bc_A)
    sh = None if A_shift is None else np.ascontiguousarray(A_shift, dtype=np.float64)
    dp = None if dprim0 is None else np.ascontiguousarray(dprim0, dtype=np.float64)
    lib().orc_loss_jvp(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)), ctypes.c_double(dgamma),
                       _p(metric), _p(curv), _p(np.ascontiguousarray(prim0)), None if dp is None else _p(dp),
                       _p(A0), _p(psi0), ctypes.c_double(dt), ctypes.c_int(nsteps), ctypes.c_int(rk), bcc, bca,
                       None if sh is None else _p(sh), _p(out), stats.ctypes.data_as(ctypes.c_void_p))
    return float(out[0]), float(out[1]), stats


def _opt(a):
    return None if a is None else _p(np.ascontiguousarray(a, dtype=np.float64))


def prim2con_jvp(layout, params, metric, A, prim, dA=None, dprim=None, dgamma=0.0):
    """(cons, dcons) of prim2con along the tangent (dprim, dA, dgamma); owned points."""
    cons = np.zeros((5,) + layout.shape3)
    dcons = np.zeros_like(cons)
    keep = [np.ascontiguousarray(x, dtype=np.float64) if x is not None else None for x in (dA, dprim)]
    lib().orc_prim2con_jvp(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)),
                           ctypes.c_double(dgamma), _p(metric), _p(A), _opt(keep[0]), _p(prim), _opt(keep[1]),
                           _p(cons), _p(dcons))
    return cons, dcons


def c2p_jvp(layout, params, metric, A, cons, guess, dA=None, dcons=None, dgamma=0.0):
    """(prim, dprim) of c2p (warm start guess) along the tangent (dcons, dA, dgamma); owned points."""
    prim = np.zeros((5,) + layout.shape3)
    dprim = np.zeros_like(prim)
    keep = [np.ascontiguousarray(x, dtype=np.float64) if x is not None else None for x in (dA, dcons)]
    lib().orc_c2p_jvp(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)), ctypes.c_double(dgamma),
                      _p(metric), _p(A), _opt(keep[0]), _p(np.ascontiguousarray(cons)), _opt(keep[1]),
                      _p(np.ascontiguousarray(guess)), _p(prim), _p(dprim))
    return prim, dprim


def stage_jvp(layout, params, metric, curv, cons, A, psi, guess, dt_max, dcons=None, dA=None, dpsi=None,
              dgamma=0.0):
    """(L, dL) of one stage's right-hand side rhs(fill(c2p(cons, A)), A, psi) along the tangent; owned points."""
    _check_ct(layout, params)
    out = np.zeros((9,) + layout.shape3)
    dout = np.zeros_like(out)
    keep = [np.ascontiguousarray(x, dtype=np.float64) if x is not None else None for x in (dcons, dA, dpsi)]
    lib().orc_stage_jvp(ctypes.byref(make_grid(layout)), ctypes.byref(make_params(params)), ctypes.c_double(dgamma),
                        _p(metric), _p(curv), _p(np.ascontiguousarray(cons)), _opt(keep[0]),
                        _p(np.ascontiguousarray(A)), _opt(keep[1]), _p(np.ascontiguousarray(psi)), _opt(keep[2]),
                        _p(np.ascontiguousarray(guess)), ctypes.c_double(dt_max), _p(out), _p(dout))
    return out, dout
