"""Seeded synthetic inputs: grid layout and initial data for the benchmark workloads.

This module holds no arithmetic of the method itself: it lays out arrays and
fills them with seeded analytic data (mode sums, piecewise-constant states,
their vector potentials and the extrinsic curvature of a static metric).  The
conserved variables are NOT computed here; each side (GPU library, CPU oracle)
maps these primitives to conserved variables with its own code.

Index space (shared by every array): padded extents ld[0] x ld[1] x ld[2],
x fastest; index (i, j, k) with owned range 0..n-1 and ghosts down to -ng and
up to n+ng is stored at [.., k+ng, j+ng, i+ng].  Positions: cell centre
((i+1/2)dx, (j+1/2)dy, (k+1/2)dz); vertex (i dx, j dy, k dz); x-edge
((i+1/2)dx, j dy, k dz), y-edge (i dx, (j+1/2)dy, k dz), z-edge (i dx, j dy,
(k+1/2)dz).

Workloads (one block, one GPU):
  riemann32  -- 32^3 + 3 ghosts, flat metric, Gamma = 5/3, seeded Riemann
                problem split at x = 1/2, MINMOD, HLLE, Noble c2p, RK2, CFL 0.25.
  curved128  -- 128^3 periodic block in a static curved metric (low-k mode
                sums), Gamma = 2, PPM or WENO-Z, RK4, CFL 0.25.
  periodic_riemann64 -- the Riemann states on a 64^3 periodic box (interfaces
                at x = 1/2 and at the wrap), flat, PPM, RK2, 20 steps, Gamma = 5/3;
                the vector potential is periodic up to a constant per wrap.
  patch_set  -- 512 Riemann-problem patches of uneven sides and levels.
  shock_tube -- an unmagnetized one-dimensional Riemann problem (tests against
                the exact solution of relativistic hydrodynamics).
All are also available at other sizes for tests.
"""
from dataclasses import dataclass, field

import numpy as np

NG_DEFAULT = 3


@dataclass
class Layout:
    n: tuple
    ng: int = NG_DEFAULT
    dx: tuple = None
    xpad: int = 8
    ld: tuple = field(init=False)

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        if self.dx is None:
            self.dx = tuple(1.0 / v for v in self.n)
        self.dx = tuple(float(v) for v in self.dx)
        ext = [v + 2 * self.ng + 1 for v in self.n]
        ext[0] = -(-ext[0] // self.xpad) * self.xpad
        self.ld = tuple(ext)

    @property
    def shape3(self):
        return (self.ld[2], self.ld[1], self.ld[0])

    @property
    def npts(self):
        return self.ld[0] * self.ld[1] * self.ld[2]

    def zeros(self, nf):
        return np.zeros((nf,) + self.shape3, dtype=np.float64)

    def owned(self, a):
        """View of the owned index range 0..n-1 of an array (..., ld2, ld1, ld0)."""
        g = self.ng
        return a[..., g:g + self.n[2], g:g + self.n[1], g:g + self.n[0]]

    def coords(self, where):
        """Coordinates (x, y, z) of every stored point, broadcastable to shape3.

        where: 'centre', 'vertex', 'xedge', 'yedge', 'zedge'."""
        g = self.ng
        off = {"centre": (0.5, 0.5, 0.5), "vertex": (0.0, 0.0, 0.0), "xedge": (0.5, 0.0, 0.0),
               "yedge": (0.0, 0.5, 0.0), "zedge": (0.0, 0.0, 0.5)}[where]
        x = (np.arange(self.ld[0]) - g + off[0]) * self.dx[0]
        y = (np.arange(self.ld[1]) - g + off[1]) * self.dx[1]
        z = (np.arange(self.ld[2]) - g + off[2]) * self.dx[2]
        return x[None, None, :], y[None, :, None], z[:, None, None]

    def periodic_wrap(self, a):
        """Fill every ghost point of a (..., ld2, ld1, ld0) array from its periodic image (in place)."""
        g = self.ng
        for ax, d in ((-1, 0), (-2, 1), (-3, 2)):
            n = self.n[d]
            L = a.shape[ax]
            idx = (np.arange(L) - g) % n + g
            a[...] = np.take(a, idx, axis=ax)
        return a


def default_params(**kw):
    p = dict(gamma=5.0 / 3.0, rho_atm=1e-10, k_atm=1.0, xi=1.5, c2p_tol=1e-14, wmax=1e3, weno_eps=1e-40,
             weno_q=1.0, c2p_maxit=50, brent_maxit=100, recon="minmod", gauge="lorenz", speeds="quartic",
             c2p_method=0, riemann="hlle", ct="fct")
    p.update(kw)
    return p


# ---- mode sums --------------------------------------------------------------------------------------------

class ModeSum:
    """f(x) = sum_m a_m sin(2 pi k_m . x + phi_m) / sum_m |a_m|, k_m in {-2..2}^3 minus 0.

    |f| <= 1 and f is periodic on the unit cube."""

    def __init__(self, seed, tag, nmodes=4):
        rng = np.random.default_rng([int(seed), int(tag)])
        ks = []
        while len(ks) < nmodes:
            k = rng.integers(-2, 3, size=3)
            if np.any(k != 0):
                ks.append(k)
        self.k = np.array(ks, dtype=np.float64)
        self.phi = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
        self.a = rng.uniform(-1.0, 1.0, size=nmodes)
        self.norm = np.sum(np.abs(self.a))

    def __call__(self, x, y, z):
        out = 0.0
        for m in range(len(self.a)):
            ph = 2.0 * np.pi * (self.k[m, 0] * x + self.k[m, 1] * y + self.k[m, 2] * z) + self.phi[m]
            out = out + self.a[m] * np.sin(ph)
        return out / self.norm

    def grad(self, x, y, z):
        g = [0.0, 0.0, 0.0]
        for m in range(len(self.a)):
            ph = 2.0 * np.pi * (self.k[m, 0] * x + self.k[m, 1] * y + self.k[m, 2] * z) + self.phi[m]
            c = self.a[m] * np.cos(ph) * 2.0 * np.pi
            for d in range(3):
                g[d] = g[d] + c * self.k[m, d]
        return [gd / self.norm for gd in g]


# ---- the Riemann-problem block (flat metric) -------------------------------------------------------------

@dataclass
class Workload:
    name: str
    layout: Layout
    params: dict
    metric: np.ndarray   # [10] vertex: alpha, beta^x..z, gxx, gxy, gxz, gyy, gyz, gzz
    curv: np.ndarray     # [6] vertex: Kxx, Kxy, Kxz, Kyy, Kyz, Kzz
    prim: np.ndarray     # [5] centre: rho, p, v^x, v^y, v^z
    A: np.ndarray        # [3] edges
    psi: np.ndarray      # [1] vertex
    dt: float
    nsteps: int
    rk: int
    bc_cell: tuple
    bc_A: tuple
    info: dict = field(default_factory=dict)
    A_shift: np.ndarray = None  # (3, 3): A_q gains A_shift[q, d] per period of wrap along axis d

    def state(self, cons):
        """9-field state array (Dt, St_x, St_y, St_z, taut, A_x, A_y, A_z, Psi) from conserved variables."""
        s = self.layout.zeros(9)
        s[0:5] = cons
        s[5:8] = self.A
        s[8] = self.psi[0]
        return s


def flat_metric(layout):
    m = layout.zeros(10)
    m[0] = 1.0
    m[4] = 1.0
    m[7] = 1.0
    m[9] = 1.0
    return m


def riemann_block(seed=0, n=32, ng=NG_DEFAULT, recon="minmod", nsteps=10, rk=2, cfl=0.25, gamma=5.0 / 3.0,
                  split=0.5, dx=None, origin=(0.0, 0.0, 0.0)):
    """Seeded relativistic MHD Riemann problem on origin + [0, n dx]^3 (dx = 1/n by default), split on the vertex
    plane x = split (coordinates include the origin, so blocks of one seed at different origins and spacings
    sample one global state and one global potential).

    Left/right: rho, p ~ U[0.1, 1], v = 0, B^x ~ U[-1, 1] shared, B^y, B^z ~ U[-1, 1] per side.
    The edge potential A = (0, int_0^x B^z dx', B^x y - int_0^x B^y dx') reproduces the
    piecewise-constant face field exactly under the discrete curl."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    L = Layout(nn, ng, dx=None if dx is None else (dx, dx, dx))
    ox, oy, oz = (float(v) for v in origin)
    rng = np.random.default_rng(int(seed))
    rhoL, rhoR = rng.uniform(0.1, 1.0, 2)
    pL, pR = rng.uniform(0.1, 1.0, 2)
    Bx = rng.uniform(-1.0, 1.0)
    ByL, BzL, ByR, BzR = rng.uniform(-1.0, 1.0, 4)
    metric = flat_metric(L)
    curv = L.zeros(6)
    prim = L.zeros(5)
    xc, _, _ = L.coords("centre")
    left = np.broadcast_to(xc + ox < split, L.shape3)
    prim[0] = np.where(left, rhoL, rhoR)
    prim[1] = np.where(left, pL, pR)

    def int_B(x, bl, br):
        return np.where(x < split, bl * x, bl * split + br * (x - split))

    A = L.zeros(3)
    xy, yy, zy = L.coords("yedge")
    A[1] = np.broadcast_to(int_B(xy + ox, BzL, BzR) + 0.0 * yy + 0.0 * zy, L.shape3)
    xz, yz, zz = L.coords("zedge")
    A[2] = np.broadcast_to(Bx * (yz + oy) - int_B(xz + ox, ByL, ByR) + 0.0 * zz, L.shape3)
    psi = L.zeros(1)
    rho_max = max(rhoL, rhoR)
    params = default_params(gamma=gamma, rho_atm=1e-7 * rho_max, recon=recon)
    dt = cfl * min(L.dx)
    info = dict(rhoL=rhoL, rhoR=rhoR, pL=pL, pR=pR, Bx=Bx, ByL=ByL, BzL=BzL, ByR=ByR, BzR=BzR, seed=seed)
    return Workload("riemann%d" % nn[0], L, params, metric, curv, prim, A, psi, dt, nsteps, rk,
                    ("copy",) * 3, ("linear",) * 3, info)


def periodic_riemann_box(seed=0, n=64, ng=NG_DEFAULT, recon="ppm", nsteps=20, rk=2, cfl=0.25, gamma=5.0 / 3.0,
                         v_amp=0.0):
    """The seeded Riemann-problem states of riemann_block on a periodic unit box: interfaces on the vertex
    planes x = 1/2 and x = 0 (the wrap).  Flat metric.

    The face field is B = Bbar + dB with Bbar the box mean and dB a zero-mean square wave in x.  The potential
    is A = Bbar x r / 2 + A_per with A_per the periodic sawtooth potential of dB, so A is periodic up to the
    constant Bbar x (L e_d) / 2 per period along axis d (kept in A_shift).  v_amp > 0 adds a seeded smooth
    velocity field of that maximum component (default 0: fluid at rest, as in the Riemann problem)."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    L = Layout(nn, ng)
    rng = np.random.default_rng(int(seed))
    rhoL, rhoR = rng.uniform(0.1, 1.0, 2)
    pL, pR = rng.uniform(0.1, 1.0, 2)
    Bx = rng.uniform(-1.0, 1.0)
    ByL, BzL, ByR, BzR = rng.uniform(-1.0, 1.0, 4)
    metric = flat_metric(L)
    curv = L.zeros(6)
    prim = L.zeros(5)
    xc, yc, zc = L.coords("centre")
    left = np.broadcast_to(np.mod(xc, 1.0) < 0.5, L.shape3)
    prim[0] = np.where(left, rhoL, rhoR)
    prim[1] = np.where(left, pL, pR)
    if v_amp > 0.0:
        for c, nm in enumerate(("vx", "vy", "vz")):
            prim[2 + c] = v_amp * np.broadcast_to(ModeSum(seed, 100 + _TAGS[nm])(xc, yc, zc), L.shape3)
    Bbar = np.array([Bx, 0.5 * (ByL + ByR), 0.5 * (BzL + BzR)])
    hy, hz = 0.5 * (ByL - ByR), 0.5 * (BzL - BzR)

    def saw(x, h):
        # integral from 0 of the square wave (+h on [0, 1/2), -h on [1/2, 1)), periodic with period 1
        xm = np.mod(x, 1.0)
        return np.where(xm < 0.5, h * xm, h * (1.0 - xm))

    A = L.zeros(3)
    x, y, z = L.coords("xedge")
    A[0] = np.broadcast_to(0.5 * (Bbar[1] * z - Bbar[2] * y) + 0.0 * x, L.shape3)
    x, y, z = L.coords("yedge")
    A[1] = np.broadcast_to(0.5 * (Bbar[2] * x - Bbar[0] * z) + saw(x, hz) + 0.0 * y, L.shape3)
    x, y, z = L.coords("zedge")
    A[2] = np.broadcast_to(0.5 * (Bbar[0] * y - Bbar[1] * x) - saw(x, hy) + 0.0 * z, L.shape3)
    ext = [nn[d] * L.dx[d] for d in range(3)]
    shift = np.zeros((3, 3))
    for d in range(3):
        e = np.zeros(3)
        e[d] = ext[d]
        shift[:, d] = 0.5 * np.cross(Bbar, e)
    psi = L.zeros(1)
    params = default_params(gamma=gamma, rho_atm=1e-7 * max(rhoL, rhoR), recon=recon)
    dt = cfl * min(L.dx)
    info = dict(rhoL=rhoL, rhoR=rhoR, pL=pL, pR=pR, Bx=Bx, ByL=ByL, BzL=BzL, ByR=ByR, BzR=BzR, seed=seed,
                v_amp=v_amp)
    return Workload("periodic_riemann%d" % nn[0], L, params, metric, curv, prim, A, psi, dt, nsteps, rk,
                    ("periodic",) * 3, ("periodic",) * 3, info, shift)


def shock_tube(left, right, n=200, axis=0, ng=NG_DEFAULT, recon="ppm", t_end=0.35, rk=2, cfl=0.25,
               gamma=5.0 / 3.0, split=0.5, Bn=0.0, Bt=None, frame=None):
    """One-dimensional Riemann problem along `axis` on [0, 1] (n cells, spacing 1/n on every axis), flat
    metric, copy boundaries for the cell fields.  left/right = (rho, p, v) with v along `axis`; the interface
    is the vertex plane at `split`.  dt = t_end / nsteps with nsteps the smallest count whose step is at most
    cfl dx, so that nsteps steps end exactly at t_end.

    No field (Bn = 0, Bt None): one cell across the other two axes, zero potential (copied into the ghosts).
    Bn: a uniform field along `axis`.  Bt = (left, right): a field along the first transverse axis t1 =
    (axis + 1) % 3, piecewise constant like the fluid.  With a field, two cells across the other axes and
    the potential's component along t2 = (axis + 2) % 3 is Bn x_t1 - int_0^x B^t1 dx (x along `axis`),
    filled linearly.

    frame = (alpha, beta, g): a constant lapse, shift component along `axis` and metric component g_aa
    (flat spacetime in coordinates that move and stretch along the tube; the other components flat).  The
    velocity given is then the contravariant component v^a."""
    t1, t2 = (axis + 1) % 3, (axis + 2) % 3
    magnetized = Bn != 0.0 or Bt is not None
    nn = [2, 2, 2] if magnetized else [1, 1, 1]
    nn[axis] = int(n)
    dx = 1.0 / n
    L = Layout(tuple(nn), ng, dx=(dx, dx, dx))
    metric = flat_metric(L)
    if frame is not None:
        metric[0] = frame[0]
        metric[1 + axis] = frame[1]
        metric[(4, 7, 9)[axis]] = frame[2]
    prim = L.zeros(5)
    pos = L.coords("centre")[axis]
    lft = np.broadcast_to(pos < split, L.shape3)
    for c, q in ((0, 0), (1, 1), (2 + axis, 2)):
        prim[c] = np.where(lft, float(left[q]), float(right[q]))
    A = L.zeros(3)
    if magnetized:
        ec = L.coords(("xedge", "yedge", "zedge")[t2])
        a2 = Bn * ec[t1]
        if Bt is not None:
            x = ec[axis]
            a2 = a2 - np.where(x < split, Bt[0] * x, Bt[0] * split + Bt[1] * (x - split))
        A[t2] = np.broadcast_to(a2, L.shape3)
    nsteps = int(np.ceil(t_end / (cfl * dx) - 1e-9))
    params = default_params(gamma=gamma, rho_atm=1e-7 * max(left[0], right[0]), recon=recon)
    info = dict(left=tuple(left), right=tuple(right), axis=axis, t_end=t_end, split=split, Bn=Bn, Bt=Bt,
                frame=frame)
    return Workload("shock_tube%d" % n, L, params, metric, L.zeros(6), prim, A, L.zeros(1), t_end / nsteps,
                    nsteps, rk, ("copy",) * 3, ("linear",) * 3 if magnetized else ("copy",) * 3, info)


def kerr_schild_block(n=32, origin=(3.0, 0.5, 0.5), extent=3.0, M=1.0, prim_fn=None, ng=NG_DEFAULT, recon="ppm",
                      nsteps=10, rk=2, cfl=0.25, gamma=4.0 / 3.0, rho_atm=1e-10, monopole=0.0):
    """A block of the Schwarzschild spacetime in Kerr-Schild coordinates (mass M at the origin), the cube
    origin + [0, extent]^3 with n cells per side.  Every stored point, ghosts included, carries the analytic
    metric: lapse 1/sqrt(1 + 2M/r), shift (2M/r) alpha^2 l^i, gamma_ij = delta_ij + (2M/r) l_i l_j (l = x/r),
    and the extrinsic curvature of the static metric, K_ij = (2 M alpha / r^2)(delta_ij - (2 + M/r) l_i l_j).
    prim_fn(x, y, z) -> (5, ...) primitives at the cell centres (ghosts included).  monopole = Q: the field
    of a magnetic monopole at the origin, densitized B = Q x / r^3, from the potential
    A = Q (1 - z/r) (-y, x, 0) / (x^2 + y^2) sampled at the edges (its string lies on the negative z axis,
    outside blocks with x^2 + y^2 > 0 throughout).  Ghosts are filled by linear extrapolation during a run."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    dx = extent / nn[0]
    L = Layout(nn, ng, dx=(dx, dx, dx))
    o = [float(v) for v in origin]

    def at(where):
        c = L.coords(where)
        x, y, z = (np.broadcast_to(c[d] + o[d], L.shape3) for d in range(3))
        r = np.sqrt(x * x + y * y + z * z)
        return x, y, z, r, (x / r, y / r, z / r)

    x, y, z, r, l = at("vertex")
    H = M / r
    alpha = 1.0 / np.sqrt(1.0 + 2.0 * H)
    metric = L.zeros(10)
    curv = L.zeros(6)
    metric[0] = alpha
    for d in range(3):
        metric[1 + d] = 2.0 * H * alpha * alpha * l[d]
    pairs = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for c, (a, b) in enumerate(pairs):
        delta = 1.0 if a == b else 0.0
        metric[4 + c] = delta + 2.0 * H * l[a] * l[b]
        curv[c] = 2.0 * M * alpha / (r * r) * (delta - (2.0 + H) * l[a] * l[b])
    xc, yc, zc, _, _ = at("centre")
    prim = np.ascontiguousarray(np.asarray(prim_fn(xc, yc, zc), dtype=np.float64).reshape((5,) + L.shape3))
    A = L.zeros(3)
    if monopole != 0.0:
        for q, where in ((0, "xedge"), (1, "yedge")):
            x, y, z, r, _ = at(where)
            f = monopole * (1.0 - z / r) / (x * x + y * y)
            A[q] = -f * y if q == 0 else f * x
    params = default_params(gamma=gamma, rho_atm=rho_atm, recon=recon)
    info = dict(M=M, origin=tuple(o), extent=extent, monopole=monopole)
    return Workload("kerr_schild%d" % nn[0], L, params, metric, curv, prim, A, L.zeros(1), cfl * dx, nsteps,
                    rk, ("linear",) * 3, ("linear",) * 3, info)


def alfven_wave(n=32, ng=NG_DEFAULT, recon="minmod", t_end=2.0, rk=2, cfl=0.2, gamma=5.0 / 3.0, A0=1.0, vA=0.5,
                Bx=1.0, rho=1.0, p=0.5):
    """The circularly polarized Alfven wave of the paper's convergence test: x in [-0.5, 0.5] (n cells, two
    across y and z, spacing 1/n), flat metric, rho = 1, p = 0.5, B = Bx (1, A0 cos kx, A0 sin kx),
    v = -vA A0 (0, cos kx, sin kx), k = 2 pi, Gamma = 5/3, MINMOD, RK2, CFL 0.2; periodic in every
    direction.  The potential A = (0, -A0 Bx cos(kx)/k, Bx y - A0 Bx sin(kx)/k) (x the physical coordinate)
    is periodic up to the constant Bx L_y that A_z gains per period along y (A_shift).  dt = t_end / nsteps
    with the step at most cfl dx."""
    L = Layout((n, 2, 2), ng, dx=(1.0 / n,) * 3)
    k = 2.0 * np.pi
    xc, _, _ = L.coords("centre")
    xc = xc - 0.5
    prim = L.zeros(5)
    prim[0] = rho
    prim[1] = p
    prim[3] = np.broadcast_to(-vA * A0 * np.cos(k * xc), L.shape3)
    prim[4] = np.broadcast_to(-vA * A0 * np.sin(k * xc), L.shape3)
    A = L.zeros(3)
    xy, _, _ = L.coords("yedge")
    A[1] = np.broadcast_to(-A0 * Bx * np.cos(k * (xy - 0.5)) / k, L.shape3)
    xz, yz, _ = L.coords("zedge")
    A[2] = np.broadcast_to(Bx * yz - A0 * Bx * np.sin(k * (xz - 0.5)) / k, L.shape3)
    nsteps = int(np.ceil(t_end / (cfl / n) - 1e-9))
    params = default_params(gamma=gamma, recon=recon)
    info = dict(t_end=t_end, A0=A0, vA=vA, Bx=Bx, rho=rho, p=p)
    shift = np.zeros((3, 3))
    shift[2, 1] = Bx * L.n[1] * L.dx[1]
    return Workload("alfven%d" % n, L, params, flat_metric(L), L.zeros(6), prim, A, L.zeros(1), t_end / nsteps,
                    nsteps, rk, ("periodic",) * 3, ("periodic",) * 3, info, shift)


def loop_advection(n=64, nz=1, ng=NG_DEFAULT, recon="minmod", t_end=1.2, rk=4, cfl=0.25, gamma=5.0 / 3.0,
                   A_loop=1e-3, R_loop=0.3, vel=(1.0 / 12.0, 1.0 / 24.0, 1.0 / 24.0), rho=1.0, p=3.0):
    """The magnetic loop advection test of Sec. 4: x, y in [-0.5, 0.5] (n x n cells, nz across z, spacing
    1/n), flat metric, uniform rho = 1, p = 3 and v = (1/12, 1/24, 1/24); the loop's potential
    A_z = max(0, A_loop (R_loop - r)), r = sqrt(x^2 + y^2), at the z edges (A_loop = 1e-3, R_loop = 0.3);
    Gamma = 5/3, MINMOD, HLLE, RK4, CFL 0.25; periodic in every direction.  dt = t_end / nsteps with the
    step at most cfl dx."""
    L = Layout((n, n, nz), ng, dx=(1.0 / n,) * 3)
    prim = L.zeros(5)
    prim[0] = rho
    prim[1] = p
    for d in range(3):
        prim[2 + d] = vel[d]
    A = L.zeros(3)
    xz, yz, _ = L.coords("zedge")
    r = np.sqrt((xz - 0.5) ** 2 + (yz - 0.5) ** 2)
    A[2] = np.broadcast_to(np.maximum(0.0, A_loop * (R_loop - r)), L.shape3)
    L.periodic_wrap(A)
    nsteps = int(np.ceil(t_end / (cfl / n) - 1e-9))
    params = default_params(gamma=gamma, recon=recon)
    info = dict(t_end=t_end, A_loop=A_loop, R_loop=R_loop, vel=tuple(vel))
    return Workload("loop%d" % n, L, params, flat_metric(L), L.zeros(6), prim, A, L.zeros(1), t_end / nsteps,
                    nsteps, rk, ("periodic",) * 3, ("periodic",) * 3, info)


def static_star_block(n=40, origin=(0.0, 0.0, 0.0), extent=10.0, star_fn=None, ng=NG_DEFAULT, recon="ppm", nsteps=10,
                      rk=4, cfl=0.25, gamma=2.0, rho_atm=1e-10, bc=("copy",) * 3):
    """A block of a static, conformally flat spacetime with a fluid at rest: the cube origin + [0, extent]^3
    with n cells per side.  star_fn(x, y, z, rho_atm) -> (alpha, psi^4, rho, p) gives the lapse and the
    conformal factor (gamma_ij = psi^4 delta_ij, zero shift and extrinsic curvature) at every vertex and the
    density and pressure at every cell centre, ghosts included."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    dx = extent / nn[0]
    L = Layout(nn, ng, dx=(dx, dx, dx))
    o = [float(v) for v in origin]

    def at(where):
        c = L.coords(where)
        return tuple(np.broadcast_to(c[d] + o[d], L.shape3) for d in range(3))

    alpha, psi4, _, _ = star_fn(*at("vertex"), rho_atm)
    metric = L.zeros(10)
    metric[0] = alpha
    for c in (4, 7, 9):
        metric[c] = psi4
    _, _, rho, p = star_fn(*at("centre"), rho_atm)
    prim = L.zeros(5)
    prim[0] = rho
    prim[1] = p
    params = default_params(gamma=gamma, rho_atm=rho_atm, recon=recon)
    info = dict(origin=tuple(o), extent=extent)
    return Workload("static_star%d" % nn[0], L, params, metric, L.zeros(6), prim, L.zeros(3), L.zeros(1), cfl * dx,
                    nsteps, rk, tuple(bc), tuple(bc), info)


GAUSS = 1.0 / 8.351e19  # one gauss in units with G = c = M_sun = 1


def magnetized_star_block(n=240, extent=40.0, B_max_gauss=1e14, ng=NG_DEFAULT, nsteps=5, rk=4, cfl=0.25):
    """The paper's Setup A (its single-GPU benchmark): a magnetized TOV star in a static (Cowling) spacetime on
    a uniform grid.  The K = 100, Gamma = 2 polytrope with central density 1.28e-3 (paper_2406_11669_amd/tov.py)
    in its isotropic metric on [-extent/2, extent/2]^3 with n cells per side; rho_atm = 1e-7 rho_c; PPM, HLLE,
    RK4, copy (Neumann) boundaries.  The field comes from A_phi = A_b varpi^2 max(p - 0.04 p_max, 0)^2, i.e.
    A = A_b max(p - p_cut, 0)^2 (-y, x, 0) at the edges, with A_b chosen so that the largest |B| (the curl
    over psi^6) is about B_max_gauss."""
    from paper_2406_11669_amd.tov import TOV
    star = TOV()
    rho_atm = 1e-7 * star.rho_c
    w = static_star_block(n=n, origin=(-0.5 * extent,) * 3, extent=extent, star_fn=star.fields, ng=ng,
                          recon="ppm", nsteps=nsteps, rk=rk, cfl=cfl, gamma=2.0, rho_atm=rho_atm)
    L = w.layout
    p_cut = 0.04 * star.K * star.rho_c ** star.G
    for q, where in ((0, "xedge"), (1, "yedge")):
        c = L.coords(where)
        x, y, z = (np.broadcast_to(c[d] - 0.5 * extent, L.shape3) for d in range(3))
        f = np.maximum(star.fields(x, y, z, rho_atm)[3] - p_cut, 0.0) ** 2
        w.A[q] = -y * f if q == 0 else x * f
    dx = L.dx[0]
    bt = np.sqrt(np.gradient(w.A[1], dx, axis=0) ** 2 + np.gradient(w.A[0], dx, axis=0) ** 2
                 + (np.gradient(w.A[1], dx, axis=2) - np.gradient(w.A[0], dx, axis=1)) ** 2)
    w.A *= B_max_gauss * GAUSS / float(np.max(bt / w.metric[4] ** 1.5))
    w.info.update(star="TOV K=100 Gamma=2 rho_c=1.28e-3", B_max_gauss=B_max_gauss)
    return w


# ---- the curved periodic block -----------------------------------------------------------------------------

_TAGS = {name: t for t, name in enumerate(
    ["alpha", "betax", "betay", "betaz", "gxx", "gxy", "gxz", "gyy", "gyz", "gzz", "rho", "p", "vx", "vy", "vz",
     "Ax", "Ay", "Az"])}


def curved_metric(layout, seed, alpha0=0.8, alpha_amp=0.15, beta_amp=0.05, gamma_amp=0.1, want_curv=True):
    """Static curved 3+1 metric at every vertex (bitwise periodic) and, optionally, its extrinsic curvature.

    gamma_ij = delta_ij + gamma_amp f_ij, alpha = alpha0 + alpha_amp f_alpha, beta^i = beta_amp f_beta^i.
    With d_t gamma_ij = 0 the extrinsic curvature (K = -L_n gamma / 2) is
    K_ij = (D_i beta_j + D_j beta_i) / (2 alpha), evaluated analytically from the modes."""
    L = layout
    x, y, z = L.coords("vertex")
    names = ["alpha", "betax", "betay", "betaz", "gxx", "gxy", "gxz", "gyy", "gyz", "gzz"]
    f = {nm: ModeSum(seed, _TAGS[nm]) for nm in names}
    m = L.zeros(10)
    m[0] = alpha0 + alpha_amp * np.broadcast_to(f["alpha"](x, y, z), L.shape3)
    for c, nm in enumerate(["betax", "betay", "betaz"]):
        m[1 + c] = beta_amp * np.broadcast_to(f[nm](x, y, z), L.shape3)
    for c, nm in enumerate(["gxx", "gxy", "gxz", "gyy", "gyz", "gzz"]):
        delta = 1.0 if nm in ("gxx", "gyy", "gzz") else 0.0
        m[4 + c] = delta + gamma_amp * np.broadcast_to(f[nm](x, y, z), L.shape3)
    L.periodic_wrap(m)
    if not want_curv:
        return m, None, f
    # analytic derivatives at vertices
    sym = [(0, 0, "gxx"), (0, 1, "gxy"), (0, 2, "gxz"), (1, 1, "gyy"), (1, 2, "gyz"), (2, 2, "gzz")]
    shape = L.shape3
    g = np.zeros((3, 3) + shape)
    dg = np.zeros((3, 3, 3) + shape)  # dg[k, a, b] = d_k gamma_ab
    for a, b, nm in sym:
        val = (1.0 if a == b else 0.0) + gamma_amp * np.broadcast_to(f[nm](x, y, z), shape)
        gr = f[nm].grad(x, y, z)
        g[a, b] = g[b, a] = val
        for k in range(3):
            dg[k, a, b] = dg[k, b, a] = gamma_amp * np.broadcast_to(gr[k], shape)
    alpha = alpha0 + alpha_amp * np.broadcast_to(f["alpha"](x, y, z), shape)
    beta = np.zeros((3,) + shape)
    dbeta = np.zeros((3, 3) + shape)  # dbeta[k, a] = d_k beta^a
    for a, nm in enumerate(["betax", "betay", "betaz"]):
        beta[a] = beta_amp * np.broadcast_to(f[nm](x, y, z), shape)
        gr = f[nm].grad(x, y, z)
        for k in range(3):
            dbeta[k, a] = beta_amp * np.broadcast_to(gr[k], shape)
    gmat = np.moveaxis(g, (0, 1), (-2, -1))
    gi = np.moveaxis(np.linalg.inv(gmat), (-2, -1), (0, 1))
    beta_l = np.einsum("ab...,b...->a...", g, beta)
    # d_i beta_j = d_i gamma_jk beta^k + gamma_jk d_i beta^k
    dbl = np.einsum("ijk...,k...->ij...", dg, beta) + np.einsum("jk...,ik...->ij...", g, dbeta)
    # Christoffel of the first kind Gamma_lij = (d_i g_lj + d_j g_li - d_l g_ij)/2
    G1 = 0.5 * (np.einsum("ilj...->lij...", dg) + np.einsum("jli...->lij...", dg) - dg)
    Gam = np.einsum("kl...,lij...->kij...", gi, G1)
    Db = dbl - np.einsum("kij...,k...->ij...", Gam, beta_l)
    K = (Db + np.swapaxes(Db, 0, 1)) / (2.0 * alpha)
    curv = L.zeros(6)
    for c, (a, b, _) in enumerate(sym):
        curv[c] = K[a, b]
    L.periodic_wrap(curv)
    return m, curv, f


def curved_block(seed=0, n=128, ng=NG_DEFAULT, recon="ppm", nsteps=5, rk=4, cfl=0.25, gamma=2.0, vmax=0.45,
                 rho_atm=1e-10):
    """Periodic block in a static curved metric with seeded low-k fluid, velocity and vector-potential modes."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    L = Layout(nn, ng)
    metric, curv, fm = curved_metric(L, seed)
    xc, yc, zc = L.coords("centre")
    f = {nm: ModeSum(seed, _TAGS[nm]) for nm in ["rho", "p", "vx", "vy", "vz", "Ax", "Ay", "Az"]}
    prim = L.zeros(5)
    prim[0] = 1.0 + 0.5 * np.broadcast_to(f["rho"](xc, yc, zc), L.shape3)
    prim[1] = 0.55 + 0.45 * np.broadcast_to(f["p"](xc, yc, zc), L.shape3)
    v = np.stack([np.broadcast_to(f[nm](xc, yc, zc), L.shape3) for nm in ("vx", "vy", "vz")])
    # scale so that max sqrt(gamma_ij v^i v^j) = vmax, with gamma_ij of the analytic modes at the centres
    gsym = {}
    for nm, (a, b) in zip(["gxx", "gxy", "gxz", "gyy", "gyz", "gzz"], [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        val = (1.0 if a == b else 0.0) + 0.1 * np.broadcast_to(fm[nm](xc, yc, zc), L.shape3)
        gsym[(a, b)] = gsym[(b, a)] = val
    vn2 = sum(gsym[(a, b)] * v[a] * v[b] for a in range(3) for b in range(3))
    scale = vmax / np.sqrt(np.max(L.owned(vn2)))
    prim[2:5] = scale * v
    L.periodic_wrap(prim)
    A = L.zeros(3)
    curl_max = 0.0
    for c, (nm, where) in enumerate((("Ax", "xedge"), ("Ay", "yedge"), ("Az", "zedge"))):
        x, y, z = L.coords(where)
        A[c] = np.broadcast_to(f[nm](x, y, z), L.shape3)
    # analytic curl magnitude at the centres sets the amplitude (max |B| = 1)
    gx = f["Ax"].grad(xc, yc, zc)
    gy = f["Ay"].grad(xc, yc, zc)
    gz = f["Az"].grad(xc, yc, zc)
    Bx = gz[1] - gy[2]
    By = gx[2] - gz[0]
    Bz = gy[0] - gx[1]
    curl_max = float(np.max(np.sqrt(Bx ** 2 + By ** 2 + Bz ** 2)))
    A *= 1.0 / curl_max
    L.periodic_wrap(A)
    psi = L.zeros(1)
    params = default_params(gamma=gamma, rho_atm=rho_atm, recon=recon)
    dt = cfl * min(L.dx)
    return Workload("curved%d" % nn[0], L, params, metric, curv, prim, A, psi, dt, nsteps, rk,
                    ("periodic",) * 3, ("periodic",) * 3, dict(seed=seed, vscale=scale, a_B=1.0 / curl_max))


# ---- AMR-like patches ---------------------------------------------------------------------------------------

def patch_set(seed=0, npatches=512, sides=(16, 24, 32, 48), levels=3, ng=NG_DEFAULT, nsteps=10, cfl=0.25,
              recon="minmod"):
    """npatches Riemann-problem blocks with seeded sides in `sides` and refinement levels 0..levels-1
    (spacing 2^-level / 32), each split at its own mid-x with its own seed; flat metric, copy/linear ghosts.
    One global time step dt = cfl * (smallest spacing) for all patches (no subcycling)."""
    rng = np.random.default_rng([int(seed), 7919])
    side = rng.choice(np.array(sides), size=npatches)
    level = rng.integers(0, levels, size=npatches)
    out = []
    for q in range(npatches):
        n = int(side[q])
        dx = 2.0 ** (-int(level[q])) / 32.0
        w = riemann_block(seed=int(seed) * 100003 + q, n=n, ng=ng, recon=recon, nsteps=nsteps, rk=2, cfl=cfl,
                          split=0.5 * n * dx, dx=dx)
        out.append(w)
    dt = cfl * 2.0 ** (-(levels - 1)) / 32.0
    rho_max = max(max(w.info["rhoL"], w.info["rhoR"]) for w in out)
    for w in out:
        w.dt = dt
        w.params["rho_atm"] = 1e-7 * rho_max  # one floor for the whole hierarchy
        w.info["level"] = int(np.log2(1.0 / (32.0 * w.layout.dx[0])) + 0.5)
    return out


def box_in_box(seed=0, n=24, levels=3, ng=NG_DEFAULT, recon="minmod", nsteps=10, cfl=0.25, split=0.375):
    """Nested refinement (box in box, as in the mesh-refinement test of Sec. 4): level 0 covers the unit box with
    n^3 cells, level l > 0 a centred box of n^3 cells at half its parent's spacing (the middle n/2 parent cells
    per axis).  One seeded Riemann problem (riemann_block) split on the vertex plane x = split, sampled by every
    level in global coordinates; the default split lies on the finest level's lower x face, so the waves cross
    refinement boundaries at once.  One global time step cfl * (finest spacing) (no subcycling).  Level 0 has
    the copy / linear ghosts of riemann_block; finer levels take their ghosts from their parent.
    Returns (workloads, parents, c0): parents[l] = l - 1 (None for level 0) and c0[l] the parent vertex index
    of the patch's vertex 0."""
    assert n % 4 == 0 and levels >= 1
    wls, parents, c0 = [], [], []
    for lev in range(levels):
        dx = 1.0 / (n * 2 ** lev)
        o = 0.5 - 0.5 * n * dx
        w = riemann_block(seed=seed, n=n, ng=ng, recon=recon, nsteps=nsteps, rk=2, cfl=cfl, split=split, dx=dx,
                          origin=(o, o, o))
        w.info["level"] = lev
        w.info["origin"] = o
        wls.append(w)
        parents.append(None if lev == 0 else lev - 1)
        c0.append(None if lev == 0 else (n // 4,) * 3)
    dt = cfl / (n * 2 ** (levels - 1))
    rho_max = max(max(w.info["rhoL"], w.info["rhoR"]) for w in wls)
    for w in wls:
        w.dt = dt
        w.params["rho_atm"] = 1e-7 * rho_max
    return wls, parents, c0


def gradient_direction(layout, seed, with_gamma=True):
    """Seeded unit direction in the space of (initial velocity field on owned cells, Gamma): independent
    standard normals, normalised.  Returns (dprim with the velocity part in fields 2..4 and periodic ghosts,
    dGamma)."""
    L = layout
    rng = np.random.default_rng([int(seed), 4099])
    d = L.zeros(5)
    L.owned(d)[2:5] = rng.normal(size=(3, L.n[2], L.n[1], L.n[0]))
    dg = float(rng.normal()) if with_gamma else 0.0
    nrm = float(np.sqrt(np.sum(L.owned(d) ** 2) + dg * dg))
    d /= nrm
    L.periodic_wrap(d)
    return d, dg / nrm


# ---- independent c2p states (learned initial guess) ---------------------------------------------------------

def metric_at_points(seed, x, y, z, alpha0=0.8, alpha_amp=0.15, beta_amp=0.05, gamma_amp=0.1):
    """The curved metric family of curved_metric evaluated at arbitrary points: (10, n) array."""
    names = ["alpha", "betax", "betay", "betaz", "gxx", "gxy", "gxz", "gyy", "gyz", "gzz"]
    f = {nm: ModeSum(seed, _TAGS[nm]) for nm in names}
    m = np.zeros((10, x.size))
    m[0] = alpha0 + alpha_amp * f["alpha"](x, y, z)
    for c, nm in enumerate(["betax", "betay", "betaz"]):
        m[1 + c] = beta_amp * f[nm](x, y, z)
    for c, nm in enumerate(["gxx", "gxy", "gxz", "gyy", "gyz", "gzz"]):
        m[4 + c] = (1.0 if nm in ("gxx", "gyy", "gzz") else 0.0) + gamma_amp * f[nm](x, y, z)
    return m


def _gmat(m):
    g = np.empty((m.shape[1], 3, 3))
    for c, (a, b) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        g[:, a, b] = g[:, b, a] = m[4 + c]
    return g


def _unit_in_metric(rng, g):
    """Isotropic directions (flat normals), normalised in the metric g: g_ij n^i n^j = 1."""
    n = rng.normal(size=(g.shape[0], 3))
    nn = np.einsum("pi,pij,pj->p", n, g, n)
    return n / np.sqrt(nn)[:, None]


def c2p_states(seed, n, log10_rho=(-8.0, 0.0), W=(1.0, 10.0), sigma=(1e-3, 10.0), p_over_rho=(1e-3, 10.0),
               gamma=(4.0 / 3.0, 2.0), flat_fraction=0.5, metric_seed=0):
    """Seeded independent primitive states for the learned c2p guess: log10 rho ~ U, W ~ U, magnetisation
    sigma = b^2 / rho ~ log-U, p / rho ~ log-U, Gamma ~ U; velocity and field directions isotropic and
    independent; metric flat for a fraction flat_fraction of the points, else the curved family at uniform
    random positions of the unit cube.  Returns dict(prim (5, n), Bt (3, n) densitized, metric (10, n), gam (n))."""
    rng = np.random.default_rng([int(seed), 8191])
    rho = 10.0 ** rng.uniform(log10_rho[0], log10_rho[1], n)
    Wl = rng.uniform(W[0], W[1], n)
    sig = np.exp(rng.uniform(np.log(sigma[0]), np.log(sigma[1]), n))
    por = np.exp(rng.uniform(np.log(p_over_rho[0]), np.log(p_over_rho[1]), n))
    gam = rng.uniform(gamma[0], gamma[1], n)
    m = np.zeros((10, n))
    m[0] = 1.0
    m[4] = m[7] = m[9] = 1.0
    curved = rng.uniform(size=n) >= flat_fraction
    if np.any(curved):
        pos = rng.uniform(size=(3, int(curved.sum())))
        m[:, curved] = metric_at_points(metric_seed, pos[0], pos[1], pos[2])
    g = _gmat(m)
    vdir = _unit_in_metric(rng, g)
    vmag = np.sqrt(1.0 - 1.0 / Wl ** 2)
    v = vdir * vmag[:, None]
    bdir = _unit_in_metric(rng, g)
    bv = np.einsum("pi,pij,pj->p", bdir, g, v)           # (Bhat . v) in the metric
    Bmag = np.sqrt(sig * rho / (1.0 / Wl ** 2 + bv ** 2))  # b^2 = B^2 / W^2 + (B . v)^2 = sigma rho
    B = bdir * Bmag[:, None]
    sqrtg = np.sqrt(np.linalg.det(g))
    prim = np.stack([rho, por * rho, v[:, 0], v[:, 1], v[:, 2]])
    Bt = (B * sqrtg[:, None]).T.copy()
    return dict(prim=prim, Bt=Bt, metric=m, gam=gam)


def c2p_block_states(seed, n=256, W=(1.0, 10.0), gamma=5.0 / 3.0):
    """n^3 per-cell states of the Riemann-problem ranges (rho, p ~ U[0.1, 1], B^i ~ U[-1, 1]) with an isotropic
    velocity of Lorentz factor W ~ U[W]; flat metric.  Returns dict(prim (5, N), Bt (3, N), gam scalar)."""
    rng = np.random.default_rng([int(seed), 131071])
    N = n ** 3
    rho = rng.uniform(0.1, 1.0, N)
    p = rng.uniform(0.1, 1.0, N)
    Wl = rng.uniform(W[0], W[1], N)
    d = rng.normal(size=(N, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    v = d * np.sqrt(1.0 - 1.0 / Wl ** 2)[:, None]
    B = rng.uniform(-1.0, 1.0, (3, N))
    prim = np.stack([rho, p, v[:, 0], v[:, 1], v[:, 2]])
    return dict(prim=prim, Bt=B, gam=gamma)
