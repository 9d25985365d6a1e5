// asterx.hip -- HIP kernels (gfx950, FP64) and the C ABI of the Valencia GRMHD right-hand side.
//
// One block, one GPU.  Per RK stage the caller runs: asterx_c2p -> asterx_fill_ghosts(prim)
// -> asterx_rhs -> asterx_rk_stage -> asterx_fill_ghosts(state).  asterx_rhs itself is
// four launches:
//   face<D> (D = x, y, z): reconstruction + face metric + prim->cons + fluxes + speeds + HLLE
//                          for every face, one thread per face, x-pencil coalesced;
//   cell:                  flux divergence + geometric sources + div B, one thread per cell;
//   vertex:                gauge quantities G_A and F_Psi at vertices;
//   edge:                  FCT electric field, dA/dt and dPsi/dt.
// Threads map to x fastest so every stencil load is coalesced across a wavefront; the
// block -> tile map keeps neighbouring tiles on one XCD (shared L2).
// Section/equation references are to AsterX, arXiv 2406.11669.

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>

#include "asterx.h"
#include "grmhd_device.h"

using namespace ax;

namespace {

thread_local std::string g_err;

int fail(int code, const char* msg) {
  g_err = msg;
  return code;
}

// ---------------------------------------------------------------------------------------
// Grid description passed by value to kernels.
struct GD {
  int n[3];
  int ng;
  int ld0, ld1;
  int sy, sz;  // strides of j and k
  size_t N;    // points per field
  double idx[3];
};

GD make_gd(const asterx_grid* g) {
  GD d;
  for (int a = 0; a < 3; ++a) {
    d.n[a] = g->n[a];
    d.idx[a] = 1.0 / g->dx[a];
  }
  d.ng = g->ng;
  d.ld0 = g->ld[0];
  d.ld1 = g->ld[1];
  d.sy = g->ld[0];
  d.sz = g->ld[0] * g->ld[1];
  d.N = (size_t)g->ld[0] * g->ld[1] * g->ld[2];
  return d;
}

DEV int at(const GD& g, int i, int j, int k) { return ((k + g.ng) * g.ld1 + (j + g.ng)) * g.ld0 + (i + g.ng); }

// Blocks are dispatched round-robin over the 8 XCDs; remap the linear block id so that
// each XCD walks a contiguous range of tiles (neighbouring tiles share its L2).
DEV unsigned xcd_block(unsigned bid, unsigned nblocks) {
  const unsigned nx = 8;
  unsigned per = nblocks / nx, rem = nblocks % nx;
  unsigned x = bid % nx, r = bid / nx;
  // XCD x owns tiles [start_x, start_x + per + (x < rem))
  unsigned start = x * per + (x < rem ? x : rem);
  return start + r;
}

// Linear tile decomposition of a 3-D box of extents e[3] into blocks of TX x TY x 1.
template <int TX, int TY>
DEV bool box_index(const int e[3], int& a, int& b, int& c) {
  unsigned nbx = (e[0] + TX - 1) / TX, nby = (e[1] + TY - 1) / TY;
  unsigned nblocks = nbx * nby * (unsigned)e[2];
  unsigned bid = xcd_block(blockIdx.x, nblocks);
  unsigned bx = bid % nbx;
  unsigned t = bid / nbx;
  unsigned by = t % nby;
  c = (int)(t / nby);
  a = (int)(bx * TX + threadIdx.x % TX);
  b = (int)(by * TY + threadIdx.x / TX);
  return a < e[0] && b < e[1] && c < e[2];
}

template <int TX, int TY>
unsigned box_blocks(const int e[3]) {
  return (unsigned)((e[0] + TX - 1) / TX) * (unsigned)((e[1] + TY - 1) / TY) * (unsigned)e[2];
}

// ---------------------------------------------------------------------------------------
// Wavefront reductions (64 lanes): max of non-negative doubles and flag counts, then one
// device atomic per wavefront.  Max is order independent, so results are deterministic.
DEV double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

DEV void atomic_max_pos(double* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax((unsigned long long*)addr, (unsigned long long)__double_as_longlong(v));
}

DEV void wave_count(bool pred, unsigned long long* ctr) {
  unsigned long long m = __ballot(pred);
  if (__lane_id() == 0 && m) atomicAdd(ctr, (unsigned long long)__popcll(m));
}

// ---------------------------------------------------------------------------------------
// Vertex -> centre/face interpolation of spacetime data (Sec. 3.2: fourth-order Lagrange).
// The centre of cell i lies midway between vertices i and i+1; stencil i-1..i+2.
DEV double lag(double a, double b, double c, double d) { return 0.5625 * (b + c) - 0.0625 * (a + d); }
DEV double dlag(double a, double b, double c, double d) { return (27.0 * (c - b) - (d - a)) * (1.0 / 24.0); }

// Value at the centre whose lower-corner vertex stencil starts at p (vertex i-1,j-1,k-1).
DEV double centre_val(const double* __restrict__ p, int sy, int sz) {
  double zz[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double yy[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double* r = p + b * sy + c * sz;
      yy[b] = lag(r[0], r[1], r[2], r[3]);
    }
    zz[c] = lag(yy[0], yy[1], yy[2], yy[3]);
  }
  return lag(zz[0], zz[1], zz[2], zz[3]);
}

// Value and first derivatives (unscaled by 1/dx) at the centre.
DEV void centre_val_der(const double* __restrict__ p, int sy, int sz, double& v, double& dx, double& dy, double& dz) {
  double vz[4], dyz[4], dxz[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double vx[4], ddx[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double* r = p + b * sy + c * sz;
      double r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
      vx[b] = lag(r0, r1, r2, r3);
      ddx[b] = dlag(r0, r1, r2, r3);
    }
    vz[c] = lag(vx[0], vx[1], vx[2], vx[3]);
    dyz[c] = dlag(vx[0], vx[1], vx[2], vx[3]);
    dxz[c] = lag(ddx[0], ddx[1], ddx[2], ddx[3]);
  }
  v = lag(vz[0], vz[1], vz[2], vz[3]);
  dz = dlag(vz[0], vz[1], vz[2], vz[3]);
  dy = lag(dyz[0], dyz[1], dyz[2], dyz[3]);
  dx = lag(dxz[0], dxz[1], dxz[2], dxz[3]);
}

DEV void centre_metric(const double* __restrict__ metric, size_t N, int base, int sy, int sz, double m[10]) {
#pragma unroll
  for (int c = 0; c < 10; ++c) m[c] = centre_val(metric + c * N + base, sy, sz);
}

// ---------------------------------------------------------------------------------------
// Staggered field (Secs. 2.3, 3.1): face Btilde = curl of the edge potential; centre value
// = average of the two faces.
DEV double faceBx(const double* Ay, const double* Az, int id, int sy, int sz, const GD& g) {
  return (Az[id + sy] - Az[id]) * g.idx[1] - (Ay[id + sz] - Ay[id]) * g.idx[2];
}
DEV double faceBy(const double* Ax, const double* Az, int id, int sy, int sz, const GD& g) {
  return (Ax[id + sz] - Ax[id]) * g.idx[2] - (Az[id + 1] - Az[id]) * g.idx[0];
}
DEV double faceBz(const double* Ax, const double* Ay, int id, int sy, int sz, const GD& g) {
  (void)sz;
  return (Ay[id + 1] - Ay[id]) * g.idx[0] - (Ax[id + sy] - Ax[id]) * g.idx[1];
}

DEV void centre_B(const double* __restrict__ A, const GD& g, int id, double Bt[3]) {
  const double* Ax = A;
  const double* Ay = A + g.N;
  const double* Az = A + 2 * g.N;
  Bt[0] = 0.5 * (faceBx(Ay, Az, id, g.sy, g.sz, g) + faceBx(Ay, Az, id + 1, g.sy, g.sz, g));
  Bt[1] = 0.5 * (faceBy(Ax, Az, id, g.sy, g.sz, g) + faceBy(Ax, Az, id + g.sy, g.sy, g.sz, g));
  Bt[2] = 0.5 * (faceBz(Ax, Ay, id, g.sy, g.sz, g) + faceBz(Ax, Ay, id + g.sz, g.sy, g.sz, g));
}

C2PParams make_c2p_params(const asterx_params* p) {
  C2PParams c;
  c.gam = p->gamma;
  c.rho_atm = p->rho_atm;
  c.k_atm = p->k_atm;
  c.tol = p->c2p_tol;
  c.wmax = p->wmax;
  c.maxit = p->c2p_maxit;
  c.brent_maxit = p->brent_maxit;
  c.method = p->c2p_method;
  return c;
}

// =======================================================================================
// prim -> cons on owned cells.
__global__ __launch_bounds__(256) void k_prim2con(GD g, double gam, const double* __restrict__ metric,
                                                  const double* __restrict__ A, const double* __restrict__ prim,
                                                  double* __restrict__ cons) {
  int i, j, k;
  if (!box_index<64, 4>(g.n, i, j, k)) return;
  int id = at(g, i, j, k);
  double m[10];
  centre_metric(metric, g.N, id - 1 - g.sy - g.sz, g.sy, g.sz, m);
  Geo G;
  geo_from(m, G);
  double Bt[3], pr[5];
  centre_B(A, g, id, Bt);
#pragma unroll
  for (int c = 0; c < 5; ++c) pr[c] = prim[c * g.N + id];
  State S;
  state_make(G, pr, Bt, gam, S);
  double U[5];
  cons_of(G, S, U);
#pragma unroll
  for (int c = 0; c < 5; ++c) cons[c * g.N + id] = U[c];
}

// c2p on owned cells (Sec. 3.5, 3.6).
__global__ __launch_bounds__(256) void k_c2p(GD g, C2PParams P, const double* __restrict__ metric,
                                             const double* __restrict__ A, double* __restrict__ cons,
                                             double* __restrict__ prim, uint8_t* __restrict__ flags,
                                             unsigned long long* __restrict__ stats) {
  int i, j, k;
  bool valid = box_index<64, 4>(g.n, i, j, k);
  uint32_t fl = 0;
  int iters = 0;
  if (valid) {
    int id = at(g, i, j, k);
    double m[10];
    centre_metric(metric, g.N, id - 1 - g.sy - g.sz, g.sy, g.sz, m);
    Geo G;
    geo_from(m, G);
    double Bt[3], U[5], prev[5], out[5];
    centre_B(A, g, id, Bt);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      U[c] = cons[c * g.N + id];
      prev[c] = prim[c * g.N + id];
    }
    fl = c2p_point(G, U, Bt, prev, P, out, iters);
#pragma unroll
    for (int c = 0; c < 5; ++c) prim[c * g.N + id] = out[c];
    if (fl & 4u) {
#pragma unroll
      for (int c = 0; c < 5; ++c) cons[c * g.N + id] = U[c];
    }
    if (flags) flags[id] = (uint8_t)fl;
  }
  if (stats) {
    wave_count(fl & 1u, stats + 0);
    wave_count(fl & 2u, stats + 1);
    wave_count(fl & 4u, stats + 2);
    wave_count(fl & 8u, stats + 3);
    wave_count(fl & 16u, stats + 4);
    double im = wave_max((double)iters);
    if (__lane_id() == 0 && im > 0.0) atomicMax(stats + 5, (unsigned long long)im);
  }
}

// Ghost fill along axis d of nf fields.
struct FillArgs {
  double* f;
  int nf;
  int d;
  int kind;
};

__global__ __launch_bounds__(256) void k_fill(GD g, FillArgs a) {
  const int d = a.d;
  int ext[3];
  for (int t = 0; t < 3; ++t) ext[t] = g.n[t] + 2 * g.ng + 1;
  int nghost = 2 * g.ng + 1;
  int cnt[3] = {ext[0], ext[1], ext[2]};
  cnt[d] = nghost;
  long long total = (long long)cnt[0] * cnt[1] * cnt[2] * a.nf;
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= total) return;
  int q0 = (int)(tid % cnt[0]);
  long long r = tid / cnt[0];
  int q1 = (int)(r % cnt[1]);
  r /= cnt[1];
  int q2 = (int)(r % cnt[2]);
  int f = (int)(r / cnt[2]);
  int idx[3] = {q0 - g.ng, q1 - g.ng, q2 - g.ng};
  int n = g.n[d];
  int q = idx[d] + g.ng;  // 0 .. nghost-1
  int s = q < g.ng ? q - g.ng : n + (q - g.ng);
  idx[d] = s;
  double* F = a.f + (size_t)f * g.N;
  int dst = at(g, idx[0], idx[1], idx[2]);
  int stride = d == 0 ? 1 : (d == 1 ? g.sy : g.sz);
  double val;
  if (a.kind == ASTERX_BC_PERIODIC) {
    int src = ((s % n) + n) % n;
    val = F[dst + (src - s) * stride];
  } else if (a.kind == ASTERX_BC_COPY) {
    int src = s < 0 ? 0 : n - 1;
    val = F[dst + (src - s) * stride];
  } else {
    if (s < 0) {
      double f0 = F[dst - s * stride], f1 = F[dst + (1 - s) * stride];
      val = f0 + (double)s * (f1 - f0);
    } else {
      double f0 = F[dst + (n - 1 - s) * stride], f1 = F[dst + (n - 2 - s) * stride];
      val = f0 + (double)(s - n + 1) * (f0 - f1);
    }
  }
  F[dst] = val;
}

// Centre field of every cell in [-ng, n+ng-1]^3 (read by the face stencils).
__global__ __launch_bounds__(256) void k_bcent(GD g, const double* __restrict__ A, double* __restrict__ bc) {
  int e[3] = {g.n[0] + 2 * g.ng, g.n[1] + 2 * g.ng, g.n[2] + 2 * g.ng};
  int a, b, c;
  if (!box_index<64, 4>(e, a, b, c)) return;
  int id = at(g, a - g.ng, b - g.ng, c - g.ng);
  double Bt[3];
  centre_B(A, g, id, Bt);
  bc[id] = Bt[0];
  bc[g.N + id] = Bt[1];
  bc[2 * g.N + id] = Bt[2];
}

// ---------------------------------------------------------------------------------------
// Face fluxes along D.  Face (i,j,k), index along D in [0, n_D], transverse in [-1, n-1]
// (the extra layer feeds the edge averages of the electric field).
struct FaceArgs {
  const double* metric;
  const double* prim;
  const double* A;
  const double* bc;
  double* flux;
  double* red;
  double gam, weno_eps, weno_q;
  int recon, speeds;
};

template <int D>
__global__ __launch_bounds__(256) void k_face(GD g, FaceArgs fa) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  int e[3] = {g.n[0] + 1, g.n[1] + 1, g.n[2] + 1};
  int a, b, c;
  bool valid = box_index<64, 4>(e, a, b, c);
  double smax = 0.0;
  if (valid) {
    int ijk[3] = {a - 1, b - 1, c - 1};
    ijk[D] += 1;
    const int i = ijk[0], j = ijk[1], k = ijk[2];
    const int id = at(g, i, j, k);
    const int st[3] = {1, g.sy, g.sz};
    const int sD = st[D], s1 = st[t1], s2 = st[t2];
    // face metric: Lagrange weights in the two transverse directions
    double m[10];
    const int mb = id - s1 - s2;
#pragma unroll
    for (int cc = 0; cc < 10; ++cc) {
      const double* p = fa.metric + cc * g.N + mb;
      double rr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double* r = p + q * s2;
        rr[q] = lag(r[0], r[s1], r[2 * s1], r[3 * s1]);
      }
      m[cc] = lag(rr[0], rr[1], rr[2], rr[3]);
    }
    Geo G;
    geo_from(m, G);
    // reconstruction of rho, p, v^x..z and the two transverse centre fields
    double L[7], R[7], cl[7], cr[7];
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      const double* f = v < 5 ? fa.prim + v * g.N : fa.bc + (v == 5 ? t1 : t2) * g.N;
      double s6[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) s6[q] = f[id + (q - 3) * sD];
      reconstruct(fa.recon, s6, L[v], R[v], fa.weno_eps, fa.weno_q);
      cl[v] = s6[2];
      cr[v] = s6[3];
    }
    // normal field on the face from the curl
    const double* Ax = fa.A;
    const double* Ay = fa.A + g.N;
    const double* Az = fa.A + 2 * g.N;
    double Bn = D == 0 ? faceBx(Ay, Az, id, g.sy, g.sz, g) : (D == 1 ? faceBy(Ax, Az, id, g.sy, g.sz, g) : faceBz(Ax, Ay, id, g.sy, g.sz, g));
    double UL[7], FL[7], UR[7], FR[7], cmL, cpL, cmR, cpR;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      double* X = side == 0 ? L : R;
      const double* C = side == 0 ? cl : cr;
      double vl[3], v[3] = {X[2], X[3], X[4]};
      lower(G.g, v, vl);
      double v2 = v[0] * vl[0] + v[1] * vl[1] + v[2] * vl[2];
      if (!(X[0] > 0.0) || !(X[1] > 0.0) || !(v2 < 1.0)) {
#pragma unroll
        for (int q = 0; q < 7; ++q) X[q] = C[q];
      }
      double Bt[3];
      Bt[D] = Bn;
      Bt[t1] = X[5];
      Bt[t2] = X[6];
      State S;
      state_make(G, X, Bt, fa.gam, S);
      if (side == 0) {
        flux_of<D>(G, S, UL, FL);
        speeds_of<D>(G, S, fa.gam, fa.speeds, cmL, cpL);
      } else {
        flux_of<D>(G, S, UR, FR);
        speeds_of<D>(G, S, fa.gam, fa.speeds, cmR, cpR);
      }
    }
    double Fo[7], sm;
    hlle7(UL, FL, cmL, cpL, UR, FR, cmR, cpR, Fo, sm);
#pragma unroll
    for (int q = 0; q < 7; ++q) fa.flux[(size_t)(D * 7 + q) * g.N + id] = Fo[q];
    if (ijk[t1] >= 0 && ijk[t2] >= 0) smax = sm;
  }
  if (fa.red) {
    double w = wave_max(smax);
    if (__lane_id() == 0) atomic_max_pos(fa.red, w);
  }
}

// ---------------------------------------------------------------------------------------
// Cells: flux divergence (eq. fluxconseqs) + geometric sources (eq. grmhdsrc) + div B.
struct CellArgs {
  const double* metric;
  const double* curv;
  const double* prim;
  const double* A;
  const double* bc;
  const double* flux;
  double* rhs;
  double* red;
  double gam;
};

__global__ __launch_bounds__(256) void k_cell(GD g, CellArgs ca) {
  int i, j, k;
  bool valid = box_index<64, 4>(g.n, i, j, k);
  double divb = 0.0;
  if (valid) {
    const int id = at(g, i, j, k);
    const int st[3] = {1, g.sy, g.sz};
    double rhs[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      double s = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double* F = ca.flux + (size_t)(d * 7 + c) * g.N;
        s += (F[id + st[d]] - F[id]) * g.idx[d];
      }
      rhs[c] = -s;
    }
    // metric, derivatives and K at the centre
    const int vb = id - 1 - g.sy - g.sz;
    double m[10], dm[3][10];
#pragma unroll
    for (int c = 0; c < 10; ++c) {
      double dx, dy, dz;
      centre_val_der(ca.metric + c * g.N + vb, g.sy, g.sz, m[c], dx, dy, dz);
      dm[0][c] = dx * g.idx[0];
      dm[1][c] = dy * g.idx[1];
      dm[2][c] = dz * g.idx[2];
    }
    double K[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) K[c] = centre_val(ca.curv + c * g.N + vb, g.sy, g.sz);
    Geo G;
    geo_from(m, G);
    double pr[5], Bt[3];
#pragma unroll
    for (int c = 0; c < 5; ++c) pr[c] = ca.prim[c * g.N + id];
    Bt[0] = ca.bc[id];
    Bt[1] = ca.bc[g.N + id];
    Bt[2] = ca.bc[2 * g.N + id];
    State S;
    state_make(G, pr, Bt, ca.gam, S);
    // T^{mu nu} = (rho h + b^2) u u + (p + b^2/2) g^{mu nu} - b b   (eq. tmunu)
    double ia = 1.0 / G.alp, ia2 = ia * ia;
    double u0 = S.W * ia, u[3], b0 = S.W * S.Bv * ia, bu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      u[a] = S.W * (S.v[a] - G.beta[a] * ia);
      bu[a] = (S.B[a] + G.alp * b0 * u[a]) / S.W;
    }
    double e = S.rhoh + S.bsq, pt = S.p + 0.5 * S.bsq;
    double T00 = e * u0 * u0 - pt * ia2 - b0 * b0;
    double T0[3], Tk[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) T0[a] = e * u0 * u[a] + pt * G.beta[a] * ia2 - b0 * bu[a];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int bb = a; bb < 3; ++bb)
        Tk[sym(a, bb)] = e * u[a] * u[bb] + pt * (G.gu[sym(a, bb)] - G.beta[a] * G.beta[bb] * ia2) - bu[a] * bu[bb];
    double bl[3];
    lower(G.g, G.beta, bl);
    double as = G.alp * G.sqrtg;
    // momentum sources: 1/2 T^{mu nu} d_j g_{mu nu}
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      const double* dg = &dm[jj][4];
      const double dal = dm[jj][0];
      const double db[3] = {dm[jj][1], dm[jj][2], dm[jj][3]};
      // beta^k beta^l d gamma_kl and T^kl d gamma_kl (symmetric sums)
      double bbdg = 0.0, Tdg = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
          bbdg += G.beta[a] * G.beta[bb] * dg[sym(a, bb)];
          Tdg += Tk[sym(a, bb)] * dg[sym(a, bb)];
        }
      double d00 = -2.0 * G.alp * dal + bbdg + 2.0 * (bl[0] * db[0] + bl[1] * db[1] + bl[2] * db[2]);
      double s0k = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double d0a = 0.0;
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) d0a += G.beta[bb] * dg[sym(a, bb)] + G.g[sym(a, bb)] * db[bb];
        s0k += T0[a] * d0a;
      }
      rhs[1 + jj] += as * (0.5 * T00 * d00 + s0k + 0.5 * Tdg);
    }
    // energy source: T^00 (beta beta K - beta.d alpha) + T^0k (2 beta^l K_kl - d_k alpha) + T^kl K_kl
    double dal[3] = {dm[0][0], dm[1][0], dm[2][0]};
    double bK[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) bK[a] = G.beta[0] * K[sym(a, 0)] + G.beta[1] * K[sym(a, 1)] + G.beta[2] * K[sym(a, 2)];
    double se = T00 * (G.beta[0] * bK[0] + G.beta[1] * bK[1] + G.beta[2] * bK[2] -
                       (G.beta[0] * dal[0] + G.beta[1] * dal[1] + G.beta[2] * dal[2]));
#pragma unroll
    for (int a = 0; a < 3; ++a) se += T0[a] * (2.0 * bK[a] - dal[a]);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) se += Tk[sym(a, bb)] * K[sym(a, bb)];
    rhs[4] += as * se;
#pragma unroll
    for (int c = 0; c < 5; ++c) ca.rhs[c * g.N + id] = rhs[c];
    if (ca.red) {
      const double* Ax = ca.A;
      const double* Ay = ca.A + g.N;
      const double* Az = ca.A + 2 * g.N;
      double dB = (faceBx(Ay, Az, id + 1, g.sy, g.sz, g) - faceBx(Ay, Az, id, g.sy, g.sz, g)) * g.idx[0] +
                  (faceBy(Ax, Az, id + g.sy, g.sy, g.sz, g) - faceBy(Ax, Az, id, g.sy, g.sz, g)) * g.idx[1] +
                  (faceBz(Ax, Ay, id + g.sz, g.sy, g.sz, g) - faceBz(Ax, Ay, id, g.sy, g.sz, g)) * g.idx[2];
      divb = fabs(dB);
    }
  }
  if (ca.red) {
    double w = wave_max(divb);
    if (__lane_id() == 0) atomic_max_pos(ca.red + 1, w);
  }
}

// ---------------------------------------------------------------------------------------
// Vertices in [-1, n]^3: G_A = alpha Psi / sqrt(gamma) - beta^j A_j and
// F_Psi^j = alpha sqrt(gamma) gamma^jk A_k - beta^j Psi, with A averaged to the vertex
// along its own direction (Sec. 3.4).
__global__ __launch_bounds__(256) void k_vertex(GD g, const double* __restrict__ metric, const double* __restrict__ A,
                                                const double* __restrict__ psi, double* __restrict__ ga,
                                                double* __restrict__ fp) {
  int e[3] = {g.n[0] + 2, g.n[1] + 2, g.n[2] + 2};
  int a, b, c;
  if (!box_index<64, 4>(e, a, b, c)) return;
  const int id = at(g, a - 1, b - 1, c - 1);
  double m[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) m[q] = metric[q * g.N + id];
  Geo G;
  geo_from(m, G);
  double Av[3];
  Av[0] = 0.5 * (A[id - 1] + A[id]);
  Av[1] = 0.5 * (A[g.N + id - g.sy] + A[g.N + id]);
  Av[2] = 0.5 * (A[2 * g.N + id - g.sz] + A[2 * g.N + id]);
  double ps = psi[id];
  ga[id] = G.alp * ps / G.sqrtg - (G.beta[0] * Av[0] + G.beta[1] * Av[1] + G.beta[2] * Av[2]);
  double as = G.alp * G.sqrtg;
  fp[id] = as * (G.gu[0] * Av[0] + G.gu[1] * Av[1] + G.gu[2] * Av[2]) - G.beta[0] * ps;
  fp[g.N + id] = as * (G.gu[1] * Av[0] + G.gu[3] * Av[1] + G.gu[4] * Av[2]) - G.beta[1] * ps;
  fp[2 * g.N + id] = as * (G.gu[2] * Av[0] + G.gu[4] * Av[1] + G.gu[5] * Av[2]) - G.beta[2] * ps;
}

// Owned edges and vertices: E by flux-CT (average of the four face induction fluxes around
// each edge; E = -vt x Btilde), dA/dt = -E - grad G_A, dPsi/dt = -div F_Psi - xi alpha Psi.
struct EdgeArgs {
  const double* metric;
  const double* psi;
  const double* flux;
  const double* ga;
  const double* fp;
  double* rhs;
  double xi;
  int gauge;
};

__global__ __launch_bounds__(256) void k_edge(GD g, EdgeArgs ea) {
  int i, j, k;
  if (!box_index<64, 4>(g.n, i, j, k)) return;
  const int id = at(g, i, j, k);
  const int sy = g.sy, sz = g.sz;
  const double* Fx_By = ea.flux + (size_t)(0 * 7 + 5) * g.N;
  const double* Fx_Bz = ea.flux + (size_t)(0 * 7 + 6) * g.N;
  const double* Fy_Bz = ea.flux + (size_t)(1 * 7 + 5) * g.N;
  const double* Fy_Bx = ea.flux + (size_t)(1 * 7 + 6) * g.N;
  const double* Fz_Bx = ea.flux + (size_t)(2 * 7 + 5) * g.N;
  const double* Fz_By = ea.flux + (size_t)(2 * 7 + 6) * g.N;
  double Ez = 0.25 * (-Fx_By[id] - Fx_By[id - sy] + Fy_Bx[id] + Fy_Bx[id - 1]);
  double Ex = 0.25 * (-Fy_Bz[id] - Fy_Bz[id - sz] + Fz_By[id] + Fz_By[id - sy]);
  double Ey = 0.25 * (-Fz_Bx[id] - Fz_Bx[id - 1] + Fx_Bz[id] + Fx_Bz[id - sz]);
  double* r = ea.rhs;
  if (ea.gauge == ASTERX_GAUGE_LORENZ) {
    double G0 = ea.ga[id];
    r[5 * g.N + id] = -Ex - (ea.ga[id + 1] - G0) * g.idx[0];
    r[6 * g.N + id] = -Ey - (ea.ga[id + sy] - G0) * g.idx[1];
    r[7 * g.N + id] = -Ez - (ea.ga[id + sz] - G0) * g.idx[2];
    const double* f0 = ea.fp;
    const double* f1 = ea.fp + g.N;
    const double* f2 = ea.fp + 2 * g.N;
    double div = (f0[id + 1] - f0[id - 1]) * (0.5 * g.idx[0]) + (f1[id + sy] - f1[id - sy]) * (0.5 * g.idx[1]) +
                 (f2[id + sz] - f2[id - sz]) * (0.5 * g.idx[2]);
    r[8 * g.N + id] = -div - ea.xi * ea.metric[id] * ea.psi[id];
  } else {
    r[5 * g.N + id] = -Ex;
    r[6 * g.N + id] = -Ey;
    r[7 * g.N + id] = -Ez;
    r[8 * g.N + id] = 0.0;
  }
}

// ---------------------------------------------------------------------------------------
// RK combine on owned points of 9 fields.
struct RKArgs {
  const double* u[4];
  double a[4];
  int nterms;
  double b_dt;
  const double* rhs;
  double* out;
};

__global__ __launch_bounds__(256) void k_rk(GD g, RKArgs ra) {
  int i, j, k;
  if (!box_index<64, 4>(g.n, i, j, k)) return;
  const int id = at(g, i, j, k);
#pragma unroll
  for (int f = 0; f < 9; ++f) {
    size_t o = (size_t)f * g.N + id;
    double s = ra.b_dt * ra.rhs[o];
    for (int m = 0; m < ra.nterms; ++m) s += ra.a[m] * ra.u[m][o];
    ra.out[o] = s;
  }
}

__global__ void k_zero(double* p, long long n) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0.0;
}

// ---------------------------------------------------------------------------------------
int check_grid(const asterx_grid* g, int min_ng) {
  if (!g) return fail(ASTERX_EARG, "grid is NULL");
  for (int a = 0; a < 3; ++a) {
    if (g->n[a] < 1) return fail(ASTERX_EARG, "grid: n must be >= 1");
    if (g->ld[a] < g->n[a] + 2 * g->ng + 1) return fail(ASTERX_EARG, "grid: ld must be >= n + 2 ng + 1");
    if (!(g->dx[a] > 0.0)) return fail(ASTERX_EARG, "grid: dx must be > 0");
  }
  if (g->ng < min_ng) return fail(ASTERX_EARG, "grid: too few ghost layers for this stencil");
  double npts = (double)g->ld[0] * g->ld[1] * g->ld[2];
  if (npts >= 2147483647.0) return fail(ASTERX_EARG, "grid: ld[0]*ld[1]*ld[2] must be below 2^31");
  return 0;
}

int check_params(const asterx_params* p) {
  if (!p) return fail(ASTERX_EARG, "params is NULL");
  if (!(p->gamma > 1.0)) return fail(ASTERX_EARG, "params: gamma must be > 1");
  if (p->recon < 0 || p->recon > 2) return fail(ASTERX_EARG, "params: unknown reconstruction");
  if (p->gauge < 0 || p->gauge > 1) return fail(ASTERX_EARG, "params: unknown gauge");
  if (p->speeds < 0 || p->speeds > 1) return fail(ASTERX_EARG, "params: unknown speed estimate");
  if (p->c2p_method < 0 || p->c2p_method > 2) return fail(ASTERX_EARG, "params: unknown c2p method");
  if (!(p->wmax > 1.0)) return fail(ASTERX_EARG, "params: wmax must be > 1");
  if (p->c2p_maxit < 1 || p->brent_maxit < 1) return fail(ASTERX_EARG, "params: iteration caps must be >= 1");
  if (!(p->rho_atm >= 0.0)) return fail(ASTERX_EARG, "params: rho_atm must be >= 0");
  return 0;
}

int launched() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_err = std::string("launch failed: ") + hipGetErrorString(e);
    return ASTERX_ELAUNCH;
  }
  return 0;
}

}  // namespace

// =======================================================================================
extern "C" {

int asterx_version(void) { return 1; }

const char* asterx_last_error(void) { return g_err.c_str(); }

size_t asterx_rhs_workspace_size(const asterx_grid* g) {
  if (!g) return 0;
  size_t N = (size_t)g->ld[0] * g->ld[1] * g->ld[2];
  return (3 + 21 + 1 + 3) * N * sizeof(double);
}

int asterx_prim2con(const asterx_grid* g, const asterx_params* p, const double* metric, const double* A,
                    const double* prim, double* cons, void* stream) {
  int rc;
  if ((rc = check_grid(g, 2)) || (rc = check_params(p))) return rc;
  if (!metric || !A || !prim || !cons) return fail(ASTERX_EARG, "prim2con: NULL array");
  GD d = make_gd(g);
  hipLaunchKernelGGL(k_prim2con, dim3(box_blocks<64, 4>(d.n)), dim3(256), 0, (hipStream_t)stream, d, p->gamma,
                     metric, A, prim, cons);
  return launched();
}

int asterx_c2p(const asterx_grid* g, const asterx_params* p, const double* metric, const double* A, double* cons,
               double* prim, uint8_t* flags, asterx_c2p_stats* stats, void* stream) {
  int rc;
  if ((rc = check_grid(g, 2)) || (rc = check_params(p))) return rc;
  if (!metric || !A || !prim || !cons) return fail(ASTERX_EARG, "c2p: NULL array");
  GD d = make_gd(g);
  hipLaunchKernelGGL(k_c2p, dim3(box_blocks<64, 4>(d.n)), dim3(256), 0, (hipStream_t)stream, d, make_c2p_params(p),
                     metric, A, cons, prim, flags, (unsigned long long*)stats);
  return launched();
}

int asterx_fill_ghosts(const asterx_grid* g, double* f, int32_t nf, const int32_t* kinds, void* stream) {
  int rc;
  if ((rc = check_grid(g, 1))) return rc;
  if (!f || !kinds || nf < 1) return fail(ASTERX_EARG, "fill_ghosts: bad arguments");
  GD d = make_gd(g);
  for (int a = 0; a < 3; ++a) {
    if (kinds[a] < 0 || kinds[a] > 2) return fail(ASTERX_EARG, "fill_ghosts: unknown boundary kind");
    if (kinds[a] == ASTERX_BC_LINEAR && g->n[a] < 2) return fail(ASTERX_EARG, "fill_ghosts: LINEAR needs n >= 2");
  }
  for (int a = 0; a < 3; ++a) {
    long long cnt = (long long)nf * (2 * g->ng + 1);
    for (int b = 0; b < 3; ++b)
      if (b != a) cnt *= (g->n[b] + 2 * g->ng + 1);
    FillArgs fa{f, nf, a, kinds[a]};
    unsigned nb = (unsigned)((cnt + 255) / 256);
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, (hipStream_t)stream, d, fa);
    if ((rc = launched())) return rc;
  }
  return 0;
}

int asterx_rhs(const asterx_grid* g, const asterx_params* p, const double* metric, const double* curv,
               const double* prim, const double* A, const double* psi, double dt_max, double* rhs, double* red,
               void* workspace, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_params(p))) return rc;
  // the face kernels load a six-cell stencil (i-3..i+2) for every scheme
  if ((rc = check_grid(g, 3))) return rc;
  if (!metric || !curv || !prim || !A || !psi || !rhs || !workspace)
    return fail(ASTERX_EARG, "rhs: NULL array");
  if (ws_bytes < asterx_rhs_workspace_size(g)) return fail(ASTERX_EARG, "rhs: workspace too small");
  if (!(dt_max > 0.0)) return fail(ASTERX_EARG, "rhs: dt_max must be > 0");
  hipStream_t s = (hipStream_t)stream;
  GD d = make_gd(g);
  double* ws = (double*)workspace;
  double* bc = ws;
  double* flux = ws + 3 * d.N;
  double* ga = ws + 24 * d.N;
  double* fp = ws + 25 * d.N;
  int ebc[3] = {d.n[0] + 2 * d.ng, d.n[1] + 2 * d.ng, d.n[2] + 2 * d.ng};
  hipLaunchKernelGGL(k_bcent, dim3(box_blocks<64, 4>(ebc)), dim3(256), 0, s, d, A, bc);
  if ((rc = launched())) return rc;
  FaceArgs fa{metric, prim, A, bc, flux, red, p->gamma, p->weno_eps, p->weno_q, p->recon, p->speeds};
  int ef[3] = {d.n[0] + 1, d.n[1] + 1, d.n[2] + 1};
  unsigned nbf = box_blocks<64, 4>(ef);
  hipLaunchKernelGGL(k_face<0>, dim3(nbf), dim3(256), 0, s, d, fa);
  hipLaunchKernelGGL(k_face<1>, dim3(nbf), dim3(256), 0, s, d, fa);
  hipLaunchKernelGGL(k_face<2>, dim3(nbf), dim3(256), 0, s, d, fa);
  if ((rc = launched())) return rc;
  CellArgs ca{metric, curv, prim, A, bc, flux, rhs, red, p->gamma};
  hipLaunchKernelGGL(k_cell, dim3(box_blocks<64, 4>(d.n)), dim3(256), 0, s, d, ca);
  if ((rc = launched())) return rc;
  if (p->gauge == ASTERX_GAUGE_LORENZ) {
    int ev[3] = {d.n[0] + 2, d.n[1] + 2, d.n[2] + 2};
    hipLaunchKernelGGL(k_vertex, dim3(box_blocks<64, 4>(ev)), dim3(256), 0, s, d, metric, A, psi, ga, fp);
    if ((rc = launched())) return rc;
  }
  EdgeArgs ea{metric, psi, flux, ga, fp, rhs, p->xi / dt_max, p->gauge};
  hipLaunchKernelGGL(k_edge, dim3(box_blocks<64, 4>(d.n)), dim3(256), 0, s, d, ea);
  return launched();
}

int asterx_rk_stage(const asterx_grid* g, int32_t nterms, const double* a, const double* const* u, double b_dt,
                    const double* rhs, double* out, void* stream) {
  int rc;
  if ((rc = check_grid(g, 1))) return rc;
  if (nterms < 1 || nterms > 4 || !a || !u || !rhs || !out) return fail(ASTERX_EARG, "rk_stage: bad arguments");
  RKArgs ra;
  for (int m = 0; m < 4; ++m) {
    ra.u[m] = m < nterms ? u[m] : nullptr;
    ra.a[m] = m < nterms ? a[m] : 0.0;
    if (m < nterms && !u[m]) return fail(ASTERX_EARG, "rk_stage: NULL state");
  }
  ra.nterms = nterms;
  ra.b_dt = b_dt;
  ra.rhs = rhs;
  ra.out = out;
  GD d = make_gd(g);
  hipLaunchKernelGGL(k_rk, dim3(box_blocks<64, 4>(d.n)), dim3(256), 0, (hipStream_t)stream, d, ra);
  return launched();
}

int asterx_zero(double* buf, int64_t count, void* stream) {
  if (!buf || count < 1) return fail(ASTERX_EARG, "zero: bad arguments");
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream, buf,
                     (long long)count);
  return launched();
}

}  // extern "C"
