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
#include <vector>

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
DEV bool box_index_t(const int e[3], unsigned tid, int& a, int& b, int& c) {
  unsigned nbx = (e[0] + TX - 1) / TX, nby = (e[1] + TY - 1) / TY;
  unsigned nblocks = nbx * nby * (unsigned)e[2];
  unsigned bid = xcd_block(blockIdx.x, nblocks);
  unsigned bx = bid % nbx;
  unsigned t = bid / nbx;
  unsigned by = t % nby;
  c = (int)(t / nby);
  a = (int)(bx * TX + tid % TX);
  b = (int)(by * TY + tid / TX);
  return a < e[0] && b < e[1] && c < e[2];
}

template <int TX, int TY>
DEV bool box_index(const int e[3], int& a, int& b, int& c) {
  return box_index_t<TX, TY>(e, threadIdx.x, a, b, c);
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

// ---------------------------------------------------------------------------------------
// Cell tiles of 16 x 4 x 4 with the spacetime data staged in LDS.  The vertex tile
// (19 x 7 x 7) of one component is loaded once, then interpolated separably -- z, then y,
// then x -- with each pass shared by all cells of the tile (Sec. 3.2 Lagrange weights).
constexpr int CTX = 16, CTY = 4, CTZ = 4;
constexpr int VX = CTX + 3, VY = CTY + 3, VZ = CTZ + 3;
constexpr int NV = VX * VY * VZ;    // vertex tile
constexpr int NZP = VX * VY * CTZ;  // after the z pass
constexpr int NYP = VX * CTY * CTZ; // after the y pass

struct TileLDS {
  double v[NV];
  double z[2 * NZP];
  double y[3 * NYP];
};

struct TileCell {
  int i0, j0, k0, cx, cy, cz;
  bool valid;
};

DEV TileCell tile_cell(const GD& g) {
  TileCell t;
  int ntx = (g.n[0] + CTX - 1) / CTX, nty = (g.n[1] + CTY - 1) / CTY, ntz = (g.n[2] + CTZ - 1) / CTZ;
  unsigned bid = xcd_block(blockIdx.x, (unsigned)(ntx * nty * ntz));
  t.i0 = (int)(bid % ntx) * CTX;
  t.j0 = (int)((bid / ntx) % nty) * CTY;
  t.k0 = (int)(bid / (ntx * nty)) * CTZ;
  t.cx = threadIdx.x % CTX;
  t.cy = (threadIdx.x / CTX) % CTY;
  t.cz = threadIdx.x / (CTX * CTY);
  t.valid = t.i0 + t.cx < g.n[0] && t.j0 + t.cy < g.n[1] && t.k0 + t.cz < g.n[2];
  return t;
}

unsigned tile_blocks(const GD& g) {
  return (unsigned)(((g.n[0] + CTX - 1) / CTX) * ((g.n[1] + CTY - 1) / CTY) * ((g.n[2] + CTZ - 1) / CTZ));
}

// Stage vertices i0-1 .. i0+CTX+1 (etc.) of field f; vertices no owned cell needs (beyond
// n+1, in a ragged last tile) are not read.
DEV void stage_vertices(const GD& g, const double* __restrict__ f, const TileCell& t, double* sv) {
  for (int q = threadIdx.x; q < NV; q += 256) {
    int vx = q % VX, vy = (q / VX) % VY, vz = q / (VX * VY);
    int i = t.i0 - 1 + vx, j = t.j0 - 1 + vy, k = t.k0 - 1 + vz;
    sv[q] = (i <= g.n[0] + 1 && j <= g.n[1] + 1 && k <= g.n[2] + 1) ? f[at(g, i, j, k)] : 0.0;
  }
}

// Centre value of the staged component (every thread of the block must call it).
DEV double tile_value(TileLDS& S, const TileCell& t) {
  __syncthreads();
  for (int q = threadIdx.x; q < NZP; q += 256) {
    int vx = q % VX, vy = (q / VX) % VY, z = q / (VX * VY);
    const double* p = S.v + vx + VX * (vy + VY * z);
    S.z[q] = lag(p[0], p[VX * VY], p[2 * VX * VY], p[3 * VX * VY]);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NYP; q += 256) {
    int vx = q % VX, y = (q / VX) % CTY, z = q / (VX * CTY);
    const double* p = S.z + vx + VX * (y + VY * z);
    S.y[q] = lag(p[0], p[VX], p[2 * VX], p[3 * VX]);
  }
  __syncthreads();
  const double* p = S.y + t.cx + VX * (t.cy + CTY * t.cz);
  return lag(p[0], p[1], p[2], p[3]);
}

// Centre derivatives (d/dx, d/dy, d/dz, scaled) of the staged component.
DEV void tile_derivs(TileLDS& S, const TileCell& t, const GD& g, double d[3]) {
  __syncthreads();
  for (int q = threadIdx.x; q < NZP; q += 256) {
    int vx = q % VX, vy = (q / VX) % VY, z = q / (VX * VY);
    const double* p = S.v + vx + VX * (vy + VY * z);
    double a = p[0], b = p[VX * VY], c = p[2 * VX * VY], e = p[3 * VX * VY];
    S.z[q] = lag(a, b, c, e);
    S.z[NZP + q] = dlag(a, b, c, e);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NYP; q += 256) {
    int vx = q % VX, y = (q / VX) % CTY, z = q / (VX * CTY);
    const double* p = S.z + vx + VX * (y + VY * z);
    const double* r = p + NZP;
    double a = p[0], b = p[VX], c = p[2 * VX], e = p[3 * VX];
    S.y[q] = lag(a, b, c, e);
    S.y[NYP + q] = dlag(a, b, c, e);
    S.y[2 * NYP + q] = lag(r[0], r[VX], r[2 * VX], r[3 * VX]);
  }
  __syncthreads();
  const double* p = S.y + t.cx + VX * (t.cy + CTY * t.cz);
  d[0] = dlag(p[0], p[1], p[2], p[3]) * g.idx[0];
  d[1] = lag(p[NYP], p[NYP + 1], p[NYP + 2], p[NYP + 3]) * g.idx[1];
  d[2] = lag(p[2 * NYP], p[2 * NYP + 1], p[2 * NYP + 2], p[2 * NYP + 3]) * g.idx[2];
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

// c2p on owned cells, tiled: the ten metric components are interpolated to the centres
// through LDS (Sec. 3.2), then each thread recovers its cell (Secs. 3.5, 3.6).
__global__ __launch_bounds__(256) void k_c2p_t(GD g, C2PParams P, const double* __restrict__ metric,
                                               const double* __restrict__ A, double* __restrict__ cons,
                                               double* __restrict__ prim, uint8_t* __restrict__ flags,
                                               unsigned long long* __restrict__ stats) {
  __shared__ TileLDS S;
  const TileCell t = tile_cell(g);
  double m[10];
#pragma unroll
  for (int c = 0; c < 10; ++c) {
    if (c > 0) __syncthreads();
    stage_vertices(g, metric + c * g.N, t, S.v);
    m[c] = tile_value(S, t);
  }
  uint32_t fl = 0;
  int iters = 0;
  if (t.valid) {
    const int id = at(g, t.i0 + t.cx, t.j0 + t.cy, t.k0 + t.cz);
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
  // ghost values are a pure function of owned values: no contraction, so that linear
  // extrapolation rounds exactly like its definition (one multiply, then one add)
#pragma clang fp contract(off)
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

// Paired-lane variant: lanes 2f and 2f+1 of a wavefront handle the left and the right state
// of face f.  Each lane reconstructs its own side (the right lane reads its stencil
// mirrored, so both run the "right face of the middle cell" formula), interpolates half of
// the face metric, and computes the conserved vector, flux and speeds of its side; the pair
// exchanges metric halves and side results through lane shuffles and both evaluate HLLE,
// the left lane storing components 0-3, the right lane 4-6.  Half the live state per lane
// of a one-lane-per-face kernel, twice the lanes in flight.
DEV double shfl1(double v) { return __shfl_xor(v, 1, 64); }

DEV double recon_right_face(int kind, const double a[5], double eps, double q) {
  if (kind == 0) return a[2] + 0.5 * mm(a[2] - a[1], a[3] - a[2]);
  if (kind == 1) {
    double s1 = mc_slope(a[0], a[1], a[2]);
    double s2 = mc_slope(a[1], a[2], a[3]);
    double s3 = mc_slope(a[2], a[3], a[4]);
    const double sixth = 1.0 / 6.0;
    double fl = 0.5 * (a[1] + a[2]) - (s2 - s1) * sixth;
    double fr = 0.5 * (a[2] + a[3]) - (s3 - s2) * sixth;
    ppm_limit(a[2], fl, fr);
    return fr;
  }
  return wenoz_face(a[0], a[1], a[2], a[3], a[4], eps, q);
}

template <int D>
__global__ __launch_bounds__(256) void k_face2(GD g, FaceArgs fa) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  const int side = threadIdx.x & 1;
  int e[3] = {g.n[0] + 1, g.n[1] + 1, g.n[2] + 1};
  int a, b, c;
  bool valid = box_index_t<32, 4>(e, threadIdx.x >> 1, a, b, c);
  // keep both lanes of a pair valid or invalid together (they share the face)
  double smax = 0.0;
  if (valid) {
    int ijk[3] = {a - 1, b - 1, c - 1};
    ijk[D] += 1;
    const int id = at(g, ijk[0], ijk[1], ijk[2]);
    const int st[3] = {1, g.sy, g.sz};
    const int sD = st[D], s1 = st[t1], s2 = st[t2];
    // reconstruction of this lane's side: left lane cells i-3..i+1, right lane i+2..i-2
    double X[7], C[7];
    const int o0 = side ? 2 : -3, os = side ? -1 : 1;
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      const double* f = v < 5 ? fa.prim + v * g.N : fa.bc + (v == 5 ? t1 : t2) * g.N;
      double s5[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) s5[q] = f[id + (o0 + os * q) * sD];
      X[v] = recon_right_face(fa.recon, s5, fa.weno_eps, fa.weno_q);
      C[v] = s5[2];
    }
    // face metric: this lane interpolates components [5 side, 5 side + 5)
    double mine[5];
    const int mb = id - s1 - s2;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const double* p = fa.metric + (size_t)(5 * side + q) * g.N + mb;
      double rr[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double* row = p + r * s2;
        rr[r] = lag(row[0], row[s1], row[2 * s1], row[3 * s1]);
      }
      mine[q] = lag(rr[0], rr[1], rr[2], rr[3]);
    }
    double m[10];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      double other = shfl1(mine[q]);
      m[q] = side ? other : mine[q];
      m[5 + q] = side ? mine[q] : other;
    }
    Geo G;
    geo_from(m, G);
    const double* Ax = fa.A;
    const double* Ay = fa.A + g.N;
    const double* Az = fa.A + 2 * g.N;
    double Bn = D == 0 ? faceBx(Ay, Az, id, g.sy, g.sz, g)
                       : (D == 1 ? faceBy(Ax, Az, id, g.sy, g.sz, g) : faceBz(Ax, Ay, id, g.sy, g.sz, g));
    // an unphysical reconstructed state falls back to the cell's own values
    {
      double vl[3], v[3] = {X[2], X[3], X[4]};
      lower(G.g, v, vl);
      double v2 = v[0] * vl[0] + v[1] * vl[1] + v[2] * vl[2];
      if (!(X[0] > 0.0) || !(X[1] > 0.0) || !(v2 < 1.0)) {
#pragma unroll
        for (int q = 0; q < 7; ++q) X[q] = C[q];
      }
    }
    double Bt[3];
    Bt[D] = Bn;
    Bt[t1] = X[5];
    Bt[t2] = X[6];
    State S;
    state_make(G, X, Bt, fa.gam, S);
    double U[7], F[7], cm, cp;
    flux_of<D>(G, S, U, F);
    speeds_of<D>(G, S, fa.gam, fa.speeds, cm, cp);
    // exchange with the partner lane and combine (HLLE, eq. HLLEfluxes)
    double Uo[7], Fo[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      Uo[q] = shfl1(U[q]);
      Fo[q] = shfl1(F[q]);
    }
    double cmo = shfl1(cm), cpo = shfl1(cp);
    double cmax = fmax(0.0, fmax(cp, cpo));
    double cmin = -fmin(0.0, fmin(cm, cmo));
    double den = cmax + cmin;
    double id_ = den > 0.0 ? 1.0 / den : 0.0;
    double cc = cmax * cmin;
    double out[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      double UL = side ? Uo[q] : U[q], UR = side ? U[q] : Uo[q];
      double FL = side ? Fo[q] : F[q], FR = side ? F[q] : Fo[q];
      out[q] = den > 0.0 ? (cmin * FR + cmax * FL - cc * (UR - UL)) * id_ : 0.5 * (FL + FR);
    }
    if (side == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) fa.flux[(size_t)(D * 7 + q) * g.N + id] = out[q];
    } else {
#pragma unroll
      for (int q = 4; q < 7; ++q) fa.flux[(size_t)(D * 7 + q) * g.N + id] = out[q];
    }
    if (ijk[t1] >= 0 && ijk[t2] >= 0) smax = fmax(cmax, cmin);
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

// Tiled cell kernel.  Pass 1 interpolates the values of the 10 metric and 6 curvature
// components through LDS; the stress tensor follows.  The momentum source
// 1/2 T^{mu nu} d_j g_{mu nu} is linear in the derivatives of the stored components,
// sum_c w_c d_j m_c with weights w_c built from T, beta and gamma, so pass 2 takes one
// component's three derivatives at a time and accumulates them (few live registers).
__global__ __launch_bounds__(256) void k_cell_t(GD g, CellArgs ca) {
  __shared__ TileLDS S;
  const TileCell t = tile_cell(g);
  double m[10], K[6];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    if (c > 0) __syncthreads();
    stage_vertices(g, c < 10 ? ca.metric + c * g.N : ca.curv + (c - 10) * g.N, t, S.v);
    double v = tile_value(S, t);
    if (c < 10) m[c] = v; else K[c - 10] = v;
  }
  const int id = t.valid ? at(g, t.i0 + t.cx, t.j0 + t.cy, t.k0 + t.cz) : 0;
  double w[10], wa[3], src[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, as = 0.0;
  if (t.valid) {
    Geo G;
    geo_from(m, G);
    double pr[5], Bt[3];
#pragma unroll
    for (int c = 0; c < 5; ++c) pr[c] = ca.prim[c * g.N + id];
    Bt[0] = ca.bc[id];
    Bt[1] = ca.bc[g.N + id];
    Bt[2] = ca.bc[2 * g.N + id];
    State St;
    state_make(G, pr, Bt, ca.gam, St);
    // T^{mu nu} = (rho h + b^2) u u + (p + b^2/2) g^{mu nu} - b b   (eq. tmunu)
    double ia = 1.0 / G.alp, ia2 = ia * ia;
    double u0 = St.W * ia, u[3], b0 = St.W * St.Bv * ia, bu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      u[a] = St.W * (St.v[a] - G.beta[a] * ia);
      bu[a] = (St.B[a] + G.alp * b0 * u[a]) / St.W;
    }
    double e = St.rhoh + St.bsq, pt = St.p + 0.5 * St.bsq;
    double T00 = e * u0 * u0 - pt * ia2 - b0 * b0;
    double T0[3], Tk[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) T0[a] = e * u0 * u[a] + pt * G.beta[a] * ia2 - b0 * bu[a];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b)
        Tk[sym(a, b)] = e * u[a] * u[b] + pt * (G.gu[sym(a, b)] - G.beta[a] * G.beta[b] * ia2) - bu[a] * bu[b];
    double bl[3];
    lower(G.g, G.beta, bl);
    as = G.alp * G.sqrtg;
    // weights of d_j alpha, d_j beta^k, d_j gamma_ab in 1/2 T^{mu nu} d_j g_{mu nu}
    w[0] = -T00 * G.alp;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      w[1 + k] = T00 * bl[k] + T0[0] * G.g[sym(0, k)] + T0[1] * G.g[sym(1, k)] + T0[2] * G.g[sym(2, k)];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) {
        if (a == b)
          w[4 + sym(a, b)] = 0.5 * T00 * G.beta[a] * G.beta[a] + T0[a] * G.beta[a] + 0.5 * Tk[sym(a, a)];
        else
          w[4 + sym(a, b)] = T00 * G.beta[a] * G.beta[b] + T0[a] * G.beta[b] + T0[b] * G.beta[a] + Tk[sym(a, b)];
      }
    // energy source: K terms now, the lapse-gradient terms with the derivatives of alpha
    double se = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        se += (T00 * G.beta[a] * G.beta[b] + 2.0 * T0[a] * G.beta[b] + Tk[sym(a, b)]) * K[sym(a, b)];
    src[4] = se;
#pragma unroll
    for (int a = 0; a < 3; ++a) wa[a] = -(T00 * G.beta[a] + T0[a]);
  }
#pragma unroll
  for (int c = 0; c < 10; ++c) {
    __syncthreads();
    stage_vertices(g, ca.metric + c * g.N, t, S.v);
    double d[3];
    tile_derivs(S, t, g, d);
    if (t.valid) {
      src[1] += w[c] * d[0];
      src[2] += w[c] * d[1];
      src[3] += w[c] * d[2];
      if (c == 0) src[4] += wa[0] * d[0] + wa[1] * d[1] + wa[2] * d[2];
    }
  }
  double divb = 0.0;
  if (t.valid) {
    const int st[3] = {1, g.sy, g.sz};
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      double sdiv = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double* F = ca.flux + (size_t)(d * 7 + c) * g.N;
        sdiv += (F[id + st[d]] - F[id]) * g.idx[d];
      }
      ca.rhs[c * g.N + id] = as * src[c] - sdiv;
    }
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
    double wm = wave_max(divb);
    if (__lane_id() == 0) atomic_max_pos(ca.red + 1, wm);
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

// ---------------------------------------------------------------------------------------
// Optional per-kernel timing: when enabled, every launch is bracketed by two HIP events on
// its own stream; asterx_timing_read waits for them and accumulates elapsed times.  Not for
// use while a stream is being captured into a graph.
enum {
  KT_PRIM2CON, KT_C2P, KT_FILL, KT_BCENT, KT_FACE_X, KT_FACE_Y, KT_FACE_Z, KT_CELL, KT_VERTEX, KT_EDGE, KT_RK,
  KT_ZERO, KT_N
};
const char* const kt_names[KT_N] = {"prim2con", "c2p", "fill_ghosts", "centre_B", "face_x", "face_y",
                                    "face_z", "cell", "vertex", "edge", "rk_stage", "zero"};
struct Pending {
  hipEvent_t a, b;
  int kind;
};
bool g_timing = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_free_events;
double g_ms[KT_N];
long long g_count[KT_N];

hipEvent_t take_event() {
  if (!g_free_events.empty()) {
    hipEvent_t e = g_free_events.back();
    g_free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

template <class F>
int timed(int kind, hipStream_t s, F&& launch) {
  if (!g_timing) {
    launch();
    return launched();
  }
  hipEvent_t a = take_event(), b = take_event();
  bool ok = a && b && hipEventRecord(a, s) == hipSuccess;
  launch();
  int rc = launched();
  ok = ok && hipEventRecord(b, s) == hipSuccess;
  if (ok) {
    g_pending.push_back(Pending{a, b, kind});
  } else {
    if (a) g_free_events.push_back(a);
    if (b) g_free_events.push_back(b);
  }
  return rc;
}

}  // namespace

// =======================================================================================
extern "C" {

int asterx_timing_enable(int32_t on) {
  g_timing = on != 0;
  return 0;
}

int asterx_timing_read(double* ms, long long* counts, int32_t n) {
  for (const Pending& p : g_pending) {
    float t = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
      g_ms[p.kind] += t;
      g_count[p.kind] += 1;
    }
    g_free_events.push_back(p.a);
    g_free_events.push_back(p.b);
  }
  g_pending.clear();
  for (int k = 0; k < n && k < KT_N; ++k) {
    if (ms) ms[k] = g_ms[k];
    if (counts) counts[k] = g_count[k];
  }
  return KT_N;
}

int asterx_timing_reset(void) {
  asterx_timing_read(nullptr, nullptr, 0);
  for (int k = 0; k < KT_N; ++k) {
    g_ms[k] = 0.0;
    g_count[k] = 0;
  }
  return 0;
}

const char* asterx_timing_name(int32_t k) { return (k >= 0 && k < KT_N) ? kt_names[k] : ""; }

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
  hipStream_t s = (hipStream_t)stream;
  return timed(KT_PRIM2CON, s, [&] {
    hipLaunchKernelGGL(k_prim2con, dim3(box_blocks<64, 4>(d.n)), dim3(256), 0, s, d, p->gamma, metric, A, prim,
                       cons);
  });
}

int asterx_c2p(const asterx_grid* g, const asterx_params* p, const double* metric, const double* A, double* cons,
               double* prim, uint8_t* flags, asterx_c2p_stats* stats, void* stream) {
  int rc;
  if ((rc = check_grid(g, 2)) || (rc = check_params(p))) return rc;
  if (!metric || !A || !prim || !cons) return fail(ASTERX_EARG, "c2p: NULL array");
  GD d = make_gd(g);
  hipStream_t s = (hipStream_t)stream;
  C2PParams cp = make_c2p_params(p);
  return timed(KT_C2P, s, [&] {
    hipLaunchKernelGGL(k_c2p_t, dim3(tile_blocks(d)), dim3(256), 0, s, d, cp, metric, A, cons, prim, flags,
                       (unsigned long long*)stats);
  });
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
    hipStream_t s = (hipStream_t)stream;
    if ((rc = timed(KT_FILL, s, [&] { hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, s, d, fa); }))) return rc;
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
  if ((rc = timed(KT_BCENT, s, [&] { hipLaunchKernelGGL(k_bcent, dim3(box_blocks<64, 4>(ebc)), dim3(256), 0, s, d, A, bc); })))
    return rc;
  FaceArgs fa{metric, prim, A, bc, flux, red, p->gamma, p->weno_eps, p->weno_q, p->recon, p->speeds};
  int ef[3] = {d.n[0] + 1, d.n[1] + 1, d.n[2] + 1};
  unsigned nbf = box_blocks<32, 4>(ef);
  if ((rc = timed(KT_FACE_X, s, [&] { hipLaunchKernelGGL(k_face2<0>, dim3(nbf), dim3(256), 0, s, d, fa); }))) return rc;
  if ((rc = timed(KT_FACE_Y, s, [&] { hipLaunchKernelGGL(k_face2<1>, dim3(nbf), dim3(256), 0, s, d, fa); }))) return rc;
  if ((rc = timed(KT_FACE_Z, s, [&] { hipLaunchKernelGGL(k_face2<2>, dim3(nbf), dim3(256), 0, s, d, fa); }))) return rc;
  CellArgs ca{metric, curv, prim, A, bc, flux, rhs, red, p->gamma};
  if ((rc = timed(KT_CELL, s, [&] { hipLaunchKernelGGL(k_cell_t, dim3(tile_blocks(d)), dim3(256), 0, s, d, ca); })))
    return rc;
  if (p->gauge == ASTERX_GAUGE_LORENZ) {
    int ev[3] = {d.n[0] + 2, d.n[1] + 2, d.n[2] + 2};
    if ((rc = timed(KT_VERTEX, s, [&] {
           hipLaunchKernelGGL(k_vertex, dim3(box_blocks<64, 4>(ev)), dim3(256), 0, s, d, metric, A, psi, ga, fp);
         })))
      return rc;
  }
  EdgeArgs ea{metric, psi, flux, ga, fp, rhs, p->xi / dt_max, p->gauge};
  return timed(KT_EDGE, s, [&] { hipLaunchKernelGGL(k_edge, dim3(box_blocks<64, 4>(d.n)), dim3(256), 0, s, d, ea); });
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
  hipStream_t s = (hipStream_t)stream;
  return timed(KT_RK, s, [&] { hipLaunchKernelGGL(k_rk, dim3(box_blocks<64, 4>(d.n)), dim3(256), 0, s, d, ra); });
}

int asterx_zero(double* buf, int64_t count, void* stream) {
  if (!buf || count < 1) return fail(ASTERX_EARG, "zero: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  return timed(KT_ZERO, s, [&] {
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, buf, (long long)count);
  });
}

}  // extern "C"
