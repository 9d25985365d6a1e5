// asterx.hip -- HIP kernels (gfx950, FP64) and the C ABI of the Valencia GRMHD right-hand side.
//
// One block, one GPU.  Per RK stage the caller runs: asterx_c2p -> asterx_fill_ghosts(prim)
// -> asterx_rhs -> asterx_rk_stage -> asterx_fill_ghosts(state).  asterx_rhs itself is
// centre field + six launches:
//   face<D> (D = x, y, z): reconstruction + face metric + prim->cons + fluxes + speeds + HLLE,
//                          two lanes per face (left and right state), x-pencil coalesced;
//   cell:                  flux divergence + geometric sources + div B, LDS-tiled metric;
//   vertex:                gauge quantities G_A and F_Psi at vertices;
//   edge:                  FCT electric field, dA/dt and dPsi/dt.
// Threads map to x fastest so every stencil load is coalesced across a wavefront; the
// block -> tile map keeps neighbouring tiles on one XCD (shared L2).  The same bodies run in
// persistent launches over work lists of (patch, tile) items for batches of patches, and the
// reverse-mode (adjoint) kernels at the end of the file transpose one stage.
// Section/equation references are to AsterX, arXiv 2406.11669.

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "asterx.h"
#include "grmhd_device.h"
#include "host_internal.h"
#include "mlp_device.h"

using namespace ax;

namespace {

thread_local std::string g_err;

// rhs workspace: centre field (3) + face fluxes (3 directions x 7) + G_A (1) + F_Psi (3)
// right-hand side workspace: centre field 3, face fluxes 21, G_A 1, F_Psi 3, upwind-CT speeds and face
// fields 9
constexpr int WS_FIELDS = 3 + 21 + 1 + 3 + 9;

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

// Element i >= 0 of a field whose base is the same for the whole wavefront: the address is
// formed by the load from the scalar base and a 32-bit per-lane byte offset (fields hold fewer
// than 2^29 points, checked on the host), instead of a 64-bit vector add per access.
template <class T>
DEV T ldu(const T* base, int i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (unsigned)i * (unsigned)sizeof(T));
}

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

// Linear tile decomposition of a 3-D box of extents e[3] into tiles of TX x TY x 1; `tile`
// is the logical tile index, `tid` the thread's index inside the tile.
template <int TX, int TY>
DEV bool box_at(const int e[3], unsigned tile, unsigned tid, int& a, int& b, int& c) {
  unsigned nbx = (e[0] + TX - 1) / TX, nby = (e[1] + TY - 1) / TY;
  unsigned bx = tile % nbx;
  unsigned t = tile / nbx;
  unsigned by = t % nby;
  c = (int)(t / nby);
  a = (int)(bx * TX + tid % TX);
  b = (int)(by * TY + tid / TX);
  return a < e[0] && b < e[1] && c < e[2];
}

// Linear decomposition of a 3-D box into tiles of 256 consecutive points (x fastest): for
// per-point kernels over extents that are not multiples of a tile row (n + 2, n + 2 ng).
DEV bool lin_at(const int e[3], unsigned tile, unsigned tid, int& a, int& b, int& c) {
  const long long q = (long long)tile * 256 + tid;
  a = (int)(q % e[0]);
  const long long t = q / e[0];
  b = (int)(t % e[1]);
  c = (int)(t / e[1]);
  return c < e[2];
}
inline unsigned lin_blocks(const int e[3]) { return (unsigned)(((long long)e[0] * e[1] * e[2] + 255) / 256); }

// Face tiles.  Face grids are n + 1 wide (129 for n = 128), so 32-wide tile rows would leave
// up to 31 of every 160 lanes idle.  In each z plane, the x range rounded down to a multiple
// of 32 is tiled 32 x 4 (x, y); the remaining x columns (fewer than 32) follow in the same
// plane, 128 faces per tile, x fastest.  Keeping them beside their plane's main tiles spreads
// these slower, uncoalesced tiles evenly over the XCDs.  Rows narrower than 32 are tiled whole.
struct FacePlan {
  int e0m, r;           // main x range [0, e0m), remainder width r
  unsigned nbx, nby;    // main tiles per plane: nbx x nby
  unsigned pm, per;     // main tiles per plane, all tiles per plane
};
__host__ __device__ inline FacePlan face_plan(const int e[3]) {
  FacePlan P;
  P.e0m = e[0] >= 32 ? (e[0] & ~31) : e[0];
  P.r = e[0] - P.e0m;
  P.nbx = (unsigned)((P.e0m + 31) / 32);
  P.nby = (unsigned)((e[1] + 3) / 4);
  P.pm = P.nbx * P.nby;
  P.per = P.pm + (unsigned)((P.r * e[1] + 127) / 128);
  return P;
}
inline unsigned face_tiles(const int e[3]) { return face_plan(e).per * (unsigned)e[2]; }
// Tile order: groups of ZG consecutive planes; inside a group, plane-tile by plane-tile (main
// tiles, then the remainder tiles) with the plane index fastest (ZG = 1: plane by plane).  For y
// and z faces (ZG = FACE_ZG) consecutive tiles of one XCD are then z-neighbours: a z face's
// stencil cells and a y face's metric rows at four z levels are shared by the next tiles and found
// in that XCD's L2, where plane by plane they were fetched again a whole plane later (reads per
// launch 0.96 -> 0.49 GB for y faces, 1.06 -> 0.50 GB for z faces; y neighbours stay FACE_ZG * nbx
// tiles apart).  x faces keep the plane order: their stencils run along x inside the tile and
// their metric is read once per face, and they measured slower in groups.
constexpr int FACE_ZG = 8;
template <int D>
constexpr int face_zg() { return D == 0 ? 1 : FACE_ZG; }
// Face f (0..127) of `tile`: position (a, b, c), whether the tile is a remainder tile (the
// same for the whole workgroup), and a main tile's origin (ax0, by0) in its plane c.
template <int ZG>
DEV bool face_at(const int e[3], unsigned tile, unsigned f, int& a, int& b, int& c, bool& rest, int& ax0,
                 int& by0) {
  const FacePlan P = face_plan(e);
  const unsigned gsz = P.per * ZG, g = tile / gsz, tl = tile - g * gsz;
  const unsigned zg = min((unsigned)ZG, (unsigned)e[2] - g * ZG);  // planes in this group
  const unsigned w = tl / zg;
  c = (int)(g * ZG + tl % zg);
  rest = w >= P.pm;
  if (!rest) {
    ax0 = (int)(w % P.nbx) * 32;
    by0 = (int)(w / P.nbx) * 4;
    a = ax0 + (int)(f % 32);
    b = by0 + (int)(f / 32);
    return a < P.e0m && b < e[1] && c < e[2];
  }
  ax0 = by0 = 0;
  const int q = (int)(w - P.pm) * 128 + (int)f;
  a = P.e0m + q % P.r;
  b = q / P.r;
  return b < e[1] && c < e[2];
}

// Logical tile of a one-tile-per-workgroup launch.
DEV unsigned my_tile() { return xcd_block(blockIdx.x, gridDim.x); }

template <int TX, int TY>
unsigned box_blocks(const int e[3]) {
  return (unsigned)((e[0] + TX - 1) / TX) * (unsigned)((e[1] + TY - 1) / TY) * (unsigned)e[2];
}

// ---------------------------------------------------------------------------------------
// Wavefront reductions (64 lanes): max of non-negative doubles and flag counts, then at most
// one device atomic per wavefront.  Max is order independent, so results are deterministic.
// Atomics to one address serialize in L2 (tens of thousands of wavefronts per launch would
// cost about a millisecond), so a maximum is only pushed when it exceeds the running value,
// read first with a device-scope load: the running value only grows, so skipping is exact.
DEV double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

DEV void atomic_max_u64(unsigned long long* addr, unsigned long long v) {
  if (__hip_atomic_load(addr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) atomicMax(addr, v);
}

DEV void atomic_max_pos(double* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomic_max_u64((unsigned long long*)addr, (unsigned long long)__double_as_longlong(v));
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

DEV TileCell tile_cell(const GD& g, unsigned bid) {
  TileCell t;
  int ntx = (g.n[0] + CTX - 1) / CTX, nty = (g.n[1] + CTY - 1) / CTY;
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

// The vertex tile of one component spans vertices i0-1 .. i0+CTX+1 (etc.).  Each thread
// fetches its (at most four) points into registers first, so that the global loads of the
// next component are in flight while the current one is interpolated; vertices no owned
// cell needs (beyond n+1, in a ragged last tile) are not read.  All per-thread offsets of
// the fetch and of the three passes are computed once per tile.
constexpr int NFETCH = (NV + 255) / 256;
constexpr int NZR = (NZP + 255) / 256;
constexpr int NYR = (NYP + 255) / 256;

struct TileIdx {
  int fetch[NFETCH];  // point index of the fetched vertex, -1 if none
  int zsrc[NZR];      // z pass: first source in S.v, -1 if no item
  int ysrc[NYR];      // y pass: first source in S.z, -1 if no item
  int xsrc;           // x pass: first source in S.y
};

DEV TileIdx tile_index(const GD& g, const TileCell& t) {
  TileIdx x;
#pragma unroll
  for (int r = 0; r < NFETCH; ++r) {
    int q = threadIdx.x + 256 * r;
    int vx = q % VX, vy = (q / VX) % VY, vz = q / (VX * VY);
    int i = t.i0 - 1 + vx, j = t.j0 - 1 + vy, k = t.k0 - 1 + vz;
    bool in = q < NV && i <= g.n[0] + 1 && j <= g.n[1] + 1 && k <= g.n[2] + 1;
    x.fetch[r] = in ? at(g, i, j, k) : (q < NV ? -2 : -1);
  }
#pragma unroll
  for (int r = 0; r < NZR; ++r) {
    int q = threadIdx.x + 256 * r;
    int vx = q % VX, vy = (q / VX) % VY, z = q / (VX * VY);
    x.zsrc[r] = q < NZP ? vx + VX * (vy + VY * z) : -1;
  }
#pragma unroll
  for (int r = 0; r < NYR; ++r) {
    int q = threadIdx.x + 256 * r;
    int vx = q % VX, y = (q / VX) % CTY, z = q / (VX * CTY);
    x.ysrc[r] = q < NYP ? vx + VX * (y + VY * z) : -1;
  }
  x.xsrc = t.cx + VX * (t.cy + CTY * t.cz);
  return x;
}

// Points a tile does not need (fetch < 0) load the component's first element instead: the
// loads stay unconditional (a load under a branch is joined by a copy that waits for it, which
// would stall the interpolation pass it was meant to overlap), and such points only feed
// cells outside the block, whose results are discarded.
DEV void tile_fetch(const double* __restrict__ f, const TileIdx& x, double pre[NFETCH]) {
#pragma unroll
  for (int r = 0; r < NFETCH; ++r) pre[r] = ldu(f, x.fetch[r] >= 0 ? x.fetch[r] : 0);
}

DEV void tile_store(const TileIdx& x, const double pre[NFETCH], double* sv) {
#pragma unroll
  for (int r = 0; r < NFETCH; ++r)
    if (x.fetch[r] != -1) sv[threadIdx.x + 256 * r] = pre[r];
}

// Centre value of the staged component (every thread of the block must call it).
DEV double tile_value(TileLDS& S, const TileIdx& x) {
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NZR; ++r)
    if (x.zsrc[r] >= 0) {
      const double* p = S.v + x.zsrc[r];
      S.z[threadIdx.x + 256 * r] = lag(p[0], p[VX * VY], p[2 * VX * VY], p[3 * VX * VY]);
    }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NYR; ++r)
    if (x.ysrc[r] >= 0) {
      const double* p = S.z + x.ysrc[r];
      S.y[threadIdx.x + 256 * r] = lag(p[0], p[VX], p[2 * VX], p[3 * VX]);
    }
  __syncthreads();
  const double* p = S.y + x.xsrc;
  return lag(p[0], p[1], p[2], p[3]);
}

// Two components per round (values only): the passes of both run between the same three
// barriers, halving the barrier count of the value rounds.
struct TileLDS2 {
  double v[2][NV];
  double z[2][NZP];
  double y[2][NYP];
};

DEV void tile_store2(const TileIdx& x, const double pre[2][NFETCH], TileLDS2& S) {
#pragma unroll
  for (int r = 0; r < NFETCH; ++r)
    if (x.fetch[r] != -1) {
      S.v[0][threadIdx.x + 256 * r] = pre[0][r];
      S.v[1][threadIdx.x + 256 * r] = pre[1][r];
    }
}

DEV void tile_value2(TileLDS2& S, const TileIdx& x, double& v0, double& v1) {
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NZR; ++r)
    if (x.zsrc[r] >= 0)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double* p = S.v[c] + x.zsrc[r];
        S.z[c][threadIdx.x + 256 * r] = lag(p[0], p[VX * VY], p[2 * VX * VY], p[3 * VX * VY]);
      }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NYR; ++r)
    if (x.ysrc[r] >= 0)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double* p = S.z[c] + x.ysrc[r];
        S.y[c][threadIdx.x + 256 * r] = lag(p[0], p[VX], p[2 * VX], p[3 * VX]);
      }
  __syncthreads();
  const double* p = S.y[0] + x.xsrc;
  v0 = lag(p[0], p[1], p[2], p[3]);
  p = S.y[1] + x.xsrc;
  v1 = lag(p[0], p[1], p[2], p[3]);
}

// Derivatives of two staged components per round (cell kernel): 2 x (value, d/dz) after the z
// pass and 2 x (value, d/dy, d/dz-carry) after the y pass.
// The y-pass output reuses the staged values' storage (dead after the z pass), so a round must not
// store new values before every wave has finished the previous round's x pass.
struct TileLDS2D {
  union {
    double v[2][NV];
    double y[6][NYP];
  };
  double z[4][NZP];
};
static_assert(6 * NYP <= 2 * NV, "y-pass output must fit in the staged values' storage");

DEV void tile_store2d(const TileIdx& x, const double pre[2][NFETCH], TileLDS2D& S) {
#pragma unroll
  for (int r = 0; r < NFETCH; ++r)
    if (x.fetch[r] != -1) {
      S.v[0][threadIdx.x + 256 * r] = pre[0][r];
      S.v[1][threadIdx.x + 256 * r] = pre[1][r];
    }
}

// xf: the two components' values after the z and y passes at the vertex x positions on both sides
// of the thread's cell, i.e. at its lower and upper x faces (the x-face metric, interpolated across z
// then y as the x-face kernel does).
DEV void tile_derivs2(TileLDS2D& S, const TileIdx& x, const GD& g, double d0[3], double d1[3], double xf[2][2]) {
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NZR; ++r)
    if (x.zsrc[r] >= 0)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double* p = S.v[c] + x.zsrc[r];
        double a = p[0], b = p[VX * VY], cc = p[2 * VX * VY], e = p[3 * VX * VY];
        S.z[2 * c][threadIdx.x + 256 * r] = lag(a, b, cc, e);
        S.z[2 * c + 1][threadIdx.x + 256 * r] = dlag(a, b, cc, e);
      }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NYR; ++r)
    if (x.ysrc[r] >= 0)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double* p = S.z[2 * c] + x.ysrc[r];
        const double* q = S.z[2 * c + 1] + x.ysrc[r];
        double a = p[0], b = p[VX], cc = p[2 * VX], e = p[3 * VX];
        S.y[3 * c][threadIdx.x + 256 * r] = lag(a, b, cc, e);
        S.y[3 * c + 1][threadIdx.x + 256 * r] = dlag(a, b, cc, e);
        S.y[3 * c + 2][threadIdx.x + 256 * r] = lag(q[0], q[VX], q[2 * VX], q[3 * VX]);
      }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    double* d = c ? d1 : d0;
    const double* p = S.y[3 * c] + x.xsrc;
    const double* q = S.y[3 * c + 1] + x.xsrc;
    const double* w = S.y[3 * c + 2] + x.xsrc;
    d[0] = dlag(p[0], p[1], p[2], p[3]) * g.idx[0];
    d[1] = lag(q[0], q[1], q[2], q[3]) * g.idx[1];
    d[2] = lag(w[0], w[1], w[2], w[3]) * g.idx[2];
    xf[c][0] = p[1];
    xf[c][1] = p[2];
  }
}

// Centre derivatives (d/dx, d/dy, d/dz, scaled) of the staged component.
DEV void tile_derivs(TileLDS& S, const TileIdx& x, const GD& g, double d[3]) {
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NZR; ++r)
    if (x.zsrc[r] >= 0) {
      const double* p = S.v + x.zsrc[r];
      double a = p[0], b = p[VX * VY], c = p[2 * VX * VY], e = p[3 * VX * VY];
      S.z[threadIdx.x + 256 * r] = lag(a, b, c, e);
      S.z[NZP + threadIdx.x + 256 * r] = dlag(a, b, c, e);
    }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NYR; ++r)
    if (x.ysrc[r] >= 0) {
      const double* p = S.z + x.ysrc[r];
      const double* q = p + NZP;
      double a = p[0], b = p[VX], c = p[2 * VX], e = p[3 * VX];
      S.y[threadIdx.x + 256 * r] = lag(a, b, c, e);
      S.y[NYP + threadIdx.x + 256 * r] = dlag(a, b, c, e);
      S.y[2 * NYP + threadIdx.x + 256 * r] = lag(q[0], q[VX], q[2 * VX], q[3 * VX]);
    }
  __syncthreads();
  const double* p = S.y + x.xsrc;
  d[0] = dlag(p[0], p[1], p[2], p[3]) * g.idx[0];
  d[1] = lag(p[NYP], p[NYP + 1], p[NYP + 2], p[NYP + 3]) * g.idx[1];
  d[2] = lag(p[2 * NYP], p[2 * NYP + 1], p[2 * NYP + 2], p[2 * NYP + 3]) * g.idx[2];
}

// T^{mu nu} = (rho h + b^2) u u + (p + b^2/2) g^{mu nu} - b b   (eq. tmunu): T^00, T^0i, T^ij (symmetric)
DEV void tmunu_upper(const Geo& G, const State& St, double& T00, double T0[3], double Tk[6]) {
  double ia = 1.0 / G.alp, ia2 = ia * ia;
  double u0 = St.W * ia, u[3], b0 = St.W * St.Bv * ia, bu[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = St.W * (St.v[a] - G.beta[a] * ia);
    bu[a] = (St.B[a] + G.alp * b0 * u[a]) / St.W;
  }
  double e = St.rhoh + St.bsq, pt = St.p + 0.5 * St.bsq;
  T00 = e * u0 * u0 - pt * ia2 - b0 * b0;
#pragma unroll
  for (int a = 0; a < 3; ++a) T0[a] = e * u0 * u[a] + pt * G.beta[a] * ia2 - b0 * bu[a];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b)
      Tk[sym(a, b)] = e * u[a] * u[b] + pt * (G.gu[sym(a, b)] - G.beta[a] * G.beta[b] * ia2) - bu[a] * bu[b];
}

// Geometric sources at a cell (eq. grmhdsrc in the 3+1 form): the momentum source
// 1/2 T^{mu nu} d_j g_{mu nu} is linear in the derivatives of the ten stored metric components,
// sum_c w_c d_j m_c, with weights w_c built from T, beta and gamma; the energy source is
// sum_q kc_q K_q over the six stored components of the extrinsic curvature (kc from T and beta)
// plus wa_j d_j alpha.  as = alpha sqrt(gamma) densitizes.  The weights need the state and the
// centre metric only, so they are formed before the curvature is interpolated.
struct SrcW {
  double w[10], wa[3], kc[6], as;
};

DEV void src_weights(const Geo& G, const double pr[5], const double Bt[3], double gam, SrcW& s) {
  State St;
  state_make(G, pr, Bt, gam, St);
  double T00, T0[3], Tk[6];
  tmunu_upper(G, St, T00, T0, Tk);
  double bl[3];
  lower(G.g, G.beta, bl);
  s.as = G.alp * G.sqrtg;
  // weights of d_j alpha, d_j beta^k, d_j gamma_ab in 1/2 T^{mu nu} d_j g_{mu nu}
  s.w[0] = -T00 * G.alp;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    s.w[1 + k] = T00 * bl[k] + T0[0] * G.g[sym(0, k)] + T0[1] * G.g[sym(1, k)] + T0[2] * G.g[sym(2, k)];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      if (a == b)
        s.w[4 + sym(a, b)] = 0.5 * T00 * G.beta[a] * G.beta[a] + T0[a] * G.beta[a] + 0.5 * Tk[sym(a, a)];
      else
        s.w[4 + sym(a, b)] = T00 * G.beta[a] * G.beta[b] + T0[a] * G.beta[b] + T0[b] * G.beta[a] + Tk[sym(a, b)];
    }
  // energy source: (T00 beta^a beta^b + 2 T^{0a} beta^b + T^{ab}) K_ab summed over a, b, the two
  // orders of an off-diagonal pair joined; the lapse-gradient terms go with the derivatives of alpha
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      const double ab = T00 * G.beta[a] * G.beta[b] + 2.0 * T0[a] * G.beta[b] + Tk[sym(a, b)];
      s.kc[sym(a, b)] = a == b ? ab : ab + (T00 * G.beta[b] * G.beta[a] + 2.0 * T0[b] * G.beta[a] + Tk[sym(a, b)]);
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) s.wa[a] = -(T00 * G.beta[a] + T0[a]);
}

// The extrinsic-curvature part of the energy source.
DEV double src_curv(const SrcW& s, const double K[6]) {
  double se = 0.0;
#pragma unroll
  for (int q = 0; q < 6; ++q) se += s.kc[q] * K[q];
  return se;
}

// Value rounds of the ten metric components at the tile's centres, two per round, round r+1's
// vertex tiles fetched during round r.  Every thread of the block must call it; the caller's
// previous LDS readers must be done (a fresh block, or a barrier since).
DEV void metric_values10(const GD& g, const double* metric, const TileIdx& x, double m[10], TileLDS2& S2) {
  double pre[2][NFETCH];
  tile_fetch(metric, x, pre[0]);
  tile_fetch(metric + g.N, x, pre[1]);
#pragma unroll
  for (int c = 0; c < 10; c += 2) {
    // the previous pair's passes no longer read S2.v (three barriers ago)
    tile_store2(x, pre, S2);
    if (c < 8) {
      tile_fetch(metric + (c + 2) * g.N, x, pre[0]);
      tile_fetch(metric + (c + 3) * g.N, x, pre[1]);
    }
    tile_value2(S2, x, m[c], m[c + 1]);
  }
}

// Value rounds of the ten metric and six curvature components at the tile's centres, two
// components per round (one set of barriers per pair), round r+1's vertex tiles fetched during
// round r.  Returns with the first metric component's tile fetched again into pre (the first
// derivative round's).  The rolled loop keeps the register footprint of one round, values
// landing by select chains (no dynamically indexed register arrays).  The leading barrier keeps
// a persistent workgroup's previous item reading the buffer the first round writes.  Every
// thread of the block must call it.
DEV void value_rounds16(const GD& g, const double* metric, const double* curv, const TileIdx& x, double m[10],
                        double K[6], double pre[NFETCH], TileLDS2& S2) {
  auto comp = [&](int r) { return r < 10 ? metric + r * g.N : (r < 16 ? curv + (r - 10) * g.N : metric); };
  double pp[2][NFETCH];
  tile_fetch(comp(0), x, pp[0]);
  tile_fetch(comp(1), x, pp[1]);
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < 16; c += 2) {
    tile_store2(x, pp, S2);
    tile_fetch(comp(c + 2), x, pp[0]);
    if (c < 14) tile_fetch(comp(c + 3), x, pp[1]);
    double v0, v1;
    tile_value2(S2, x, v0, v1);
#pragma unroll
    for (int q = 0; q < 10; ++q) m[q] = c == q ? v0 : (c + 1 == q ? v1 : m[q]);
#pragma unroll
    for (int q = 0; q < 6; ++q) K[q] = c == 10 + q ? v0 : (c + 1 == 10 + q ? v1 : K[q]);
  }
  // comp(16) (metric component 0, the first derivative round's) is already in pp[0]
#pragma unroll
  for (int r = 0; r < NFETCH; ++r) pre[r] = pp[0][r];
}

// Value rounds of the six curvature components alone (the pairs of value_rounds16, so the same
// arithmetic), then metric component 0's vertex tile fetched into pre.  Leading barrier: the
// block's previous LDS readers are done.  Every thread of the block must call it.
DEV void curv_rounds(const GD& g, const double* metric, const double* curv, const TileIdx& x, double K[6],
                     double pre[NFETCH], TileLDS2& S2) {
  double pp[2][NFETCH];
  tile_fetch(curv, x, pp[0]);
  tile_fetch(curv + g.N, x, pp[1]);
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < 6; c += 2) {
    tile_store2(x, pp, S2);
    tile_fetch(c < 4 ? curv + (c + 2) * g.N : metric, x, pp[0]);
    if (c < 4) tile_fetch(curv + (c + 3) * g.N, x, pp[1]);
    double v0, v1;
    tile_value2(S2, x, v0, v1);
#pragma unroll
    for (int q = 0; q < 6; ++q) K[q] = c == q ? v0 : (c + 1 == q ? v1 : K[q]);
  }
#pragma unroll
  for (int r = 0; r < NFETCH; ++r) pre[r] = pp[0][r];
}

// Derivative rounds of the ten metric components, two per round, accumulated into the sources:
// src[1 + j] += w_c d_j m_c and, with alpha's, src[4] += wa_j d_j alpha.  pre0: metric
// component 0's vertex tile, already fetched.  Every thread of the block must call it.
// xfm (or NULL): the x-face metric of the tile's cells' faces is stored there, ten fields indexed like
// the fluxes (the face between cells i-1 and i at cell i): each cell its lower face, the last cell of
// a row also its upper one.  cell: the thread's cell (i, j, k), valid with `valid`.
DEV void src_deriv_rounds(const GD& g, const double* metric, const TileIdx& x, bool valid, const double pre0[NFETCH],
                          const SrcW& s, double src[5], TileLDS2D& SD, double* xfm = nullptr, int fid = 0,
                          bool last_x = false) {
  double pp[2][NFETCH];
#pragma unroll
  for (int r = 0; r < NFETCH; ++r) pp[0][r] = pre0[r];
  tile_fetch(metric + g.N, x, pp[1]);
#pragma unroll 1
  for (int c = 0; c < 10; c += 2) {
    __syncthreads();
    tile_store2d(x, pp, SD);
    if (c < 8) {
      tile_fetch(metric + (c + 2) * g.N, x, pp[0]);
      tile_fetch(metric + (c + 3) * g.N, x, pp[1]);
    }
    double d0[3], d1[3], xf[2][2];
    tile_derivs2(SD, x, g, d0, d1, xf);
    if (xfm && valid) {
      xfm[(size_t)c * g.N + fid] = xf[0][0];
      xfm[(size_t)(c + 1) * g.N + fid] = xf[1][0];
      if (last_x) {
        xfm[(size_t)c * g.N + fid + 1] = xf[0][1];
        xfm[(size_t)(c + 1) * g.N + fid + 1] = xf[1][1];
      }
    }
    if (valid) {
      double w0 = s.w[0], w1 = s.w[1];
#pragma unroll
      for (int q = 2; q < 10; ++q) {
        w0 = c == q ? s.w[q] : w0;
        w1 = c + 1 == q ? s.w[q] : w1;
      }
      src[1] += w0 * d0[0];
      src[2] += w0 * d0[1];
      src[3] += w0 * d0[2];
      if (c == 0) src[4] += s.wa[0] * d0[0] + s.wa[1] * d0[1] + s.wa[2] * d0[2];
      src[1] += w1 * d1[0];
      src[2] += w1 * d1[1];
      src[3] += w1 * d1[2];
    }
  }
}

// Derivative rounds of the ten metric components, two per round, contracted with a cotangent:
// E[c] = sum_j r[j] d_j m_c at the tile's centres (derivatives scaled by 1/dx_j), dal[j] = d_j alpha,
// and flat = every derivative is zero.  pre0: metric component 0's vertex tile, already fetched.
// Every thread of the block must call it.
DEV void metric_derivs_dot(const GD& g, const double* metric, const TileIdx& x, const double pre0[NFETCH],
                           const double r[3], double E[10], double dal[3], bool& flat, TileLDS2D& SD) {
  double pp[2][NFETCH];
#pragma unroll
  for (int q = 0; q < NFETCH; ++q) pp[0][q] = pre0[q];
  tile_fetch(metric + g.N, x, pp[1]);
  flat = true;
#pragma unroll 1
  for (int c = 0; c < 10; c += 2) {
    __syncthreads();
    tile_store2d(x, pp, SD);
    if (c < 8) {
      tile_fetch(metric + (c + 2) * g.N, x, pp[0]);
      tile_fetch(metric + (c + 3) * g.N, x, pp[1]);
    }
    double d0[3], d1[3], xf[2][2];
    tile_derivs2(SD, x, g, d0, d1, xf);
    const double e0 = r[0] * d0[0] + r[1] * d0[1] + r[2] * d0[2];
    const double e1 = r[0] * d1[0] + r[1] * d1[1] + r[2] * d1[2];
#pragma unroll
    for (int q = 0; q < 10; ++q) E[q] = c == q ? e0 : (c + 1 == q ? e1 : E[q]);
    if (c == 0) {
      dal[0] = d0[0];
      dal[1] = d0[1];
      dal[2] = d0[2];
    }
    flat = flat && d0[0] == 0.0 && d0[1] == 0.0 && d0[2] == 0.0 && d1[0] == 0.0 && d1[1] == 0.0 && d1[2] == 0.0;
  }
}

// =======================================================================================
// prim -> cons on owned cells.
DEV void prim2con_body(const GD& g, double gam, const double* __restrict__ metric, const double* __restrict__ A,
                       const double* __restrict__ prim, double* __restrict__ cons, unsigned tile) {
  int i, j, k;
  if (!box_at<64, 4>(g.n, tile, threadIdx.x, i, j, k)) return;
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

// LDS written by this wavefront and read back by it only: its accesses execute in order, and a
// wavefront barrier keeps the compiler from moving the reads above the writes.
DEV void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// c2p on owned cells, tiled: the ten metric components are interpolated to the centres
// through LDS (Sec. 3.2), then each thread recovers its cell (Secs. 3.5, 3.6).
struct C2PArgs {
  const double* metric;
  const double* A;
  double* cons;
  double* prim;
  uint8_t* flags;
  unsigned long long* stats;
  const float* mlp;  // learned guess (LEARNED instantiation only)
  mlpd::Stdz z;
  const double* curv;  // SRC instantiation: curvature at vertices
  double* src;         // SRC instantiation: densitized sources out, [4] (S_x, S_y, S_z, tau)
};

// LEARNED: a wavefront with cells that have no usable warm start (previous primitives that are
// not a physical state: the first recovery of a block, reset or prolonged cells) evaluates the
// learned guess's network on its 64 cells (through its own part of the tile's LDS, free once the
// metric passes are done) and seeds Noble's iteration of those cells with it; the other cells,
// and wavefronts without such cells, start from their previous primitives as in the plain form.
// SRC: the cell's geometric sources (eq. grmhdsrc) follow from the recovered state, with the
// centre metric of the recovery's own value rounds (the six curvature components join them) and
// the metric derivative rounds after it; stored densitized, alpha sqrt(gamma) S (rounded on its own).
template <bool LEARNED, bool SRC = false>
DEV void c2p_body(const GD& g, const C2PParams& P, const C2PArgs& a, TileLDS& S, unsigned tile) {
  const double* __restrict__ metric = a.metric;
  const double* __restrict__ A = a.A;
  double* __restrict__ cons = a.cons;
  double* __restrict__ prim = a.prim;
  uint8_t* __restrict__ flags = a.flags;
  unsigned long long* __restrict__ stats = a.stats;
  const TileCell t = tile_cell(g, tile);
  const TileIdx x = tile_index(g, t);
  double m[10];
  double K[6], pre0[NFETCH];  // SRC only
  TileLDS2& S2 = *reinterpret_cast<TileLDS2*>(&S);
  metric_values10(g, metric, x, m, S2);
  uint32_t fl = 0;
  int iters = 0;
  const int id = t.valid ? at(g, t.i0 + t.cx, t.j0 + t.cy, t.k0 + t.cz) : 0;
  Geo G;
  double Bt[3], U[5], prev[5], out[5];
  if (t.valid) {
    geo_from(m, G);
    centre_B(A, g, id, Bt);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      U[c] = cons[c * g.N + id];
      prev[c] = prim[c * g.N + id];
    }
  }
  double zw[2] = {0.0, 0.0};
  bool use_guess = false;
  if constexpr (LEARNED) {
    using namespace mlpd;
    // F and Y (one part per wavefront) lie in TileLDS's z and y arrays, i.e. over the value rounds'
    // staged vertices and z-pass output, which every thread has finished reading at the barrier
    // before the last x pass; that x pass reads the y-pass output, which lies beyond both
    float(*F)[64][NI] = reinterpret_cast<float(*)[64][NI]>(S.z);
    float(*Y)[64][NO] = reinterpret_cast<float(*)[64][NO]>(S.y);
    const int w = threadIdx.x >> 6, l = __lane_id(), lr = l & 15, lg = l >> 4;
    float f[NI];
    bool usable = false;
    C2PIn c;
    bool in = t.valid && isfinite(U[0]) && isfinite(U[1]) && isfinite(U[2]) && isfinite(U[3]) && isfinite(U[4]) &&
              U[0] >= G.sqrtg * P.rho_atm;
    if (in) in = !warm_usable(G, prev, P);
    // the network runs for whole wavefronts only (matrix instructions), and only where it is needed
    if (__ballot(in) != 0) {
      if (in) {
        c2p_input(G, U, Bt, c);
        features(G, c, P.gam, f, usable);
      }
#pragma unroll
      for (int k = 0; k < NI; ++k) F[w][l][k] = usable ? (f[k] - a.z.is[k]) * a.z.isc[k] : 0.0f;
      wave_lds_sync();
      f4 y[4];
      mlp_fwd<false>(a.mlp, F[w], y, nullptr);
      if (lg == 0)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int q = 0; q < NO; ++q) Y[w][nt * 16 + lr][q] = a.z.os[q] + y[nt][q] / a.z.osc[q];
      wave_lds_sync();
    }
    if (usable) {
      const double W = (double)__expf(Y[w][l][0]);
      const double wcap = 1.0 - 1.0 / (P.wmax * P.wmax);
      zw[0] = c.D * (double)__expf(Y[w][l][1]);
      zw[1] = fmin(fmax(1.0 - 1.0 / (W * W), 0.0), wcap);
      use_guess = isfinite(zw[0]) && zw[0] > 0.0;
    }
  }
  if (t.valid) {
    fl = c2p_point(G, U, Bt, prev, P, out, iters, use_guess ? zw : nullptr);
#pragma unroll
    for (int c = 0; c < 5; ++c) prim[c * g.N + id] = out[c];
    if (fl & 4u) {
#pragma unroll
      for (int c = 0; c < 5; ++c) cons[c * g.N + id] = U[c];
    }
    if (flags) flags[id] = (uint8_t)fl;
  }
  if constexpr (SRC) {
    SrcW sw;
    sw.as = 0.0;
    double src[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (t.valid) src_weights(G, out, Bt, P.gam, sw);
    // curvature rounds after the recovery and the weights (fewer live registers); the tile's LDS
    // offsets are formed again (from an opaque copy of the tile id, so they are not held across the
    // recovery)
    const TileIdx x2 = tile_index(g, tile_cell(g, (unsigned)__builtin_amdgcn_readfirstlane((int)tile)));
    curv_rounds(g, metric, a.curv, x2, K, pre0, S2);
    if (t.valid) src[4] = src_curv(sw, K);
    src_deriv_rounds(g, metric, x2, t.valid, pre0, sw, src, *reinterpret_cast<TileLDS2D*>(&S), a.src + 4 * g.N, id,
                     t.i0 + t.cx == g.n[0] - 1);
    if (t.valid)
#pragma unroll
      for (int c = 1; c < 5; ++c) a.src[(c - 1) * g.N + id] = __dmul_rn(sw.as, src[c]);
  }
  if (stats) {
    wave_count(fl & 1u, stats + 0);
    wave_count(fl & 2u, stats + 1);
    wave_count(fl & 4u, stats + 2);
    wave_count(fl & 8u, stats + 3);
    wave_count(fl & 16u, stats + 4);
    double im = wave_max((double)iters);
    if (__lane_id() == 0 && im > 0.0) atomic_max_u64(stats + 5, (unsigned long long)im);
  }
}

// Ghost fill along axis d of nf fields.
struct FillArgs {
  double* f;
  int nf;
  int d;
  int kind;
  double shift[3];  // periodic kind: added per period of wrap, for fields 0..2 (else 0)
};

// Ghost points along axis d: the ghost index set of axis d times the full extents of the
// other two axes; one thread per point, looping over the nf fields.
DEV long long fill_points(const GD& g, int d) {
  long long cnt = 2 * g.ng + 1;
  for (int t = 0; t < 3; ++t)
    if (t != d) cnt *= (g.n[t] + 2 * g.ng + 1);
  return cnt;
}

DEV void fill_body(const GD& g, const FillArgs& a, unsigned tile) {
  // ghost values are a pure function of owned values: no contraction, so that linear
  // extrapolation rounds exactly like its definition (one multiply, then one add)
#pragma clang fp contract(off)
  const int d = a.d;
  int cnt[3] = {g.n[0] + 2 * g.ng + 1, g.n[1] + 2 * g.ng + 1, g.n[2] + 2 * g.ng + 1};
  cnt[d] = 2 * g.ng + 1;
  long long tid = (long long)tile * 256 + threadIdx.x;
  if (tid >= (long long)cnt[0] * cnt[1] * cnt[2]) return;
  int q0 = (int)(tid % cnt[0]);
  long long r = tid / cnt[0];
  int q1 = (int)(r % cnt[1]);
  int q2 = (int)(r / cnt[1]);
  int idx[3] = {q0 - g.ng, q1 - g.ng, q2 - g.ng};
  int n = g.n[d];
  int q = idx[d] + g.ng;  // 0 .. 2 ng
  int s = q < g.ng ? q - g.ng : n + (q - g.ng);
  idx[d] = s;
  int dst = at(g, idx[0], idx[1], idx[2]);
  int stride = d == 0 ? 1 : (d == 1 ? g.sy : g.sz);
  for (int f = 0; f < a.nf; ++f) {
    double* F = a.f + (size_t)f * g.N;
    double val;
    if (a.kind == ASTERX_BC_PERIODIC) {
      int src = ((s % n) + n) % n;
      val = F[dst + (src - s) * stride];
      if (f < 3 && a.shift[f] != 0.0) val = val + (double)((s - src) / n) * a.shift[f];
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
}

// One-pass ghost fill when no axis extrapolates (periodic and copy kinds: every ghost point is a
// remapped owned point): the ghost points of x (all y, z), of y (owned x, all z) and of z (owned x,
// y) in one launch, each read from the owned point its per-axis maps reach; periodic offsets are
// added axis by axis in x, y, z order, exactly as the three axis passes add them, so the result is
// the same bit for bit.
struct Fill1Args {
  double* f;
  int nf;
  int kind[3];
  double shift[3][3];  // [field][axis], fields 0..2
};

DEV long long fill1_points(const GD& g) {
  const long long G = 2 * g.ng + 1, E1 = g.n[1] + 2 * g.ng + 1, E2 = g.n[2] + 2 * g.ng + 1;
  return G * E1 * E2 + (long long)g.n[0] * G * E2 + (long long)g.n[0] * g.n[1] * G;
}

DEV void fill1_body(const GD& g, const Fill1Args& a, unsigned tile) {
#pragma clang fp contract(off)
  const int ng = g.ng, G = 2 * ng + 1;
  const int E1 = g.n[1] + 2 * ng + 1;
  const long long s0 = (long long)G * E1 * (g.n[2] + 2 * ng + 1), s1 = (long long)g.n[0] * G * (g.n[2] + 2 * ng + 1),
                  s2 = (long long)g.n[0] * g.n[1] * G;
  long long t = (long long)tile * 256 + threadIdx.x;
  auto gh = [&](int q, int n) { return q < ng ? q - ng : n + (q - ng); };
  int idx[3];
  if (t < s0) {
    idx[0] = gh((int)(t % G), g.n[0]);
    const long long r = t / G;
    idx[1] = (int)(r % E1) - ng;
    idx[2] = (int)(r / E1) - ng;
  } else if ((t -= s0) < s1) {
    idx[0] = (int)(t % g.n[0]);
    const long long r = t / g.n[0];
    idx[1] = gh((int)(r % G), g.n[1]);
    idx[2] = (int)(r / G) - ng;
  } else if ((t -= s1) < s2) {
    idx[0] = (int)(t % g.n[0]);
    const long long r = t / g.n[0];
    idx[1] = (int)(r % g.n[1]);
    idx[2] = gh((int)(r / g.n[1]), g.n[2]);
  } else {
    return;
  }
  int src[3], wrap[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int sd = idx[d], n = g.n[d];
    if (sd >= 0 && sd < n) {
      src[d] = sd;
      wrap[d] = 0;
    } else if (a.kind[d] == ASTERX_BC_PERIODIC) {
      src[d] = ((sd % n) + n) % n;
      wrap[d] = (sd - src[d]) / n;
    } else {
      src[d] = sd < 0 ? 0 : n - 1;
      wrap[d] = 0;
    }
  }
  const int dst = at(g, idx[0], idx[1], idx[2]), so = at(g, src[0], src[1], src[2]);
  for (int f = 0; f < a.nf; ++f) {
    double* F = a.f + (size_t)f * g.N;
    double val = F[so];
    if (f < 3)
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (wrap[d] != 0 && a.shift[f][d] != 0.0) val = val + (double)wrap[d] * a.shift[f][d];
    F[dst] = val;
  }
}

// Centre field of every cell in [-ng, n+ng-1]^3 (read by the face stencils).
DEV void bcent_body(const GD& g, const double* __restrict__ A, double* __restrict__ bc, unsigned tile) {
  int e[3] = {g.n[0] + 2 * g.ng, g.n[1] + 2 * g.ng, g.n[2] + 2 * g.ng};
  int a, b, c;
  if (!lin_at(e, tile, threadIdx.x, a, b, c)) return;
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
  double gam, weno_eps, weno_q, gfac;
  int recon, speeds, riemann;
  double* apm;  // UCT: a_+, a_- and the normal field per direction
  // x faces: the x-face metric stored by the recovery with sources over the faces with owned
  // transverse indices (ten fields indexed like the fluxes), or NULL
  const double* xfm;
};

// Paired-lane variant: lanes 2f and 2f+1 of a wavefront handle the left and the right state
// of face f.  Each lane reconstructs its own side (the right lane reads its stencil
// mirrored, so both run the "right face of the middle cell" formula), interpolates half of
// the face metric, and computes the conserved vector, flux and speeds of its side; the pair
// exchanges metric halves and side results through lane shuffles and both evaluate HLLE,
// the left lane storing components 0-3, the right lane 4-6.  Half the live state per lane
// of a one-lane-per-face kernel, twice the lanes in flight.
// The swap is a DPP quad permutation (1, 0, 3, 2) of the two 32-bit halves: a VALU move, with no
// round trip through the LDS crossbar; both lanes of a pair are always active together.
DEV double shfl1(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, 0xB1, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int kind, class T>
DEV T recon_right_face(const T a[5], double eps, double q) {
  if (kind == ASTERX_RECON_MINMOD) return a[2] + 0.5 * mm(a[2] - a[1], a[3] - a[2]);
  if (kind == ASTERX_RECON_PPM) {
    T s1 = mc_slope(a[0], a[1], a[2]);
    T s2 = mc_slope(a[1], a[2], a[3]);
    T s3 = mc_slope(a[2], a[3], a[4]);
    const double sixth = 1.0 / 6.0;
    T fl = 0.5 * (a[1] + a[2]) - (s2 - s1) * sixth;
    T fr = 0.5 * (a[2] + a[3]) - (s3 - s2) * sixth;
    ppm_limit(a[2], fl, fr);
    return fr;
  }
  if (kind == ASTERX_RECON_MP5) return mp5_face(a[0], a[1], a[2], a[3], a[4]);
  return wenoz_face(a[0], a[1], a[2], a[3], a[4], eps, q);
}

// Transpose of recon_right_face on its active branch: ab[k] = xb d(face value) / d(a[k]).
template <int kind>
DEV void recon_right_face_vjp(const double a[5], double xb, double eps, double q, double ab[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) ab[k] = 0.0;
  if (kind == ASTERX_RECON_MINMOD) {
    // a2 + (a2 - a1) / 2 or a2 + (a3 - a2) / 2, whichever difference is smaller; a2 at an extremum
    const double x = a[2] - a[1], y = a[3] - a[2], h = 0.5 * xb;
    ab[2] = xb;
    if (x * y > 0.0) {
      if (fabs(x) <= fabs(y)) {
        ab[2] += h;
        ab[1] -= h;
      } else {
        ab[3] += h;
        ab[2] -= h;
      }
    }
  } else if (kind == ASTERX_RECON_PPM) {
    ppm_right_vjp(a, xb, ab);
  } else if (kind == ASTERX_RECON_MP5) {
    Lin5 s[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      s[k] = Lin5(a[k]);
      s[k].c[k] = 1.0;
    }
    const Lin5 r = mp5_face(s[0], s[1], s[2], s[3], s[4]);
#pragma unroll
    for (int k = 0; k < 5; ++k) ab[k] = xb * r.c[k];
  } else {
    // WENO-Z: one dual-number pass per stencil value.  Forward mode keeps the tangent of the
    // Z ratio tau / (beta + eps) exact where a smoothness indicator vanishes (eps ~ 1e-40); a
    // reverse sweep would form it as a difference of two terms of order 1 / eps.
#pragma unroll 1
    for (int k = 0; k < 5; ++k) {
      Dual s[5];
#pragma unroll
      for (int r = 0; r < 5; ++r) s[r] = Dual(a[r], r == k ? 1.0 : 0.0);
      ab[k] = xb * recon_right_face<kind>(s, eps, q).d;
    }
  }
}

// The x-face metric goes through LDS: a workgroup's 32 x 4 x 1 faces need a vertex block of
// 32 x 7 x 4 points per component (interpolation in y and z only), loaded once, coalesced
// along x, into a double buffer (one barrier per component, the next component's loads in
// flight meanwhile); gathered directly, each wavefront would touch 16 separate rows.  (The
// same staging serves z faces under WENO-Z, with a 35 x 7 x 1 block.)  The two lanes of a face each
// interpolate two of the four Lagrange rows and swap them, so both hold all ten components;
// the arithmetic (rows along t1, then across t2) is the direct 16-point formula's.
template <int D>
struct FaceBlk {
  static constexpr int BX = D == 0 ? 32 : 35, BY = D == 1 ? 4 : 7, BZ = D == 2 ? 1 : 4;
  static constexpr int N = BX * BY * BZ, NR = (N + 255) / 256;
};
constexpr int FACE_LDS = 32 * 7 * 4;
// y faces stage their reconstruction stencils instead: 7 variables x 9 rows (y) x 32 cells (x)
constexpr int FACE_RY = 9, FACE_RX = 32, FACE_RV = FACE_RY * FACE_RX, FACE_RN = 7 * FACE_RV;
// y and z faces of a main tile interpolate their metric in two passes: each lane the 4-point pass
// across its x column, through a wavefront-private row of 35 columns per component and side, then the
// 4-point pass along x from that row (a wavefront is one 32-face row of the tile).
constexpr int FACE_GC = 35;
struct FaceLDS {
  union {
    double m[2][FACE_LDS];
    double r[FACE_RN];
    double g[4][5][2][FACE_GC];
  };
};
static_assert(FaceBlk<0>::N <= FACE_LDS && FaceBlk<1>::N <= FACE_LDS && FaceBlk<2>::N <= FACE_LDS, "face LDS");

// UCT: the faces cover transverse indices [-3, n+1] (the upwind edge field reconstructs face
// values three faces beyond each edge) instead of [-1, n-1], gather directly, and also store the
// upwind transverse velocities (slots 5, 6 in place of the induction fluxes) and the two speeds.
template <int D, int RECON, bool UCT = false>
DEV void face_body(const GD& g, const FaceArgs& fa, unsigned tile, FaceLDS& L) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  constexpr int LO = UCT ? 3 : 1;
  using FB = FaceBlk<D>;
  const int side = threadIdx.x & 1;
  int e[3] = {g.n[0] + 2 * LO - 1, g.n[1] + 2 * LO - 1, g.n[2] + 2 * LO - 1};
  e[D] = g.n[D] + 1;
  int a, b, c;
  bool rest;
  int ax0, by0;
  // both lanes of a pair are valid or invalid together (they share the face); LDS staging
  // assumes a 32 x 4 tile, so remainder tiles gather directly
  const bool valid = face_at<face_zg<D>()>(e, tile, threadIdx.x >> 1, a, b, c, rest, ax0, by0);
  const int cz = c;
  int ijk[3] = {a - LO, b - LO, c - LO};
  ijk[D] += LO;
  const int id = valid ? at(g, ijk[0], ijk[1], ijk[2]) : 0;
  const int st[3] = {1, g.sy, g.sz};
  const int sD = st[D];
  // reconstruction of this lane's side: left lane cells i-3..i+1, right lane i+2..i-2
  double X[7];
  auto direct_recon = [&]() {
    const int o0 = side ? 2 : -3, os = side ? -1 : 1;
    if constexpr (RECON == ASTERX_RECON_WENOZ && D == 2) {
      // one variable at a time (the WENO-Z weights of seven variables interleaved would not
      // fit the register file), the next variable's stencil loading meanwhile (z faces: their
      // stencil rows are a plane apart; x faces measured faster without the extra registers)
      auto field = [&](int v) { return v < 5 ? fa.prim + v * g.N : fa.bc + (v == 5 ? t1 : t2) * g.N; };
      double nx[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) nx[q] = ldu(field(0), id + (o0 + os * q) * sD);
#pragma unroll 1
      for (int v = 0; v < 7; ++v) {
        double s5[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) s5[q] = nx[q];
        if (v < 6) {
          const double* f = field(v + 1);
#pragma unroll
          for (int q = 0; q < 5; ++q) nx[q] = ldu(f, id + (o0 + os * q) * sD);
        }
        const double xv = recon_right_face<RECON>(s5, fa.weno_eps, fa.weno_q);
#pragma unroll
        for (int k = 0; k < 7; ++k) X[k] = v == k ? xv : X[k];
      }
    } else if constexpr (RECON == ASTERX_RECON_WENOZ) {
#pragma unroll 1
      for (int v = 0; v < 7; ++v) {
        const double* f = v < 5 ? fa.prim + v * g.N : fa.bc + (v == 5 ? t1 : t2) * g.N;
        double s5[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) s5[q] = ldu(f, id + (o0 + os * q) * sD);
        const double xv = recon_right_face<RECON>(s5, fa.weno_eps, fa.weno_q);
#pragma unroll
        for (int k = 0; k < 7; ++k) X[k] = v == k ? xv : X[k];
      }
    } else {
      // all 35 stencil values are loaded before the first reconstruction
      double s5[7][5];
#pragma unroll
      for (int v = 0; v < 7; ++v) {
        const double* f = v < 5 ? fa.prim + v * g.N : fa.bc + (v == 5 ? t1 : t2) * g.N;
#pragma unroll
        for (int q = 0; q < 5; ++q) s5[v][q] = ldu(f, id + (o0 + os * q) * sD);
      }
#pragma unroll
      for (int v = 0; v < 7; ++v) X[v] = recon_right_face<RECON>(s5[v], fa.weno_eps, fa.weno_q);
    }
  };
  if (D == 1 && RECON == ASTERX_RECON_WENOZ && !UCT && !rest) {
    // y faces under WENO-Z: the seven stencil fields of the workgroup's 32 x 4 faces (cells y
    // in [by0 - 3, by0 + 5], x in [ax0 - 1, ax0 + 30]) go through LDS once, coalesced along x
    // (measured faster for WENO-Z only; PPM and MINMOD keep the direct gather).  The leading
    // barrier keeps a persistent workgroup's previous item from being overwritten.
    __syncthreads();
#pragma unroll
    for (int r = 0; r < (FACE_RN + 255) / 256; ++r) {
      const int q = threadIdx.x + 256 * r;
      if (q < FACE_RN) {
        const int v = q / FACE_RV, rem = q % FACE_RV;
        const int Y = by0 - 3 + rem / FACE_RX, X0 = ax0 - 1 + rem % FACE_RX, Z = cz - 1;
        const double* f = v < 5 ? fa.prim + v * g.N : fa.bc + (v == 5 ? t1 : t2) * g.N;
        L.r[q] = (X0 <= g.n[0] + g.ng && Y <= g.n[1] + g.ng) ? f[at(g, X0, Y, Z)] : 0.0;
      }
    }
    __syncthreads();
    if (valid) {
      const int o0 = side ? 2 : -3, os = side ? -1 : 1;
      const int base = (ijk[1] - (by0 - 3)) * FACE_RX + (ijk[0] - (ax0 - 1));
      auto stencil = [&](int v, double s5[5]) {
#pragma unroll
        for (int q = 0; q < 5; ++q) s5[q] = L.r[v * FACE_RV + base + (o0 + os * q) * FACE_RX];
      };
#pragma unroll 1
      for (int v = 0; v < 7; ++v) {
        double s5[5];
        stencil(v, s5);
        const double xv = recon_right_face<RECON>(s5, fa.weno_eps, fa.weno_q);
#pragma unroll
        for (int k = 0; k < 7; ++k) X[k] = v == k ? xv : X[k];
      }
    }
  } else if (valid) {
    direct_recon();
  }
  double m[10];
  // x faces whose transverse indices are all owned (not the y = -1 row block, not the z = -1 plane):
  // the x-face metric stored by the recovery kernel (each lane loads five components and the pair
  // swaps them), a workgroup-uniform choice
  const bool xstored = D == 0 && !UCT && fa.xfm && !rest && by0 >= LO && cz >= LO;
  // y and z faces: the direct 16-point gather (one transverse direction is x, so a
  // wavefront's loads are contiguous rows) measured faster than the staged block, except
  // for z faces under WENO-Z
  constexpr bool METRIC_LDS = !(D == 1 || (D == 2 && RECON != ASTERX_RECON_WENOZ));
  // y faces (other than WENO-Z's, whose stencils occupy the LDS) and gathered z faces of main tiles:
  // the x pass of the face metric is shared through a wavefront-private LDS row
  // (main tiles are 32 faces wide when the face row is; narrower rows gather directly)
  constexpr bool METRIC_ROW = !METRIC_LDS && !(D == 1 && RECON == ASTERX_RECON_WENOZ);
  if (xstored) {
    if (valid) {
      double mine[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) mine[q] = ldu(fa.xfm + (size_t)(5 * side + q) * g.N, id);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        double other = shfl1(mine[q]);
        m[q] = side ? other : mine[q];
        m[5 + q] = side ? mine[q] : other;
      }
    }
  } else if (METRIC_ROW && !rest && e[0] >= 32) {
    if (valid) {
      // the other transverse direction (z for y faces, y for z faces); x is the wavefront's row
      const int so = D == 1 ? g.sz : g.sy;
      const int w = threadIdx.x >> 6, f = (threadIdx.x >> 1) & 31;
      // vertex column x = i - 1 of this lane's face i
      const int mb = id - so - 1;
      const double* p0 = fa.metric + (size_t)(5 * side) * g.N + mb;
      double zc[5], mine[5];
      // all 20 column loads in one block, so they are in flight together
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const double* p = p0 + (size_t)q * g.N;
        zc[q] = lag(p[0], p[so], p[2 * so], p[3 * so]);
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) L.g[w][q][side][f] = zc[q];
      if (f < 15) {
        // the 3 columns past the row's end, one (component, column) pair per lane
        const int q = f / 3, c = f % 3;
        const double* p = p0 + (size_t)q * g.N + (32 + c - f);
        L.g[w][q][side][32 + c] = lag(p[0], p[so], p[2 * so], p[3 * so]);
      }
      // the row is written and read by this wavefront only (its LDS accesses execute in order): a
      // wavefront-level barrier keeps the compiler from moving the reads above the writes
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const double* row = L.g[w][q][side] + f;
        mine[q] = lag(row[0], row[1], row[2], row[3]);
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        double other = shfl1(mine[q]);
        m[q] = side ? other : mine[q];
        m[5 + q] = side ? mine[q] : other;
      }
    }
  } else if (!METRIC_LDS || rest) {
    if (valid) {
      const int s1 = st[t1], s2 = st[t2];
      const int mb = id - s1 - s2;
      double mine[5];
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
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        double other = shfl1(mine[q]);
        m[q] = side ? other : mine[q];
        m[5 + q] = side ? mine[q] : other;
      }
    }
  } else if constexpr (D == 0) {
    // x faces of a main tile: the pass across z is shared by the tile's 4 rows (y).  Each round takes
    // two components, q for the left lanes and q + 5 for the right ones: the workgroup forms the
    // z-interpolated values at the tile's 32 x positions and 7 vertex rows y (2 x 7 x 32 items, the
    // next round's loads in flight meanwhile), stores them in LDS (double-buffered, one barrier per
    // round), and each lane takes the pass along y over its row's 4 vertex rows.
    constexpr int NI = 2 * 7 * 32, NIR = (NI + 255) / 256;
    const int Y0 = by0 - LO - 1, Z0 = cz - LO - 1;
    int ioff[NIR], isel[NIR];
#pragma unroll
    for (int r = 0; r < NIR; ++r) {
      const int it = threadIdx.x + 256 * r, rem = it % 224;
      const int X = ax0 + rem % 32, Y = Y0 + rem / 32;
      const bool in = it < NI && X <= g.n[0] + g.ng && Y <= g.n[1] + g.ng && Z0 + 3 <= g.n[2] + g.ng;
      ioff[r] = in ? at(g, X, Y, Z0) : -1;
      isel[r] = it < NI ? it / 224 : 0;  // items past NI (no load) keep a component in range
    }
    double pre[NIR][4];
    auto fetch = [&](int q) {
#pragma unroll
      for (int r = 0; r < NIR; ++r) {
        const double* f = fa.metric + (size_t)(q + 5 * isel[r]) * g.N;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) pre[r][kk] = ioff[r] >= 0 ? ldu(f, ioff[r] + kk * g.sz) : 0.0;
      }
    };
    fetch(0);
    const int w = threadIdx.x >> 6, f = (threadIdx.x >> 1) & 31;
    // a persistent workgroup's previous item read its last round from the buffer the first round
    // here writes (five rounds, two buffers)
    __syncthreads();
#pragma unroll 1
    for (int q = 0; q < 5; ++q) {
      double* buf = L.m[q & 1];
#pragma unroll
      for (int r = 0; r < NIR; ++r)
        if (threadIdx.x + 256 * r < NI) buf[threadIdx.x + 256 * r] = lag(pre[r][0], pre[r][1], pre[r][2], pre[r][3]);
      __syncthreads();
      if (q < 4) fetch(q + 1);
      double v = 0.0;
      if (valid) {
        const double* p = buf + side * 224 + w * 32 + f;
        v = lag(p[0], p[32], p[64], p[96]);
      }
      const double o = shfl1(v);
      const double v0 = side ? o : v, v1 = side ? v : o;
#pragma unroll
      for (int k = 0; k < 10; ++k) m[k] = k == q ? v0 : (k == q + 5 ? v1 : m[k]);
    }
  } else {
    // the block starts one vertex below the first face's transverse position (face index - LO)
    const int X0 = D == 0 ? ax0 : ax0 - LO - 1, Y0 = D == 1 ? by0 : by0 - LO - 1, Z0 = D == 2 ? cz : cz - LO - 1;
    int foff[FB::NR];
    double pre[FB::NR];
#pragma unroll
    for (int r = 0; r < FB::NR; ++r) {
      const int q = threadIdx.x + 256 * r;
      const int X = X0 + q % FB::BX, Y = Y0 + (q / FB::BX) % FB::BY, Z = Z0 + q / (FB::BX * FB::BY);
      const bool in = q < FB::N && X <= g.n[0] + g.ng && Y <= g.n[1] + g.ng && Z <= g.n[2] + g.ng;
      foff[r] = in ? at(g, X, Y, Z) : -1;
      pre[r] = in ? ldu(fa.metric, foff[r]) : 0.0;
    }
    const int lst[3] = {1, FB::BX, FB::BX * FB::BY};
    const int ls1 = lst[t1], ls2 = lst[t2];
    const int lbase = valid ? (a - ax0) + FB::BX * (b - by0) + 2 * side * ls2 : 0;
#pragma unroll 1
    for (int q = 0; q < 10; ++q) {
      double* buf = L.m[q & 1];
#pragma unroll
      for (int r = 0; r < FB::NR; ++r)
        if (threadIdx.x + 256 * r < FB::N) buf[threadIdx.x + 256 * r] = pre[r];
      __syncthreads();
      if (q < 9)
#pragma unroll
        for (int r = 0; r < FB::NR; ++r) pre[r] = foff[r] >= 0 ? ldu(fa.metric + (size_t)(q + 1) * g.N, foff[r]) : 0.0;
      double ra = 0.0, rb = 0.0;
      if (valid) {
        const double* p = buf + lbase;
        ra = lag(p[0], p[ls1], p[2 * ls1], p[3 * ls1]);
        p += ls2;
        rb = lag(p[0], p[ls1], p[2 * ls1], p[3 * ls1]);
      }
      const double oa = shfl1(ra), ob = shfl1(rb);
      const double v = side ? lag(oa, ob, ra, rb) : lag(ra, rb, oa, ob);
#pragma unroll
      for (int k = 0; k < 10; ++k) m[k] = q == k ? v : m[k];
    }
  }
  double smax = 0.0;
  if (valid) {
    Geo G;
    geo_from(m, G);
    const double* Ax = fa.A;
    const double* Ay = fa.A + g.N;
    const double* Az = fa.A + 2 * g.N;
    double Bn = D == 0 ? faceBx(Ay, Az, id, g.sy, g.sz, g)
                       : (D == 1 ? faceBy(Ax, Az, id, g.sy, g.sz, g) : faceBz(Ax, Ay, id, g.sy, g.sz, g));
    // an unphysical reconstructed state falls back to the values of this side's own cell (i-1 for
    // the left lane, i for the right one), read again (rare) rather than kept in registers
    {
      double vl[3], v[3] = {X[2], X[3], X[4]};
      lower(G.g, v, vl);
      double v2 = v[0] * vl[0] + v[1] * vl[1] + v[2] * vl[2];
      if (!(X[0] > 0.0) || !(X[1] > 0.0) || !(v2 < 1.0)) {
        const int own = side ? id : id - sD;
#pragma unroll
        for (int q = 0; q < 7; ++q) X[q] = ldu(q < 5 ? fa.prim + q * g.N : fa.bc + (q == 5 ? t1 : t2) * g.N, own);
      }
    }
    double Bt[3];
    Bt[D] = Bn;
    Bt[t1] = X[5];
    Bt[t2] = X[6];
    State S;
    state_make(G, X, Bt, fa.gam, S, fa.gfac);
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
    // HLLE: (cmin F_R + cmax F_L - cmax cmin (U_R - U_L)) / (cmax + cmin); LxF (eq. LxFfluxes):
    // (F_R + F_L - c_wave (U_R - U_L)) / 2, c_wave = max(cmax, cmin).  Written from this lane's
    // point of view (own side, other side) so no per-component side selects.
    double w_own, w_oth, w_u;
    if (fa.riemann == ASTERX_RIEMANN_LXF) {
      const double hw = 0.5 * fmax(cmax, cmin);
      w_own = w_oth = 0.5;
      w_u = side ? -hw : hw;
    } else {
      double id_ = den > 0.0 ? recip(den) : 0.0;
      double cc = cmax * cmin;
      w_own = den > 0.0 ? (side ? cmin : cmax) * id_ : 0.5;
      w_oth = den > 0.0 ? (side ? cmax : cmin) * id_ : 0.5;
      w_u = den > 0.0 ? (side ? -cc : cc) * id_ : 0.0;
    }
    double out[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) out[q] = w_own * F[q] + w_oth * Fo[q] + w_u * (U[q] - Uo[q]);
    if constexpr (UCT) {
      // upwind transverse velocities (eq. uct1) with a_+ = cmax, a_- = cmin (eq. uct2)
      double vbar[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int t = k ? t2 : t1;
        const double vown = G.alp * X[2 + t] - G.beta[t], voth = shfl1(vown);
        const double vl = side ? voth : vown, vr = side ? vown : voth;
        vbar[k] = den > 0.0 ? (cmax * vl + cmin * vr) / den : 0.5 * (vl + vr);
      }
      if (side == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) fa.flux[(size_t)(D * 7 + q) * g.N + id] = out[q];
        fa.apm[(size_t)(D * 3) * g.N + id] = cmax;
        fa.apm[(size_t)(D * 3 + 1) * g.N + id] = cmin;
        fa.apm[(size_t)(D * 3 + 2) * g.N + id] = Bn;
      } else {
        fa.flux[(size_t)(D * 7 + 4) * g.N + id] = out[4];
        fa.flux[(size_t)(D * 7 + 5) * g.N + id] = vbar[0];
        fa.flux[(size_t)(D * 7 + 6) * g.N + id] = vbar[1];
      }
      if ((unsigned)ijk[t1] < (unsigned)g.n[t1] && (unsigned)ijk[t2] < (unsigned)g.n[t2]) smax = fmax(cmax, cmin);
    } else {
      if (side == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) fa.flux[(size_t)(D * 7 + q) * g.N + id] = out[q];
      } else {
#pragma unroll
        for (int q = 4; q < 7; ++q) fa.flux[(size_t)(D * 7 + q) * g.N + id] = out[q];
      }
      if (ijk[t1] >= 0 && ijk[t2] >= 0) smax = fmax(cmax, cmin);
    }
  }
  if (fa.red) {
    double w = wave_max(smax);
    if (__lane_id() == 0) atomic_max_pos(fa.red, w);
  }
}

// ---------------------------------------------------------------------------------------
// Cells: flux divergence (eq. fluxconseqs) + geometric sources (eq. grmhdsrc) + div B.
// Runge-Kutta stage outputs written in place of the right-hand side: per owned point,
// out = b_dt rhs + sum_m a[m] u[m], with the products and sums in the order of the
// stage-combine kernel (so the two paths agree bit for bit).
struct RKOut {
  const double* u[2];
  double a[2];
  double b_dt;
  double* out;
  int nterms;
};
struct Combine {
  RKOut o[2];
  int nout;  // 0: the right-hand side itself is stored
};

template <int MAXT>
DEV double rk_point(double b_dt, double r, const double* const* u, const double* a, int nterms, size_t o) {
  double s = b_dt * r;
#pragma unroll
  for (int m = 0; m < MAXT; ++m)
    if (m < nterms) s = fma(a[m], u[m][o], s);
  return s;
}

DEV void emit(const Combine& cb, double* rhs, size_t o, double v) {
  if (cb.nout == 0) {
    rhs[o] = v;
    return;
  }
#pragma unroll
  for (int k = 0; k < 2; ++k)
    if (k < cb.nout) cb.o[k].out[o] = rk_point<2>(cb.o[k].b_dt, v, cb.o[k].u, cb.o[k].a, cb.o[k].nterms, o);
}

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
  Combine cmb;
};

// Tiled cell kernel.  Pass 1 interpolates the values of the 10 metric and 6 curvature
// components through LDS; the stress tensor follows.  The momentum source
// 1/2 T^{mu nu} d_j g_{mu nu} is linear in the derivatives of the stored components,
// sum_c w_c d_j m_c with weights w_c built from T, beta and gamma, so pass 2 takes one
// component's three derivatives at a time and accumulates them (few live registers).
DEV void cell_body(const GD& g, const CellArgs& ca, TileLDS& S, unsigned tile) {
  const TileCell t = tile_cell(g, tile);
  const TileIdx x = tile_index(g, t);
  double m[10], K[6], pre[NFETCH];
  value_rounds16(g, ca.metric, ca.curv, x, m, K, pre, *reinterpret_cast<TileLDS2*>(&S));
  const int id = t.valid ? at(g, t.i0 + t.cx, t.j0 + t.cy, t.k0 + t.cz) : 0;
  SrcW sw;
  sw.as = 0.0;
  double src[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (t.valid) {
    Geo G;
    geo_from(m, G);
    double pr[5], Bt[3];
#pragma unroll
    for (int c = 0; c < 5; ++c) pr[c] = ca.prim[c * g.N + id];
    Bt[0] = ca.bc[id];
    Bt[1] = ca.bc[g.N + id];
    Bt[2] = ca.bc[2 * g.N + id];
    src_weights(G, pr, Bt, ca.gam, sw);
    src[4] = src_curv(sw, K);
  }
  src_deriv_rounds(g, ca.metric, x, t.valid, pre, sw, src, *reinterpret_cast<TileLDS2D*>(&S));
  double divb = 0.0;
  if (t.valid) {
    const int st[3] = {1, g.sy, g.sz};
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      double sdiv = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double* F = ca.flux + (size_t)(d * 7 + c) * g.N;
        sdiv += (ldu(F, id + st[d]) - ldu(F, id)) * g.idx[d];
      }
      // the densitized source rounded on its own, as the recovery kernel with sources stores it
      emit(ca.cmb, ca.rhs, (size_t)c * g.N + id, __dmul_rn(sw.as, src[c]) - sdiv);
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
// Cells with their sources given (stored by the recovery kernel with sources): flux divergence
// (eq. fluxconseqs) plus the densitized source, div B, and the stage outputs, with the cell
// kernel's arithmetic (bitwise the same results).  One thread per owned cell, x fastest, no LDS:
// a streaming kernel over the fluxes, sources and stage states.
struct DivArgs {
  const double* src;  // [4] alpha sqrt(gamma) times the S_x, S_y, S_z, tau sources
  const double* flux;
  const double* A;
  double* rhs;
  double* red;
  Combine cmb;
};

DEV void div_body(const GD& g, const DivArgs& da, unsigned tile) {
  int i, j, k;
  const bool in = box_at<64, 4>(g.n, tile, threadIdx.x, i, j, k);
  double divb = 0.0;
  if (in) {
    const int id = at(g, i, j, k);
    const int st[3] = {1, g.sy, g.sz};
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      double sdiv = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double* F = da.flux + (size_t)(d * 7 + c) * g.N;
        sdiv += (ldu(F, id + st[d]) - ldu(F, id)) * g.idx[d];
      }
      const double sc = c ? ldu(da.src + (size_t)(c - 1) * g.N, id) : 0.0;
      emit(da.cmb, da.rhs, (size_t)c * g.N + id, sc - sdiv);
    }
    if (da.red) {
      const double* Ax = da.A;
      const double* Ay = da.A + g.N;
      const double* Az = da.A + 2 * g.N;
      double dB = (faceBx(Ay, Az, id + 1, g.sy, g.sz, g) - faceBx(Ay, Az, id, g.sy, g.sz, g)) * g.idx[0] +
                  (faceBy(Ax, Az, id + g.sy, g.sy, g.sz, g) - faceBy(Ax, Az, id, g.sy, g.sz, g)) * g.idx[1] +
                  (faceBz(Ax, Ay, id + g.sz, g.sy, g.sz, g) - faceBz(Ax, Ay, id, g.sy, g.sz, g)) * g.idx[2];
      divb = fabs(dB);
    }
  }
  if (da.red) {
    double wm = wave_max(divb);
    if (__lane_id() == 0) atomic_max_pos(da.red + 1, wm);
  }
}

// ---------------------------------------------------------------------------------------
// Covariant stress-energy tensor at the vertices [0, n]^3 (Sec. 3.1: stored with the spacetime
// variables, for a spacetime solver): the vertex fluid state is the mean of the primitives and
// centre fields of the 8 cells sharing the vertex, the metric the vertex's own;
// T_{mu nu} = g_{mu a} g_{nu b} T^{ab}.  Output fields 00, 0x, 0y, 0z, xx, xy, xz, yy, yz, zz.
struct TmunuArgs {
  const double* metric;
  const double* prim;
  const double* A;
  double* out;
  double gam;
};

// Tiles of 16 x 4 x 4 vertices: the primitives and centre fields of the 17 x 5 x 5 cells they share are
// staged through LDS once (the centre field from the curl of A), then each vertex averages its 8 cells.
constexpr int TV_X = 16, TV_Y = 4, TV_Z = 4, TC_X = TV_X + 1, TC_Y = TV_Y + 1, TC_Z = TV_Z + 1;
constexpr int TC_N = TC_X * TC_Y * TC_Z;
struct TmunuLDS {
  double c[8][TC_N];
};

unsigned tmunu_tiles(const GD& g) {
  return (unsigned)(((g.n[0] + TV_X) / TV_X) * ((g.n[1] + TV_Y) / TV_Y) * ((g.n[2] + TV_Z) / TV_Z));
}

DEV void tmunu_body(const GD& g, const TmunuArgs& ta, unsigned tile, TmunuLDS& L) {
  const int nbx = (g.n[0] + TV_X) / TV_X, nby = (g.n[1] + TV_Y) / TV_Y;
  const int i0 = (int)(tile % nbx) * TV_X, j0 = (int)((tile / nbx) % nby) * TV_Y, k0 = (int)(tile / (nbx * nby)) * TV_Z;
  for (int q = threadIdx.x; q < TC_N; q += 256) {
    const int ci = i0 - 1 + q % TC_X, cj = j0 - 1 + (q / TC_X) % TC_Y, ck = k0 - 1 + q / (TC_X * TC_Y);
    // cells -1 .. n serve the vertices 0 .. n; cells beyond are not staged (no vertex reads them)
    if (ci <= g.n[0] && cj <= g.n[1] && ck <= g.n[2]) {
      const int c = at(g, ci, cj, ck);
#pragma unroll
      for (int v = 0; v < 5; ++v) L.c[v][q] = ta.prim[v * g.N + c];
      double b[3];
      centre_B(ta.A, g, c, b);
#pragma unroll
      for (int v = 0; v < 3; ++v) L.c[5 + v][q] = b[v];
    }
  }
  __syncthreads();
  const int vx = threadIdx.x % TV_X, vy = (threadIdx.x / TV_X) % TV_Y, vz = threadIdx.x / (TV_X * TV_Y);
  const int i = i0 + vx, j = j0 + vy, k = k0 + vz;
  if (i > g.n[0] || j > g.n[1] || k > g.n[2]) return;
  double pr[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, Bt[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int dk = -1; dk <= 0; ++dk)
#pragma unroll
    for (int dj = -1; dj <= 0; ++dj)
#pragma unroll
      for (int di = -1; di <= 0; ++di) {
        const int q = (vx + 1 + di) + TC_X * ((vy + 1 + dj) + TC_Y * (vz + 1 + dk));
#pragma unroll
        for (int v = 0; v < 5; ++v) pr[v] += L.c[v][q];
#pragma unroll
        for (int v = 0; v < 3; ++v) Bt[v] += L.c[5 + v][q];
      }
#pragma unroll
  for (int q = 0; q < 5; ++q) pr[q] *= 0.125;
#pragma unroll
  for (int q = 0; q < 3; ++q) Bt[q] *= 0.125;
  const int id = at(g, i, j, k);
  double m[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) m[q] = ta.metric[q * g.N + id];
  Geo G;
  geo_from(m, G);
  State St;
  state_make(G, pr, Bt, ta.gam, St);
  double T00, T0[3], Tk[6];
  tmunu_upper(G, St, T00, T0, Tk);
  double bl[3];
  lower(G.g, G.beta, bl);
  double g4[4][4], Tu[4][4];
  g4[0][0] = -G.alp * G.alp + bl[0] * G.beta[0] + bl[1] * G.beta[1] + bl[2] * G.beta[2];
  Tu[0][0] = T00;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    g4[0][a + 1] = g4[a + 1][0] = bl[a];
    Tu[0][a + 1] = Tu[a + 1][0] = T0[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      g4[a + 1][b + 1] = G.g[sym(a, b)];
      Tu[a + 1][b + 1] = Tk[sym(a, b)];
    }
  }
  double X[4][4];  // T^{a}_{nu}
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int n = 0; n < 4; ++n) X[a][n] = Tu[a][0] * g4[0][n] + Tu[a][1] * g4[1][n] + Tu[a][2] * g4[2][n] + Tu[a][3] * g4[3][n];
  const int mu[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3}, nu[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
#pragma unroll
  for (int c = 0; c < 10; ++c) {
    const int a = mu[c], b = nu[c];
    ta.out[(size_t)c * g.N + id] = g4[a][0] * X[0][b] + g4[a][1] * X[1][b] + g4[a][2] * X[2][b] + g4[a][3] * X[3][b];
  }
}

// ---------------------------------------------------------------------------------------
// Factor-2 inter-level operators (refinement boundaries, Sec. 3.9 and the AMR tests of Sec. 4).  The
// fine grid's vertex 0 sits on coarse vertex c0; each axis of a field is cell- (stag 0) or
// vertex-centred (stag 1).  Prolongation per axis: vertex directions inject on coincident points
// and take (-1, 9, 9, -1)/16 at midpoints; cell directions give the children of coarse cell c the
// conservative quadratic values u_c -+ (u_{c+1} - u_{c-1})/8; tensor product.  Cell fields fall
// back per coarse cell to minmod-limited linear children when a third-order child leaves the
// [min, max] of the 27 coarse cells around it.  Restriction: children's mean along cell
// directions, injection along vertex directions.
struct InterArgs {
  GD gc, gf;
  int c0[3], stag[3], lo[3], hi[3];
  int nf;
  const double* src;
  double* dst;
};

DEV int fdiv2(int f) { return f >= 0 ? f / 2 : -((1 - f) / 2); }

// 1-D prolongation stencil: first coarse index, count and weights
DEV int pstencil(int f, int c0, int vertex, int& first, double w[4]) {
  if (vertex) {
    if ((f & 1) == 0) {
      first = c0 + f / 2;
      w[0] = 1.0;
      return 1;
    }
    first = c0 + fdiv2(f) - 1;
    w[0] = -1.0 / 16.0;
    w[1] = 9.0 / 16.0;
    w[2] = 9.0 / 16.0;
    w[3] = -1.0 / 16.0;
    return 4;
  }
  const int child = f - 2 * fdiv2(f);
  first = c0 + fdiv2(f) - 1;
  w[0] = child ? -1.0 / 8.0 : 1.0 / 8.0;
  w[1] = 1.0;
  w[2] = child ? 1.0 / 8.0 : -1.0 / 8.0;
  return 3;
}

// Fields vertex-centred along at least one axis: one thread per fine point.
DEV void prolong_body(const InterArgs& a, unsigned tile) {
  const int e[3] = {a.hi[0] - a.lo[0] + 1, a.hi[1] - a.lo[1] + 1, a.hi[2] - a.lo[2] + 1};
  int i, j, k;
  if (!lin_at(e, tile, threadIdx.x, i, j, k)) return;
  const int f[3] = {a.lo[0] + i, a.lo[1] + j, a.lo[2] + k};
  int first[3], n[3];
  double w[3][4];
#pragma unroll
  for (int d = 0; d < 3; ++d) n[d] = pstencil(f[d], a.c0[d], a.stag[d], first[d], w[d]);
  for (int q = 0; q < a.nf; ++q) {
    const double* c = a.src + (size_t)q * a.gc.N;
    double sum = 0.0;
    for (int r = 0; r < n[2]; ++r)
      for (int p2 = 0; p2 < n[1]; ++p2)
        for (int p1 = 0; p1 < n[0]; ++p1)
          sum += w[0][p1] * w[1][p2] * w[2][r] * c[at(a.gc, first[0] + p1, first[1] + p2, first[2] + r)];
    a.dst[(size_t)q * a.gf.N + at(a.gf, f[0], f[1], f[2])] = sum;
  }
}

// Cell fields: one thread per coarse parent of the fine box; the 27 parent-centred values, the fallback
// decision and all 8 children computed once, the children inside the box stored.
DEV void prolong_cells_body(const InterArgs& a, unsigned tile) {
  int pl[3], e[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    pl[d] = a.c0[d] + fdiv2(a.lo[d]);
    e[d] = a.c0[d] + fdiv2(a.hi[d]) - pl[d] + 1;
  }
  int i, j, k;
  if (!lin_at(e, tile, threadIdx.x, i, j, k)) return;
  const int cc[3] = {pl[0] + i, pl[1] + j, pl[2] + k};
  const size_t Nc = a.gc.N, Nf = a.gf.N;
  for (int q = 0; q < a.nf; ++q) {
    const double* c = a.src + (size_t)q * Nc;
    double u[27];
#pragma unroll
    for (int r = 0; r < 27; ++r) u[r] = c[at(a.gc, cc[0] - 1 + r % 3, cc[1] - 1 + (r / 3) % 3, cc[2] - 1 + r / 9)];
    double mn = u[13], mx = u[13];
#pragma unroll
    for (int r = 0; r < 27; ++r) {
      mn = fmin(mn, u[r]);
      mx = fmax(mx, u[r]);
    }
    double ch[8];
    bool fall = false;
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int cx = h & 1, cy = (h >> 1) & 1, cz = h >> 2;
      const double wx[3] = {cx ? -0.125 : 0.125, 1.0, cx ? 0.125 : -0.125};
      const double wy[3] = {cy ? -0.125 : 0.125, 1.0, cy ? 0.125 : -0.125};
      const double wz[3] = {cz ? -0.125 : 0.125, 1.0, cz ? 0.125 : -0.125};
      double sum = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int p2 = 0; p2 < 3; ++p2)
#pragma unroll
          for (int p1 = 0; p1 < 3; ++p1) sum += wx[p1] * wy[p2] * wz[r] * u[p1 + 3 * p2 + 9 * r];
      ch[h] = sum;
      fall = fall || sum < mn || sum > mx;
    }
    if (fall) {
      const double uc = u[13];
      const double sx = mm(u[14] - uc, uc - u[12]), sy = mm(u[16] - uc, uc - u[10]), sz = mm(u[22] - uc, uc - u[4]);
#pragma unroll
      for (int h = 0; h < 8; ++h)
        ch[h] = uc + ((h & 1) ? 0.25 : -0.25) * sx + (((h >> 1) & 1) ? 0.25 : -0.25) * sy + ((h >> 2) ? 0.25 : -0.25) * sz;
    }
    double* o = a.dst + (size_t)q * Nf;
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int f0 = 2 * (cc[0] - a.c0[0]) + (h & 1), f1 = 2 * (cc[1] - a.c0[1]) + ((h >> 1) & 1),
                f2 = 2 * (cc[2] - a.c0[2]) + (h >> 2);
      if (f0 >= a.lo[0] && f0 <= a.hi[0] && f1 >= a.lo[1] && f1 <= a.hi[1] && f2 >= a.lo[2] && f2 <= a.hi[2])
        o[at(a.gf, f0, f1, f2)] = ch[h];
    }
  }
}

DEV void restrict_body(const InterArgs& a, unsigned tile) {
  const int e[3] = {a.hi[0] - a.lo[0] + 1, a.hi[1] - a.lo[1] + 1, a.hi[2] - a.lo[2] + 1};
  int i, j, k;
  if (!lin_at(e, tile, threadIdx.x, i, j, k)) return;
  const int c[3] = {a.lo[0] + i, a.lo[1] + j, a.lo[2] + k};
  int n[3], b[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    b[d] = 2 * (c[d] - a.c0[d]);
    n[d] = a.stag[d] ? 1 : 2;
  }
  const double inv = 1.0 / (double)(n[0] * n[1] * n[2]);
  for (int q = 0; q < a.nf; ++q) {
    const double* f = a.src + (size_t)q * a.gf.N;
    double s = 0.0;
    for (int r = 0; r < n[2]; ++r)
      for (int p2 = 0; p2 < n[1]; ++p2)
        for (int p1 = 0; p1 < n[0]; ++p1) s += f[at(a.gf, b[0] + p1, b[1] + p2, b[2] + r)];
    a.dst[(size_t)q * a.gc.N + at(a.gc, c[0], c[1], c[2])] = s * inv;
  }
}

// ---------------------------------------------------------------------------------------
// Vertices in [-1, n]^3: G_A = alpha Psi / sqrt(gamma) - beta^j A_j and
// F_Psi^j = alpha sqrt(gamma) gamma^jk A_k - beta^j Psi, with A averaged to the vertex
// along its own direction (Sec. 3.4).
struct VertexArgs {
  const double* metric;
  const double* A;
  const double* psi;
  double* ga;
  double* fp;
};

DEV void vertex_body(const GD& g, const VertexArgs& va, unsigned tile) {
  const double* __restrict__ metric = va.metric;
  const double* __restrict__ A = va.A;
  const double* __restrict__ psi = va.psi;
  double* __restrict__ ga = va.ga;
  double* __restrict__ fp = va.fp;
  int e[3] = {g.n[0] + 2, g.n[1] + 2, g.n[2] + 2};
  int a, b, c;
  if (!lin_at(e, tile, threadIdx.x, a, b, c)) return;
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
  Combine cmb;
  const double* apm;  // UCT: a_+, a_- and the normal field per face direction (stored by the face kernel)
};

// One term of the upwind edge field (Sec. 3.4, eq. eq3.20) at the edge owned by point id: the 1-D
// Riemann problem along DIR, from the FD-faces in the row through the edge along DIR (their upwind
// velocity component DIR and normal field, both stored by the UCT face kernel, PPM-reconstructed to
// the edge from below (L) and above (R)), with the larger speeds of the two DIR-faces meeting at the
// edge (offset along SDIR).
template <int DIR, int FD, int SDIR>
DEV double uct_term(const GD& g, const EdgeArgs& ea, int id) {
  const int st[3] = {1, g.sy, g.sz};
  const int sd = st[DIR];
  constexpr int slot = DIR == (FD + 1) % 3 ? 5 : 6;
  const double* vb = ea.flux + (size_t)(FD * 7 + slot) * g.N;
  const double* bn = ea.apm + (size_t)(FD * 3 + 2) * g.N;
  double v6[6], b6[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    v6[s] = vb[id + (s - 3) * sd];
    b6[s] = bn[id + (s - 3) * sd];
  }
  const double vm[5] = {v6[5], v6[4], v6[3], v6[2], v6[1]}, bm[5] = {b6[5], b6[4], b6[3], b6[2], b6[1]};
  const double vl = recon_right_face<ASTERX_RECON_PPM>(v6, 0.0, 1.0), vr = recon_right_face<ASTERX_RECON_PPM>(vm, 0.0, 1.0);
  const double bl = recon_right_face<ASTERX_RECON_PPM>(b6, 0.0, 1.0), br = recon_right_face<ASTERX_RECON_PPM>(bm, 0.0, 1.0);
  const double* ap = ea.apm + (size_t)(DIR * 3) * g.N;
  const double* am = ea.apm + (size_t)(DIR * 3 + 1) * g.N;
  const int o = st[SDIR];
  const double a_p = fmax(ap[id], ap[id - o]), a_m = fmax(am[id], am[id - o]);
  const double den = a_p + a_m;
  if (!(den > 0.0)) return 0.5 * (vl * bl + vr * br);
  return (a_p * vl * bl + a_m * vr * br - a_p * a_m * (br - bl)) / den;
}

template <bool UCT = false>
DEV void edge_body(const GD& g, const EdgeArgs& ea, unsigned tile) {
  int i, j, k;
  if (!box_at<64, 4>(g.n, tile, threadIdx.x, i, j, k)) return;
  const int id = at(g, i, j, k);
  const int sy = g.sy, sz = g.sz;
  double Ex, Ey, Ez;
  if constexpr (UCT) {
    // E_c = -(term along c+1 from the (c+2)-faces) + (term along c+2 from the (c+1)-faces)
    Ex = -uct_term<1, 2, 2>(g, ea, id) + uct_term<2, 1, 1>(g, ea, id);
    Ey = -uct_term<2, 0, 0>(g, ea, id) + uct_term<0, 2, 2>(g, ea, id);
    Ez = -uct_term<0, 1, 1>(g, ea, id) + uct_term<1, 0, 0>(g, ea, id);
  } else {
    const double* Fx_By = ea.flux + (size_t)(0 * 7 + 5) * g.N;
    const double* Fx_Bz = ea.flux + (size_t)(0 * 7 + 6) * g.N;
    const double* Fy_Bz = ea.flux + (size_t)(1 * 7 + 5) * g.N;
    const double* Fy_Bx = ea.flux + (size_t)(1 * 7 + 6) * g.N;
    const double* Fz_Bx = ea.flux + (size_t)(2 * 7 + 5) * g.N;
    const double* Fz_By = ea.flux + (size_t)(2 * 7 + 6) * g.N;
    Ez = 0.25 * (-Fx_By[id] - Fx_By[id - sy] + Fy_Bx[id] + Fy_Bx[id - 1]);
    Ex = 0.25 * (-Fy_Bz[id] - Fy_Bz[id - sz] + Fz_By[id] + Fz_By[id - sy]);
    Ey = 0.25 * (-Fz_Bx[id] - Fz_Bx[id - 1] + Fx_Bz[id] + Fx_Bz[id - sz]);
  }
  double* r = ea.rhs;
  const size_t N = g.N;
  if (ea.gauge == ASTERX_GAUGE_LORENZ) {
    double G0 = ea.ga[id];
    const double* f0 = ea.fp;
    const double* f1 = ea.fp + g.N;
    const double* f2 = ea.fp + 2 * g.N;
    double div = (f0[id + 1] - f0[id - 1]) * (0.5 * g.idx[0]) + (f1[id + sy] - f1[id - sy]) * (0.5 * g.idx[1]) +
                 (f2[id + sz] - f2[id - sz]) * (0.5 * g.idx[2]);
    emit(ea.cmb, r, 5 * N + id, -Ex - (ea.ga[id + 1] - G0) * g.idx[0]);
    emit(ea.cmb, r, 6 * N + id, -Ey - (ea.ga[id + sy] - G0) * g.idx[1]);
    emit(ea.cmb, r, 7 * N + id, -Ez - (ea.ga[id + sz] - G0) * g.idx[2]);
    emit(ea.cmb, r, 8 * N + id, -div - ea.xi * ea.metric[id] * ea.psi[id]);
  } else {
    emit(ea.cmb, r, 5 * N + id, -Ex);
    emit(ea.cmb, r, 6 * N + id, -Ey);
    emit(ea.cmb, r, 7 * N + id, -Ez);
    emit(ea.cmb, r, 8 * N + id, 0.0);
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

DEV void rk_body(const GD& g, const RKArgs& ra, unsigned tile) {
  int i, j, k;
  if (!box_at<64, 4>(g.n, tile, threadIdx.x, i, j, k)) return;
  const int id = at(g, i, j, k);
#pragma unroll
  for (int f = 0; f < 9; ++f) {
    size_t o = (size_t)f * g.N + id;
    ra.out[o] = rk_point<4>(ra.b_dt, ra.rhs[o], ra.u, ra.a, ra.nterms, o);
  }
}

// =======================================================================================
// Kernels.  Single block: one workgroup per logical tile of the block.  Batched: a
// persistent grid of workgroups walks a list of (patch, tile) items; every patch is a grid
// descriptor plus a base offset into field-major pools whose field stride is the total
// point count of all patches, so the same bodies run unchanged.
struct PatchDesc {
  GD g;
  long long off;
};
struct Item {
  int patch;
  int tile;
};

template <class T>
DEV T* shifted(T* p, long long off) {
  return p ? p + off : p;
}
DEV Combine shifted(const Combine& c, long long off) {
  Combine r = c;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    r.o[k].out = shifted(c.o[k].out, off);
#pragma unroll
    for (int m = 0; m < 2; ++m) r.o[k].u[m] = shifted(c.o[k].u[m], off);
  }
  return r;
}

__global__ __launch_bounds__(256) void k_prim2con(GD g, double gam, const double* metric, const double* A,
                                                  const double* prim, double* cons) {
  prim2con_body(g, gam, metric, A, prim, cons, my_tile());
}
__global__ __launch_bounds__(256) void kb_prim2con(const PatchDesc* __restrict__ P, const Item* __restrict__ it,
                                                   int nit, double gam, const double* metric, const double* A,
                                                   const double* prim, double* cons) {
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item m = it[w];
    const PatchDesc d = P[m.patch];
    prim2con_body(d.g, gam, metric + d.off, A + d.off, prim + d.off, cons + d.off, (unsigned)m.tile);
  }
}

// c2p stages two components per value round (TileLDS2); the learned guess reuses the buffer
union C2PLDS {
  TileLDS t;
  TileLDS2 t2;
};
// the cell kernel's value and derivative rounds share one buffer
union CellLDS {
  TileLDS t;
  TileLDS2 t2;
  TileLDS2D t2d;
};

__global__ __launch_bounds__(256) void k_c2p(GD g, C2PParams cp, C2PArgs a) {
  __shared__ C2PLDS S;
  c2p_body<false>(g, cp, a, S.t, my_tile());
}
__global__ __launch_bounds__(256) void k_c2p_learned(GD g, C2PParams cp, C2PArgs a) {
  __shared__ C2PLDS S;
  c2p_body<true>(g, cp, a, S.t, my_tile());
}
// 3 waves per SIMD: the stress tensor and the source weights after the recovery take about 160
// registers; held at 4 waves the kernel spills across the recovery and measured slower.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_c2p_src(GD g, C2PParams cp, C2PArgs a) {
  __shared__ CellLDS S;
  c2p_body<false, true>(g, cp, a, S.t, my_tile());
}
__global__ __launch_bounds__(256) void k_c2p_learned_src(GD g, C2PParams cp, C2PArgs a) {
  __shared__ CellLDS S;
  c2p_body<true, true>(g, cp, a, S.t, my_tile());
}
__global__ __launch_bounds__(256) void kb_c2p(const PatchDesc* __restrict__ P, const Item* __restrict__ it, int nit,
                                              C2PParams cp, C2PArgs a) {
  __shared__ C2PLDS S;
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item m = it[w];
    const PatchDesc d = P[m.patch];
    C2PArgs b = a;
    b.metric = a.metric + d.off;
    b.A = a.A + d.off;
    b.cons = a.cons + d.off;
    b.prim = a.prim + d.off;
    b.flags = shifted(a.flags, d.off);
    c2p_body<false>(d.g, cp, b, S.t, (unsigned)m.tile);
  }
}

__global__ __launch_bounds__(256) void k_fill(GD g, FillArgs a) { fill_body(g, a, blockIdx.x); }
__global__ __launch_bounds__(256) void k_fill1(GD g, Fill1Args a) { fill1_body(g, a, blockIdx.x); }
__global__ __launch_bounds__(256) void kb_fill1(const PatchDesc* __restrict__ P, const Item* __restrict__ it, int nit,
                                                Fill1Args a) {
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item m = it[w];
    const PatchDesc d = P[m.patch];
    Fill1Args b = a;
    b.f = a.f + d.off;
    fill1_body(d.g, b, (unsigned)m.tile);
  }
}
__global__ __launch_bounds__(256) void kb_fill(const PatchDesc* __restrict__ P, const Item* __restrict__ it, int nit,
                                               FillArgs a) {
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item m = it[w];
    const PatchDesc d = P[m.patch];
    FillArgs b = a;
    b.f = a.f + d.off;
    fill_body(d.g, b, (unsigned)m.tile);
  }
}

__global__ __launch_bounds__(256) void k_bcent(GD g, const double* A, double* bc) { bcent_body(g, A, bc, my_tile()); }
__global__ __launch_bounds__(256) void kb_bcent(const PatchDesc* __restrict__ P, const Item* __restrict__ it, int nit,
                                                const double* A, double* bc) {
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item m = it[w];
    const PatchDesc d = P[m.patch];
    bcent_body(d.g, A + d.off, bc + d.off, (unsigned)m.tile);
  }
}

template <int D, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(R == ASTERX_RECON_WENOZ ? 5 : 4))) void k_face(GD g, FaceArgs fa) {
  __shared__ FaceLDS L;
  face_body<D, R>(g, fa, my_tile(), L);
}
template <int D, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_face_uct(GD g, FaceArgs fa) {
  __shared__ FaceLDS L;
  face_body<D, R, true>(g, fa, my_tile(), L);
}
template <int D, int R>
__global__ __launch_bounds__(256) void kb_face(const PatchDesc* __restrict__ P, const Item* __restrict__ it, int nit,
                                               FaceArgs fa) {
  __shared__ FaceLDS L;
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item m = it[w];
    const PatchDesc d = P[m.patch];
    FaceArgs b = fa;
    b.metric = fa.metric + d.off;
    b.prim = fa.prim + d.off;
    b.A = fa.A + d.off;
    b.bc = fa.bc + d.off;
    b.flux = fa.flux + d.off;
    face_body<D, R>(d.g, b, (unsigned)m.tile, L);
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_cell(GD g, CellArgs ca) {
  __shared__ CellLDS S;
  cell_body(g, ca, S.t, my_tile());
}
__global__ __launch_bounds__(256) void kb_cell(const PatchDesc* __restrict__ P, const Item* __restrict__ it, int nit,
                                               CellArgs ca) {
  __shared__ CellLDS S;
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item m = it[w];
    const PatchDesc d = P[m.patch];
    CellArgs b = ca;
    b.metric = ca.metric + d.off;
    b.curv = ca.curv + d.off;
    b.prim = ca.prim + d.off;
    b.A = ca.A + d.off;
    b.bc = ca.bc + d.off;
    b.flux = ca.flux + d.off;
    b.rhs = shifted(ca.rhs, d.off);
    b.cmb = shifted(ca.cmb, d.off);
    cell_body(d.g, b, S.t, (unsigned)m.tile);
  }
}

__global__ __launch_bounds__(256) void k_div(GD g, DivArgs da) { div_body(g, da, my_tile()); }
__global__ __launch_bounds__(256) void k_vertex(GD g, VertexArgs va) { vertex_body(g, va, my_tile()); }
__global__ __launch_bounds__(256) void k_tmunu(GD g, TmunuArgs ta) {
  __shared__ TmunuLDS L;
  tmunu_body(g, ta, my_tile(), L);
}
__global__ __launch_bounds__(256) void k_prolong(InterArgs a) { prolong_body(a, my_tile()); }
__global__ __launch_bounds__(256) void k_prolong_cells(InterArgs a) { prolong_cells_body(a, my_tile()); }
__global__ __launch_bounds__(256) void k_restrict(InterArgs a) { restrict_body(a, my_tile()); }
__global__ __launch_bounds__(256) void kb_vertex(const PatchDesc* __restrict__ P, const Item* __restrict__ it, int nit,
                                                 VertexArgs va) {
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item m = it[w];
    const PatchDesc d = P[m.patch];
    VertexArgs b{va.metric + d.off, va.A + d.off, va.psi + d.off, va.ga + d.off, va.fp + d.off};
    vertex_body(d.g, b, (unsigned)m.tile);
  }
}

__global__ __launch_bounds__(256) void k_edge(GD g, EdgeArgs ea) { edge_body(g, ea, my_tile()); }
__global__ __launch_bounds__(256) void k_edge_uct(GD g, EdgeArgs ea) { edge_body<true>(g, ea, my_tile()); }
__global__ __launch_bounds__(256) void kb_edge(const PatchDesc* __restrict__ P, const Item* __restrict__ it, int nit,
                                               EdgeArgs ea) {
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item m = it[w];
    const PatchDesc d = P[m.patch];
    EdgeArgs b = ea;
    b.metric = ea.metric + d.off;
    b.psi = ea.psi + d.off;
    b.flux = ea.flux + d.off;
    b.ga = ea.ga + d.off;
    b.fp = ea.fp + d.off;
    b.rhs = shifted(ea.rhs, d.off);
    b.cmb = shifted(ea.cmb, d.off);
    edge_body(d.g, b, (unsigned)m.tile);
  }
}

__global__ __launch_bounds__(256) void k_rk(GD g, RKArgs ra) { rk_body(g, ra, my_tile()); }
__global__ __launch_bounds__(256) void kb_rk(const PatchDesc* __restrict__ P, const Item* __restrict__ it, int nit,
                                             RKArgs ra) {
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item m = it[w];
    const PatchDesc d = P[m.patch];
    RKArgs b = ra;
#pragma unroll
    for (int q = 0; q < 4; ++q) b.u[q] = shifted(ra.u[q], d.off);
    b.rhs = ra.rhs + d.off;
    b.out = ra.out + d.off;
    rk_body(d.g, b, (unsigned)m.tile);
  }
}

// =======================================================================================
// Adjoint (vector-Jacobian products) of one right-hand side evaluation with its c2p.
// The linear parts (flux divergence, FCT averages, gauge terms, staggered curl and averages,
// periodic ghost fills) are transposed exactly; the face physics of each side runs one
// hand-written reverse sweep (side_vjp), the other pointwise nonlinear parts (reconstruction,
// sources) build local Jacobians with dual numbers (forward mode) and contract them with the
// incoming cotangents; converged iterations (quartic roots, c2p) are differentiated through
// the implicit-function theorem.  Non-smooth points take the active branch; an exact tie of
// the two sides in the HLLE max/min splits the cotangent equally (the central derivative).

// Adjoint workspace: fields of the block's index space.
enum {
  AW_CONS = 0, AW_PRIM = 5, AW_BC = 10, AW_PBAR = 13, AW_BCBAR = 18, AW_BFBAR = 21, AW_ABAR = 24, AW_PSIBAR = 27,
  AW_AVBAR = 28, AW_FBAR = 31, AW_FIELDS = 52
};
// The Gamma cotangent is accumulated into GSLOTS workspace slots (workgroup id modulo GSLOTS):
// per-wavefront FP64 atomics to one address would serialize in L2.  The slots are summed in a
// fixed order into the caller's gamma_bar at the end of each adjoint call.
constexpr int GSLOTS = 64;

DEV void gslots_body(const double* __restrict__ slots, double* __restrict__ gamma_bar) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < GSLOTS; ++q) t += slots[q];
    gamma_bar[0] += t;
  }
}

DEV bool owned3(const GD& g, int i, int j, int k) {
  return i >= 0 && j >= 0 && k >= 0 && i < g.n[0] && j < g.n[1] && k < g.n[2];
}

// Cotangent of one field at (i, j, k) if that point is owned, else 0.
DEV double rb_at(const GD& g, const double* r, int i, int j, int k) {
  return owned3(g, i, j, k) ? r[at(g, i, j, k)] : 0.0;
}

// Face-flux cotangents from the right-hand-side cotangent rbar (9 fields, owned points):
// hydro components through the divergence (rhs[i] = -(F[i+e] - F[i]) / dx, so
// Fbar[f] = (rbar[f] - rbar[f-e]) / dx), induction components through the FCT averages.
struct FluxBarArgs {
  const double* rbar;
  double* fbar;
};

DEV void fluxbar_body(const GD& g, const FluxBarArgs& a, unsigned tile) {
  int e[3] = {g.n[0] + 2, g.n[1] + 2, g.n[2] + 2};
  int p, q, r;
  if (!box_at<64, 4>(e, tile, threadIdx.x, p, q, r)) return;
  const int i = p - 1, j = q - 1, k = r - 1;  // every index in [-1, n]
  const int id = at(g, i, j, k);
  const double* R = a.rbar;
  auto rc = [&](int c, int ii, int jj, int kk) { return rb_at(g, R + (size_t)c * g.N, ii, jj, kk); };
  const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int d = 0; d < 3; ++d) {
    const int il = i - off[d][0], jl = j - off[d][1], kl = k - off[d][2];
#pragma unroll
    for (int c = 0; c < 5; ++c)
      a.fbar[(size_t)(d * 7 + c) * g.N + id] = (rc(c, i, j, k) - rc(c, il, jl, kl)) * g.idx[d];
  }
  // dA/dt = -E: Ebar = -rbar_A; E components are quarter-sums of induction fluxes
  double* fb = a.fbar;
  fb[(size_t)(0 * 7 + 5) * g.N + id] = 0.25 * (rc(7, i, j, k) + rc(7, i, j + 1, k));   // Fx_By <- E_z
  fb[(size_t)(0 * 7 + 6) * g.N + id] = -0.25 * (rc(6, i, j, k) + rc(6, i, j, k + 1));  // Fx_Bz <- E_y
  fb[(size_t)(1 * 7 + 5) * g.N + id] = 0.25 * (rc(5, i, j, k) + rc(5, i, j, k + 1));   // Fy_Bz <- E_x
  fb[(size_t)(1 * 7 + 6) * g.N + id] = -0.25 * (rc(7, i, j, k) + rc(7, i + 1, j, k));  // Fy_Bx <- E_z
  fb[(size_t)(2 * 7 + 5) * g.N + id] = 0.25 * (rc(6, i, j, k) + rc(6, i + 1, j, k));   // Fz_Bx <- E_y
  fb[(size_t)(2 * 7 + 6) * g.N + id] = -0.25 * (rc(5, i, j, k) + rc(5, i, j + 1, k));  // Fz_By <- E_x
}

struct FaceAdjArgs {
  const double* metric;
  const double* prim;
  const double* A;
  const double* bc;
  const double* fbar;
  double* pbar;
  double* bcbar;
  double* bfbar;
  double* gbar;
  double gam, weno_eps, weno_q;
  int speeds, riemann;
};

template <int D, int RECON>
DEV void face_adj_body(const GD& g, const FaceAdjArgs& fa, unsigned tile) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  const int side = threadIdx.x & 1;
  int e[3] = {g.n[0] + 1, g.n[1] + 1, g.n[2] + 1};
  int a, b, c;
  bool rest;
  int ax0, by0;
  bool valid = face_at<face_zg<D>()>(e, tile, threadIdx.x >> 1, a, b, c, rest, ax0, by0);
  double gsum = 0.0;
  if (valid) {
    int ijk[3] = {a - 1, b - 1, c - 1};
    ijk[D] += 1;
    const int id = at(g, ijk[0], ijk[1], ijk[2]);
    const int st[3] = {1, g.sy, g.sz};
    const int sD = st[D], s1 = st[t1], s2 = st[t2];
    const int o0 = side ? 2 : -3, os = side ? -1 : 1;
    // forward recomputation of this lane's side (the stencils are loaded again for the transposed
    // reconstruction at the end rather than held in registers through the reverse sweep)
    auto field = [&](int v) { return v < 5 ? fa.prim + v * g.N : fa.bc + (v == 5 ? t1 : t2) * g.N; };
    double X[7];
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      double sten[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) sten[q] = field(v)[id + (o0 + os * q) * sD];
      X[v] = recon_right_face<RECON>(sten, fa.weno_eps, fa.weno_q);
    }
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
    bool fallback;
    {
      double vl[3], v[3] = {X[2], X[3], X[4]};
      lower(G.g, v, vl);
      double v2 = v[0] * vl[0] + v[1] * vl[1] + v[2] * vl[2];
      fallback = !(X[0] > 0.0) || !(X[1] > 0.0) || !(v2 < 1.0);
      if (fallback) {
        // this side's own cell (stencil point 2)
#pragma unroll
        for (int q = 0; q < 7; ++q) X[q] = field(q)[id + (o0 + os * 2) * sD];
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
    // HLLE transposed for this lane's side
    double fbar[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) fbar[q] = fa.fbar[(size_t)(D * 7 + q) * g.N + id];
    double Ub[7], Fb[7], cmb = 0.0, cpb = 0.0;
    if (fa.riemann == ASTERX_RIEMANN_LXF) {
      // (F_L + F_R - c_wave (U_R - U_L)) / 2 transposed; c_wave = max(cmax, cmin)
      const double cw = fmax(cmax, cmin);
      double dcw = 0.0;
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        Fb[q] = 0.5 * fbar[q];
        Ub[q] = (side ? -0.5 : 0.5) * cw * fbar[q];
        const double UL = side ? Uo[q] : U[q], UR = side ? U[q] : Uo[q];
        dcw -= 0.5 * fbar[q] * (UR - UL);
      }
      double dcmax = cmax > cmin ? dcw : (cmax == cmin ? 0.5 * dcw : 0.0);
      double dcmin = cmin > cmax ? dcw : (cmax == cmin ? 0.5 * dcw : 0.0);
      if (cmax > 0.0) {
        if (cp == cpo) cpb = 0.5 * dcmax;
        else if (cp > cpo) cpb = dcmax;
      }
      if (cmin > 0.0) {
        if (cm == cmo) cmb = -0.5 * dcmin;
        else if (cm < cmo) cmb = -dcmin;
      }
    } else if (den > 0.0) {
      double id_ = 1.0 / den, cc = cmax * cmin;
      double wF = (side ? cmin : cmax) * id_, wU = (side ? -cc : cc) * id_;
      double dcmax = 0.0, dcmin = 0.0;
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        Fb[q] = fbar[q] * wF;
        Ub[q] = fbar[q] * wU;
        double FL = side ? Fo[q] : F[q], FR = side ? F[q] : Fo[q];
        double UL = side ? Uo[q] : U[q], UR = side ? U[q] : Uo[q];
        double fo = (cmin * FR + cmax * FL - cc * (UR - UL)) * id_;
        dcmax += fbar[q] * (FL - cmin * (UR - UL) - fo) * id_;
        dcmin += fbar[q] * (FR - cmax * (UR - UL) - fo) * id_;
      }
      // cmax = max(0, c+_L, c+_R), cmin = -min(0, c-_L, c-_R): to the active side, half each on a tie
      if (cmax > 0.0) {
        if (cp == cpo) cpb = 0.5 * dcmax;
        else if (cp > cpo) cpb = dcmax;
      }
      if (cmin > 0.0) {
        if (cm == cmo) cmb = -0.5 * dcmin;
        else if (cm < cmo) cmb = -dcmin;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        Fb[q] = 0.5 * fbar[q];
        Ub[q] = 0.0;
      }
    }
    // local VJP through (X, Bn, Gamma) -> (U, F, c-, c+): one reverse sweep
    double Xb[7], Bnb, gb;
    side_vjp<D>(G, X, Bn, fa.gam, fa.speeds, cp, cm, Ub, Fb, cmb, cpb, Xb, Bnb, gb);
    // the normal field is shared by both sides: sum the pair, one store per face.  It and the
    // stencil loads below come before the scatter: atomics and loads share one counter, so a
    // load issued after an atomic waits for that atomic to complete.
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      double* dst = v < 5 ? fa.pbar + v * g.N : fa.bcbar + (v == 5 ? t1 : t2) * g.N;
      if (fallback) {
        atomicAdd(dst + id + (o0 + os * 2) * sD, Xb[v]);
        continue;
      }
      double sten[5], ab[5];
#pragma unroll
      for (int r = 0; r < 5; ++r) sten[r] = field(v)[id + (o0 + os * r) * sD];
      recon_right_face_vjp<RECON>(sten, Xb[v], fa.weno_eps, fa.weno_q, ab);
#pragma unroll
      for (int q = 0; q < 5; ++q)
        if (ab[q] != 0.0) atomicAdd(dst + id + (o0 + os * q) * sD, ab[q]);
    }
    double bn_total = Bnb + shfl1(Bnb);
    if (side == 0) fa.bfbar[(size_t)D * g.N + id] += bn_total;
    gsum = gb;
  }
  double w = gsum;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) w += __shfl_xor(w, o, 64);
  if (__lane_id() == 0 && w != 0.0) atomicAdd(fa.gbar + (blockIdx.x & (GSLOTS - 1)), w);
}

// Geometric sources transposed, one owned cell per thread, over the cell tiles of the forward
// kernels: the metric's centre values and derivatives and the curvature come from the same
// LDS-staged separable passes (metric_values10 / value_rounds16, metric_derivs_dot).
struct CellAdjArgs {
  const double* metric;
  const double* curv;
  const double* prim;
  const double* bc;
  const double* rbar;
  double* pbar;
  double* bcbar;
  double* gbar;
  double gam;
};

// sum_k rb_k src_k of the densitized sources alpha sqrt(gamma) (1/2 T^{mu nu} d_j g_{mu nu}, energy
// term) of one state, in dual numbers (the formulas of the forward cell kernel).  The momentum source
// along j is linear in the metric derivatives along j, so its contraction with rb_{1+j} is the
// momentum formula evaluated once on E_c = sum_j rb_{1+j} d_j m_c; dal = d_j alpha, K the curvature.
DEV Dual sources_dot_dual(const Geo& G, const double E[10], const double dal[3], const double K[6], double rb4,
                          const Dual pr[5], const Dual Bt[3], Dual gam) {
  StateT<Dual> St;
  state_make(G, pr, Bt, gam, St, gam / (gam - 1.0));
  double ia = 1.0 / G.alp, ia2 = ia * ia;
  Dual u0 = St.W * ia, b0 = St.W * St.Bv * ia, u[3], bu[3];
  for (int a = 0; a < 3; ++a) {
    u[a] = St.W * (St.v[a] - G.beta[a] * ia);
    bu[a] = (St.B[a] + G.alp * b0 * u[a]) / St.W;
  }
  Dual e = St.rhoh + St.bsq, pt = St.p + 0.5 * St.bsq;
  Dual T00 = e * u0 * u0 - pt * ia2 - b0 * b0;
  Dual T0[3], Tk[6];
  for (int a = 0; a < 3; ++a) T0[a] = e * u0 * u[a] + pt * G.beta[a] * ia2 - b0 * bu[a];
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b)
      Tk[sym(a, b)] = e * u[a] * u[b] + pt * (G.gu[sym(a, b)] - G.beta[a] * G.beta[b] * ia2) - bu[a] * bu[b];
  double bl[3];
  lower(G.g, G.beta, bl);
  double as = G.alp * G.sqrtg;
  // momentum, contracted
  const double* dg = &E[4];
  const double dalE = E[0], db[3] = {E[1], E[2], E[3]};
  double bbdg = 0.0;
  Dual Tdg(0.0);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      bbdg += G.beta[a] * G.beta[b] * dg[sym(a, b)];
      Tdg += Tk[sym(a, b)] * dg[sym(a, b)];
    }
  double d00 = -2.0 * G.alp * dalE + bbdg + 2.0 * (bl[0] * db[0] + bl[1] * db[1] + bl[2] * db[2]);
  Dual s0k(0.0);
  for (int a = 0; a < 3; ++a) {
    double d0a = 0.0;
    for (int b = 0; b < 3; ++b) d0a += G.beta[b] * dg[sym(a, b)] + G.g[sym(a, b)] * db[b];
    s0k += T0[a] * d0a;
  }
  Dual mom = 0.5 * T00 * d00 + s0k + 0.5 * Tdg;
  // energy
  double bK[3];
  for (int a = 0; a < 3; ++a) bK[a] = G.beta[0] * K[sym(a, 0)] + G.beta[1] * K[sym(a, 1)] + G.beta[2] * K[sym(a, 2)];
  Dual se = T00 * (G.beta[0] * bK[0] + G.beta[1] * bK[1] + G.beta[2] * bK[2] -
                   (G.beta[0] * dal[0] + G.beta[1] * dal[1] + G.beta[2] * dal[2]));
  for (int a = 0; a < 3; ++a) se += T0[a] * (2.0 * bK[a] - dal[a]);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) se += Tk[sym(a, b)] * K[sym(a, b)];
  return as * (mom + rb4 * se);
}

DEV void cell_adj_body(const GD& g, const CellAdjArgs& ca, CellLDS& S, unsigned tile) {
  const TileCell t = tile_cell(g, tile);
  const TileIdx x = tile_index(g, t);
  const int id = t.valid ? at(g, t.i0 + t.cx, t.j0 + t.cy, t.k0 + t.cz) : 0;
  double rb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (t.valid)
    for (int c = 0; c < 5; ++c) rb[c] = ca.rbar[(size_t)c * g.N + id];
  double m[10], K[6], pre[NFETCH], E[10], dal[3];
  bool flat;
  value_rounds16(g, ca.metric, ca.curv, x, m, K, pre, S.t2);
  metric_derivs_dot(g, ca.metric, x, pre, rb + 1, E, dal, flat, S.t2d);
  for (int c = 0; c < 6; ++c) flat = flat && K[c] == 0.0;
  double gsum = 0.0;
  // a metric with no derivatives and no curvature has no sources
  if (t.valid && !flat && (rb[1] != 0.0 || rb[2] != 0.0 || rb[3] != 0.0 || rb[4] != 0.0)) {
    Geo G;
    geo_from(m, G);
    double pr[5], Bt[3];
    for (int c = 0; c < 5; ++c) pr[c] = ca.prim[c * g.N + id];
    for (int c = 0; c < 3; ++c) Bt[c] = ca.bc[c * g.N + id];
#pragma unroll 1
    for (int dir = 0; dir < 9; ++dir) {
      Dual pd[5], bd[3];
      for (int c = 0; c < 5; ++c) pd[c] = Dual(pr[c], dir == c ? 1.0 : 0.0);
      for (int c = 0; c < 3; ++c) bd[c] = Dual(Bt[c], dir == 5 + c ? 1.0 : 0.0);
      const double s = sources_dot_dual(G, E, dal, K, rb[4], pd, bd, Dual(ca.gam, dir == 8 ? 1.0 : 0.0)).d;
      if (dir < 5) ca.pbar[(size_t)dir * g.N + id] += s;
      else if (dir < 8) ca.bcbar[(size_t)(dir - 5) * g.N + id] += s;
      else gsum = s;
    }
  }
  double w = gsum;
  for (int o = 32; o >= 1; o >>= 1) w += __shfl_xor(w, o, 64);
  if (__lane_id() == 0 && w != 0.0) atomicAdd(ca.gbar + (blockIdx.x & (GSLOTS - 1)), w);
}

// Gauge terms transposed at vertices [-1, n]^3: G_A and F_Psi cotangents from the A and Psi
// right-hand-side cotangents, then to Psi and to the vertex-averaged potential.
struct VertexAdjArgs {
  const double* metric;
  const double* rbar;
  double* psibar;
  double* avbar;
  double xi;
  int gauge;
};

DEV void vertex_adj_body(const GD& g, const VertexAdjArgs& va, unsigned tile) {
  int e[3] = {g.n[0] + 2, g.n[1] + 2, g.n[2] + 2};
  int p, q, r;
  if (!box_at<64, 4>(e, tile, threadIdx.x, p, q, r)) return;
  const int i = p - 1, j = q - 1, k = r - 1;
  const int id = at(g, i, j, k);
  const double* R = va.rbar;
  auto rc = [&](int c, int ii, int jj, int kk) { return rb_at(g, R + (size_t)c * g.N, ii, jj, kk); };
  double mm_[10];
  for (int c = 0; c < 10; ++c) mm_[c] = va.metric[(size_t)c * g.N + id];
  Geo G;
  geo_from(mm_, G);
  double psb = 0.0, avb[3] = {0.0, 0.0, 0.0};
  if (va.gauge == ASTERX_GAUGE_LORENZ) {
    // dA_d/dt[edge] -= (G_A[edge + e_d] - G_A[edge]) / dx_d, so G_A's cotangent at vertex v is
    // sum_d (rbar_A_d[v] - rbar_A_d[v - e_d]) / dx_d
    double gb = (rc(5, i, j, k) - rc(5, i - 1, j, k)) * g.idx[0] + (rc(6, i, j, k) - rc(6, i, j - 1, k)) * g.idx[1] +
                (rc(7, i, j, k) - rc(7, i, j, k - 1)) * g.idx[2];
    // dPsi/dt[v] = -(F[v + e] - F[v - e]) / (2 dx) - xi alpha Psi[v]
    double fb[3] = {(rc(8, i + 1, j, k) - rc(8, i - 1, j, k)) * 0.5 * g.idx[0],
                    (rc(8, i, j + 1, k) - rc(8, i, j - 1, k)) * 0.5 * g.idx[1],
                    (rc(8, i, j, k + 1) - rc(8, i, j, k - 1)) * 0.5 * g.idx[2]};
    double as = G.alp * G.sqrtg;
    psb = gb * G.alp / G.sqrtg - (fb[0] * G.beta[0] + fb[1] * G.beta[1] + fb[2] * G.beta[2]) -
          va.xi * G.alp * rc(8, i, j, k);
    for (int kk = 0; kk < 3; ++kk)
      avb[kk] = -gb * G.beta[kk] +
                as * (fb[0] * G.gu[sym(0, kk)] + fb[1] * G.gu[sym(1, kk)] + fb[2] * G.gu[sym(2, kk)]);
  }
  va.psibar[id] += psb;
  for (int c = 0; c < 3; ++c) va.avbar[(size_t)c * g.N + id] = avb[c];
}

// Edge potential from the vertex averages (A^v_d[v] = (A_d[v - e_d] + A_d[v]) / 2), edges
// [-2, n]^3 (gather, one edge per thread).
DEV void edge_adj_body(const GD& g, const double* __restrict__ avbar, double* __restrict__ abar, unsigned tile) {
  int e[3] = {g.n[0] + 3, g.n[1] + 3, g.n[2] + 3};
  int p, q, r;
  if (!box_at<64, 4>(e, tile, threadIdx.x, p, q, r)) return;
  const int i = p - 2, j = q - 2, k = r - 2;
  const int id = at(g, i, j, k);
  const int st[3] = {1, g.sy, g.sz};
  const int ijk[3] = {i, j, k};
  for (int d = 0; d < 3; ++d) {
    auto inv = [&](int dd) {  // vertex index shifted by dd along d within [-1, n]^3
      for (int a = 0; a < 3; ++a) {
        int v = ijk[a] + (a == d ? dd : 0);
        if (v < -1 || v > g.n[a]) return false;
      }
      return true;
    };
    double s = 0.0;
    if (inv(0)) s += 0.5 * avbar[(size_t)d * g.N + id];
    if (inv(1)) s += 0.5 * avbar[(size_t)d * g.N + id + st[d]];
    abar[(size_t)d * g.N + id] += s;
  }
}

// Periodic ghost fill transposed along axis d: every ghost cotangent is added to its image
// and cleared (axes are undone in the reverse order of the fill).
struct FillTArgs {
  double* f;
  int nf;
  int d;
};

DEV void fillT_body(const GD& g, const FillTArgs& a, unsigned tile) {
  const int d = a.d;
  int cnt[3] = {g.n[0] + 2 * g.ng + 1, g.n[1] + 2 * g.ng + 1, g.n[2] + 2 * g.ng + 1};
  cnt[d] = 2 * g.ng + 1;
  long long tid = (long long)tile * 256 + threadIdx.x;
  if (tid >= (long long)cnt[0] * cnt[1] * cnt[2]) return;
  int q0 = (int)(tid % cnt[0]);
  long long r = tid / cnt[0];
  int q1 = (int)(r % cnt[1]);
  int q2 = (int)(r / cnt[1]);
  int idx[3] = {q0 - g.ng, q1 - g.ng, q2 - g.ng};
  int n = g.n[d];
  int q = idx[d] + g.ng;
  int s = q < g.ng ? q - g.ng : n + (q - g.ng);
  idx[d] = s;
  int dst = at(g, idx[0], idx[1], idx[2]);
  int stride = d == 0 ? 1 : (d == 1 ? g.sy : g.sz);
  int src = ((s % n) + n) % n;
  for (int f = 0; f < a.nf; ++f) {
    double* F = a.f + (size_t)f * g.N;
    double v = F[dst];
    if (v != 0.0) atomicAdd(F + dst + (src - s) * stride, v);
    F[dst] = 0.0;
  }
}

// c2p transposed at owned cells: cons = f(prim, Btilde, Gamma) at the recovered state, so
// prim_bar -> lambda = J_prim^{-T} prim_bar, cons_bar += lambda, Btilde_bar -= J_B^T lambda,
// Gamma_bar -= J_Gamma^T lambda.  Atmosphere cells (constant primitives) pass nothing.
struct C2PAdjArgs {
  const double* metric;
  const double* prim;
  const double* bc;
  const uint8_t* flags;
  const double* pbar;
  double* consbar;
  double* bcbar;
  double* gbar;
  double gam;
  int mode;  // 0: c2p (solve with J_prim^T), 1: prim -> cons (multiply by J^T)
};

DEV void c2p_adj_body(const GD& g, const C2PAdjArgs& ca, TileLDS2& S2, unsigned tile) {
  const TileCell t = tile_cell(g, tile);
  const TileIdx x = tile_index(g, t);
  double m[10];
  metric_values10(g, ca.metric, x, m, S2);
  double gsum = 0.0;
  if (t.valid) {
    const int id = at(g, t.i0 + t.cx, t.j0 + t.cy, t.k0 + t.cz);
    double pb[5];
    bool any = false;
    for (int c = 0; c < 5; ++c) {
      pb[c] = ca.pbar[(size_t)c * g.N + id];
      any = any || pb[c] != 0.0;
    }
    bool atmo = ca.mode == 0 && ca.flags && (ca.flags[id] & 4u);
    if (any && !atmo) {
      Geo G;
      geo_from(m, G);
      double pr[5], Bt[3];
      for (int c = 0; c < 5; ++c) pr[c] = ca.prim[(size_t)c * g.N + id];
      for (int c = 0; c < 3; ++c) Bt[c] = ca.bc[(size_t)c * g.N + id];
      double J[5][9];
      for (int dir = 0; dir < 9; ++dir) {
        Dual pd[5], bd[3];
        for (int c = 0; c < 5; ++c) pd[c] = Dual(pr[c], dir == c ? 1.0 : 0.0);
        for (int c = 0; c < 3; ++c) bd[c] = Dual(Bt[c], dir == 5 + c ? 1.0 : 0.0);
        Dual gd(ca.gam, dir == 8 ? 1.0 : 0.0);
        StateT<Dual> S;
        state_make(G, pd, bd, gd, S, gd / (gd - 1.0));
        Dual U[5];
        cons_of(G, S, U);
        for (int c = 0; c < 5; ++c) J[c][dir] = U[c].d;
      }
      double lam[5];
      if (ca.mode == 0) {
        // solve J_prim^T lam = pb (Gaussian elimination with partial pivoting)
        double M[5][6];
        for (int r = 0; r < 5; ++r) {
          for (int c = 0; c < 5; ++c) M[r][c] = J[c][r];
          M[r][5] = pb[r];
        }
        // partial pivoting by row swaps with fixed indices (the first largest |M[r][c]|, r >= c, ends
        // in row c), so that M stays in registers
#pragma unroll
        for (int c = 0; c < 5; ++c) {
#pragma unroll
          for (int r = c + 1; r < 5; ++r) {
            const bool sw = fabs(M[r][c]) > fabs(M[c][c]);
#pragma unroll
            for (int q = c; q < 6; ++q) {
              const double a = M[c][q], b = M[r][q];
              M[c][q] = sw ? b : a;
              M[r][q] = sw ? a : b;
            }
          }
          const double inv = 1.0 / M[c][c];
#pragma unroll
          for (int r = c + 1; r < 5; ++r) {
            const double f = M[r][c] * inv;
#pragma unroll
            for (int q = c; q < 6; ++q) M[r][q] -= f * M[c][q];
          }
        }
#pragma unroll
        for (int r = 4; r >= 0; --r) {
          double s = M[r][5];
#pragma unroll
          for (int q = r + 1; q < 5; ++q) s -= M[r][q] * lam[q];
          lam[r] = s / M[r][r];
        }
        for (int c = 0; c < 5; ++c) ca.consbar[(size_t)c * g.N + id] += lam[c];
        for (int b = 0; b < 3; ++b) {
          double s = 0.0;
          for (int c = 0; c < 5; ++c) s += J[c][5 + b] * lam[c];
          ca.bcbar[(size_t)b * g.N + id] -= s;
        }
        double s = 0.0;
        for (int c = 0; c < 5; ++c) s += J[c][8] * lam[c];
        gsum = -s;
      } else {
        // cons = f(prim, B, Gamma): prim_bar' += J_prim^T cons_bar (pbar holds cons_bar here)
        for (int r = 0; r < 5; ++r) {
          double s = 0.0;
          for (int c = 0; c < 5; ++c) s += J[c][r] * pb[c];
          ca.consbar[(size_t)r * g.N + id] += s;  // consbar holds prim_bar in this mode
        }
        for (int b = 0; b < 3; ++b) {
          double s = 0.0;
          for (int c = 0; c < 5; ++c) s += J[c][5 + b] * pb[c];
          ca.bcbar[(size_t)b * g.N + id] += s;
        }
        double s = 0.0;
        for (int c = 0; c < 5; ++c) s += J[c][8] * pb[c];
        gsum = s;
      }
    }
  }
  double w = gsum;
  for (int o = 32; o >= 1; o >>= 1) w += __shfl_xor(w, o, 64);
  if (__lane_id() == 0 && w != 0.0) atomicAdd(ca.gbar + (blockIdx.x & (GSLOTS - 1)), w);
}

// Centre-field cotangents to face-field cotangents (gather over the two adjacent cells),
// faces [-ng+1, n+ng]^3.
DEV void bcface_adj_body(const GD& g, const double* __restrict__ bcbar, double* __restrict__ bfbar, unsigned tile) {
  // faces [-ng, n+ng]^3: the centre of cell c (in [-ng, n+ng-1]) averages faces c and c + e_d
  int e[3] = {g.n[0] + 2 * g.ng + 1, g.n[1] + 2 * g.ng + 1, g.n[2] + 2 * g.ng + 1};
  int p, q, r;
  if (!box_at<64, 4>(e, tile, threadIdx.x, p, q, r)) return;
  const int i = p - g.ng, j = q - g.ng, k = r - g.ng;
  const int id = at(g, i, j, k);
  const int st[3] = {1, g.sy, g.sz};
  const int ijk[3] = {i, j, k};
  for (int d = 0; d < 3; ++d) {
    double s = 0.0;
    if (ijk[d] <= g.n[d] + g.ng - 1) s += 0.5 * bcbar[(size_t)d * g.N + id];
    if (ijk[d] - 1 >= -g.ng) s += 0.5 * bcbar[(size_t)d * g.N + id - st[d]];
    bfbar[(size_t)d * g.N + id] += s;
  }
}

// Face-field cotangents to the edge potential (transposed curl, gather), edges [-ng, n+ng]^3
// (a face f feeds the edges f and f + e_t of its two transverse directions t).
DEV void curlT_body(const GD& g, const double* __restrict__ bf, double* __restrict__ abar, unsigned tile) {
  int e[3] = {g.n[0] + 2 * g.ng + 1, g.n[1] + 2 * g.ng + 1, g.n[2] + 2 * g.ng + 1};
  int p, q, r;
  if (!box_at<64, 4>(e, tile, threadIdx.x, p, q, r)) return;
  const int i = p - g.ng, j = q - g.ng, k = r - g.ng;
  const int id = at(g, i, j, k);
  const double* Bx = bf;
  const double* By = bf + g.N;
  const double* Bz = bf + 2 * g.N;
  const int sy = g.sy, sz = g.sz;
  const bool im = i > -g.ng, jm = j > -g.ng, km = k > -g.ng;  // the face below exists
  auto F = [](const double* f, int o, bool ok) { return ok ? f[o] : 0.0; };
  abar[id] += (F(By, id - sz, km) - By[id]) * g.idx[2] + (Bz[id] - F(Bz, id - sy, jm)) * g.idx[1];
  abar[g.N + id] += (Bx[id] - F(Bx, id - sz, km)) * g.idx[2] + (F(Bz, id - 1, im) - Bz[id]) * g.idx[0];
  abar[2 * g.N + id] += (F(Bx, id - sy, jm) - Bx[id]) * g.idx[1] + (By[id] - F(By, id - 1, im)) * g.idx[0];
}

// dst[owned] += src[owned] for nf fields.
struct AccumArgs {
  const double* src;
  double* dst;
  int nf;
};

DEV void accum_body(const GD& g, const AccumArgs& a, unsigned tile) {
  int i, j, k;
  if (!box_at<64, 4>(g.n, tile, threadIdx.x, i, j, k)) return;
  const int id = at(g, i, j, k);
  for (int f = 0; f < a.nf; ++f) a.dst[(size_t)f * g.N + id] += a.src[(size_t)f * g.N + id];
}

template <class T>
DEV void copy_body(const GD& g, const T* __restrict__ src, T* __restrict__ dst, long long n, unsigned tile) {
  long long t = (long long)tile * 256 + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

__global__ __launch_bounds__(256) void k_fluxbar(GD g, FluxBarArgs a) { fluxbar_body(g, a, my_tile()); }
// At the 2-wave floor (256 registers) the kernel spills 24-32 doubles per lane (PPM, WENO-Z, MP5)
// yet hides more latency: one wavefront per SIMD leaves every load and FP64 dependency chain exposed.
template <int D, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_face_adj(GD g, FaceAdjArgs fa) {
  face_adj_body<D, R>(g, fa, my_tile());
}
__global__ __launch_bounds__(256) void k_cell_adj(GD g, CellAdjArgs ca) {
  __shared__ CellLDS S;
  cell_adj_body(g, ca, S, my_tile());
}
__global__ __launch_bounds__(256) void k_vertex_adj(GD g, VertexAdjArgs va) { vertex_adj_body(g, va, my_tile()); }
__global__ __launch_bounds__(256) void k_edge_adj(GD g, const double* avbar, double* abar) {
  edge_adj_body(g, avbar, abar, my_tile());
}
__global__ __launch_bounds__(256) void k_fillT(GD g, FillTArgs a) { fillT_body(g, a, blockIdx.x); }
__global__ __launch_bounds__(256) void k_c2p_adj(GD g, C2PAdjArgs ca) {
  __shared__ TileLDS2 S2;
  c2p_adj_body(g, ca, S2, my_tile());
}
__global__ __launch_bounds__(64) void k_gslots(const double* slots, double* gamma_bar) { gslots_body(slots, gamma_bar); }
__global__ __launch_bounds__(256) void k_bcface_adj(GD g, const double* bcbar, double* bfbar) {
  bcface_adj_body(g, bcbar, bfbar, my_tile());
}
__global__ __launch_bounds__(256) void k_curlT(GD g, const double* bf, double* abar) { curlT_body(g, bf, abar, my_tile()); }
__global__ __launch_bounds__(256) void k_accum(GD g, AccumArgs a) { accum_body(g, a, my_tile()); }
__global__ __launch_bounds__(256) void k_copy(GD g, const double* src, double* dst, long long n) {
  copy_body(g, src, dst, n, blockIdx.x);
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
  if (npts >= 536870912.0) return fail(ASTERX_EARG, "grid: ld[0]*ld[1]*ld[2] must be below 2^29");
  return 0;
}

int check_params(const asterx_params* p) {
  if (!p) return fail(ASTERX_EARG, "params is NULL");
  if (!(p->gamma > 1.0)) return fail(ASTERX_EARG, "params: gamma must be > 1");
  if (p->recon < 0 || p->recon > 3) return fail(ASTERX_EARG, "params: unknown reconstruction");
  if (p->riemann < 0 || p->riemann > 1) return fail(ASTERX_EARG, "params: unknown Riemann solver");
  if (p->ct < 0 || p->ct > 1) return fail(ASTERX_EARG, "params: unknown electric-field scheme");
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
  KT_ZERO, KT_ADJ, KT_TMUNU, KT_INTER, KT_N
};
const char* const kt_names[KT_N] = {"prim2con", "c2p", "fill_ghosts", "centre_B", "face_x", "face_y",
                                    "face_z", "cell", "vertex", "edge", "rk_stage", "zero", "adjoint", "tmunu",
                                    "inter_level"};
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

// ---------------------------------------------------------------------------------------
// Launch targets.  A single block launches one workgroup per tile of each phase; a batch
// of patches launches a persistent grid over that phase's (patch, tile) work list.
enum { PH_P2C, PH_C2P, PH_FILLX, PH_FILLY, PH_FILLZ, PH_BCENT, PH_FACE, PH_CELL, PH_VERTEX, PH_EDGE, PH_RK, PH_FILL1,
       PH_N };

unsigned host_tile_blocks(const GD& g) {
  return (unsigned)(((g.n[0] + CTX - 1) / CTX) * ((g.n[1] + CTY - 1) / CTY) * ((g.n[2] + CTZ - 1) / CTZ));
}

unsigned tiles_for(int phase, const GD& g) {
  int e[3];
  switch (phase) {
    case PH_C2P:
    case PH_CELL:
      return host_tile_blocks(g);
    case PH_FILLX:
    case PH_FILLY:
    case PH_FILLZ: {
      int d = phase - PH_FILLX;
      long long cnt = 2 * g.ng + 1;
      for (int t = 0; t < 3; ++t)
        if (t != d) cnt *= (g.n[t] + 2 * g.ng + 1);
      return (unsigned)((cnt + 255) / 256);
    }
    case PH_BCENT:
      for (int a = 0; a < 3; ++a) e[a] = g.n[a] + 2 * g.ng;
      return lin_blocks(e);
    case PH_FILL1: {
      const long long G = 2 * g.ng + 1, E1 = g.n[1] + 2 * g.ng + 1, E2 = g.n[2] + 2 * g.ng + 1;
      const long long cnt = G * E1 * E2 + (long long)g.n[0] * G * E2 + (long long)g.n[0] * g.n[1] * G;
      return (unsigned)((cnt + 255) / 256);
    }
    case PH_FACE:
      for (int a = 0; a < 3; ++a) e[a] = g.n[a] + 1;
      return face_tiles(e);
    case PH_VERTEX:
      for (int a = 0; a < 3; ++a) e[a] = g.n[a] + 2;
      return lin_blocks(e);
    default:
      return box_blocks<64, 4>(g.n);
  }
}

}  // namespace

struct asterx_batch {
  int np = 0;
  long long ntot = 0;
  int blocks = 0;
  std::vector<GD> gds;
  std::vector<long long> off;
  PatchDesc* d_patches = nullptr;
  Item* d_items[PH_N] = {};
  int nitems[PH_N] = {};
};

namespace {

unsigned bgrid(const asterx_batch* b, int phase) {
  return (unsigned)(b->nitems[phase] < b->blocks ? b->nitems[phase] : b->blocks);
}

// One phase on either target: KS(g, args...) one workgroup per tile, or
// KB(patches, items, nitems, args...) persistent over the batch's work list.
#define RUN_PHASE(KT, PHASE, KS, KB, ...)                                                                     \
  (b ? (b->nitems[PHASE] ? timed(KT, s,                                                                      \
                                 [&] {                                                                       \
                                   hipLaunchKernelGGL(KB, dim3(bgrid(b, PHASE)), dim3(256), 0, s,           \
                                                      b->d_patches, b->d_items[PHASE], b->nitems[PHASE],     \
                                                      __VA_ARGS__);                                          \
                                 })                                                                          \
                         : 0)                                                                                \
     : timed(KT, s, [&] { hipLaunchKernelGGL(KS, dim3(tiles_for(PHASE, g)), dim3(256), 0, s, g, __VA_ARGS__); }))

template <int R>
int faces_r(const GD& g, const asterx_batch* b, const FaceArgs& fa, hipStream_t s) {
  int rc;
  if ((rc = RUN_PHASE(KT_FACE_X, PH_FACE, (k_face<0, R>), (kb_face<0, R>), fa))) return rc;
  if ((rc = RUN_PHASE(KT_FACE_Y, PH_FACE, (k_face<1, R>), (kb_face<1, R>), fa))) return rc;
  return RUN_PHASE(KT_FACE_Z, PH_FACE, (k_face<2, R>), (kb_face<2, R>), fa);
}

// Upwind CT (single blocks): faces over transverse indices [-3, n+1].
template <int R>
int faces_uct_r(const GD& g, const FaceArgs& fa, hipStream_t s) {
  int rc;
  auto tiles = [&](int D) {
    int e[3] = {g.n[0] + 5, g.n[1] + 5, g.n[2] + 5};
    e[D] = g.n[D] + 1;
    return face_tiles(e);
  };
  if ((rc = timed(KT_FACE_X, s, [&] { hipLaunchKernelGGL((k_face_uct<0, R>), dim3(tiles(0)), dim3(256), 0, s, g, fa); })))
    return rc;
  if ((rc = timed(KT_FACE_Y, s, [&] { hipLaunchKernelGGL((k_face_uct<1, R>), dim3(tiles(1)), dim3(256), 0, s, g, fa); })))
    return rc;
  return timed(KT_FACE_Z, s, [&] { hipLaunchKernelGGL((k_face_uct<2, R>), dim3(tiles(2)), dim3(256), 0, s, g, fa); });
}

int faces_uct(const GD& g, const FaceArgs& fa, int recon, hipStream_t s) {
  if (recon == ASTERX_RECON_MINMOD) return faces_uct_r<ASTERX_RECON_MINMOD>(g, fa, s);
  if (recon == ASTERX_RECON_PPM) return faces_uct_r<ASTERX_RECON_PPM>(g, fa, s);
  if (recon == ASTERX_RECON_MP5) return faces_uct_r<ASTERX_RECON_MP5>(g, fa, s);
  return faces_uct_r<ASTERX_RECON_WENOZ>(g, fa, s);
}

int faces(const GD& g, const asterx_batch* b, const FaceArgs& fa, int recon, hipStream_t s) {
  if (recon == ASTERX_RECON_MINMOD) return faces_r<ASTERX_RECON_MINMOD>(g, b, fa, s);
  if (recon == ASTERX_RECON_PPM) return faces_r<ASTERX_RECON_PPM>(g, b, fa, s);
  if (recon == ASTERX_RECON_MP5) return faces_r<ASTERX_RECON_MP5>(g, b, fa, s);
  return faces_r<ASTERX_RECON_WENOZ>(g, b, fa, s);
}

// ---- the phases, shared by the single-block and the batched entry points ----
int do_prim2con(const GD& g, const asterx_batch* b, const asterx_params* p, const double* metric, const double* A,
                const double* prim, double* cons, hipStream_t s) {
  return RUN_PHASE(KT_PRIM2CON, PH_P2C, k_prim2con, kb_prim2con, p->gamma, metric, A, prim, cons);
}

int do_c2p(const GD& g, const asterx_batch* b, const asterx_params* p, const double* metric, const double* A,
           double* cons, double* prim, uint8_t* flags, asterx_c2p_stats* stats, hipStream_t s) {
  C2PParams cp = make_c2p_params(p);
  C2PArgs a{metric, A, cons, prim, flags, (unsigned long long*)stats, nullptr, {}};
  return RUN_PHASE(KT_C2P, PH_C2P, k_c2p, kb_c2p, cp, a);
}

int do_c2p_learned(const GD& g, const asterx_params* p, const double* metric, const double* A, double* cons,
                   double* prim, uint8_t* flags, asterx_c2p_stats* stats, const float* mlp, const mlpd::Stdz& z,
                   hipStream_t s) {
  C2PParams cp = make_c2p_params(p);
  C2PArgs a{metric, A, cons, prim, flags, (unsigned long long*)stats, mlp, z};
  return timed(KT_C2P, s, [&] {
    hipLaunchKernelGGL(k_c2p_learned, dim3(tiles_for(PH_C2P, g)), dim3(256), 0, s, g, cp, a);
  });
}

int do_c2p_src(const GD& g, const asterx_params* p, const double* metric, const double* curv, const double* A,
               double* cons, double* prim, uint8_t* flags, asterx_c2p_stats* stats, const float* mlp,
               const mlpd::Stdz& z, double* src, hipStream_t s) {
  C2PParams cp = make_c2p_params(p);
  C2PArgs a{metric, A, cons, prim, flags, (unsigned long long*)stats, mlp, z, curv, src};
  return timed(KT_C2P, s, [&] {
    if (mlp)
      hipLaunchKernelGGL(k_c2p_learned_src, dim3(tiles_for(PH_C2P, g)), dim3(256), 0, s, g, cp, a);
    else
      hipLaunchKernelGGL(k_c2p_src, dim3(tiles_for(PH_C2P, g)), dim3(256), 0, s, g, cp, a);
  });
}

// The network's standardisation from an asterx_mlp (scales must be positive).
int make_stdz(const asterx_mlp* mlp, mlpd::Stdz& z, const char* who) {
  for (int k = 0; k < mlpd::NI; ++k) {
    if (!(mlp->in_scale[k] > 0.0f)) return fail(ASTERX_EARG, (std::string(who) + ": network scales must be > 0").c_str());
    z.is[k] = mlp->in_shift[k];
    z.isc[k] = mlp->in_scale[k];
  }
  for (int k = 0; k < mlpd::NO; ++k) {
    if (!(mlp->out_scale[k] > 0.0f)) return fail(ASTERX_EARG, (std::string(who) + ": network scales must be > 0").c_str());
    z.os[k] = mlp->out_shift[k];
    z.osc[k] = 1.0f / mlp->out_scale[k];
  }
  return 0;
}

int do_fill(const GD& g, const asterx_batch* b, double* f, int nf, const int32_t* kinds, hipStream_t s,
            const double* shift = nullptr) {
  int rc;
  if (kinds[0] != ASTERX_BC_LINEAR && kinds[1] != ASTERX_BC_LINEAR && kinds[2] != ASTERX_BC_LINEAR) {
    Fill1Args fa{f, nf, {kinds[0], kinds[1], kinds[2]}, {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}}};
    if (shift)
      for (int q = 0; q < 3 && q < nf; ++q)
        for (int a = 0; a < 3; ++a) fa.shift[q][a] = shift[q * 3 + a];
    return RUN_PHASE(KT_FILL, PH_FILL1, k_fill1, kb_fill1, fa);
  }
  for (int a = 0; a < 3; ++a) {
    FillArgs fa{f, nf, a, kinds[a], {0.0, 0.0, 0.0}};
    if (shift)
      for (int q = 0; q < 3 && q < nf; ++q) fa.shift[q] = shift[q * 3 + a];
    if ((rc = RUN_PHASE(KT_FILL, PH_FILLX + a, k_fill, kb_fill, fa))) return rc;
  }
  return 0;
}

int do_bcent(const GD& g, const double* A, double* bc, hipStream_t s) {
  const asterx_batch* b = nullptr;
  return RUN_PHASE(KT_BCENT, PH_BCENT, k_bcent, kb_bcent, A, bc);
}

// src (single blocks): densitized sources stored by the recovery with sources; the cell phase is
// then the divergence kernel instead of the cell kernel.
int do_rhs(const GD& g, const asterx_batch* b, const asterx_params* p, const double* metric, const double* curv,
           const double* prim, const double* A, const double* psi, double dt_max, double* rhs, double* red,
           double* ws, hipStream_t s, const Combine& cmb = Combine{}, const double* src = nullptr) {
  int rc;
  double* bc = ws;
  double* flux = ws + 3 * g.N;
  double* ga = ws + 24 * g.N;
  double* fp = ws + 25 * g.N;
  double* apm = ws + 28 * g.N;
  const bool uct = p->ct == ASTERX_CT_UCT;
  if ((rc = RUN_PHASE(KT_BCENT, PH_BCENT, k_bcent, kb_bcent, A, bc))) return rc;
  FaceArgs fa{metric, prim, A, bc, flux, red, p->gamma, p->weno_eps, p->weno_q, p->gamma / (p->gamma - 1.0),
              p->recon, p->speeds, p->riemann, apm, (src && !uct) ? src + 4 * g.N : nullptr};
  if ((rc = uct ? faces_uct(g, fa, p->recon, s) : faces(g, b, fa, p->recon, s))) return rc;
  if (src) {
    const DivArgs da{src, flux, A, rhs, red, cmb};
    if ((rc = timed(KT_CELL, s, [&] {
           hipLaunchKernelGGL(k_div, dim3(box_blocks<64, 4>(g.n)), dim3(256), 0, s, g, da);
         })))
      return rc;
  } else {
    CellArgs ca{metric, curv, prim, A, bc, flux, rhs, red, p->gamma, cmb};
    if ((rc = RUN_PHASE(KT_CELL, PH_CELL, k_cell, kb_cell, ca))) return rc;
  }
  if (p->gauge == ASTERX_GAUGE_LORENZ) {
    VertexArgs va{metric, A, psi, ga, fp};
    if ((rc = RUN_PHASE(KT_VERTEX, PH_VERTEX, k_vertex, kb_vertex, va))) return rc;
  }
  EdgeArgs ea{metric, psi, flux, ga, fp, rhs, p->xi / dt_max, p->gauge, cmb, apm};
  if (uct)
    return timed(KT_EDGE, s, [&] {
      hipLaunchKernelGGL(k_edge_uct, dim3(tiles_for(PH_EDGE, g)), dim3(256), 0, s, g, ea);
    });
  return RUN_PHASE(KT_EDGE, PH_EDGE, k_edge, kb_edge, ea);
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char *pa = (const char*)a, *pb = (const char*)b;
  return a && b && pa < pb + nb && pb < pa + na;
}

// Checks of the stage outputs against the right-hand side's inputs and each other; npts is the
// per-field stride (the block's points, or a batch's pool).
int make_combine(int32_t nout, const asterx_rk_out* outs, size_t npts, const double* const* ins, const size_t* nin,
                 int nins, Combine& cmb) {
  if (nout < 1 || nout > 2 || !outs) return fail(ASTERX_EARG, "rhs_rk: nout must be 1 or 2");
  const size_t st = 9 * npts * sizeof(double);
  cmb = Combine{};
  cmb.nout = nout;
  for (int k = 0; k < nout; ++k) {
    const asterx_rk_out& o = outs[k];
    if (o.nterms < 1 || o.nterms > 2 || !o.out) return fail(ASTERX_EARG, "rhs_rk: bad output");
    for (int m = 0; m < o.nterms; ++m)
      if (!o.u[m]) return fail(ASTERX_EARG, "rhs_rk: NULL state");
    for (int i = 0; i < nins; ++i)
      if (overlap(o.out, st, ins[i], nin[i] * sizeof(double)))
        return fail(ASTERX_EARG, "rhs_rk: an output overlaps an input of the right-hand side");
    for (int m = 0; m < o.nterms; ++m)
      if (o.u[m] != o.out && overlap(o.out, st, o.u[m], st))
        return fail(ASTERX_EARG, "rhs_rk: an output partially overlaps one of its own states");
    for (int j = 0; j < nout; ++j) {
      if (j == k) continue;
      if (overlap(o.out, st, outs[j].out, st)) return fail(ASTERX_EARG, "rhs_rk: outputs overlap");
      for (int m = 0; m < outs[j].nterms; ++m)
        if (overlap(o.out, st, outs[j].u[m], st))
          return fail(ASTERX_EARG, "rhs_rk: an output overlaps a state the other output reads");
    }
    RKOut& r = cmb.o[k];
    r.nterms = o.nterms;
    r.b_dt = o.b_dt;
    r.out = o.out;
    for (int m = 0; m < 2; ++m) {
      r.u[m] = m < o.nterms ? o.u[m] : nullptr;
      r.a[m] = m < o.nterms ? o.a[m] : 0.0;
    }
  }
  return 0;
}

int do_rk(const GD& g, const asterx_batch* b, int32_t nterms, const double* a, const double* const* u, double b_dt,
          const double* rhs, double* out, hipStream_t s) {
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
  return RUN_PHASE(KT_RK, PH_RK, k_rk, kb_rk, ra);
}

int check_kinds(const asterx_grid* gr, const int32_t* kinds) {
  for (int a = 0; a < 3; ++a) {
    if (kinds[a] < 0 || kinds[a] > 2) return fail(ASTERX_EARG, "fill_ghosts: unknown boundary kind");
    if (kinds[a] == ASTERX_BC_LINEAR && gr->n[a] < 2) return fail(ASTERX_EARG, "fill_ghosts: LINEAR needs n >= 2");
  }
  return 0;
}

}  // namespace

// =======================================================================================
namespace axh {
int set_error(int code, const char* msg) { return fail(code, msg); }
}  // namespace axh

// ---------------------------------------------------------------------------------------
// Library-held right-hand side workspace of asterx_rhs_rk_noalloc, for callers that cannot
// allocate.  Each device holds its own copy of the array until the process ends; host code
// reaches it only through the device address hipGetSymbolAddress returns with that device
// current (the array's name in host code is not a device address).  Every call on a device
// shares its copy, so calls that overlap on one device race.
static __device__ __align__(256) double scratch[ASTERX_NOALLOC_WS_BYTES / sizeof(double)];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[SCRATCH_MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`, looked up once per device.
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(ASTERX_ELAUNCH, "rhs_rk_noalloc: no current device");
  if (dev >= SCRATCH_MAX_DEVICES) return fail(ASTERX_EARG, "rhs_rk_noalloc: device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      g_err = std::string("rhs_rk_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e);
      return ASTERX_ELAUNCH;
    }
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return 0;
}
}  // namespace

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

int asterx_version(void) { return 7; }

const char* asterx_last_error(void) { return g_err.c_str(); }

size_t asterx_rhs_workspace_size(const asterx_grid* g) {
  if (!g) return 0;
  size_t N = (size_t)g->ld[0] * g->ld[1] * g->ld[2];
  return (size_t)WS_FIELDS * N * sizeof(double);
}

int asterx_prim2con(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* A,
                    const double* prim, double* cons, void* stream) {
  int rc;
  if ((rc = check_grid(gr, 2)) || (rc = check_params(p))) return rc;
  if (!metric || !A || !prim || !cons) return fail(ASTERX_EARG, "prim2con: NULL array");
  GD g = make_gd(gr);
  const asterx_batch* b = nullptr;
  return do_prim2con(g, b, p, metric, A, prim, cons, (hipStream_t)stream);
}

int asterx_c2p(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* A, double* cons,
               double* prim, uint8_t* flags, asterx_c2p_stats* stats, void* stream) {
  int rc;
  if ((rc = check_grid(gr, 2)) || (rc = check_params(p))) return rc;
  if (!metric || !A || !prim || !cons) return fail(ASTERX_EARG, "c2p: NULL array");
  GD g = make_gd(gr);
  const asterx_batch* b = nullptr;
  return do_c2p(g, b, p, metric, A, cons, prim, flags, stats, (hipStream_t)stream);
}

int asterx_c2p_learned(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* A,
                       double* cons, double* prim, uint8_t* flags, asterx_c2p_stats* stats, const asterx_mlp* mlp,
                       void* stream) {
  int rc;
  if ((rc = check_grid(gr, 2)) || (rc = check_params(p))) return rc;
  if (!metric || !A || !prim || !cons || !mlp || !mlp->params) return fail(ASTERX_EARG, "c2p_learned: NULL array");
  mlpd::Stdz z;
  if ((rc = make_stdz(mlp, z, "c2p_learned"))) return rc;
  GD g = make_gd(gr);
  return do_c2p_learned(g, p, metric, A, cons, prim, flags, stats, mlp->params, z, (hipStream_t)stream);
}

int asterx_c2p_src(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* curv,
                   const double* A, double* cons, double* prim, uint8_t* flags, asterx_c2p_stats* stats,
                   const asterx_mlp* mlp, double* src, void* stream) {
  int rc;
  if ((rc = check_grid(gr, 2)) || (rc = check_params(p))) return rc;
  if (!metric || !curv || !A || !prim || !cons || !src) return fail(ASTERX_EARG, "c2p_src: NULL array");
  mlpd::Stdz z{};
  if (mlp) {
    if (!mlp->params) return fail(ASTERX_EARG, "c2p_src: NULL network parameters");
    if ((rc = make_stdz(mlp, z, "c2p_src"))) return rc;
  }
  GD g = make_gd(gr);
  return do_c2p_src(g, p, metric, curv, A, cons, prim, flags, stats, mlp ? mlp->params : nullptr, z, src,
                    (hipStream_t)stream);
}

int asterx_fill_ghosts(const asterx_grid* gr, double* f, int32_t nf, const int32_t* kinds, void* stream) {
  int rc;
  if ((rc = check_grid(gr, 1))) return rc;
  if (!f || !kinds || nf < 1) return fail(ASTERX_EARG, "fill_ghosts: bad arguments");
  if ((rc = check_kinds(gr, kinds))) return rc;
  GD g = make_gd(gr);
  const asterx_batch* b = nullptr;
  return do_fill(g, b, f, nf, kinds, (hipStream_t)stream);
}

int asterx_fill_ghosts_shift(const asterx_grid* gr, double* f, int32_t nf, const double* shift, void* stream) {
  int rc;
  if ((rc = check_grid(gr, 1))) return rc;
  if (!f || !shift || nf < 1 || nf > 3) return fail(ASTERX_EARG, "fill_ghosts_shift: bad arguments");
  GD g = make_gd(gr);
  const asterx_batch* b = nullptr;
  const int32_t per[3] = {ASTERX_BC_PERIODIC, ASTERX_BC_PERIODIC, ASTERX_BC_PERIODIC};
  return do_fill(g, b, f, nf, per, (hipStream_t)stream, shift);
}

int asterx_rhs(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* curv,
               const double* prim, const double* A, const double* psi, double dt_max, double* rhs, double* red,
               void* workspace, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_params(p))) return rc;
  // the face kernels load a six-cell stencil (i-3..i+2) for every scheme
  if ((rc = check_grid(gr, 3))) return rc;
  if (p->ct == ASTERX_CT_UCT && gr->ng < 4) return fail(ASTERX_EARG, "rhs: upwind CT needs ng >= 4");
  if (!metric || !curv || !prim || !A || !psi || !rhs || !workspace) return fail(ASTERX_EARG, "rhs: NULL array");
  if (ws_bytes < asterx_rhs_workspace_size(gr)) return fail(ASTERX_EARG, "rhs: workspace too small");
  if (!(dt_max > 0.0)) return fail(ASTERX_EARG, "rhs: dt_max must be > 0");
  GD g = make_gd(gr);
  const asterx_batch* b = nullptr;
  return do_rhs(g, b, p, metric, curv, prim, A, psi, dt_max, rhs, red, (double*)workspace, (hipStream_t)stream);
}

int asterx_rk_stage(const asterx_grid* gr, int32_t nterms, const double* a, const double* const* u, double b_dt,
                    const double* rhs, double* out, void* stream) {
  int rc;
  if ((rc = check_grid(gr, 1))) return rc;
  GD g = make_gd(gr);
  const asterx_batch* b = nullptr;
  return do_rk(g, b, nterms, a, u, b_dt, rhs, out, (hipStream_t)stream);
}

int asterx_rhs_rk(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* curv,
                  const double* prim, const double* A, const double* psi, double dt_max, int32_t nout,
                  const asterx_rk_out* outs, double* red, void* workspace, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_params(p)) || (rc = check_grid(gr, 3))) return rc;
  if (p->ct == ASTERX_CT_UCT && gr->ng < 4) return fail(ASTERX_EARG, "rhs_rk: upwind CT needs ng >= 4");
  if (!metric || !curv || !prim || !A || !psi || !workspace) return fail(ASTERX_EARG, "rhs_rk: NULL array");
  if (ws_bytes < asterx_rhs_workspace_size(gr)) return fail(ASTERX_EARG, "rhs_rk: workspace too small");
  if (!(dt_max > 0.0)) return fail(ASTERX_EARG, "rhs_rk: dt_max must be > 0");
  GD g = make_gd(gr);
  const double* ins[6] = {metric, curv, prim, A, psi, (const double*)workspace};
  const size_t nin[6] = {10 * g.N, 6 * g.N, 5 * g.N, 3 * g.N, g.N, ws_bytes / sizeof(double)};
  Combine cmb;
  if ((rc = make_combine(nout, outs, g.N, ins, nin, 6, cmb))) return rc;
  return do_rhs(g, nullptr, p, metric, curv, prim, A, psi, dt_max, nullptr, red, (double*)workspace,
                (hipStream_t)stream, cmb);
}

int asterx_rhs_rk_src(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* prim,
                      const double* A, const double* psi, const double* src, double dt_max, int32_t nout,
                      const asterx_rk_out* outs, double* red, void* workspace, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_params(p)) || (rc = check_grid(gr, 3))) return rc;
  if (p->ct == ASTERX_CT_UCT && gr->ng < 4) return fail(ASTERX_EARG, "rhs_rk_src: upwind CT needs ng >= 4");
  if (!metric || !prim || !A || !psi || !src || !workspace) return fail(ASTERX_EARG, "rhs_rk_src: NULL array");
  if (ws_bytes < asterx_rhs_workspace_size(gr)) return fail(ASTERX_EARG, "rhs_rk_src: workspace too small");
  if (!(dt_max > 0.0)) return fail(ASTERX_EARG, "rhs_rk_src: dt_max must be > 0");
  GD g = make_gd(gr);
  const double* ins[6] = {metric, prim, A, psi, src, (const double*)workspace};
  const size_t nin[6] = {10 * g.N, 5 * g.N, 3 * g.N, g.N, ASTERX_SRC_FIELDS * g.N, ws_bytes / sizeof(double)};
  Combine cmb;
  if ((rc = make_combine(nout, outs, g.N, ins, nin, 6, cmb))) return rc;
  return do_rhs(g, nullptr, p, metric, nullptr, prim, A, psi, dt_max, nullptr, red, (double*)workspace,
                (hipStream_t)stream, cmb, src);
}

int asterx_rhs_rk_noalloc(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* curv,
                          const double* prim, const double* A, const double* psi, double dt_max, int32_t nout,
                          const asterx_rk_out* outs, double* red, void* stream) {
  int rc;
  if ((rc = check_params(p)) || (rc = check_grid(gr, 3))) return rc;
  const size_t need = asterx_rhs_workspace_size(gr);
  if (need > ASTERX_NOALLOC_WS_BYTES)
    return fail(ASTERX_EARG, "rhs_rk_noalloc: the grid needs more workspace than the library holds (64 MiB)");
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  return asterx_rhs_rk(gr, p, metric, curv, prim, A, psi, dt_max, nout, outs, red, ws, need, stream);
}

int asterx_tmunu(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* prim,
                 const double* A, double* tmunu, void* stream) {
  int rc;
  if ((rc = check_params(p)) || (rc = check_grid(gr, 2))) return rc;
  if (!metric || !prim || !A || !tmunu) return fail(ASTERX_EARG, "tmunu: NULL array");
  GD g = make_gd(gr);
  TmunuArgs ta{metric, prim, A, tmunu, p->gamma};
  hipStream_t s = (hipStream_t)stream;
  return timed(KT_TMUNU, s, [&] { hipLaunchKernelGGL(k_tmunu, dim3(tmunu_tiles(g)), dim3(256), 0, s, g, ta); });
}

// Coarse index range reached by prolonging fine indices [lo, hi] along one axis.
void prolong_reach(int lo, int hi, int c0, int vertex, int& cmin, int& cmax) {
  auto fd = [](int f) { return f >= 0 ? f / 2 : -((1 - f) / 2); };
  cmin = c0 + fd(lo) - 1;
  cmax = c0 + fd(hi) + (vertex ? 2 : 1);
}

int check_inter(const asterx_grid* gc, const asterx_grid* gf, const int32_t* c0, const int32_t* stag, int32_t nf,
                const void* src, const void* dst, const int32_t* lo, const int32_t* hi, bool prolong) {
  int rc;
  if ((rc = check_grid(gc, 2)) || (rc = check_grid(gf, 2))) return rc;
  if (!c0 || !stag || !lo || !hi || !src || !dst || nf < 1) return fail(ASTERX_EARG, "inter-level: bad arguments");
  for (int d = 0; d < 3; ++d) {
    if (stag[d] != 0 && stag[d] != 1) return fail(ASTERX_EARG, "inter-level: stag must be 0 (cell) or 1 (vertex)");
    if (lo[d] > hi[d]) return fail(ASTERX_EARG, "inter-level: empty box");
    const asterx_grid* out = prolong ? gf : gc;
    if (lo[d] < -out->ng || hi[d] > out->n[d] + out->ng) return fail(ASTERX_EARG, "inter-level: box outside the target grid");
    int rmin, rmax;
    const asterx_grid* in = prolong ? gc : gf;
    if (prolong) {
      prolong_reach(lo[d], hi[d], c0[d], stag[d], rmin, rmax);
    } else {
      rmin = 2 * (lo[d] - c0[d]);
      rmax = 2 * (hi[d] - c0[d]) + 1;
    }
    if (rmin < -in->ng || rmax > in->n[d] + in->ng) return fail(ASTERX_EARG, "inter-level: stencil outside the source grid");
  }
  return 0;
}

int inter_launch(const asterx_grid* gc, const asterx_grid* gf, const int32_t* c0, const int32_t* stag, int32_t nf,
                 const double* src, double* dst, const int32_t* lo, const int32_t* hi, bool prolong, void* stream) {
  InterArgs a;
  a.gc = make_gd(gc);
  a.gf = make_gd(gf);
  for (int d = 0; d < 3; ++d) {
    a.c0[d] = c0[d];
    a.stag[d] = stag[d];
    a.lo[d] = lo[d];
    a.hi[d] = hi[d];
  }
  a.nf = nf;
  a.src = src;
  a.dst = dst;
  int e[3] = {hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1};
  const bool cells = !stag[0] && !stag[1] && !stag[2];
  if (prolong && cells)
    for (int d = 0; d < 3; ++d) {
      auto fd = [](int f) { return f >= 0 ? f / 2 : -((1 - f) / 2); };
      e[d] = fd(hi[d]) - fd(lo[d]) + 1;  // coarse parents of the fine box
    }
  hipStream_t s = (hipStream_t)stream;
  return timed(KT_INTER, s, [&] {
    if (prolong && cells) hipLaunchKernelGGL(k_prolong_cells, dim3(lin_blocks(e)), dim3(256), 0, s, a);
    else if (prolong) hipLaunchKernelGGL(k_prolong, dim3(lin_blocks(e)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_restrict, dim3(lin_blocks(e)), dim3(256), 0, s, a);
  });
}

int asterx_prolong(const asterx_grid* coarse, const asterx_grid* fine, const int32_t* c0, const int32_t* stag,
                   int32_t nf, const double* cf, double* ff, const int32_t* lo, const int32_t* hi, void* stream) {
  int rc;
  if ((rc = check_inter(coarse, fine, c0, stag, nf, cf, ff, lo, hi, true))) return rc;
  return inter_launch(coarse, fine, c0, stag, nf, cf, ff, lo, hi, true, stream);
}

int asterx_restrict(const asterx_grid* coarse, const asterx_grid* fine, const int32_t* c0, const int32_t* stag,
                    int32_t nf, const double* ff, double* cf, const int32_t* lo, const int32_t* hi, void* stream) {
  int rc;
  if ((rc = check_inter(coarse, fine, c0, stag, nf, ff, cf, lo, hi, false))) return rc;
  return inter_launch(coarse, fine, c0, stag, nf, ff, cf, lo, hi, false, stream);
}

int asterx_zero(double* buf, int64_t count, void* stream) {
  if (!buf || count < 1) return fail(ASTERX_EARG, "zero: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  return timed(KT_ZERO, s, [&] {
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, buf, (long long)count);
  });
}

// ---- batches of patches -------------------------------------------------------------------

int asterx_batch_create(int32_t npatches, const asterx_grid* grids, const asterx_batch_tuning* tuning,
                        asterx_batch** out) {
  if (!out || npatches < 1 || !grids) return fail(ASTERX_EARG, "batch_create: bad arguments");
  *out = nullptr;
  int order = tuning ? tuning->order : 1;
  int per_cu = tuning ? tuning->blocks_per_cu : 4;
  if (order < 0 || order > 2 || per_cu < 1 || per_cu > 64) return fail(ASTERX_EARG, "batch_create: bad tuning");
  asterx_batch* b = new asterx_batch();
  b->np = npatches;
  long long tot = 0;
  for (int q = 0; q < npatches; ++q) {
    int rc = check_grid(&grids[q], 3);
    if (rc) {
      delete b;
      return rc;
    }
    b->off.push_back(tot);
    tot += (long long)grids[q].ld[0] * grids[q].ld[1] * grids[q].ld[2];
  }
  b->ntot = tot;
  std::vector<PatchDesc> pd(npatches);
  for (int q = 0; q < npatches; ++q) {
    GD g = make_gd(&grids[q]);
    g.N = (size_t)tot;  // field stride of the pools
    b->gds.push_back(g);
    pd[q].g = g;
    pd[q].off = b->off[q];
  }
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  b->blocks = per_cu * ncu;
  std::vector<std::vector<Item>> lists(PH_N);
  for (int ph = 0; ph < PH_N; ++ph) {
    std::vector<int> porder(npatches);
    for (int q = 0; q < npatches; ++q) porder[q] = q;
    if (order == 1)
      std::stable_sort(porder.begin(), porder.end(),
                       [&](int x, int y) { return tiles_for(ph, b->gds[x]) > tiles_for(ph, b->gds[y]); });
    std::vector<Item>& L = lists[ph];
    if (order == 2) {  // round robin over patches, largest first
      std::stable_sort(porder.begin(), porder.end(),
                       [&](int x, int y) { return tiles_for(ph, b->gds[x]) > tiles_for(ph, b->gds[y]); });
      unsigned maxt = 0;
      for (int q = 0; q < npatches; ++q) maxt = std::max(maxt, tiles_for(ph, b->gds[q]));
      for (unsigned t = 0; t < maxt; ++t)
        for (int q : porder)
          if (t < tiles_for(ph, b->gds[q])) L.push_back(Item{q, (int)t});
    } else {
      for (int q : porder)
        for (unsigned t = 0; t < tiles_for(ph, b->gds[q]); ++t) L.push_back(Item{q, (int)t});
    }
    b->nitems[ph] = (int)L.size();
  }
  bool ok = hipMalloc((void**)&b->d_patches, sizeof(PatchDesc) * npatches) == hipSuccess &&
            hipMemcpy(b->d_patches, pd.data(), sizeof(PatchDesc) * npatches, hipMemcpyHostToDevice) == hipSuccess;
  for (int ph = 0; ph < PH_N && ok; ++ph) {
    ok = hipMalloc((void**)&b->d_items[ph], sizeof(Item) * lists[ph].size()) == hipSuccess &&
         hipMemcpy(b->d_items[ph], lists[ph].data(), sizeof(Item) * lists[ph].size(), hipMemcpyHostToDevice) ==
             hipSuccess;
  }
  if (!ok) {
    asterx_batch_destroy(b);
    return fail(ASTERX_ELAUNCH, "batch_create: device allocation failed");
  }
  *out = b;
  return 0;
}

int asterx_batch_destroy(asterx_batch* b) {
  if (!b) return 0;
  if (b->d_patches) (void)hipFree(b->d_patches);
  for (int ph = 0; ph < PH_N; ++ph)
    if (b->d_items[ph]) (void)hipFree(b->d_items[ph]);
  delete b;
  return 0;
}

int64_t asterx_batch_points(const asterx_batch* b) { return b ? b->ntot : -1; }

int64_t asterx_batch_offset(const asterx_batch* b, int32_t p) {
  return (b && p >= 0 && p < b->np) ? b->off[p] : -1;
}

size_t asterx_batch_workspace_size(const asterx_batch* b) {
  return b ? (size_t)WS_FIELDS * (size_t)b->ntot * sizeof(double) : 0;
}

int asterx_batch_prim2con(const asterx_batch* b, const asterx_params* p, const double* metric, const double* A,
                          const double* prim, double* cons, void* stream) {
  int rc;
  if (!b) return fail(ASTERX_EARG, "batch is NULL");
  if ((rc = check_params(p))) return rc;
  if (!metric || !A || !prim || !cons) return fail(ASTERX_EARG, "batch_prim2con: NULL array");
  const GD& g = b->gds[0];
  return do_prim2con(g, b, p, metric, A, prim, cons, (hipStream_t)stream);
}

int asterx_batch_c2p(const asterx_batch* b, const asterx_params* p, const double* metric, const double* A,
                     double* cons, double* prim, uint8_t* flags, asterx_c2p_stats* stats, void* stream) {
  int rc;
  if (!b) return fail(ASTERX_EARG, "batch is NULL");
  if ((rc = check_params(p))) return rc;
  if (!metric || !A || !prim || !cons) return fail(ASTERX_EARG, "batch_c2p: NULL array");
  const GD& g = b->gds[0];
  return do_c2p(g, b, p, metric, A, cons, prim, flags, stats, (hipStream_t)stream);
}

int asterx_batch_fill_ghosts(const asterx_batch* b, double* f, int32_t nf, const int32_t* kinds, void* stream) {
  if (!b || !f || !kinds || nf < 1) return fail(ASTERX_EARG, "batch_fill_ghosts: bad arguments");
  for (int a = 0; a < 3; ++a) {
    if (kinds[a] < 0 || kinds[a] > 2) return fail(ASTERX_EARG, "fill_ghosts: unknown boundary kind");
    for (int q = 0; q < b->np; ++q)
      if (kinds[a] == ASTERX_BC_LINEAR && b->gds[q].n[a] < 2)
        return fail(ASTERX_EARG, "fill_ghosts: LINEAR needs n >= 2");
  }
  const GD& g = b->gds[0];
  return do_fill(g, b, f, nf, kinds, (hipStream_t)stream);
}

int asterx_batch_rhs(const asterx_batch* b, const asterx_params* p, const double* metric, const double* curv,
                     const double* prim, const double* A, const double* psi, double dt_max, double* rhs, double* red,
                     void* workspace, size_t ws_bytes, void* stream) {
  int rc;
  if (!b) return fail(ASTERX_EARG, "batch is NULL");
  if ((rc = check_params(p))) return rc;
  if (p->ct == ASTERX_CT_UCT) return fail(ASTERX_EARG, "batch: upwind CT is available for single blocks only");
  if (!metric || !curv || !prim || !A || !psi || !rhs || !workspace) return fail(ASTERX_EARG, "rhs: NULL array");
  if (ws_bytes < asterx_batch_workspace_size(b)) return fail(ASTERX_EARG, "rhs: workspace too small");
  if (!(dt_max > 0.0)) return fail(ASTERX_EARG, "rhs: dt_max must be > 0");
  const GD& g = b->gds[0];
  return do_rhs(g, b, p, metric, curv, prim, A, psi, dt_max, rhs, red, (double*)workspace, (hipStream_t)stream);
}

int asterx_batch_rhs_rk(const asterx_batch* b, const asterx_params* p, const double* metric, const double* curv,
                        const double* prim, const double* A, const double* psi, double dt_max, int32_t nout,
                        const asterx_rk_out* outs, double* red, void* workspace, size_t ws_bytes, void* stream) {
  int rc;
  if (!b) return fail(ASTERX_EARG, "batch is NULL");
  if ((rc = check_params(p))) return rc;
  if (p->ct == ASTERX_CT_UCT) return fail(ASTERX_EARG, "batch: upwind CT is available for single blocks only");
  if (!metric || !curv || !prim || !A || !psi || !workspace) return fail(ASTERX_EARG, "rhs_rk: NULL array");
  if (ws_bytes < asterx_batch_workspace_size(b)) return fail(ASTERX_EARG, "rhs_rk: workspace too small");
  if (!(dt_max > 0.0)) return fail(ASTERX_EARG, "rhs_rk: dt_max must be > 0");
  const size_t n = (size_t)b->ntot;
  const double* ins[6] = {metric, curv, prim, A, psi, (const double*)workspace};
  const size_t nin[6] = {10 * n, 6 * n, 5 * n, 3 * n, n, ws_bytes / sizeof(double)};
  Combine cmb;
  if ((rc = make_combine(nout, outs, n, ins, nin, 6, cmb))) return rc;
  const GD& g = b->gds[0];
  return do_rhs(g, b, p, metric, curv, prim, A, psi, dt_max, nullptr, red, (double*)workspace, (hipStream_t)stream,
                cmb);
}

int asterx_batch_rk_stage(const asterx_batch* b, int32_t nterms, const double* a, const double* const* u,
                          double b_dt, const double* rhs, double* out, void* stream) {
  if (!b) return fail(ASTERX_EARG, "batch is NULL");
  const GD& g = b->gds[0];
  return do_rk(g, b, nterms, a, u, b_dt, rhs, out, (hipStream_t)stream);
}

}  // extern "C"

// ---- adjoint -------------------------------------------------------------------------------

namespace {

unsigned pts_blocks(long long n) { return (unsigned)((n + 255) / 256); }

int adj_fillT(const GD& g, double* f, int nf, hipStream_t s) {
  int rc;
  for (int a = 2; a >= 0; --a) {
    FillTArgs fa{f, nf, a};
    unsigned nb = tiles_for(PH_FILLX + a, g);
    if ((rc = timed(KT_ADJ, s, [&] { hipLaunchKernelGGL(k_fillT, dim3(nb), dim3(256), 0, s, g, fa); }))) return rc;
  }
  return 0;
}

template <int R>
int adj_faces_r(const GD& g, const FaceAdjArgs& fa, hipStream_t s) {
  int rc;
  unsigned nb = tiles_for(PH_FACE, g);
  if ((rc = timed(KT_ADJ, s, [&] { hipLaunchKernelGGL((k_face_adj<0, R>), dim3(nb), dim3(256), 0, s, g, fa); })))
    return rc;
  if ((rc = timed(KT_ADJ, s, [&] { hipLaunchKernelGGL((k_face_adj<1, R>), dim3(nb), dim3(256), 0, s, g, fa); })))
    return rc;
  return timed(KT_ADJ, s, [&] { hipLaunchKernelGGL((k_face_adj<2, R>), dim3(nb), dim3(256), 0, s, g, fa); });
}

int check_adjoint(const asterx_grid* gr, const asterx_params* p, size_t ws_bytes) {
  int rc;
  if ((rc = check_params(p)) || (rc = check_grid(gr, 3))) return rc;
  for (int a = 0; a < 3; ++a)
    if (gr->n[a] < gr->ng + 1) return fail(ASTERX_EARG, "adjoint: periodic blocks need n > ng on every axis");
  if (ws_bytes < asterx_adjoint_workspace_size(gr)) return fail(ASTERX_EARG, "adjoint: workspace too small");
  return 0;
}

// Zero the workspace, copy the stage input, recompute c2p (flags in the workspace tail) and the
// centre field.
int adj_prologue(const GD& g, const asterx_params* p, const double* metric, const double* cons,
                 const double* prim_guess, const double* A, double* ws, uint8_t* flags, hipStream_t s, bool with_c2p) {
  int rc;
  long long nzero = (long long)AW_FIELDS * (long long)g.N;
  if ((rc = timed(KT_ZERO, s, [&] { hipLaunchKernelGGL(k_zero, dim3(pts_blocks(nzero)), dim3(256), 0, s, ws, nzero); })))
    return rc;
  if ((rc = do_bcent(g, A, ws + AW_BC * g.N, s))) return rc;
  if (!with_c2p) return 0;
  long long n5 = 5LL * (long long)g.N;
  if ((rc = timed(KT_ADJ, s, [&] {
         hipLaunchKernelGGL(k_copy, dim3(pts_blocks(n5)), dim3(256), 0, s, g, cons, ws + AW_CONS * g.N, n5);
       })))
    return rc;
  if ((rc = timed(KT_ADJ, s, [&] {
         hipLaunchKernelGGL(k_copy, dim3(pts_blocks(n5)), dim3(256), 0, s, g, prim_guess, ws + AW_PRIM * g.N, n5);
       })))
    return rc;
  const asterx_batch* b = nullptr;
  if ((rc = do_c2p(g, b, p, metric, A, ws + AW_CONS * g.N, ws + AW_PRIM * g.N, flags, nullptr, s))) return rc;
  const int32_t per[3] = {ASTERX_BC_PERIODIC, ASTERX_BC_PERIODIC, ASTERX_BC_PERIODIC};
  return do_fill(g, b, ws + AW_PRIM * g.N, 5, per, s);
}

// Gamma cotangent slots: after the flags in the workspace tail.
double* gamma_slots(const GD& g, double* ws) { return ws + (size_t)AW_FIELDS * g.N + ((size_t)g.N + 7) / 8; }

int gslots_zero(double* slots, hipStream_t s) {
  return timed(KT_ZERO, s, [&] { hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, slots, (long long)GSLOTS); });
}

int gslots_finish(const double* slots, double* gamma_bar, hipStream_t s) {
  return timed(KT_ADJ, s, [&] { hipLaunchKernelGGL(k_gslots, dim3(1), dim3(64), 0, s, slots, gamma_bar); });
}

// Centre-field and face-field cotangents to the edge potential, fold ghosts, add to A_bar.
int adj_epilogue(const GD& g, double* ws, double* A_bar, double* psi_bar, hipStream_t s) {
  int rc;
  int ef[3] = {g.n[0] + 2 * g.ng + 1, g.n[1] + 2 * g.ng + 1, g.n[2] + 2 * g.ng + 1};
  unsigned nb = box_blocks<64, 4>(ef);
  if ((rc = timed(KT_ADJ, s, [&] {
         hipLaunchKernelGGL(k_bcface_adj, dim3(nb), dim3(256), 0, s, g, ws + AW_BCBAR * g.N, ws + AW_BFBAR * g.N);
       })))
    return rc;
  if ((rc = timed(KT_ADJ, s, [&] {
         hipLaunchKernelGGL(k_curlT, dim3(nb), dim3(256), 0, s, g, ws + AW_BFBAR * g.N, ws + AW_ABAR * g.N);
       })))
    return rc;
  if ((rc = adj_fillT(g, ws + AW_ABAR * g.N, 3, s))) return rc;
  unsigned no = tiles_for(PH_RK, g);
  if (A_bar) {
    AccumArgs aa{ws + AW_ABAR * g.N, A_bar, 3};
    if ((rc = timed(KT_ADJ, s, [&] { hipLaunchKernelGGL(k_accum, dim3(no), dim3(256), 0, s, g, aa); }))) return rc;
  }
  if (psi_bar) {
    if ((rc = adj_fillT(g, ws + AW_PSIBAR * g.N, 1, s))) return rc;
    AccumArgs pa{ws + AW_PSIBAR * g.N, psi_bar, 1};
    if ((rc = timed(KT_ADJ, s, [&] { hipLaunchKernelGGL(k_accum, dim3(no), dim3(256), 0, s, g, pa); }))) return rc;
  }
  return 0;
}

}  // namespace

extern "C" {

size_t asterx_adjoint_workspace_size(const asterx_grid* g) {
  if (!g) return 0;
  size_t N = (size_t)g->ld[0] * g->ld[1] * g->ld[2];
  return (size_t)AW_FIELDS * N * sizeof(double) + ((N + 7) / 8) * 8 + GSLOTS * sizeof(double);
}

int asterx_rhs_adjoint(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* curv,
                       const double* cons, const double* prim_guess, const double* A, const double* psi,
                       double dt_max, const double* rhs_bar, double* cons_bar, double* A_bar, double* psi_bar,
                       double* gamma_bar, void* workspace, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_adjoint(gr, p, ws_bytes))) return rc;
  if (p->ct == ASTERX_CT_UCT) return fail(ASTERX_EARG, "rhs_adjoint: upwind CT is not differentiated");
  if (!metric || !curv || !cons || !prim_guess || !A || !psi || !rhs_bar || !cons_bar || !A_bar || !psi_bar ||
      !gamma_bar || !workspace)
    return fail(ASTERX_EARG, "rhs_adjoint: NULL array");
  if (!(dt_max > 0.0)) return fail(ASTERX_EARG, "rhs_adjoint: dt_max must be > 0");
  hipStream_t s = (hipStream_t)stream;
  GD g = make_gd(gr);
  double* ws = (double*)workspace;
  uint8_t* flags = (uint8_t*)(ws + (size_t)AW_FIELDS * g.N);
  double* slots = gamma_slots(g, ws);
  if ((rc = adj_prologue(g, p, metric, cons, prim_guess, A, ws, flags, s, true))) return rc;
  if ((rc = gslots_zero(slots, s))) return rc;
  unsigned nb;
  // fluxbar and vertex_adj tile the (n + 2)^3 vertex box 64 x 4
  int ev[3] = {g.n[0] + 2, g.n[1] + 2, g.n[2] + 2};
  FluxBarArgs fb{rhs_bar, ws + AW_FBAR * g.N};
  nb = box_blocks<64, 4>(ev);
  if ((rc = timed(KT_ADJ, s, [&] { hipLaunchKernelGGL(k_fluxbar, dim3(nb), dim3(256), 0, s, g, fb); }))) return rc;
  FaceAdjArgs fa{metric, ws + AW_PRIM * g.N, A, ws + AW_BC * g.N, ws + AW_FBAR * g.N, ws + AW_PBAR * g.N,
                 ws + AW_BCBAR * g.N, ws + AW_BFBAR * g.N, slots, p->gamma, p->weno_eps, p->weno_q, p->speeds,
                 p->riemann};
  if (p->recon == ASTERX_RECON_MINMOD) rc = adj_faces_r<ASTERX_RECON_MINMOD>(g, fa, s);
  else if (p->recon == ASTERX_RECON_PPM) rc = adj_faces_r<ASTERX_RECON_PPM>(g, fa, s);
  else if (p->recon == ASTERX_RECON_MP5) rc = adj_faces_r<ASTERX_RECON_MP5>(g, fa, s);
  else rc = adj_faces_r<ASTERX_RECON_WENOZ>(g, fa, s);
  if (rc) return rc;
  CellAdjArgs ca{metric, curv, ws + AW_PRIM * g.N, ws + AW_BC * g.N, rhs_bar, ws + AW_PBAR * g.N,
                 ws + AW_BCBAR * g.N, slots, p->gamma};
  if ((rc = timed(KT_ADJ, s, [&] {
         hipLaunchKernelGGL(k_cell_adj, dim3(tiles_for(PH_CELL, g)), dim3(256), 0, s, g, ca);
       })))
    return rc;
  VertexAdjArgs va{metric, rhs_bar, ws + AW_PSIBAR * g.N, ws + AW_AVBAR * g.N, p->xi / dt_max, p->gauge};
  nb = box_blocks<64, 4>(ev);
  if ((rc = timed(KT_ADJ, s, [&] { hipLaunchKernelGGL(k_vertex_adj, dim3(nb), dim3(256), 0, s, g, va); }))) return rc;
  int ee[3] = {g.n[0] + 3, g.n[1] + 3, g.n[2] + 3};
  nb = box_blocks<64, 4>(ee);
  if ((rc = timed(KT_ADJ, s, [&] {
         hipLaunchKernelGGL(k_edge_adj, dim3(nb), dim3(256), 0, s, g, ws + AW_AVBAR * g.N, ws + AW_ABAR * g.N);
       })))
    return rc;
  if ((rc = adj_fillT(g, ws + AW_PBAR * g.N, 5, s))) return rc;
  C2PAdjArgs cpa{metric, ws + AW_PRIM * g.N, ws + AW_BC * g.N, flags, ws + AW_PBAR * g.N, cons_bar,
                 ws + AW_BCBAR * g.N, slots, p->gamma, 0};
  if ((rc = timed(KT_ADJ, s, [&] {
         hipLaunchKernelGGL(k_c2p_adj, dim3(tiles_for(PH_C2P, g)), dim3(256), 0, s, g, cpa);
       })))
    return rc;
  if ((rc = adj_epilogue(g, ws, A_bar, psi_bar, s))) return rc;
  return gslots_finish(slots, gamma_bar, s);
}

int asterx_c2p_adjoint(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* cons,
                       const double* prim_guess, const double* A, const double* prim_bar, double* cons_bar,
                       double* A_bar, double* gamma_bar, void* workspace, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_adjoint(gr, p, ws_bytes))) return rc;
  if (!metric || !cons || !prim_guess || !A || !prim_bar || !cons_bar || !A_bar || !gamma_bar || !workspace)
    return fail(ASTERX_EARG, "c2p_adjoint: NULL array");
  hipStream_t s = (hipStream_t)stream;
  GD g = make_gd(gr);
  double* ws = (double*)workspace;
  uint8_t* flags = (uint8_t*)(ws + (size_t)AW_FIELDS * g.N);
  double* slots = gamma_slots(g, ws);
  if ((rc = adj_prologue(g, p, metric, cons, prim_guess, A, ws, flags, s, true))) return rc;
  if ((rc = gslots_zero(slots, s))) return rc;
  unsigned no = tiles_for(PH_RK, g);
  AccumArgs cp{prim_bar, ws + AW_PBAR * g.N, 5};
  if ((rc = timed(KT_ADJ, s, [&] { hipLaunchKernelGGL(k_accum, dim3(no), dim3(256), 0, s, g, cp); }))) return rc;
  C2PAdjArgs cpa{metric, ws + AW_PRIM * g.N, ws + AW_BC * g.N, flags, ws + AW_PBAR * g.N, cons_bar,
                 ws + AW_BCBAR * g.N, slots, p->gamma, 0};
  if ((rc = timed(KT_ADJ, s, [&] {
         hipLaunchKernelGGL(k_c2p_adj, dim3(tiles_for(PH_C2P, g)), dim3(256), 0, s, g, cpa);
       })))
    return rc;
  if ((rc = adj_epilogue(g, ws, A_bar, nullptr, s))) return rc;
  return gslots_finish(slots, gamma_bar, s);
}

int asterx_prim2con_adjoint(const asterx_grid* gr, const asterx_params* p, const double* metric, const double* A,
                            const double* prim, const double* cons_bar, double* prim_bar, double* A_bar,
                            double* gamma_bar, void* workspace, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_adjoint(gr, p, ws_bytes))) return rc;
  if (!metric || !A || !prim || !cons_bar || !prim_bar || !A_bar || !gamma_bar || !workspace)
    return fail(ASTERX_EARG, "prim2con_adjoint: NULL array");
  hipStream_t s = (hipStream_t)stream;
  GD g = make_gd(gr);
  double* ws = (double*)workspace;
  double* slots = gamma_slots(g, ws);
  if ((rc = adj_prologue(g, p, metric, nullptr, nullptr, A, ws, nullptr, s, false))) return rc;
  if ((rc = gslots_zero(slots, s))) return rc;
  unsigned no = tiles_for(PH_RK, g);
  AccumArgs cp{cons_bar, ws + AW_PBAR * g.N, 5};
  if ((rc = timed(KT_ADJ, s, [&] { hipLaunchKernelGGL(k_accum, dim3(no), dim3(256), 0, s, g, cp); }))) return rc;
  C2PAdjArgs cpa{metric, prim, ws + AW_BC * g.N, nullptr, ws + AW_PBAR * g.N, prim_bar, ws + AW_BCBAR * g.N,
                 slots, p->gamma, 1};
  if ((rc = timed(KT_ADJ, s, [&] {
         hipLaunchKernelGGL(k_c2p_adj, dim3(tiles_for(PH_C2P, g)), dim3(256), 0, s, g, cpa);
       })))
    return rc;
  if ((rc = adj_epilogue(g, ws, A_bar, nullptr, s))) return rc;
  return gslots_finish(slots, gamma_bar, s);
}

}  // extern "C"
