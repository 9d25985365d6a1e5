// asterx_oracle.cpp -- serial FP64 CPU oracle of the Valencia GRMHD right-hand side.
//
// TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the GPU
// library is checked against.  Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark may build, load or call it.  It shares no code,
// header, table or constant with the GPU library (paper_2406_11669_amd/csrc).
//
// Everything here follows the paper (AsterX, arXiv 2406.11669) in its own order
// and notation, written plainly: loops over every face, cell, edge and vertex,
// no tiling, no fusion, no fast-math.  Build: g++ -O2 -ffp-contract=off.  The same
// source built with -fopenmp spreads the k-planes of the grid loops over threads
// (for the all-core CPU baseline); the serial build ignores those pragmas.
// Where the paper is silent or ambiguous the reading taken is stated inline and
// listed, with its reason, in the design notes of the repository.
//
// Index space (Sec. 3.1, storage locations): one padded array per field with
// extents ld[0] x ld[1] x ld[2] (x fastest).  Index (i,j,k) names the cell
// centre (i,j,k), the x-face (i-1/2,j,k), the y-face (i,j-1/2,k), the z-face
// (i,j,k-1/2), the x-edge (i,j-1/2,k-1/2), the y-edge (i-1/2,j,k-1/2), the
// z-edge (i-1/2,j-1/2,k) and the vertex (i-1/2,j-1/2,k-1/2).  Owned indices are
// 0..n-1 per axis; the rest (down to -ng, up to n+ng) are ghosts.
//
// Templated on the scalar type T so the same code can run on dual numbers
// (forward-mode directional derivatives) as well as on double.

#include <cmath>
#include <cstdint>
#include <cstddef>
#include <cstring>
#include <cfloat>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <algorithm>

namespace orc {

using std::sqrt;
using std::fabs;

// ---------------------------------------------------------------------------
// Plain-old-data descriptors passed in from Python (ctypes); the oracle keeps
// its own definitions and does not include the GPU library's header.
struct Grid {
  int32_t n[3];   // owned cells per axis
  int32_t ng;     // ghost layers
  int32_t ld[3];  // allocated extents per axis (>= n + 2 ng + 1)
  int32_t pad_;
  double dx[3];   // grid spacing
};

struct Params {
  double gamma;     // adiabatic index of the ideal-gas EOS (Sec. 3.7)
  double rho_atm;   // atmosphere density floor (Sec. 3.6)
  double k_atm;     // polytropic constant of the atmosphere EOS
  double xi;        // generalized-Lorenz damping, in units of 1/dt_max (Sec. 3.4: 1.5)
  double c2p_tol;   // Noble Newton tolerance on max(|dz/z|, |dw|)
  double wmax;      // Lorentz-factor safety cap used by the c2p clamps
  double weno_eps;  // WENO-Z epsilon
  double weno_q;    // WENO-Z exponent
  int32_t c2p_maxit;    // Noble Newton iteration cap
  int32_t brent_maxit;  // Brent iteration cap
  int32_t recon;        // 0 MINMOD, 1 PPM, 2 WENO-Z
  int32_t gauge;        // 0 generalized Lorenz, 1 algebraic
  int32_t speeds;       // 0 quartic, 1 quadratic bound
  int32_t c2p_method;   // 0 Noble then Palenzuela, 1 Noble only, 2 Palenzuela only
  int32_t riemann;      // 0 HLLE, 1 Lax-Friedrichs
  int32_t ct;           // electric field on edges: 0 flux CT, 1 upwind CT
};

enum { REC_MINMOD = 0, REC_PPM = 1, REC_WENOZ = 2, REC_MP5 = 3 };
enum { RIEMANN_HLLE = 0, RIEMANN_LXF = 1 };
enum { CT_FCT = 0, CT_UCT = 1 };
enum { GAUGE_LORENZ = 0, GAUGE_ALGEBRAIC = 1 };
enum { SPEED_QUARTIC = 0, SPEED_BOUND = 1 };
enum { BC_PERIODIC = 0, BC_COPY = 1, BC_LINEAR = 2 };

// c2p flags (per cell bits) and counters
enum { FL_NOBLE_FAIL = 1, FL_FALLBACK = 2, FL_ATMO = 4, FL_HARD_FAIL = 8, FL_NAN_IN = 16 };
enum { ST_NOBLE_FAIL = 0, ST_FALLBACK = 1, ST_ATMO = 2, ST_HARD_FAIL = 3, ST_NAN_IN = 4, ST_ITERS_MAX = 5 };

static inline size_t npts(const Grid& g) { return (size_t)g.ld[0] * g.ld[1] * g.ld[2]; }
static inline size_t at(const Grid& g, int i, int j, int k) {
  return ((size_t)(k + g.ng) * g.ld[1] + (size_t)(j + g.ng)) * g.ld[0] + (size_t)(i + g.ng);
}

using std::pow;

static inline double value_of(double x) { return x; }
template <class T> static inline T sq(const T& x) { return x * x; }
template <class T> static inline bool is_finite(const T& x) { return std::isfinite(value_of(x)); }

// ---------------------------------------------------------------------------
// Operation-counting scalar: a double that counts its floating-point operations
// (+, -, *, /, sqrt, pow each count one) so that the algorithmic FLOPs of a
// kernel can be measured by running the plain implementation on it.
struct Cnt {
  double v;
  static unsigned long long ops;
  Cnt() : v(0.0) {}
  Cnt(double x) : v(x) {}
};
unsigned long long Cnt::ops = 0;
static inline double value_of(const Cnt& x) { return x.v; }
static inline Cnt operator+(const Cnt& a, const Cnt& b) { ++Cnt::ops; return Cnt(a.v + b.v); }
static inline Cnt operator-(const Cnt& a, const Cnt& b) { ++Cnt::ops; return Cnt(a.v - b.v); }
static inline Cnt operator*(const Cnt& a, const Cnt& b) { ++Cnt::ops; return Cnt(a.v * b.v); }
static inline Cnt operator/(const Cnt& a, const Cnt& b) { ++Cnt::ops; return Cnt(a.v / b.v); }
static inline Cnt operator-(const Cnt& a) { return Cnt(-a.v); }
static inline bool operator<(const Cnt& a, const Cnt& b) { return a.v < b.v; }
static inline bool operator>(const Cnt& a, const Cnt& b) { return a.v > b.v; }
static inline bool operator<=(const Cnt& a, const Cnt& b) { return a.v <= b.v; }
static inline bool operator>=(const Cnt& a, const Cnt& b) { return a.v >= b.v; }
static inline bool operator==(const Cnt& a, const Cnt& b) { return a.v == b.v; }
static inline bool operator!=(const Cnt& a, const Cnt& b) { return a.v != b.v; }
static inline Cnt sqrt(const Cnt& a) { ++Cnt::ops; return Cnt(std::sqrt(a.v)); }
static inline Cnt fabs(const Cnt& a) { return Cnt(std::fabs(a.v)); }
static inline Cnt pow(const Cnt& a, const Cnt& b) { ++Cnt::ops; return Cnt(std::pow(a.v, b.v)); }
static inline Cnt pow(const Cnt& a, double b) { ++Cnt::ops; return Cnt(std::pow(a.v, b)); }

// ---------------------------------------------------------------------------
// Forward-mode dual number: value v and tangent d, so that running the plain
// implementation on it yields the directional derivative (JVP) of any output
// along a chosen input tangent.  Branches compare values only; converged
// iterations carry the tangent of their final iterate (within a relative
// error of the order of the last Newton step).
struct Dl {
  double v, d;
  Dl() : v(0.0), d(0.0) {}
  Dl(double x) : v(x), d(0.0) {}
  Dl(double x, double t) : v(x), d(t) {}
};
static inline double value_of(const Dl& x) { return x.v; }
static inline Dl operator+(const Dl& a, const Dl& b) { return Dl(a.v + b.v, a.d + b.d); }
static inline Dl operator-(const Dl& a, const Dl& b) { return Dl(a.v - b.v, a.d - b.d); }
static inline Dl operator*(const Dl& a, const Dl& b) { return Dl(a.v * b.v, a.d * b.v + a.v * b.d); }
static inline Dl operator/(const Dl& a, const Dl& b) {
  double q = a.v / b.v;
  return Dl(q, (a.d - q * b.d) / b.v);
}
static inline Dl operator-(const Dl& a) { return Dl(-a.v, -a.d); }
static inline bool operator<(const Dl& a, const Dl& b) { return a.v < b.v; }
static inline bool operator>(const Dl& a, const Dl& b) { return a.v > b.v; }
static inline bool operator<=(const Dl& a, const Dl& b) { return a.v <= b.v; }
static inline bool operator>=(const Dl& a, const Dl& b) { return a.v >= b.v; }
static inline bool operator==(const Dl& a, const Dl& b) { return a.v == b.v; }
static inline bool operator!=(const Dl& a, const Dl& b) { return a.v != b.v; }
static inline Dl sqrt(const Dl& a) {
  double r = std::sqrt(a.v);
  return Dl(r, a.d / (2.0 * r));
}
static inline Dl fabs(const Dl& a) { return a.v < 0.0 ? -a : a; }
static inline Dl pow(const Dl& a, const Dl& b) {
  double r = std::pow(a.v, b.v);
  double t = (a.d != 0.0 ? b.v * std::pow(a.v, b.v - 1.0) * a.d : 0.0) + (b.d != 0.0 ? r * std::log(a.v) * b.d : 0.0);
  return Dl(r, t);
}
static inline Dl pow(const Dl& a, double b) { return Dl(std::pow(a.v, b), a.d != 0.0 ? b * std::pow(a.v, b - 1.0) * a.d : 0.0); }

// Phase marks: rhs_grid calls phase_mark(k) at the boundaries of its parts; for the
// counting type the operations of each part are accumulated into g_phase_ops.
static unsigned long long g_phase_ops[4];
static unsigned long long g_phase_last = 0;
template <class T> static inline void phase_mark(int) {}
template <> inline void phase_mark<Cnt>(int k) {
  if (k >= 0) g_phase_ops[k] += Cnt::ops - g_phase_last;
  g_phase_last = Cnt::ops;
}

// ---------------------------------------------------------------------------
// 3+1 geometry at a point (Sec. 2.1, line element): lapse alpha, shift beta^i,
// spatial metric gamma_ij; derived inverse, determinant, sqrt(gamma).
// Metric storage order: alpha, beta^x, beta^y, beta^z, gxx, gxy, gxz, gyy, gyz, gzz.
template <class T> struct Geom {
  T alp, beta[3], g[3][3], gi[3][3], det, sqrtg, betal[3];
};

template <class T> Geom<T> make_geom(const T m[10]) {
  Geom<T> G;
  G.alp = m[0];
  for (int i = 0; i < 3; ++i) G.beta[i] = m[1 + i];
  G.g[0][0] = m[4]; G.g[0][1] = m[5]; G.g[0][2] = m[6];
  G.g[1][0] = m[5]; G.g[1][1] = m[7]; G.g[1][2] = m[8];
  G.g[2][0] = m[6]; G.g[2][1] = m[8]; G.g[2][2] = m[9];
  // inverse by cofactors
  T c[3][3];
  c[0][0] = G.g[1][1] * G.g[2][2] - G.g[1][2] * G.g[2][1];
  c[0][1] = G.g[0][2] * G.g[2][1] - G.g[0][1] * G.g[2][2];
  c[0][2] = G.g[0][1] * G.g[1][2] - G.g[0][2] * G.g[1][1];
  c[1][0] = G.g[1][2] * G.g[2][0] - G.g[1][0] * G.g[2][2];
  c[1][1] = G.g[0][0] * G.g[2][2] - G.g[0][2] * G.g[2][0];
  c[1][2] = G.g[0][2] * G.g[1][0] - G.g[0][0] * G.g[1][2];
  c[2][0] = G.g[1][0] * G.g[2][1] - G.g[1][1] * G.g[2][0];
  c[2][1] = G.g[0][1] * G.g[2][0] - G.g[0][0] * G.g[2][1];
  c[2][2] = G.g[0][0] * G.g[1][1] - G.g[0][1] * G.g[1][0];
  G.det = G.g[0][0] * c[0][0] + G.g[0][1] * c[1][0] + G.g[0][2] * c[2][0];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) G.gi[i][j] = c[i][j] / G.det;
  G.sqrtg = sqrt(G.det);
  for (int i = 0; i < 3; ++i) {
    G.betal[i] = T(0);
    for (int j = 0; j < 3; ++j) G.betal[i] = G.betal[i] + G.g[i][j] * G.beta[j];
  }
  return G;
}

// Inverse 4-metric (from the line element of Sec. 2.1):
// g^00 = -1/alpha^2, g^0i = beta^i/alpha^2, g^ij = gamma^ij - beta^i beta^j/alpha^2.
template <class T> void inverse_4metric(const Geom<T>& G, T gu[4][4]) {
  T ia2 = T(1) / (G.alp * G.alp);
  gu[0][0] = -ia2;
  for (int i = 0; i < 3; ++i) {
    gu[0][i + 1] = G.beta[i] * ia2;
    gu[i + 1][0] = gu[0][i + 1];
    for (int j = 0; j < 3; ++j) gu[i + 1][j + 1] = G.gi[i][j] - G.beta[i] * G.beta[j] * ia2;
  }
}

// ---------------------------------------------------------------------------
// Equation of state (Sec. 3.7).  Ideal fluid p = (Gamma-1) rho eps; polytrope
// p = K rho^Gamma, eps = p/((Gamma-1) rho).  h = 1 + eps + p/rho (Sec. 2.2).
template <class T> T eos_eps_from_p(const T& rho, const T& p, const T& gam) { return p / ((gam - T(1)) * rho); }
template <class T> T eos_p_from_eps(const T& rho, const T& eps, const T& gam) { return (gam - T(1)) * rho * eps; }
template <class T> T polytrope_p(const T& rho, double K, const T& gam) { return T(K) * pow(rho, gam); }

// ---------------------------------------------------------------------------
// Fluid state at a point (Sec. 2.2).  Primitives: rho, p, v^i (Eulerian
// 3-velocity, contravariant).  Btilde^i = sqrt(gamma) B^i.
// W = 1/sqrt(1 - v^i v_i); comoving field b^mu from the Eulerian field (eq.
// eulerianB), with u^0 = W/alpha, u^i = W (v^i - beta^i/alpha), and the
// covariant spatial b_i = B_i/W + alpha b^0 v_i (Sec. 3.5).
template <class T> struct Fluid {
  T rho, p, eps, h, v[3], vl[3], v2, W, B[3], Bl[3], B2, Bv, b0, b[3], bl[3], bsq, u0, u[3];
};

template <class T> Fluid<T> make_fluid(const Geom<T>& G, const T prim[5], const T Bt[3], const T& gam) {
  Fluid<T> F;
  F.rho = prim[0];
  F.p = prim[1];
  F.eps = eos_eps_from_p(F.rho, F.p, gam);
  F.h = T(1) + F.eps + F.p / F.rho;
  for (int i = 0; i < 3; ++i) F.v[i] = prim[2 + i];
  for (int i = 0; i < 3; ++i) {
    F.vl[i] = T(0);
    for (int j = 0; j < 3; ++j) F.vl[i] = F.vl[i] + G.g[i][j] * F.v[j];
  }
  F.v2 = F.v[0] * F.vl[0] + F.v[1] * F.vl[1] + F.v[2] * F.vl[2];
  F.W = T(1) / sqrt(T(1) - F.v2);
  for (int i = 0; i < 3; ++i) F.B[i] = Bt[i] / G.sqrtg;
  for (int i = 0; i < 3; ++i) {
    F.Bl[i] = T(0);
    for (int j = 0; j < 3; ++j) F.Bl[i] = F.Bl[i] + G.g[i][j] * F.B[j];
  }
  F.B2 = F.B[0] * F.Bl[0] + F.B[1] * F.Bl[1] + F.B[2] * F.Bl[2];
  F.Bv = F.B[0] * F.vl[0] + F.B[1] * F.vl[1] + F.B[2] * F.vl[2];
  F.b0 = F.W * F.Bv / G.alp;
  F.u0 = F.W / G.alp;
  for (int i = 0; i < 3; ++i) F.u[i] = F.W * (F.v[i] - G.beta[i] / G.alp);
  for (int i = 0; i < 3; ++i) F.b[i] = (F.B[i] + G.alp * F.b0 * F.u[i]) / F.W;
  F.bsq = (F.B2 + G.alp * G.alp * F.b0 * F.b0) / (F.W * F.W);
  for (int i = 0; i < 3; ++i) F.bl[i] = F.Bl[i] / F.W + G.alp * F.b0 * F.vl[i];
  return F;
}

// ---------------------------------------------------------------------------
// Primitive -> conserved map, Sec. 2.2 (conserved-variable definitions, eq. cons):
//   D = rho W,  S_j = (rho h + b^2) W^2 v_j - alpha b^0 b_j,
//   tau = (rho h + b^2) W^2 - (p + b^2/2) - alpha^2 (b^0)^2 - D,
// evolved densitized by sqrt(gamma) (flux-conservative form, eq. fluxconseqs).
// Output order: Dt, St_x, St_y, St_z, taut.
template <class T> void prim2con_point(const Geom<T>& G, const Fluid<T>& F, T cons[5]) {
  T rhohb = F.rho * F.h + F.bsq;
  T D = F.rho * F.W;
  T S[3];
  for (int j = 0; j < 3; ++j) S[j] = rhohb * F.W * F.W * F.vl[j] - G.alp * F.b0 * F.bl[j];
  T tau = rhohb * F.W * F.W - (F.p + F.bsq / T(2)) - G.alp * G.alp * F.b0 * F.b0 - D;
  cons[0] = G.sqrtg * D;
  for (int j = 0; j < 3; ++j) cons[1 + j] = G.sqrtg * S[j];
  cons[4] = G.sqrtg * tau;
}

// ---------------------------------------------------------------------------
// Physical fluxes along direction d, eq. grmhdeqs, multiplied by
// sqrt(-g) = alpha sqrt(gamma) (eq. fluxconseqs).  vt^i = alpha v^i - beta^i.
// Returns 7 components: Dt, St_x, St_y, St_z, taut, and the induction fluxes of
// the two transverse densitized field components t1 = (d+1)%3, t2 = (d+2)%3:
//   Btilde^k vt^d - Btilde^d vt^k  (eq. inductioneq).
// U receives the matching 7 conserved components (the HLLE state vector).
template <class T> void flux_point(const Geom<T>& G, const Fluid<T>& F, int d, T U[7], T Fx[7]) {
  T cons[5];
  prim2con_point(G, F, cons);
  T vt[3];
  for (int i = 0; i < 3; ++i) vt[i] = G.alp * F.v[i] - G.beta[i];
  T ptot = F.p + F.bsq / T(2);
  // undensitized D, S_j, tau
  T D = cons[0] / G.sqrtg, tau = cons[4] / G.sqrtg, S[3];
  for (int j = 0; j < 3; ++j) S[j] = cons[1 + j] / G.sqrtg;
  // F^d / alpha pieces
  Fx[0] = G.sqrtg * (D * vt[d]);
  for (int j = 0; j < 3; ++j) {
    T delta = (j == d) ? T(1) : T(0);
    Fx[1 + j] = G.sqrtg * (S[j] * vt[d] + G.alp * (ptot * delta - F.bl[j] * F.B[d] / F.W));
  }
  Fx[4] = G.sqrtg * (tau * vt[d] + G.alp * (ptot * F.v[d] - G.alp * F.b0 * F.B[d] / F.W));
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  Fx[5] = G.sqrtg * (F.B[t1] * vt[d] - F.B[d] * vt[t1]);
  Fx[6] = G.sqrtg * (F.B[t2] * vt[d] - F.B[d] * vt[t2]);
  for (int c = 0; c < 5; ++c) U[c] = cons[c];
  U[5] = G.sqrtg * F.B[t1];
  U[6] = G.sqrtg * F.B[t2];
}

// ---------------------------------------------------------------------------
// Characteristic speeds along direction d (Sec. 3.3: outer roots of the
// fast-magnetosonic quartic).  Reading: the covariant dispersion relation of
// ideal MHD for a wave front phi = x^d - lambda t, with covector
// phi_mu = (-lambda, e_d):  a = phi_mu u^mu, bb = phi_mu b^mu,
// G = g^{mu nu} phi_mu phi_nu,
//   Q(lambda) = rho h (1 - cs^2) a^4 - (rho h cs^2 + b^2) a^2 G + cs^2 bb^2 G.
// Its largest/smallest real roots are c_+/c_-.  Root finding: Newton from the
// outer roots of the isotropic bound (1 - w2) a^2 - w2 G = 0 with
// w2 = cs^2 + cA^2 - cs^2 cA^2 (which lies outside every fast root), inward.
template <class T> struct Disp {
  T A4, Bq, Cq, a0, a1, bb0, bb1, G0, G1, G2;
};

template <class T> Disp<T> make_disp(const Geom<T>& G, const Fluid<T>& F, int d, const T& gam, T& w2) {
  Disp<T> Q;
  T gu[4][4];
  inverse_4metric(G, gu);
  T rhoh = F.rho * F.h;
  T cs2 = gam * F.p / rhoh;
  Q.A4 = rhoh * (T(1) - cs2);
  Q.Bq = rhoh * cs2 + F.bsq;
  Q.Cq = cs2;
  Q.a0 = F.u[d];
  Q.a1 = -F.u0;
  Q.bb0 = F.b[d];
  Q.bb1 = -F.b0;
  Q.G0 = gu[d + 1][d + 1];
  Q.G1 = T(-2) * gu[0][d + 1];
  Q.G2 = gu[0][0];
  T cA2 = F.bsq / (rhoh + F.bsq);
  w2 = cs2 + cA2 - cs2 * cA2;
  return Q;
}

template <class T> void disp_eval(const Disp<T>& Q, const T& lam, T& q, T& dq) {
  T a = Q.a0 + Q.a1 * lam;
  T bb = Q.bb0 + Q.bb1 * lam;
  T Gm = Q.G0 + Q.G1 * lam + Q.G2 * lam * lam;
  T dG = Q.G1 + T(2) * Q.G2 * lam;
  q = Q.A4 * a * a * a * a - Q.Bq * a * a * Gm + Q.Cq * bb * bb * Gm;
  dq = T(4) * Q.A4 * a * a * a * Q.a1 - Q.Bq * (T(2) * a * Q.a1 * Gm + a * a * dG) +
       Q.Cq * (T(2) * bb * Q.bb1 * Gm + bb * bb * dG);
}

// Roots of qa x^2 + qb x + qc (qa > 0), larger first, in the cancellation-free form.
template <class T> void quad_roots(const T& qa, const T& qb, const T& qc, T& rp, T& rm) {
  T disc = qb * qb - T(4) * qa * qc;
  if (disc < T(0)) disc = T(0);
  T sd = sqrt(disc);
  T qq = (qb >= T(0)) ? T(-0.5) * (qb + sd) : T(-0.5) * (qb - sd);
  T r1, r2;
  if (qq == T(0)) {
    r1 = r2 = T(0);
  } else {
    r1 = qq / qa;
    r2 = qc / qq;
  }
  if (r1 >= r2) { rp = r1; rm = r2; } else { rp = r2; rm = r1; }
}

template <class T> void bound_roots(const Disp<T>& Q, const T& w2, T& lp, T& lm) {
  T om = T(1) - w2;
  T qa = om * Q.a1 * Q.a1 - w2 * Q.G2;
  T qb = T(2) * om * Q.a0 * Q.a1 - w2 * Q.G1;
  T qc = om * Q.a0 * Q.a0 - w2 * Q.G0;
  quad_roots(qa, qb, qc, lp, lm);
}

template <class T> T quartic_newton(const Disp<T>& Q, T lam) {
  for (int it = 0; it < 30; ++it) {
    T q, dq;
    disp_eval(Q, lam, q, dq);
    if (dq == T(0)) break;
    T step = q / dq;
    lam = lam - step;
    T ref = fabs(lam) > T(1) ? fabs(lam) : T(1);
    if (fabs(step) <= T(4.0 * DBL_EPSILON) * ref) break;
  }
  return lam;
}

template <class T> void speeds_point(const Geom<T>& G, const Fluid<T>& F, int d, const T& gam, int kind, T& cm, T& cp) {
  T w2;
  Disp<T> Q = make_disp(G, F, d, gam, w2);
  T lp, lm;
  bound_roots(Q, w2, lp, lm);
  if (kind == SPEED_BOUND) { cp = lp; cm = lm; return; }
  cp = quartic_newton(Q, lp);
  cm = quartic_newton(Q, lm);
}

// ---------------------------------------------------------------------------
// HLLE flux (Sec. 3.3, eq. HLLEfluxes) with c_max = max(0, c+_l, c+_r),
// c_min = -min(0, c-_l, c-_r).
template <class T> void hlle(const T UL[7], const T FL[7], const T& cmL, const T& cpL, const T UR[7], const T FR[7],
                             const T& cmR, const T& cpR, T Fo[7], T& cmax_out, T& cmin_out) {
  T cmax = T(0);
  if (cpL > cmax) cmax = cpL;
  if (cpR > cmax) cmax = cpR;
  T mn = T(0);
  if (cmL < mn) mn = cmL;
  if (cmR < mn) mn = cmR;
  T cmin = -mn;
  cmax_out = cmax;
  cmin_out = cmin;
  T den = cmax + cmin;
  for (int c = 0; c < 7; ++c) {
    if (den > T(0))
      Fo[c] = (cmin * FR[c] + cmax * FL[c] - cmax * cmin * (UR[c] - UL[c])) / den;
    else
      Fo[c] = T(0.5) * (FL[c] + FR[c]);
  }
}

// Lax-Friedrichs flux (Sec. 3.3, eq. LxFfluxes): the mean of the two side fluxes
// minus c_wave/2 times the jump of the state vector, with c_wave = max(c_max,
// c_min) and c_max, c_min as for HLLE.
template <class T> void lxf(const T UL[7], const T FL[7], const T& cmL, const T& cpL, const T UR[7], const T FR[7],
                            const T& cmR, const T& cpR, T Fo[7], T& cmax_out, T& cmin_out) {
  T cmax = T(0);
  if (cpL > cmax) cmax = cpL;
  if (cpR > cmax) cmax = cpR;
  T mn = T(0);
  if (cmL < mn) mn = cmL;
  if (cmR < mn) mn = cmR;
  T cmin = -mn;
  cmax_out = cmax;
  cmin_out = cmin;
  T cwave = cmax > cmin ? cmax : cmin;
  for (int c = 0; c < 7; ++c) Fo[c] = (FR[c] + FL[c] - cwave * (UR[c] - UL[c])) / T(2);
}

template <class T> void riemann_flux(int kind, const T UL[7], const T FL[7], const T& cmL, const T& cpL,
                                     const T UR[7], const T FR[7], const T& cmR, const T& cpR, T Fo[7], T& cmax,
                                     T& cmin) {
  if (kind == RIEMANN_LXF)
    lxf(UL, FL, cmL, cpL, UR, FR, cmR, cpR, Fo, cmax, cmin);
  else
    hlle(UL, FL, cmL, cpL, UR, FR, cmR, cpR, Fo, cmax, cmin);
}

// ---------------------------------------------------------------------------
// Reconstruction (Sec. 3.3).  Each routine takes the five cell values
// a[0..4] = a_{c-2}..a_{c+2} around cell c and returns the values at its left
// face (c-1/2) and right face (c+1/2).
// Near ties of the discontinuous limiter decisions, PPM's monotonicity constraints (serial build only;
// the counts do not enter any result; minmod and the MC slope are continuous across their switching
// points, so their branches cannot change a result).  A comparison of p with q whose sides differ but
// agree to 1e-12 of their magnitude is one that a different but equally valid rounding of p or q (fused
// multiply-adds, another summation order) can decide the other way; exact equalities (uniform data) are
// computed exactly by any rounding order.  The tests report the count beside the agreement of two
// implementations.
static unsigned long long g_tie_decisions = 0, g_tie_near = 0;
template <class T> inline void note_tie(const T&, const T&) {}
inline void note_tie(double p, double q) {
#ifndef _OPENMP
  ++g_tie_decisions;
  if (p != q && std::fabs(p - q) <= 1e-12 * (std::fabs(p) + std::fabs(q))) ++g_tie_near;
#else
  (void)p;
  (void)q;
#endif
}

template <class T> T minmod2(const T& x, const T& y) {
  if (x * y > T(0)) return (x > T(0) ? T(1) : T(-1)) * (fabs(x) < fabs(y) ? fabs(x) : fabs(y));
  return T(0);
}

// MINMOD: slope sigma = minmod(a_c - a_{c-1}, a_{c+1} - a_c); faces a_c -+ sigma/2.
template <class T> void rec_minmod(const T a[5], T& aL, T& aR) {
  T s = minmod2(a[2] - a[1], a[3] - a[2]);
  aL = a[2] - s / T(2);
  aR = a[2] + s / T(2);
}

// PPM (Colella & Woodward 1984): monotonized-central slopes, the quartic face
// interpolant, then the two monotonicity constraints.  No contact steepening
// and no flattening (the paper names neither).
template <class T> T ppm_slope(const T& am, const T& a0, const T& ap) {
  T da = (ap - am) / T(2);
  if ((ap - a0) * (a0 - am) > T(0)) {
    T m = fabs(da);
    T l = T(2) * fabs(a0 - am);
    T r = T(2) * fabs(ap - a0);
    if (l < m) m = l;
    if (r < m) m = r;
    return (da >= T(0) ? T(1) : T(-1)) * m;
  }
  return T(0);
}

template <class T> void rec_ppm(const T a[5], T& aL, T& aR) {
  T dm1 = ppm_slope(a[0], a[1], a[2]);
  T d0 = ppm_slope(a[1], a[2], a[3]);
  T dp1 = ppm_slope(a[2], a[3], a[4]);
  aL = (a[1] + a[2]) / T(2) - (d0 - dm1) / T(6);
  aR = (a[2] + a[3]) / T(2) - (dp1 - d0) / T(6);
  T ac = a[2];
  note_tie(aR, ac);
  note_tie(aL, ac);
  if ((aR - ac) * (ac - aL) <= T(0)) {
    aL = ac;
    aR = ac;
  } else {
    T dd = aR - aL;
    T a6 = dd * (ac - (aL + aR) / T(2));
    T d2 = dd * dd / T(6);
    note_tie(a6, d2);
    note_tie(-d2, a6);
    if (a6 > d2)
      aL = T(3) * ac - T(2) * aR;
    else if (-d2 > a6)
      aR = T(3) * ac - T(2) * aL;
  }
}

// WENO-Z (Borges et al. 2008) on the fifth-order Jiang-Shu stencils.
// Left-biased value at c+1/2 from a_{c-2..c+2}:
template <class T> T wenoz_right_face(const T& am2, const T& am1, const T& a0, const T& ap1, const T& ap2, double eps,
                                      double qexp) {
  T q0 = (T(2) * am2 - T(7) * am1 + T(11) * a0) / T(6);
  T q1 = (-am1 + T(5) * a0 + T(2) * ap1) / T(6);
  T q2 = (T(2) * a0 + T(5) * ap1 - ap2) / T(6);
  T b0 = T(13.0 / 12.0) * sq(am2 - T(2) * am1 + a0) + T(0.25) * sq(am2 - T(4) * am1 + T(3) * a0);
  T b1 = T(13.0 / 12.0) * sq(am1 - T(2) * a0 + ap1) + T(0.25) * sq(am1 - ap1);
  T b2 = T(13.0 / 12.0) * sq(a0 - T(2) * ap1 + ap2) + T(0.25) * sq(T(3) * a0 - T(4) * ap1 + ap2);
  T tau5 = fabs(b0 - b2);
  T w0 = T(0.1) * (T(1) + pow(tau5 / (b0 + T(eps)), qexp));
  T w1 = T(0.6) * (T(1) + pow(tau5 / (b1 + T(eps)), qexp));
  T w2 = T(0.3) * (T(1) + pow(tau5 / (b2 + T(eps)), qexp));
  T s = w0 + w1 + w2;
  return (w0 * q0 + w1 * q1 + w2 * q2) / s;
}

template <class T> void rec_wenoz(const T a[5], T& aL, T& aR, double eps, double qexp) {
  aR = wenoz_right_face(a[0], a[1], a[2], a[3], a[4], eps, qexp);
  // the left face is the mirror image
  aL = wenoz_right_face(a[4], a[3], a[2], a[1], a[0], eps, qexp);
}

// MP5 (Suresh & Huynh 1997), the paper's fifth scheme (Sec. 3.3, cited only).
// Left-biased value at c+1/2 from a_{c-2..c+2}: the fifth-order interpolant is
// kept when it lies between a_c and the monotonicity-preserving bound
// a_c + minmod(a_{c+1} - a_c, alpha (a_c - a_{c-1})); otherwise it is replaced by
// the median of itself and the accuracy-preserving interval [f_min, f_max]
// built from the M4 curvature measures.  alpha = 4.
template <class T> T tmin(const T& x, const T& y) { return y < x ? y : x; }
template <class T> T tmax(const T& x, const T& y) { return y > x ? y : x; }

// minmod of four numbers: the one of least magnitude if all share a sign, else 0
template <class T> T minmod4(const T& w, const T& x, const T& y, const T& z) {
  if (w > T(0) && x > T(0) && y > T(0) && z > T(0)) return tmin(tmin(w, x), tmin(y, z));
  if (w < T(0) && x < T(0) && y < T(0) && z < T(0)) return tmax(tmax(w, x), tmax(y, z));
  return T(0);
}

// median of three numbers
template <class T> T median3(const T& x, const T& y, const T& z) { return x + minmod2(y - x, z - x); }

template <class T> T mp5_right_face(const T& am2, const T& am1, const T& a0, const T& ap1, const T& ap2) {
  const T alpha = T(4);
  T f_or = (T(2) * am2 - T(13) * am1 + T(47) * a0 + T(27) * ap1 - T(3) * ap2) / T(60);
  T f_mp = a0 + minmod2(ap1 - a0, alpha * (a0 - am1));
  if ((f_or - a0) * (f_or - f_mp) <= T(0)) return f_or;
  T d_m = am2 - T(2) * am1 + a0;
  T d_0 = am1 - T(2) * a0 + ap1;
  T d_p = a0 - T(2) * ap1 + ap2;
  T dm4_right = minmod4(T(4) * d_0 - d_p, T(4) * d_p - d_0, d_0, d_p);
  T dm4_left = minmod4(T(4) * d_0 - d_m, T(4) * d_m - d_0, d_0, d_m);
  T f_ul = a0 + alpha * (a0 - am1);
  T f_av = (a0 + ap1) / T(2);
  T f_md = f_av - dm4_right / T(2);
  T f_lc = a0 + (a0 - am1) / T(2) + T(4) / T(3) * dm4_left;
  T f_min = tmax(tmin(tmin(a0, ap1), f_md), tmin(tmin(a0, f_ul), f_lc));
  T f_max = tmin(tmax(tmax(a0, ap1), f_md), tmax(tmax(a0, f_ul), f_lc));
  return median3(f_or, f_min, f_max);
}

template <class T> void rec_mp5(const T a[5], T& aL, T& aR) {
  aR = mp5_right_face(a[0], a[1], a[2], a[3], a[4]);
  aL = mp5_right_face(a[4], a[3], a[2], a[1], a[0]);
}

template <class T> void reconstruct_cell(int kind, const T a[5], T& aL, T& aR, const Params& P) {
  if (kind == REC_MINMOD)
    rec_minmod(a, aL, aR);
  else if (kind == REC_PPM)
    rec_ppm(a, aL, aR);
  else if (kind == REC_MP5)
    rec_mp5(a, aL, aR);
  else
    rec_wenoz(a, aL, aR, P.weno_eps, P.weno_q);
}

// Face i-1/2 from the six cells a[0..5] = a_{i-3}..a_{i+2}:
// left state = right face of cell i-1, right state = left face of cell i.
template <class T> void reconstruct_face(int kind, const T a[6], T& L, T& R, const Params& P) {
  T dummy;
  reconstruct_cell(kind, a, dummy, L, P);
  reconstruct_cell(kind, a + 1, R, dummy, P);
}

// ---------------------------------------------------------------------------
// Vertex -> centre/face interpolation of the spacetime data (Sec. 3.2: fourth
// order Lagrange).  A cell centre lies midway between vertices i and i+1; the
// four-point stencil uses vertices i-1..i+2.  Weights at the midpoint
// (-1, 9, 9, -1)/16; the derivative of the same cubic at the midpoint is
// (27 (f_{i+1} - f_i) - (f_{i+2} - f_{i-1})) / (24 dx).
static const double LAG[4] = {-1.0 / 16.0, 9.0 / 16.0, 9.0 / 16.0, -1.0 / 16.0};

template <class T> T lag_deriv(const T f[4], double dx) {
  return (T(27) * (f[2] - f[1]) - (f[3] - f[0])) / T(24.0 * dx);
}
template <class T> T lag_value(const T f[4]) {
  return T(LAG[0]) * f[0] + T(LAG[1]) * f[1] + T(LAG[2]) * f[2] + T(LAG[3]) * f[3];
}

// Value and the three first derivatives of field f at cell centre (i,j,k).
template <class T> void centre_interp(const Grid& g, const T* f, int i, int j, int k, T& val, T der[3]) {
  // collapse z, then y, then x, keeping value and derivative lines
  T vz[4][4], dz[4][4];  // [b][a] after z
  for (int b = 0; b < 4; ++b)
    for (int a = 0; a < 4; ++a) {
      T col[4];
      for (int c = 0; c < 4; ++c) col[c] = f[at(g, i - 1 + a, j - 1 + b, k - 1 + c)];
      vz[b][a] = lag_value(col);
      dz[b][a] = lag_deriv(col, g.dx[2]);
    }
  T vy[4], dy[4], dzy[4];  // [a]
  for (int a = 0; a < 4; ++a) {
    T c1[4], c2[4];
    for (int b = 0; b < 4; ++b) { c1[b] = vz[b][a]; c2[b] = dz[b][a]; }
    vy[a] = lag_value(c1);
    dy[a] = lag_deriv(c1, g.dx[1]);
    dzy[a] = lag_value(c2);
  }
  val = lag_value(vy);
  der[0] = lag_deriv(vy, g.dx[0]);
  der[1] = lag_value(dy);
  der[2] = lag_value(dzy);
}

// Value only of field f at cell centre (i,j,k): the same z, y and x passes as
// centre_interp without the derivative lines (the recovery and prim -> cons need
// no metric derivatives), so the value is bitwise the same.
template <class T> T centre_value(const Grid& g, const T* f, int i, int j, int k) {
  T vy[4];
  for (int a = 0; a < 4; ++a) {
    T c1[4];
    for (int b = 0; b < 4; ++b) {
      T col[4];
      for (int c = 0; c < 4; ++c) col[c] = f[at(g, i - 1 + a, j - 1 + b, k - 1 + c)];
      c1[b] = lag_value(col);
    }
    vy[a] = lag_value(c1);
  }
  return lag_value(vy);
}

// Value of field f at the face of direction d with index (i,j,k): the face
// lies on vertex plane i (d = x) and midway in the two transverse directions.
template <class T> T face_interp(const Grid& g, const T* f, int d, int i, int j, int k) {
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  T rows[4];
  for (int b = 0; b < 4; ++b) {
    T col[4];
    for (int c = 0; c < 4; ++c) {
      int id[3] = {i, j, k};
      id[t1] += b - 1;
      id[t2] += c - 1;
      col[c] = f[at(g, id[0], id[1], id[2])];
    }
    rows[b] = lag_value(col);
  }
  return lag_value(rows);
}

// ---------------------------------------------------------------------------
// Magnetic field from the staggered vector potential (Sec. 2.3, B = curl A,
// and Sec. 3.1): the densitized face field is the coordinate curl of the edge
// potential,
//   Bx[i,j,k] = (Az[i,j+1,k]-Az[i,j,k])/dy - (Ay[i,j,k+1]-Ay[i,j,k])/dz
//   By[i,j,k] = (Ax[i,j,k+1]-Ax[i,j,k])/dz - (Az[i+1,j,k]-Az[i,j,k])/dx
//   Bz[i,j,k] = (Ay[i+1,j,k]-Ay[i,j,k])/dx - (Ax[i,j+1,k]-Ax[i,j,k])/dy
// (Levi-Civita symbol; the divergence of this face field vanishes identically).
template <class T> T face_B(const Grid& g, const T* A, int d, int i, int j, int k) {
  size_t N = npts(g);
  const T* Ax = A;
  const T* Ay = A + N;
  const T* Az = A + 2 * N;
  if (d == 0)
    return (Az[at(g, i, j + 1, k)] - Az[at(g, i, j, k)]) / T(g.dx[1]) -
           (Ay[at(g, i, j, k + 1)] - Ay[at(g, i, j, k)]) / T(g.dx[2]);
  if (d == 1)
    return (Ax[at(g, i, j, k + 1)] - Ax[at(g, i, j, k)]) / T(g.dx[2]) -
           (Az[at(g, i + 1, j, k)] - Az[at(g, i, j, k)]) / T(g.dx[0]);
  return (Ay[at(g, i + 1, j, k)] - Ay[at(g, i, j, k)]) / T(g.dx[0]) -
         (Ax[at(g, i, j + 1, k)] - Ax[at(g, i, j, k)]) / T(g.dx[1]);
}

// Centre field: linear interpolation of the two adjacent faces (Sec. 3.1).
template <class T> void centre_B(const Grid& g, const T* A, int i, int j, int k, T Bt[3]) {
  Bt[0] = (face_B(g, A, 0, i, j, k) + face_B(g, A, 0, i + 1, j, k)) / T(2);
  Bt[1] = (face_B(g, A, 1, i, j, k) + face_B(g, A, 1, i, j + 1, k)) / T(2);
  Bt[2] = (face_B(g, A, 2, i, j, k) + face_B(g, A, 2, i, j, k + 1)) / T(2);
}

template <class T> void centre_metric_values(const Grid& g, const T* metric, int i, int j, int k, T m[10]) {
  size_t N = npts(g);
  for (int c = 0; c < 10; ++c) m[c] = centre_value(g, metric + c * N, i, j, k);
}

template <class T> void centre_metric(const Grid& g, const T* metric, int i, int j, int k, T m[10], T dm[3][10]) {
  size_t N = npts(g);
  for (int c = 0; c < 10; ++c) {
    T der[3];
    centre_interp(g, metric + c * N, i, j, k, m[c], der);
    for (int d = 0; d < 3; ++d) dm[d][c] = der[d];
  }
}

// ---------------------------------------------------------------------------
// Conservative-to-primitive recovery (Sec. 3.5).
template <class T> struct C2PInput {
  T D, S[3], tau, B[3];  // undensitized; S covariant, B contravariant
  T S2, B2, BS;
};

template <class T> C2PInput<T> make_c2p_input(const Geom<T>& G, const T cons[5], const T Bt[3]) {
  C2PInput<T> c;
  c.D = cons[0] / G.sqrtg;
  for (int j = 0; j < 3; ++j) c.S[j] = cons[1 + j] / G.sqrtg;
  c.tau = cons[4] / G.sqrtg;
  for (int j = 0; j < 3; ++j) c.B[j] = Bt[j] / G.sqrtg;
  c.S2 = T(0);
  c.B2 = T(0);
  c.BS = T(0);
  for (int i = 0; i < 3; ++i) {
    c.BS = c.BS + c.B[i] * c.S[i];
    for (int j = 0; j < 3; ++j) {
      c.S2 = c.S2 + G.gi[i][j] * c.S[i] * c.S[j];
      c.B2 = c.B2 + G.g[i][j] * c.B[i] * c.B[j];
    }
  }
  return c;
}

// The two residuals of the Noble et al. 2D scheme in the unknowns z = rho h W^2
// and w = v^2 (eqs. Noble2D momentum and Noble2D energy), with the ideal-gas
// pressure written in (z, w): p = ((Gamma-1)/Gamma) (z (1-w) - D sqrt(1-w)).
template <class T> void noble_residual(const C2PInput<T>& c, const T& gam, const T& z, const T& w, T R[2], T J[2][2]) {
  T gm = (gam - T(1)) / gam;
  T sw = sqrt(T(1) - w);
  T p = gm * (z * (T(1) - w) - c.D * sw);
  T BS2 = c.BS * c.BS;
  T Bz = c.B2 + z;
  R[0] = w * Bz * Bz - BS2 * (c.B2 + T(2) * z) / (z * z) - c.S2;
  R[1] = c.tau + c.D - c.B2 * (T(1) + w) / T(2) + BS2 / (T(2) * z * z) - z + p;
  J[0][0] = T(2) * w * Bz + T(2) * BS2 * Bz / (z * z * z);
  J[0][1] = Bz * Bz;
  J[1][0] = -BS2 / (z * z * z) - T(1) + gm * (T(1) - w);
  J[1][1] = -c.B2 / T(2) + gm * (-z + c.D / (T(2) * sw));
}

// Primitive velocity from z (eq. Noble2D v):
// v^i = gamma^ij S_j/(z + B^2) + (B^j S_j) B^i/(z (z + B^2)).
template <class T> void velocity_from_z(const Geom<T>& G, const C2PInput<T>& c, const T& z, T v[3]) {
  for (int i = 0; i < 3; ++i) {
    T Su = T(0);
    for (int j = 0; j < 3; ++j) Su = Su + G.gi[i][j] * c.S[j];
    v[i] = Su / (z + c.B2) + c.BS * c.B[i] / (z * (z + c.B2));
  }
}

// Newton-Raphson on (z, w).  Returns true on convergence with the primitives.
template <class T> bool c2p_noble(const Geom<T>& G, const C2PInput<T>& c, const T& gam, const Params& P, T z, T w,
                                  T prim[5], int& iters) {
  T wcap = T(1) - T(1) / (T(P.wmax) * T(P.wmax));
  bool ok = false;
  iters = 0;
  for (int it = 1; it <= P.c2p_maxit; ++it) {
    iters = it;
    T R[2], J[2][2];
    noble_residual(c, gam, z, w, R, J);
    T det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    T dz = (-R[0] * J[1][1] + J[0][1] * R[1]) / det;
    T dw = (-J[0][0] * R[1] + J[1][0] * R[0]) / det;
    z = z + dz;
    w = w + dw;
    if (w < T(0)) w = T(0);
    if (w > wcap) w = wcap;
    if (!is_finite(z) || !is_finite(w) || !(z > T(0))) return false;
    T ez = fabs(dz) / fabs(z);
    T err = ez > fabs(dw) ? ez : fabs(dw);
    if (err < T(P.c2p_tol)) { ok = true; break; }
  }
  if (!ok) return false;
  // recovery in the order of the paper: W, rho, v^i, eps, p
  T W = T(1) / sqrt(T(1) - w);
  T rho = c.D / W;
  T v[3];
  velocity_from_z(G, c, z, v);
  T eps = (z / (rho * W * W) - T(1)) / gam;  // (eq. Noble2D epsilon; the 1/gamma there is 1/Gamma)
  T p = eos_p_from_eps(rho, eps, gam);
  if (!(eps >= T(0)) || !is_finite(p)) return false;
  prim[0] = rho;
  prim[1] = p;
  for (int i = 0; i < 3; ++i) prim[2 + i] = v[i];
  return true;
}

// Palenzuela et al. 1D scheme: q, r, s, t (eq. Palenzuela qrst) and the
// master function f(x) = x - h W (eq. Palenzuela Brent) for x = h W.
// 1/W^2 = 1 - (r x^2 + t^2 (2x + s)) / (x^2 (x + s)^2);  rho = D/W;
// eps = -1 + (x/W)(1 - W^2) + W [1 + q - s + (t^2/x^2 + s/W^2)/2]
// (the printed t^2/x is read as t^2/x^2: rederived from the energy equation
// with z = D x).
template <class T> struct Palen {
  T q, r, s, t, D;
};

template <class T> void palen_eval(const Palen<T>& P5, const T& x, const T& gam, double wmax, T& f, T& W, T& rho, T& eps,
                                   T& p) {
  T v2 = (P5.r * x * x + P5.t * P5.t * (T(2) * x + P5.s)) / (x * x * (x + P5.s) * (x + P5.s));
  T iW2 = T(1) - v2;
  T floor = T(1) / (T(wmax) * T(wmax));
  if (iW2 < floor) iW2 = floor;  // safety clamp (reading: keeps W finite inside the bracket)
  W = T(1) / sqrt(iW2);
  rho = P5.D / W;
  eps = T(-1) + (x / W) * (T(1) - W * W) + W * (T(1) + P5.q - P5.s + (P5.t * P5.t / (x * x) + P5.s * iW2) / T(2));
  p = eos_p_from_eps(rho, eps, gam);
  T h = T(1) + eps + p / rho;
  f = x - h * W;
}

// Brent's method (Brent 1973): keeps a bracket [b, c] with a sign change,
// takes inverse-quadratic or secant steps when they stay well inside the
// bracket and shrink fast enough, bisects otherwise.
template <class T> bool c2p_palenzuela(const Geom<T>& G, const C2PInput<T>& c, const T& gam, const Params& P,
                                       T prim[5]) {
  Palen<T> P5;
  P5.D = c.D;
  P5.q = c.tau / c.D;
  P5.r = c.S2 / (c.D * c.D);
  P5.s = c.B2 / c.D;
  P5.t = c.BS / pow(c.D, 1.5);
  T lo = T(1) + P5.q - P5.s;
  T hi = T(2) + T(2) * P5.q - P5.s;
  if (lo < T(1)) lo = T(1);  // x = h W >= 1 for any physical state
  if (!(hi > lo)) return false;
  T W, rho, eps, p;
  T a = lo, b = hi, fa, fb;
  palen_eval(P5, a, gam, P.wmax, fa, W, rho, eps, p);
  palen_eval(P5, b, gam, P.wmax, fb, W, rho, eps, p);
  if (!is_finite(fa) || !is_finite(fb)) return false;
  if ((fa > T(0) && fb > T(0)) || (fa < T(0) && fb < T(0))) return false;
  T cc = a, fc = fa, dstep = b - a, estep = dstep;
  bool conv = false;
  for (int it = 0; it < P.brent_maxit; ++it) {
    if ((fb > T(0) && fc > T(0)) || (fb < T(0) && fc < T(0))) {
      cc = a; fc = fa; dstep = b - a; estep = dstep;
    }
    if (fabs(fc) < fabs(fb)) {  // make b the best estimate
      a = b; fa = fb;
      b = cc; fb = fc;
      cc = a; fc = fa;
    }
    T tol = T(2.0 * DBL_EPSILON) * fabs(b);
    T m = (cc - b) / T(2);
    if (fabs(m) <= tol || fb == T(0)) { conv = true; break; }
    if (fabs(estep) >= tol && fabs(fa) > fabs(fb)) {
      T s = fb / fa, pp, qq;
      if (a == cc) {  // secant
        pp = T(2) * m * s;
        qq = T(1) - s;
      } else {  // inverse quadratic interpolation
        T qa = fa / fc, r = fb / fc;
        pp = s * (T(2) * m * qa * (qa - r) - (b - a) * (r - T(1)));
        qq = (qa - T(1)) * (r - T(1)) * (s - T(1));
      }
      if (pp > T(0)) qq = -qq; else pp = -pp;
      T lim1 = T(3) * m * qq - fabs(tol * qq);
      T lim2 = fabs(estep * qq);
      if (T(2) * pp < (lim1 < lim2 ? lim1 : lim2)) {
        estep = dstep;
        dstep = pp / qq;
      } else {
        dstep = m; estep = m;
      }
    } else {
      dstep = m; estep = m;
    }
    a = b; fa = fb;
    if (fabs(dstep) > tol) b = b + dstep;
    else b = b + (m > T(0) ? tol : -tol);
    palen_eval(P5, b, gam, P.wmax, fb, W, rho, eps, p);
    if (!is_finite(fb)) return false;
  }
  if (!conv) return false;
  T f;
  palen_eval(P5, b, gam, P.wmax, f, W, rho, eps, p);
  if (!(eps >= T(0)) || !is_finite(p)) return false;
  T z = c.D * b;  // z = rho h W^2 = D x
  T v[3];
  velocity_from_z(G, c, z, v);
  prim[0] = rho;
  prim[1] = p;
  for (int i = 0; i < 3; ++i) prim[2 + i] = v[i];
  return true;
}

// Atmosphere (Sec. 3.6): rho = rho_atm, p and eps from the polytrope, v = 0,
// conserved variables recomputed from these primitives, field kept.
template <class T> void atmosphere(const Geom<T>& G, const T Bt[3], const T& gam, const Params& P, T prim[5], T cons[5]) {
  prim[0] = T(P.rho_atm);
  prim[1] = polytrope_p(T(P.rho_atm), P.k_atm, gam);
  prim[2] = prim[3] = prim[4] = T(0);
  Fluid<T> F = make_fluid(G, prim, Bt, gam);
  prim2con_point(G, F, cons);
}

// Warm start from the previous primitives: z0 = rho h W^2, w0 = v^2.  When the
// previous state is unusable, a cold start z0 = tau + D (+ B^2-free), w0 from
// S^2 / (z0 + B^2)^2 is used.
template <class T> void c2p_guess(const Geom<T>& G, const C2PInput<T>& c, const T prev[5], const T& gam, const Params& P,
                                  T& z0, T& w0) {
  T wcap = T(1) - T(1) / (T(P.wmax) * T(P.wmax));
  T v2 = T(0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) v2 = v2 + G.g[i][j] * prev[2 + i] * prev[2 + j];
  bool good = prev[0] > T(0) && prev[1] >= T(0) && v2 < wcap && is_finite(v2) && is_finite(prev[1]);
  if (good) {
    T eps = eos_eps_from_p(prev[0], prev[1], gam);
    T h = T(1) + eps + prev[1] / prev[0];
    z0 = prev[0] * h / (T(1) - v2);
    w0 = v2;
  } else {
    z0 = c.tau + c.D;
    T den = z0 + c.B2;
    w0 = c.S2 / (den * den);
    if (w0 > wcap) w0 = wcap;
  }
}

// Full point recovery: Noble -> Palenzuela -> atmosphere.
// cons (densitized) is updated in place when the atmosphere is applied.
template <class T> uint8_t c2p_point(const Geom<T>& G, T cons[5], const T Bt[3], const T prev[5], const T& gam,
                                     const Params& P, T prim[5], int& iters) {
  uint8_t fl = 0;
  iters = 0;
  bool nan_in = false;
  for (int c = 0; c < 5; ++c)
    if (!is_finite(cons[c])) nan_in = true;
  if (nan_in || !(cons[0] >= G.sqrtg * T(P.rho_atm))) {
    if (nan_in) fl |= FL_NAN_IN;
    fl |= FL_ATMO;
    atmosphere(G, Bt, gam, P, prim, cons);
    return fl;
  }
  C2PInput<T> c = make_c2p_input(G, cons, Bt);
  // Without a field and with Gamma <= 2, every physical state of the ideal gas has tau > 0 and
  // E^2 > S^2 + D^2, i.e. S^2 < tau (tau + 2D) (E^2 - S^2 - D^2 = W^2 rho^2 (2 eps + eps^2 (1 - (Gamma-1)^2))
  // + p^2).  A state beyond that bound by more than a relative 1e-10 has no solution for either solver to
  // find; it takes the failure branch with the flags the two failed solvers set (Sec. 3.6).
  if (c.B2 <= T(0) && gam <= T(2) &&
      (!(c.tau > T(0)) || c.S2 > T(1.0 + 1e-10) * c.tau * (c.tau + T(2) * c.D))) {
    if (P.c2p_method != 2) fl |= FL_NOBLE_FAIL;
    fl |= FL_HARD_FAIL | FL_ATMO;
    atmosphere(G, Bt, gam, P, prim, cons);
    return fl;
  }
  bool ok = false;
  if (P.c2p_method != 2) {
    T z0, w0;
    c2p_guess(G, c, prev, gam, P, z0, w0);
    ok = c2p_noble(G, c, gam, P, z0, w0, prim, iters);
    if (!ok) fl |= FL_NOBLE_FAIL;
  }
  if (!ok && P.c2p_method != 1) {
    ok = c2p_palenzuela(G, c, gam, P, prim);
    if (ok && P.c2p_method == 0) fl |= FL_FALLBACK;
  }
  if (!ok) {
    fl |= FL_HARD_FAIL | FL_ATMO;
    atmosphere(G, Bt, gam, P, prim, cons);
    return fl;
  }
  if (prim[0] < T(P.rho_atm)) {
    fl |= FL_ATMO;
    atmosphere(G, Bt, gam, P, prim, cons);
  }
  return fl;
}

// ---------------------------------------------------------------------------
// Energy-momentum tensor (eq. tmunu) and the geometric sources (eq. grmhdsrc).
template <class T> void stress_tensor(const Geom<T>& G, const Fluid<T>& F, T Tu[4][4]) {
  T gu[4][4];
  inverse_4metric(G, gu);
  T uu[4] = {F.u0, F.u[0], F.u[1], F.u[2]};
  T bu[4] = {F.b0, F.b[0], F.b[1], F.b[2]};
  T e = F.rho * F.h + F.bsq;
  T ptot = F.p + F.bsq / T(2);
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) Tu[m][n] = e * uu[m] * uu[n] + ptot * gu[m][n] - bu[m] * bu[n];
}

// Densitized sources alpha sqrt(gamma) S (eq. fluxconseqs).
//  S_j: T^{mu nu}(d_mu g_{nu j} - Gamma^delta_{nu mu} g_{delta j}) = 1/2 T^{mu nu} d_j g_{mu nu}
//       (identity for a symmetric T); the spatial derivatives of g_{mu nu}
//       follow from g_00 = -alpha^2 + beta_k beta^k, g_0k = beta_k, g_kl = gamma_kl.
//  tau: alpha (T^{mu 0} d_mu ln alpha - T^{mu nu} Gamma^0_{nu mu}) in its 3+1 form
//       T^00 (beta^k beta^l K_kl - beta^k d_k alpha) + T^0k (2 beta^l K_kl - d_k alpha) + T^kl K_kl.
// dm[j][c]: d_j of metric component c; K: Kxx, Kxy, Kxz, Kyy, Kyz, Kzz.
template <class T> void sources_point(const Geom<T>& G, const T dm[3][10], const T K6[6], const Fluid<T>& F, T src[5]) {
  T Tu[4][4];
  stress_tensor(G, F, Tu);
  T K[3][3];
  K[0][0] = K6[0]; K[0][1] = K[1][0] = K6[1]; K[0][2] = K[2][0] = K6[2];
  K[1][1] = K6[3]; K[1][2] = K[2][1] = K6[4]; K[2][2] = K6[5];
  const int gidx[3][3] = {{4, 5, 6}, {5, 7, 8}, {6, 8, 9}};
  src[0] = T(0);
  for (int j = 0; j < 3; ++j) {
    // d_j g_{mu nu}
    T dg[4][4];
    T dal = dm[j][0];
    T dbeta[3] = {dm[j][1], dm[j][2], dm[j][3]};
    T dgam[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) dgam[a][b] = dm[j][gidx[a][b]];
    T d00 = T(-2) * G.alp * dal;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        d00 = d00 + dgam[a][b] * G.beta[a] * G.beta[b] + T(2) * G.g[a][b] * G.beta[a] * dbeta[b];
    dg[0][0] = d00;
    for (int a = 0; a < 3; ++a) {
      T d0a = T(0);
      for (int b = 0; b < 3; ++b) d0a = d0a + dgam[a][b] * G.beta[b] + G.g[a][b] * dbeta[b];
      dg[0][a + 1] = d0a;
      dg[a + 1][0] = d0a;
      for (int b = 0; b < 3; ++b) dg[a + 1][b + 1] = dgam[a][b];
    }
    T s = T(0);
    for (int m = 0; m < 4; ++m)
      for (int n = 0; n < 4; ++n) s = s + Tu[m][n] * dg[m][n];
    src[1 + j] = G.alp * G.sqrtg * s / T(2);
  }
  T dal[3] = {dm[0][0], dm[1][0], dm[2][0]};
  T e = T(0);
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) e = e + Tu[0][0] * G.beta[k] * G.beta[l] * K[k][l];
  for (int k = 0; k < 3; ++k) e = e - Tu[0][0] * G.beta[k] * dal[k];
  for (int k = 0; k < 3; ++k) {
    T t = T(0);
    for (int l = 0; l < 3; ++l) t = t + T(2) * G.beta[l] * K[k][l];
    e = e + Tu[0][k + 1] * (t - dal[k]);
  }
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) e = e + Tu[k + 1][l + 1] * K[k][l];
  src[4] = G.alp * G.sqrtg * e;
}

// ---------------------------------------------------------------------------
// Grid operations.

template <class T> static inline T load_metric_point(const Grid& g, const T* metric, int i, int j, int k, T m[10]) {
  size_t N = npts(g);
  for (int c = 0; c < 10; ++c) m[c] = metric[c * N + at(g, i, j, k)];
  return m[0];
}

// Covariant stress-energy tensor T_{mu nu} at vertices (Sec. 3.1: it lives at the vertices with the
// spacetime variables, for the spacetime solver; eq. tmunu for T^{mu nu}), on every vertex of the block,
// indices [0, n] per axis.  The vertex fluid state is the arithmetic mean of the primitives and of the
// centre fields of the 8 cells sharing the vertex (the paper does not say how the cell data reach the
// vertex); the metric is the vertex's own.  T_{mu nu} = g_{mu a} g_{nu b} T^{ab} with g_00 = -alpha^2 +
// beta_k beta^k, g_0i = beta_i, g_ij = gamma_ij.  out: 10 fields T_00, T_0x, T_0y, T_0z, T_xx, T_xy,
// T_xz, T_yy, T_yz, T_zz.
template <class T> void tmunu_vertices(const Grid& g, const T& gam, const T* metric, const T* prim, const T* A,
                                       T* out) {
  size_t N = npts(g);
  for (int k = 0; k <= g.n[2]; ++k)
    for (int j = 0; j <= g.n[1]; ++j)
      for (int i = 0; i <= g.n[0]; ++i) {
        T pr[5], Bt[3];
        for (int c = 0; c < 5; ++c) pr[c] = T(0);
        for (int c = 0; c < 3; ++c) Bt[c] = T(0);
        for (int dk = -1; dk <= 0; ++dk)
          for (int dj = -1; dj <= 0; ++dj)
            for (int di = -1; di <= 0; ++di) {
              for (int c = 0; c < 5; ++c) pr[c] = pr[c] + prim[c * N + at(g, i + di, j + dj, k + dk)];
              T b[3];
              centre_B(g, A, i + di, j + dj, k + dk, b);
              for (int c = 0; c < 3; ++c) Bt[c] = Bt[c] + b[c];
            }
        for (int c = 0; c < 5; ++c) pr[c] = pr[c] / T(8);
        for (int c = 0; c < 3; ++c) Bt[c] = Bt[c] / T(8);
        T m[10];
        load_metric_point(g, metric, i, j, k, m);
        Geom<T> G = make_geom(m);
        Fluid<T> F = make_fluid(G, pr, Bt, gam);
        T Tu[4][4];
        stress_tensor(G, F, Tu);
        T g4[4][4];
        T bb = T(0);
        for (int a = 0; a < 3; ++a) bb = bb + G.beta[a] * G.betal[a];
        g4[0][0] = -G.alp * G.alp + bb;
        for (int a = 0; a < 3; ++a) {
          g4[0][a + 1] = g4[a + 1][0] = G.betal[a];
          for (int b = 0; b < 3; ++b) g4[a + 1][b + 1] = G.g[a][b];
        }
        const int idx[10][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 1}, {1, 2}, {1, 3}, {2, 2}, {2, 3}, {3, 3}};
        for (int c = 0; c < 10; ++c) {
          int mu = idx[c][0], nu = idx[c][1];
          T s = T(0);
          for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) s = s + g4[mu][a] * g4[nu][b] * Tu[a][b];
          out[c * N + at(g, i, j, k)] = s;
        }
      }
}

// Initial prim -> cons on owned cells (Sec. 3.12: analytical expressions
// initialise the conserved variables).
template <class T> void prim2con_grid(const Grid& g, const Params& /*P*/, const T& gam, const T* metric, const T* A,
                                      const T* prim, T* cons) {
  size_t N = npts(g);
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        T m[10];
        centre_metric_values(g, metric, i, j, k, m);
        Geom<T> G = make_geom(m);
        T Bt[3];
        centre_B(g, A, i, j, k, Bt);
        size_t id = at(g, i, j, k);
        T pr[5];
        for (int c = 0; c < 5; ++c) pr[c] = prim[c * N + id];
        Fluid<T> F = make_fluid(G, pr, Bt, gam);
        T cs[5];
        prim2con_point(G, F, cs);
        for (int c = 0; c < 5; ++c) cons[c * N + id] = cs[c];
      }
}

// c2p on owned cells.  prim holds the previous primitives on entry (warm
// start) and the recovered ones on exit; cons is reset where the atmosphere
// applies.  stats (6 counters) accumulates.
template <class T> void c2p_grid(const Grid& g, const Params& P, const T& gam, const T* metric, const T* A, T* cons,
                                 T* prim, uint8_t* flags, unsigned long long* stats) {
  size_t N = npts(g);
  unsigned long long n_noble = 0, n_fallback = 0, n_atmo = 0, n_hard = 0, n_nan = 0, it_max = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_noble, n_fallback, n_atmo, n_hard, n_nan) \
    reduction(max : it_max)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        T m[10];
        centre_metric_values(g, metric, i, j, k, m);
        Geom<T> G = make_geom(m);
        T Bt[3];
        centre_B(g, A, i, j, k, Bt);
        size_t id = at(g, i, j, k);
        T cs[5], prev[5], pr[5];
        for (int c = 0; c < 5; ++c) {
          cs[c] = cons[c * N + id];
          prev[c] = prim[c * N + id];
        }
        int iters = 0;
        uint8_t fl = c2p_point(G, cs, Bt, prev, gam, P, pr, iters);
        for (int c = 0; c < 5; ++c) {
          prim[c * N + id] = pr[c];
          cons[c * N + id] = cs[c];
        }
        if (flags) flags[id] = fl;
        if (fl & FL_NOBLE_FAIL) n_noble++;
        if (fl & FL_FALLBACK) n_fallback++;
        if (fl & FL_ATMO) n_atmo++;
        if (fl & FL_HARD_FAIL) n_hard++;
        if (fl & FL_NAN_IN) n_nan++;
        if ((unsigned long long)iters > it_max) it_max = (unsigned long long)iters;
      }
  if (stats) {
    stats[ST_NOBLE_FAIL] += n_noble;
    stats[ST_FALLBACK] += n_fallback;
    stats[ST_ATMO] += n_atmo;
    stats[ST_HARD_FAIL] += n_hard;
    stats[ST_NAN_IN] += n_nan;
    if (it_max > stats[ST_ITERS_MAX]) stats[ST_ITERS_MAX] = it_max;
  }
}

// Ghost fill of nf fields, axis by axis over the full extent of the other
// axes (so edges and corners are filled).  kind per axis.
template <class T> void fill_ghosts(const Grid& g, T* f, int nf, const int kinds[3], const double* shift = nullptr) {
  size_t N = npts(g);
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) { lo[d] = -g.ng; hi[d] = g.n[d] + g.ng; }
  for (int d = 0; d < 3; ++d) {
    int n = g.n[d];
    for (int q = 0; q < nf; ++q) {
      T* F = f + q * N;
      int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
      for (int b = lo[e2]; b <= hi[e2]; ++b)
        for (int a = lo[e1]; a <= hi[e1]; ++a)
          for (int s = lo[d]; s <= hi[d]; ++s) {
            if (s >= 0 && s < n) continue;
            int id[3], src0[3], src1[3];
            id[d] = s; id[e1] = a; id[e2] = b;
            for (int t = 0; t < 3; ++t) { src0[t] = id[t]; src1[t] = id[t]; }
            T val;
            if (kinds[d] == BC_PERIODIC) {
              src0[d] = ((s % n) + n) % n;  // periodic image (also for blocks thinner than the ghost width)
              val = F[at(g, src0[0], src0[1], src0[2])];
              // a potential of a field with a uniform mean changes by a constant per period
              if (shift && q < 3) val = val + T(shift[q * 3 + d] * (double)((s - src0[d]) / n));
            } else if (kinds[d] == BC_COPY) {
              src0[d] = s < 0 ? 0 : n - 1;
              val = F[at(g, src0[0], src0[1], src0[2])];
            } else {
              // linear extrapolation from the two nearest owned points
              if (s < 0) {
                src0[d] = 0; src1[d] = 1;
                T f0 = F[at(g, src0[0], src0[1], src0[2])], f1 = F[at(g, src1[0], src1[1], src1[2])];
                val = f0 + T(s) * (f1 - f0);
              } else {
                src0[d] = n - 1; src1[d] = n - 2;
                T f0 = F[at(g, src0[0], src0[1], src0[2])], f1 = F[at(g, src1[0], src1[1], src1[2])];
                val = f0 + T(s - n + 1) * (f0 - f1);
              }
            }
            F[at(g, id[0], id[1], id[2])] = val;
          }
    }
  }
}

// Reconstructed left/right primitive states (rho, p, v^x, v^y, v^z, Bt^{t1},
// Bt^{t2}) at the face of direction d with index (i,j,k).  A side whose
// reconstructed state is unphysical (rho <= 0, p <= 0 or v^2 >= 1 at the face
// metric) falls back to the adjacent cell's own values.
template <class T> int face_states(const Grid& g, const Params& P, const T* prim, const T* Bc, const Geom<T>& Gf, int d,
                                   int i, int j, int k, T L[7], T R[7]) {
  size_t N = npts(g);
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  T cellL[7], cellR[7];
  for (int v = 0; v < 7; ++v) {
    const T* f = (v < 5) ? prim + v * N : (v == 5 ? Bc + t1 * N : Bc + t2 * N);
    T a[6];
    for (int s = 0; s < 6; ++s) {
      int id[3] = {i, j, k};
      id[d] += s - 3;
      a[s] = f[at(g, id[0], id[1], id[2])];
    }
    reconstruct_face(P.recon, a, L[v], R[v], P);
    cellL[v] = a[2];
    cellR[v] = a[3];
  }
  int nfix = 0;
  for (int side = 0; side < 2; ++side) {
    T* X = side == 0 ? L : R;
    T* C = side == 0 ? cellL : cellR;
    T v2 = T(0);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) v2 = v2 + Gf.g[a][b] * X[2 + a] * X[2 + b];
    if (!(X[0] > T(0)) || !(X[1] > T(0)) || !(v2 < T(1))) {
      for (int v = 0; v < 7; ++v) X[v] = C[v];
      ++nfix;
    }
  }
  return nfix;
}

// Right-hand side on owned points (Sec. 3.12 workflow, steps 2-4, and Sec. 3.4).
// rhs: 9 fields Dt, St_x, St_y, St_z, taut, A_x, A_y, A_z, Psi.
// red[0] = max characteristic speed over faces of owned cells,
// red[1] = max |div Btilde| over owned cells.
template <class T> void rhs_grid(const Grid& g, const Params& P, const T& gam, const T* metric, const T* curv,
                                 const T* prim, const T* A, const T* psi, double dt_max, T* rhs, double* red,
                                 long long* nfix_out) {
  size_t N = npts(g);
  phase_mark<T>(-1);
  // centre field everywhere it can be formed
  std::vector<T> Bc(3 * N, T(0));
#pragma omp parallel for schedule(static)
  for (int k = -g.ng; k < g.n[2] + g.ng; ++k)
    for (int j = -g.ng; j < g.n[1] + g.ng; ++j)
      for (int i = -g.ng; i < g.n[0] + g.ng; ++i) {
        T b[3];
        centre_B(g, A, i, j, k, b);
        for (int c = 0; c < 3; ++c) Bc[c * N + at(g, i, j, k)] = b[c];
      }
  phase_mark<T>(0);
  // face fluxes: 3 directions x 7 components.  Upwind CT also keeps, per face, the upwind
  // transverse velocities (eq. uct1) and the two speeds a_+ = c_max, a_- = c_min (eq. uct2), on
  // the faces its PPM reconstruction to the edges reaches: transverse indices [-3, n+1].
  const bool uct = P.ct == CT_UCT;
  const int tlo = uct ? -3 : -1, thi_ext = uct ? 1 : -1;
  std::vector<T> flux(21 * N, T(0));
  std::vector<T> vbar(uct ? 9 * N : 0, T(0));  // [d][component]: transverse ones set
  std::vector<T> apm(uct ? 6 * N : 0, T(0));   // [d][+/-]
  double vmax = 0.0;
  long long nfix = 0;
  for (int d = 0; d < 3; ++d) {
    int lo[3] = {tlo, tlo, tlo}, hi[3] = {g.n[0] + thi_ext, g.n[1] + thi_ext, g.n[2] + thi_ext};
    lo[d] = 0;
    hi[d] = g.n[d];
#pragma omp parallel for schedule(static) reduction(+ : nfix) reduction(max : vmax)
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          T m[10];
          for (int c = 0; c < 10; ++c) m[c] = face_interp(g, metric + c * N, d, i, j, k);
          Geom<T> G = make_geom(m);
          T L[7], R[7];
          nfix += face_states(g, P, prim, Bc.data(), G, d, i, j, k, L, R);
          T BtL[3], BtR[3];
          int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
          T Bn = face_B(g, A, d, i, j, k);
          BtL[d] = Bn; BtL[t1] = L[5]; BtL[t2] = L[6];
          BtR[d] = Bn; BtR[t1] = R[5]; BtR[t2] = R[6];
          Fluid<T> FLd = make_fluid(G, L, BtL, gam);
          Fluid<T> FRd = make_fluid(G, R, BtR, gam);
          T UL[7], FL[7], UR[7], FR[7], cmL, cpL, cmR, cpR;
          flux_point(G, FLd, d, UL, FL);
          flux_point(G, FRd, d, UR, FR);
          speeds_point(G, FLd, d, gam, P.speeds, cmL, cpL);
          speeds_point(G, FRd, d, gam, P.speeds, cmR, cpR);
          T Fo[7], cmax, cmin;
          riemann_flux(P.riemann, UL, FL, cmL, cpL, UR, FR, cmR, cpR, Fo, cmax, cmin);
          for (int c = 0; c < 7; ++c) flux[(d * 7 + c) * N + at(g, i, j, k)] = Fo[c];
          if (uct) {
            // transport velocities vt^j = alpha v^j - beta^j of both sides, upwinded (eq. uct1)
            for (int t : {t1, t2}) {
              T vL = G.alp * L[2 + t] - G.beta[t], vR = G.alp * R[2 + t] - G.beta[t];
              T den = cmax + cmin;
              vbar[(d * 3 + t) * N + at(g, i, j, k)] =
                  den > T(0) ? (cmax * vL + cmin * vR) / den : (vL + vR) / T(2);
            }
            apm[(d * 2 + 0) * N + at(g, i, j, k)] = cmax;
            apm[(d * 2 + 1) * N + at(g, i, j, k)] = cmin;
          }
          bool owned = true;
          int id[3] = {i, j, k};
          for (int t = 0; t < 3; ++t)
            if (t != d && (id[t] < 0 || id[t] >= g.n[t])) owned = false;
          if (owned) {
            double s = std::max(value_of(cmax), value_of(cmin));
            if (s > vmax) vmax = s;
          }
        }
  }
  phase_mark<T>(1);
  // hydro: flux divergence (eq. fluxconseqs) plus sources, owned cells
  const size_t CURV = 6;
  double divmax = 0.0;
#pragma omp parallel for schedule(static) reduction(max : divmax)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        size_t id = at(g, i, j, k);
        size_t nb[3] = {at(g, i + 1, j, k), at(g, i, j + 1, k), at(g, i, j, k + 1)};
        T m[10], dm[3][10], K6[CURV];
        centre_metric(g, metric, i, j, k, m, dm);
        for (int c = 0; c < 6; ++c) K6[c] = centre_value(g, curv + c * N, i, j, k);
        Geom<T> G = make_geom(m);
        T pr[5], Bt[3];
        for (int c = 0; c < 5; ++c) pr[c] = prim[c * N + id];
        for (int c = 0; c < 3; ++c) Bt[c] = Bc[c * N + id];
        Fluid<T> F = make_fluid(G, pr, Bt, gam);
        T src[5];
        sources_point(G, dm, K6, F, src);
        for (int c = 0; c < 5; ++c) {
          T div = T(0);
          for (int d = 0; d < 3; ++d)
            div = div + (flux[(d * 7 + c) * N + nb[d]] - flux[(d * 7 + c) * N + id]) / T(g.dx[d]);
          rhs[c * N + id] = -div + src[c];
        }
        // discrete divergence of the face field (Sec. 2.2, divergence-free condition)
        T dB = (face_B(g, A, 0, i + 1, j, k) - face_B(g, A, 0, i, j, k)) / T(g.dx[0]) +
               (face_B(g, A, 1, i, j + 1, k) - face_B(g, A, 1, i, j, k)) / T(g.dx[1]) +
               (face_B(g, A, 2, i, j, k + 1) - face_B(g, A, 2, i, j, k)) / T(g.dx[2]);
        double adb = std::fabs(value_of(dB));
        if (adb > divmax) divmax = adb;
      }
  phase_mark<T>(2);
  // electric field on edges by flux-CT (Sec. 3.4, FCT): each component is the
  // average of the four induction fluxes on the faces that share the edge.
  // Induction flux slots: direction d stores (B^{(d+1)%3}, B^{(d+2)%3}) in
  // components 5 and 6.  With E = -vt x Btilde:
  //   E_z = -F^x_{By} = +F^y_{Bx}; E_x = -F^y_{Bz} = +F^z_{By}; E_y = -F^z_{Bx} = +F^x_{Bz}.
  auto FX = [&](int d, int comp, int i, int j, int k) -> T {
    int slot = ((comp - d + 3) % 3 == 1) ? 5 : 6;
    return flux[(d * 7 + slot) * N + at(g, i, j, k)];
  };
  const T* Ax = A;
  const T* Ay = A + N;
  const T* Az = A + 2 * N;
  // G_A = alpha Psi / sqrt(gamma) - beta^j A_j at vertices (A averaged to the
  // vertex along its own direction), and F_Psi^j = alpha sqrt(gamma) gamma^jk A_k - beta^j Psi.
  std::vector<T> GA(N, T(0)), FP(3 * N, T(0));
#pragma omp parallel for schedule(static)
  for (int k = -1; k <= g.n[2]; ++k)
    for (int j = -1; j <= g.n[1]; ++j)
      for (int i = -1; i <= g.n[0]; ++i) {
        T m[10];
        load_metric_point(g, metric, i, j, k, m);
        Geom<T> G = make_geom(m);
        T Av[3];
        Av[0] = (Ax[at(g, i - 1, j, k)] + Ax[at(g, i, j, k)]) / T(2);
        Av[1] = (Ay[at(g, i, j - 1, k)] + Ay[at(g, i, j, k)]) / T(2);
        Av[2] = (Az[at(g, i, j, k - 1)] + Az[at(g, i, j, k)]) / T(2);
        T ps = psi[at(g, i, j, k)];
        T bA = G.beta[0] * Av[0] + G.beta[1] * Av[1] + G.beta[2] * Av[2];
        GA[at(g, i, j, k)] = G.alp * ps / G.sqrtg - bA;
        for (int a = 0; a < 3; ++a) {
          T Au = G.gi[a][0] * Av[0] + G.gi[a][1] * Av[1] + G.gi[a][2] * Av[2];
          FP[a * N + at(g, i, j, k)] = G.alp * G.sqrtg * Au - G.beta[a] * ps;
        }
      }
  // Upwind CT (Sec. 3.4, eq. eq3.20): E_c on the c-edge owned by point p, with a = c+1, b = c+2
  // (cyclic).  The a-directed term takes the b-faces in the row through the edge along a: their
  // upwind velocity component a and their normal field B^b, PPM-reconstructed to the edge from
  // either side (L: right face of the element below the edge, R: left face of the element above),
  // with the speeds of the two a-faces that meet at the edge (the larger of each); the b-directed
  // term likewise with a and b exchanged.  E_c = -(a term) + (b term); for c = z this is eq3.20.
  auto uct_term = [&](int dir, int fd, const int p[3], int sdir) -> T {
    // dir: direction of the 1-D Riemann problem at the edge; fd: normal of the faces sampled along
    // dir; sdir: the direction separating the two dir-faces that meet at the edge
    T v6[6], b6[6];
    for (int s = 0; s < 6; ++s) {
      int q[3] = {p[0], p[1], p[2]};
      q[dir] += s - 3;
      v6[s] = vbar[(fd * 3 + dir) * N + at(g, q[0], q[1], q[2])];
      b6[s] = face_B(g, A, fd, q[0], q[1], q[2]);
    }
    T vL, vR, bL, bR;
    reconstruct_face(REC_PPM, v6, vL, vR, P);
    reconstruct_face(REC_PPM, b6, bL, bR, P);
    int q[3] = {p[0], p[1], p[2]};
    q[sdir] -= 1;
    T ap0 = apm[(dir * 2 + 0) * N + at(g, p[0], p[1], p[2])], ap1 = apm[(dir * 2 + 0) * N + at(g, q[0], q[1], q[2])];
    T am0 = apm[(dir * 2 + 1) * N + at(g, p[0], p[1], p[2])], am1 = apm[(dir * 2 + 1) * N + at(g, q[0], q[1], q[2])];
    T ap = ap0 > ap1 ? ap0 : ap1, am = am0 > am1 ? am0 : am1;
    T den = ap + am;
    if (!(den > T(0))) return (vL * bL + vR * bR) / T(2);
    return (ap * vL * bL + am * vR * bR - ap * am * (bR - bL)) / den;
  };
  double xi = P.xi / dt_max;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        size_t id = at(g, i, j, k);
        T E[3];
        if (uct) {
          const int p[3] = {i, j, k};
          for (int c = 0; c < 3; ++c) {
            int a = (c + 1) % 3, b = (c + 2) % 3;
            E[c] = -uct_term(a, b, p, b) + uct_term(b, a, p, a);
          }
        } else {
          E[2] = (-FX(0, 1, i, j, k) - FX(0, 1, i, j - 1, k) + FX(1, 0, i, j, k) + FX(1, 0, i - 1, j, k)) / T(4);
          E[0] = (-FX(1, 2, i, j, k) - FX(1, 2, i, j, k - 1) + FX(2, 1, i, j, k) + FX(2, 1, i, j - 1, k)) / T(4);
          E[1] = (-FX(2, 0, i, j, k) - FX(2, 0, i - 1, j, k) + FX(0, 2, i, j, k) + FX(0, 2, i, j, k - 1)) / T(4);
        }
        size_t nb[3] = {at(g, i + 1, j, k), at(g, i, j + 1, k), at(g, i, j, k + 1)};
        for (int a = 0; a < 3; ++a) {
          T r = -E[a];
          if (P.gauge == GAUGE_LORENZ) r = r - (GA[nb[a]] - GA[id]) / T(g.dx[a]);
          rhs[(5 + a) * N + id] = r;
        }
        if (P.gauge == GAUGE_LORENZ) {
          T m[10];
          load_metric_point(g, metric, i, j, k, m);
          size_t dn[3] = {at(g, i - 1, j, k), at(g, i, j - 1, k), at(g, i, j, k - 1)};
          T div = T(0);
          for (int a = 0; a < 3; ++a) div = div + (FP[a * N + nb[a]] - FP[a * N + dn[a]]) / T(2.0 * g.dx[a]);
          rhs[8 * N + id] = -div - T(xi) * m[0] * psi[id];
        } else {
          rhs[8 * N + id] = T(0);
        }
      }
  phase_mark<T>(3);
  if (red) {
    red[0] = vmax;
    red[1] = divmax;
  }
  if (nfix_out) *nfix_out = nfix;
}

// ---------------------------------------------------------------------------
// Inter-level operators for factor-2 mesh refinement (Sec. 3.9, the prolongation used at refinement
// boundaries in the AMR tests of Sec. 4).  The fine grid's vertex 0 sits on coarse vertex c0 (per
// axis), so fine spacing is half the coarse one.  Each axis of a field is cell- or vertex-centred
// (cell fields: all cell; vertex fields: all vertex; the x-edge potential: cell in x, vertex in y, z).
//   Prolongation, per axis: a vertex-centred direction injects where a fine vertex sits on a coarse
//   one and takes the cubic Lagrange midpoint value (-1, 9, 9, -1)/16 in between; a cell-centred
//   direction gives the two children of coarse cell c the conservative quadratic values
//   u_c -+ (u_{c+1} - u_{c-1})/8 (lower child -, upper child +), whose mean is u_c.  Applied as a
//   tensor product.  Fields centred in all three directions fall back, per coarse cell, to the
//   minmod-limited linear children u_c + sum_a (+-1/4) minmod(u_{c+e_a} - u_c, u_c - u_{c-e_a})
//   when any of the 8 third-order children leaves [min, max] of the 27 coarse cells around c (the
//   shock fallback; one decision per coarse cell keeps the children's mean equal to u_c).
//   Restriction, per axis: the mean of the two children in a cell-centred direction, injection in
//   a vertex-centred one (tensor product).
static inline int floordiv2(int f) { return f >= 0 ? f / 2 : -((1 - f) / 2); }

// 1-D prolongation stencil of fine index f: coarse indices c[0..n-1] and weights w[0..n-1].
static int prolong_stencil(int f, int c0, int vertex, int c[4], double w[4]) {
  if (vertex) {
    if (f % 2 == 0) {
      c[0] = c0 + f / 2;
      w[0] = 1.0;
      return 1;
    }
    int b = c0 + floordiv2(f);
    for (int q = 0; q < 4; ++q) c[q] = b - 1 + q;
    w[0] = -1.0 / 16.0; w[1] = 9.0 / 16.0; w[2] = 9.0 / 16.0; w[3] = -1.0 / 16.0;
    return 4;
  }
  int cc = c0 + floordiv2(f);
  int child = f - 2 * floordiv2(f);  // 0 lower, 1 upper
  c[0] = cc - 1; c[1] = cc; c[2] = cc + 1;
  w[0] = child ? -1.0 / 8.0 : 1.0 / 8.0;
  w[1] = 1.0;
  w[2] = child ? 1.0 / 8.0 : -1.0 / 8.0;
  return 3;
}

static double prolong_point(const Grid& gc, const double* cf, const int c0[3], const int stag[3], int fi, int fj,
                            int fk) {
  int ci[3][4], n[3];
  double w[3][4];
  int f[3] = {fi, fj, fk};
  for (int a = 0; a < 3; ++a) n[a] = prolong_stencil(f[a], c0[a], stag[a], ci[a], w[a]);
  double s = 0.0;
  for (int r = 0; r < n[2]; ++r)
    for (int q = 0; q < n[1]; ++q)
      for (int p = 0; p < n[0]; ++p) s += w[0][p] * w[1][q] * w[2][r] * cf[at(gc, ci[0][p], ci[1][q], ci[2][r])];
  return s;
}

template <class T> static T minmod_s(const T& x, const T& y) { return minmod2(x, y); }

void prolong_grid(const Grid& gc, const Grid& gf, const int c0[3], const int stag[3], int nf, const double* cf,
                  double* ff, const int lo[3], const int hi[3]) {
  size_t Nc = npts(gc), Nf = npts(gf);
  const bool allcell = !stag[0] && !stag[1] && !stag[2];
  for (int q = 0; q < nf; ++q) {
    const double* c = cf + q * Nc;
    double* o = ff + q * Nf;
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          double v = prolong_point(gc, c, c0, stag, i, j, k);
          if (allcell) {
            // the coarse cell of (i, j, k) and its 8 children's third-order values
            int cc[3] = {c0[0] + floordiv2(i), c0[1] + floordiv2(j), c0[2] + floordiv2(k)};
            int f0[3] = {2 * floordiv2(i), 2 * floordiv2(j), 2 * floordiv2(k)};
            double mn = c[at(gc, cc[0], cc[1], cc[2])], mx = mn;
            for (int dk = -1; dk <= 1; ++dk)
              for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                  double u = c[at(gc, cc[0] + di, cc[1] + dj, cc[2] + dk)];
                  mn = std::min(mn, u);
                  mx = std::max(mx, u);
                }
            bool fall = false;
            for (int dk = 0; dk <= 1; ++dk)
              for (int dj = 0; dj <= 1; ++dj)
                for (int di = 0; di <= 1; ++di) {
                  double u = prolong_point(gc, c, c0, stag, f0[0] + di, f0[1] + dj, f0[2] + dk);
                  if (u < mn || u > mx) fall = true;
                }
            if (fall) {
              double uc = c[at(gc, cc[0], cc[1], cc[2])];
              int fid[3] = {i, j, k};
              v = uc;
              for (int a = 0; a < 3; ++a) {
                int e[3] = {0, 0, 0};
                e[a] = 1;
                double up = c[at(gc, cc[0] + e[0], cc[1] + e[1], cc[2] + e[2])];
                double dn = c[at(gc, cc[0] - e[0], cc[1] - e[1], cc[2] - e[2])];
                double sl = minmod_s(up - uc, uc - dn);
                int child = fid[a] - 2 * floordiv2(fid[a]);
                v += (child ? 0.25 : -0.25) * sl;
              }
            }
          }
          o[at(gf, i, j, k)] = v;
        }
  }
}

void restrict_grid(const Grid& gc, const Grid& gf, const int c0[3], const int stag[3], int nf, const double* ff,
                   double* cf, const int lo[3], const int hi[3]) {
  size_t Nc = npts(gc), Nf = npts(gf);
  for (int q = 0; q < nf; ++q) {
    const double* f = ff + q * Nf;
    double* o = cf + q * Nc;
    for (int k = lo[2]; k <= hi[2]; ++k)
      for (int j = lo[1]; j <= hi[1]; ++j)
        for (int i = lo[0]; i <= hi[0]; ++i) {
          int c[3] = {i, j, k};
          int n[3], fs[3][2];
          for (int a = 0; a < 3; ++a) {
            int base = 2 * (c[a] - c0[a]);
            if (stag[a]) {
              n[a] = 1;
              fs[a][0] = base;
            } else {
              n[a] = 2;
              fs[a][0] = base;
              fs[a][1] = base + 1;
            }
          }
          double s = 0.0;
          for (int r = 0; r < n[2]; ++r)
            for (int p2 = 0; p2 < n[1]; ++p2)
              for (int p1 = 0; p1 < n[0]; ++p1) s += f[at(gf, fs[0][p1], fs[1][p2], fs[2][r])];
          o[at(gc, i, j, k)] = s / double(n[0] * n[1] * n[2]);
        }
  }
}

// out = sum_m a_m u_m + b_dt rhs on owned points of 9 fields.
template <class T> void rk_combine(const Grid& g, int nterms, const double* a, const T* const* u, double b_dt, const T* rhs,
                                   T* out) {
  size_t N = npts(g);
  for (int f = 0; f < 9; ++f)
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          size_t id = f * N + at(g, i, j, k);
          T s = T(0);
          for (int m = 0; m < nterms; ++m) s = s + T(a[m]) * u[m][id];
          out[id] = s + T(b_dt) * rhs[id];
        }
}


// Whole time steps (Sec. 3.12 workflow): every stage runs c2p on the stage
// input (resetting atmosphere cells in place), fills the primitive ghosts,
// evaluates the right-hand side and combines.  RK2 is read as Heun's method,
// RK4 as the classical scheme (the paper names neither tableau).
// state: 9 fields (Dt, St_x, St_y, St_z, taut, A_x, A_y, A_z, Psi).
template <class T> void run_steps(const Grid& g, const Params& P, const T& gam, const T* metric, const T* curv, T* state,
                                  T* prim, double dt, int nsteps, int rk, const int bc_cell[3], const int bc_A[3],
                                  uint8_t* flags, unsigned long long* stats, double* redmax,
                                  const double* shiftA = nullptr) {
  size_t N = npts(g);
  std::vector<T> U0(9 * N), U1(9 * N), U2(9 * N), U3(9 * N), k1(9 * N), k2(9 * N), k3(9 * N), k4(9 * N);
  auto fill_state = [&](T* U) {
    fill_ghosts(g, U, 5, bc_cell);
    fill_ghosts(g, U + 5 * N, 3, bc_A, shiftA);
    fill_ghosts(g, U + 8 * N, 1, bc_cell);
  };
  auto stage = [&](T* U, T* k) {
    c2p_grid(g, P, gam, metric, U + 5 * N, U, prim, flags, stats);
    fill_ghosts(g, prim, 5, bc_cell);
    double red[2];
    rhs_grid(g, P, gam, metric, curv, prim, U + 5 * N, U + 8 * N, dt, k, red, (long long*)nullptr);
    if (redmax) {
      redmax[0] = std::max(redmax[0], red[0]);
      redmax[1] = std::max(redmax[1], red[1]);
    }
  };
  auto owned_loop = [&](auto fn) {
    for (int f = 0; f < 9; ++f)
#pragma omp parallel for schedule(static)
      for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
          for (int i = 0; i < g.n[0]; ++i) fn(f * N + at(g, i, j, k));
  };
  for (int step = 0; step < nsteps; ++step) {
    std::copy(state, state + 9 * N, U0.begin());
    if (rk == 2) {
      stage(U0.data(), k1.data());
      U1 = U0;
      owned_loop([&](size_t id) { U1[id] = U0[id] + T(dt) * k1[id]; });
      fill_state(U1.data());
      stage(U1.data(), k2.data());
      std::copy(U1.begin(), U1.end(), state);
      owned_loop([&](size_t id) { state[id] = U0[id] / T(2) + U1[id] / T(2) + T(dt / 2) * k2[id]; });
      fill_state(state);
    } else {
      stage(U0.data(), k1.data());
      U1 = U0;
      owned_loop([&](size_t id) { U1[id] = U0[id] + T(dt / 2) * k1[id]; });
      fill_state(U1.data());
      stage(U1.data(), k2.data());
      U2 = U0;
      owned_loop([&](size_t id) { U2[id] = U0[id] + T(dt / 2) * k2[id]; });
      fill_state(U2.data());
      stage(U2.data(), k3.data());
      U3 = U0;
      owned_loop([&](size_t id) { U3[id] = U0[id] + T(dt) * k3[id]; });
      fill_state(U3.data());
      stage(U3.data(), k4.data());
      std::copy(U0.begin(), U0.end(), state);
      owned_loop([&](size_t id) {
        state[id] = U0[id] + T(dt / 6) * k1[id] + T(dt / 3) * k2[id] + T(dt / 3) * k3[id] + T(dt / 6) * k4[id];
      });
      fill_state(state);
    }
  }
}

}  // namespace orc

// ---------------------------------------------------------------------------
// C entry points (double precision).
using namespace orc;

extern "C" {

// Limiter decisions counted by note_tie since the last reset: out[0] all, out[1] near ties.
void orc_tie_counts(unsigned long long* out, int reset) {
  out[0] = g_tie_decisions;
  out[1] = g_tie_near;
  if (reset) g_tie_decisions = g_tie_near = 0;
}

int orc_version(void) { return 1; }

void orc_prim2con(const Grid* g, const Params* P, const double* metric, const double* A, const double* prim,
                  double* cons) {
  prim2con_grid<double>(*g, *P, P->gamma, metric, A, prim, cons);
}

void orc_c2p(const Grid* g, const Params* P, const double* metric, const double* A, double* cons, double* prim,
             uint8_t* flags, unsigned long long* stats) {
  c2p_grid<double>(*g, *P, P->gamma, metric, A, cons, prim, flags, stats);
}

void orc_fill_ghosts(const Grid* g, double* f, int nf, const int* kinds) { fill_ghosts<double>(*g, f, nf, kinds); }

void orc_fill_ghosts_shift(const Grid* g, double* f, int nf, const double* shift) {
  const int per[3] = {BC_PERIODIC, BC_PERIODIC, BC_PERIODIC};
  fill_ghosts<double>(*g, f, nf, per, shift);
}

void orc_tmunu(const Grid* g, const Params* P, const double* metric, const double* prim, const double* A,
               double* out) {
  tmunu_vertices<double>(*g, P->gamma, metric, prim, A, out);
}

void orc_rhs(const Grid* g, const Params* P, const double* metric, const double* curv, const double* prim,
             const double* A, const double* psi, double dt_max, double* rhs, double* red, long long* nfix) {
  rhs_grid<double>(*g, *P, P->gamma, metric, curv, prim, A, psi, dt_max, rhs, red, nfix);
}

void orc_run(const Grid* g, const Params* P, const double* metric, const double* curv, double* state, double* prim,
             double dt, int nsteps, int rk, const int* bc_cell, const int* bc_A, uint8_t* flags,
             unsigned long long* stats, double* redmax, const double* shiftA) {
  run_steps<double>(*g, *P, P->gamma, metric, curv, state, prim, dt, nsteps, rk, bc_cell, bc_A, flags, stats, redmax,
                    shiftA);
}

// Loss of the differentiation workload, (sum over owned cells of rho^2 dV)^(1/2) after nsteps
// from the primitives prim0 (conserved variables by prim2con, cell ghosts by bc_cell), and its
// directional derivative along the tangent (dprim0, dgamma) by forward-mode dual numbers.
// out[0] = loss, out[1] = directional derivative.  stats: c2p counters of the whole run.
void orc_loss_jvp(const Grid* g, const Params* P, double dgamma, const double* metric, const double* curv,
                  const double* prim0, const double* dprim0, const double* A0, const double* psi0, double dt,
                  int nsteps, int rk, const int* bc_cell, const int* bc_A, const double* shiftA, double* out,
                  unsigned long long* stats) {
  size_t N = npts(*g);
  auto lift = [&](const double* a, const double* da, int nf) {
    std::vector<Dl> r((size_t)nf * N);
    for (size_t q = 0; q < (size_t)nf * N; ++q) r[q] = Dl(a[q], da ? da[q] : 0.0);
    return r;
  };
  std::vector<Dl> m = lift(metric, nullptr, 10), K = lift(curv, nullptr, 6), prim = lift(prim0, dprim0, 5);
  std::vector<Dl> state(9 * N);
  std::vector<Dl> A = lift(A0, nullptr, 3), psi = lift(psi0, nullptr, 1);
  Dl gam(P->gamma, dgamma);
  prim2con_grid<Dl>(*g, *P, gam, m.data(), A.data(), prim.data(), state.data());
  fill_ghosts<Dl>(*g, state.data(), 5, bc_cell);
  std::copy(A.begin(), A.end(), state.begin() + 5 * N);
  std::copy(psi.begin(), psi.end(), state.begin() + 8 * N);
  std::vector<uint8_t> flags(N);
  run_steps<Dl>(*g, *P, gam, m.data(), K.data(), state.data(), prim.data(), dt, nsteps, rk, bc_cell, bc_A,
                flags.data(), stats, nullptr, shiftA);
  c2p_grid<Dl>(*g, *P, gam, m.data(), state.data() + 5 * N, state.data(), prim.data(), flags.data(), stats);
  Dl acc(0.0);
  double dV = g->dx[0] * g->dx[1] * g->dx[2];
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        Dl r = prim[at(*g, i, j, k)];
        acc = acc + r * r * Dl(dV);
      }
  Dl L = sqrt(acc);
  out[0] = L.v;
  out[1] = L.d;
}

// Directional derivatives of the pieces of one stage, by forward-mode dual numbers (arrays with
// ghosts as given; tangents d* with the same layout; NULL tangent = 0).
static std::vector<Dl> lift_dl(const double* a, const double* da, size_t n) {
  std::vector<Dl> r(n);
  for (size_t q = 0; q < n; ++q) r[q] = Dl(a[q], da ? da[q] : 0.0);
  return r;
}

// cons = prim2con(prim, A): writes cons and its tangent on owned points.
void orc_prim2con_jvp(const Grid* g, const Params* P, double dgamma, const double* metric, const double* A,
                      const double* dA, const double* prim, const double* dprim, double* cons, double* dcons) {
  size_t N = npts(*g);
  std::vector<Dl> m = lift_dl(metric, nullptr, 10 * N), a = lift_dl(A, dA, 3 * N), pr = lift_dl(prim, dprim, 5 * N);
  std::vector<Dl> c(5 * N);
  prim2con_grid<Dl>(*g, *P, Dl(P->gamma, dgamma), m.data(), a.data(), pr.data(), c.data());
  for (size_t q = 0; q < 5 * N; ++q) {
    cons[q] = c[q].v;
    dcons[q] = c[q].d;
  }
}

// prim = c2p(cons, A) warm-started from guess: writes prim and its tangent on owned points.
void orc_c2p_jvp(const Grid* g, const Params* P, double dgamma, const double* metric, const double* A, const double* dA,
                 const double* cons, const double* dcons, const double* guess, double* prim, double* dprim) {
  size_t N = npts(*g);
  std::vector<Dl> m = lift_dl(metric, nullptr, 10 * N), a = lift_dl(A, dA, 3 * N), c = lift_dl(cons, dcons, 5 * N);
  std::vector<Dl> pr = lift_dl(guess, nullptr, 5 * N);
  std::vector<uint8_t> flags(N);
  unsigned long long st[6] = {0, 0, 0, 0, 0, 0};
  c2p_grid<Dl>(*g, *P, Dl(P->gamma, dgamma), m.data(), a.data(), c.data(), pr.data(), flags.data(), st);
  for (size_t q = 0; q < 5 * N; ++q) {
    prim[q] = pr[q].v;
    dprim[q] = pr[q].d;
  }
}

// One stage's right-hand side L(cons, A, psi) = rhs(fill(c2p(cons, A)), A, psi) with the primitive
// ghosts filled periodically: writes L (9 fields) and its tangent on owned points.
void orc_stage_jvp(const Grid* g, const Params* P, double dgamma, const double* metric, const double* curv,
                   const double* cons, const double* dcons, const double* A, const double* dA, const double* psi,
                   const double* dpsi, const double* guess, double dt_max, double* out, double* dout) {
  size_t N = npts(*g);
  std::vector<Dl> m = lift_dl(metric, nullptr, 10 * N), K = lift_dl(curv, nullptr, 6 * N);
  std::vector<Dl> a = lift_dl(A, dA, 3 * N), c = lift_dl(cons, dcons, 5 * N), ps = lift_dl(psi, dpsi, N);
  std::vector<Dl> pr = lift_dl(guess, nullptr, 5 * N), r(9 * N);
  std::vector<uint8_t> flags(N);
  unsigned long long st[6] = {0, 0, 0, 0, 0, 0};
  Dl gam(P->gamma, dgamma);
  c2p_grid<Dl>(*g, *P, gam, m.data(), a.data(), c.data(), pr.data(), flags.data(), st);
  const int per[3] = {BC_PERIODIC, BC_PERIODIC, BC_PERIODIC};
  fill_ghosts<Dl>(*g, pr.data(), 5, per);
  double red[2];
  rhs_grid<Dl>(*g, *P, gam, m.data(), K.data(), pr.data(), a.data(), ps.data(), dt_max, r.data(), red,
               (long long*)nullptr);
  for (size_t q = 0; q < 9 * N; ++q) {
    out[q] = r[q].v;
    dout[q] = r[q].d;
  }
}

void orc_prolong(const Grid* gc, const Grid* gf, const int* c0, const int* stag, int nf, const double* cf, double* ff,
                 const int* lo, const int* hi) {
  prolong_grid(*gc, *gf, c0, stag, nf, cf, ff, lo, hi);
}

void orc_restrict(const Grid* gc, const Grid* gf, const int* c0, const int* stag, int nf, const double* ff,
                  double* cf, const int* lo, const int* hi) {
  restrict_grid(*gc, *gf, c0, stag, nf, ff, cf, lo, hi);
}

void orc_rk_stage(const Grid* g, int nterms, const double* a, const double* const* u, double b_dt, const double* rhs,
                  double* out) {
  rk_combine<double>(*g, nterms, a, u, b_dt, rhs, out);
}

// Algorithmic operation counts of one right-hand side and one c2p on this block,
// measured with the counting scalar: out[0..3] = centre field, faces (all three
// directions), cells (divergence + sources), constrained transport; out[4] = c2p.
void orc_count_ops(const Grid* g, const Params* P, const double* metric, const double* curv, const double* prim,
                   const double* A, const double* psi, double dt_max, unsigned long long* out) {
  size_t N = npts(*g);
  auto conv = [&](const double* a, size_t n) {
    std::vector<Cnt> v(n);
    for (size_t i = 0; i < n; ++i) v[i] = Cnt(a[i]);
    return v;
  };
  std::vector<Cnt> m = conv(metric, 10 * N), k = conv(curv, 6 * N), pr = conv(prim, 5 * N), a = conv(A, 3 * N),
                   ps = conv(psi, N), rhs(9 * N);
  for (int q = 0; q < 4; ++q) g_phase_ops[q] = 0;
  Cnt::ops = 0;
  g_phase_last = 0;
  rhs_grid<Cnt>(*g, *P, Cnt(P->gamma), m.data(), k.data(), pr.data(), a.data(), ps.data(), dt_max, rhs.data(),
                nullptr, nullptr);
  for (int q = 0; q < 4; ++q) out[q] = g_phase_ops[q];
  // c2p from the conserved variables of these primitives, warm-started from them
  std::vector<Cnt> cons(5 * N);
  prim2con_grid<Cnt>(*g, *P, Cnt(P->gamma), m.data(), a.data(), pr.data(), cons.data());
  Cnt::ops = 0;
  c2p_grid<Cnt>(*g, *P, Cnt(P->gamma), m.data(), a.data(), cons.data(), pr.data(), nullptr, nullptr);
  out[4] = Cnt::ops;
}

// Threads of the OpenMP build (OpenMP over k-planes of the grid loops; every cell is computed
// as in the serial build and the reductions are integer sums and maxima, so results are bitwise
// the same).  The serial build ignores the pragmas and reports 1.
int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

// Counts of the counting scalar on single building blocks, for the pins of the
// counter itself: out[0] lag_value, [1] lag_deriv, [2] face_interp of one field,
// [3] centre_value of one field, [4] centre_interp (value and three derivatives),
// [5] face_B, [6] centre_B, [7] make_geom, [8] a fixed expression mixing every
// counted operation with the uncounted ones (negation, fabs, comparisons).
void orc_count_probe(unsigned long long* out) {
  Grid g{};
  for (int d = 0; d < 3; ++d) {
    g.n[d] = 2;
    g.ld[d] = 2 + 2 * 3 + 1;
    g.dx[d] = 0.25;
  }
  g.ng = 3;
  size_t N = npts(g);
  std::vector<Cnt> f(3 * N);
  for (size_t q = 0; q < 3 * N; ++q) f[q] = Cnt(1.0 + 0.001 * double(q % 97));
  Cnt col[4] = {Cnt(1.0), Cnt(2.0), Cnt(4.0), Cnt(3.0)};
  auto count = [](auto fn) {
    Cnt::ops = 0;
    fn();
    return Cnt::ops;
  };
  Cnt sink(0.0);
  out[0] = count([&] { sink = lag_value(col); });
  out[1] = count([&] { sink = lag_deriv(col, 0.25); });
  out[2] = count([&] { sink = face_interp(g, f.data(), 1, 0, 0, 0); });
  out[3] = count([&] { sink = centre_value(g, f.data(), 0, 0, 0); });
  out[4] = count([&] {
    Cnt der[3];
    centre_interp(g, f.data(), 0, 0, 0, sink, der);
  });
  out[5] = count([&] { sink = face_B(g, f.data(), 2, 0, 0, 0); });
  out[6] = count([&] {
    Cnt b[3];
    centre_B(g, f.data(), 0, 0, 0, b);
  });
  out[7] = count([&] {
    Cnt m[10] = {Cnt(0.9), Cnt(0.1), Cnt(0.0), Cnt(-0.1), Cnt(1.1), Cnt(0.05), Cnt(0.0), Cnt(1.0), Cnt(0.02),
                 Cnt(0.95)};
    Geom<Cnt> G = make_geom(m);
    sink = G.sqrtg;
  });
  out[8] = count([&] {
    Cnt a(1.5), b(-0.5), c(2.0), d(0.25), e(4.0);
    Cnt t = -(((a + b) * c - d) / e);        // 4
    t = fabs(t) + sqrt(e) + pow(a, 2.0);     // 2 additions, sqrt, pow: 4
    if (t > a && !(t <= b) && t != c) sink = t;
  });
  (void)value_of(sink);
}

// Operations of one point recovery on the counting scalar (same inputs as
// orc_pt_c2p); iters out.
unsigned long long orc_count_c2p_point(const Params* P, const double* m10, const double* cons5, const double* Bt3,
                                       const double* prev5, int* iters) {
  Cnt m[10], cs[5], bt[3], pv[5], pr[5];
  for (int c = 0; c < 10; ++c) m[c] = Cnt(m10[c]);
  for (int c = 0; c < 5; ++c) {
    cs[c] = Cnt(cons5[c]);
    pv[c] = Cnt(prev5[c]);
  }
  for (int c = 0; c < 3; ++c) bt[c] = Cnt(Bt3[c]);
  Geom<Cnt> G = make_geom(m);
  Cnt::ops = 0;
  int it = 0;
  c2p_point(G, cs, bt, pv, Cnt(P->gamma), *P, pr, it);
  if (iters) *iters = it;
  return Cnt::ops;
}

// Face B (densitized) of direction d for every index in [-ng+?]: fills all
// points where the curl stencil is inside the array (for pins).
void orc_face_B(const Grid* g, const double* A, double* Bf) {
  size_t N = npts(*g);
  for (int d = 0; d < 3; ++d)
    for (int k = -g->ng; k < g->n[2] + g->ng; ++k)
      for (int j = -g->ng; j < g->n[1] + g->ng; ++j)
        for (int i = -g->ng; i < g->n[0] + g->ng; ++i) Bf[d * N + at(*g, i, j, k)] = face_B(*g, A, d, i, j, k);
}

// Centre metric value and derivatives for owned cells: out[40][N] ordered
// (value of 10 components, d_x of 10, d_y of 10, d_z of 10).
void orc_centre_metric(const Grid* g, const double* metric, double* out) {
  size_t N = npts(*g);
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) {
        double m[10], dm[3][10];
        centre_metric(*g, metric, i, j, k, m, dm);
        size_t id = at(*g, i, j, k);
        for (int c = 0; c < 10; ++c) {
          out[c * N + id] = m[c];
          for (int d = 0; d < 3; ++d) out[(10 * (d + 1) + c) * N + id] = dm[d][c];
        }
      }
}

// Face-interpolated field f of direction d at owned-range faces.
void orc_face_interp(const Grid* g, const double* f, int d, double* out) {
  for (int k = 0; k < g->n[2]; ++k)
    for (int j = 0; j < g->n[1]; ++j)
      for (int i = 0; i < g->n[0]; ++i) out[at(*g, i, j, k)] = face_interp(*g, f, d, i, j, k);
}

// ---- pointwise entry points (for the pins) ----
// metric10 = alpha, beta^i, gamma_ij; prim5 = rho, p, v^i; Bt3 densitized.

void orc_pt_prim2con(const double* m10, const double* prim5, const double* Bt3, double gam, double* cons5) {
  Geom<double> G = make_geom(m10);
  Fluid<double> F = make_fluid(G, prim5, Bt3, gam);
  prim2con_point(G, F, cons5);
}

// Auxiliary fluid quantities: W, b0, b^x..z, bsq, u0, u^x..z, h, eps (13 values)
void orc_pt_fluid(const double* m10, const double* prim5, const double* Bt3, double gam, double* out) {
  Geom<double> G = make_geom(m10);
  Fluid<double> F = make_fluid(G, prim5, Bt3, gam);
  out[0] = F.W; out[1] = F.b0;
  for (int i = 0; i < 3; ++i) out[2 + i] = F.b[i];
  out[5] = F.bsq; out[6] = F.u0;
  for (int i = 0; i < 3; ++i) out[7 + i] = F.u[i];
  out[10] = F.h; out[11] = F.eps; out[12] = F.v2;
}

void orc_pt_flux(const double* m10, const double* prim5, const double* Bt3, double gam, int d, double* U7,
                 double* F7) {
  Geom<double> G = make_geom(m10);
  Fluid<double> F = make_fluid(G, prim5, Bt3, gam);
  flux_point(G, F, d, U7, F7);
}

// out: c-, c+, bound-, bound+ ; coeffs: the five polynomial coefficients of Q
// (lambda^0..lambda^4) obtained by evaluating Q at five points (test helper).
void orc_pt_speeds(const double* m10, const double* prim5, const double* Bt3, double gam, int d, double* out) {
  Geom<double> G = make_geom(m10);
  Fluid<double> F = make_fluid(G, prim5, Bt3, gam);
  double cm, cp, bm, bp;
  speeds_point(G, F, d, gam, SPEED_QUARTIC, cm, cp);
  speeds_point(G, F, d, gam, SPEED_BOUND, bm, bp);
  out[0] = cm; out[1] = cp; out[2] = bm; out[3] = bp;
}

void orc_pt_quartic_eval(const double* m10, const double* prim5, const double* Bt3, double gam, int d, int n,
                         const double* lam, double* q) {
  Geom<double> G = make_geom(m10);
  Fluid<double> F = make_fluid(G, prim5, Bt3, gam);
  double w2;
  Disp<double> Q = make_disp(G, F, d, gam, w2);
  for (int i = 0; i < n; ++i) {
    double dq;
    disp_eval(Q, lam[i], q[i], dq);
  }
}

void orc_pt_hlle(const double* UL, const double* FL, double cmL, double cpL, const double* UR, const double* FR,
                 double cmR, double cpR, double* Fo) {
  double a, b;
  hlle(UL, FL, cmL, cpL, UR, FR, cmR, cpR, Fo, a, b);
}

void orc_pt_lxf(const double* UL, const double* FL, double cmL, double cpL, const double* UR, const double* FR,
                double cmR, double cpR, double* Fo) {
  double a, b;
  lxf(UL, FL, cmL, cpL, UR, FR, cmR, cpR, Fo, a, b);
}

// 1-D reconstruction of an array a[0..n): for every cell c in [2, n-3] the
// values at its left and right faces.
void orc_recon_1d(const Params* P, int kind, int n, const double* a, double* aL, double* aR) {
  for (int c = 2; c < n - 2; ++c) reconstruct_cell(kind, a + c - 2, aL[c], aR[c], *P);
}

// Point c2p. cons5 densitized (updated if the atmosphere applies), prev5 the
// warm start; returns flags; iters out.
int orc_pt_c2p(const Params* P, const double* m10, double* cons5, const double* Bt3, const double* prev5,
               double* prim5, int* iters) {
  Geom<double> G = make_geom(m10);
  int it = 0;
  uint8_t fl = c2p_point(G, cons5, Bt3, prev5, P->gamma, *P, prim5, it);
  if (iters) *iters = it;
  return fl;
}

// Noble residuals and Jacobian at (z, w) for the given conserved state.
void orc_pt_noble_residual(const double* m10, const double* cons5, const double* Bt3, double gam, double z, double w,
                           double* R2, double* J4) {
  Geom<double> G = make_geom(m10);
  C2PInput<double> c = make_c2p_input(G, cons5, Bt3);
  double J[2][2];
  noble_residual(c, gam, z, w, R2, J);
  J4[0] = J[0][0]; J4[1] = J[0][1]; J4[2] = J[1][0]; J4[3] = J[1][1];
}

// Palenzuela master function f(x) and its bracket [lo, hi] (unclamped lower bound).
void orc_pt_palen(const double* m10, const double* cons5, const double* Bt3, double gam, double wmax, int n,
                  const double* x, double* f, double* bracket) {
  Geom<double> G = make_geom(m10);
  C2PInput<double> c = make_c2p_input(G, cons5, Bt3);
  Palen<double> P5;
  P5.D = c.D; P5.q = c.tau / c.D; P5.r = c.S2 / (c.D * c.D); P5.s = c.B2 / c.D; P5.t = c.BS / std::pow(c.D, 1.5);
  bracket[0] = 1.0 + P5.q - P5.s;
  bracket[1] = 2.0 + 2.0 * P5.q - P5.s;
  for (int i = 0; i < n; ++i) {
    double W, rho, eps, p;
    palen_eval(P5, x[i], gam, wmax, f[i], W, rho, eps, p);
  }
}

// Sources at a point from the metric, its first derivatives dm[3][10], K6.
void orc_pt_sources(const double* m10, const double* dm30, const double* K6, const double* prim5, const double* Bt3,
                    double gam, double* src5) {
  Geom<double> G = make_geom(m10);
  Fluid<double> F = make_fluid(G, prim5, Bt3, gam);
  double dm[3][10];
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 10; ++c) dm[d][c] = dm30[d * 10 + c];
  sources_point(G, dm, K6, F, src5);
}

// T^{mu nu} (16 values, row-major).
void orc_pt_tmunu(const double* m10, const double* prim5, const double* Bt3, double gam, double* T16) {
  Geom<double> G = make_geom(m10);
  Fluid<double> F = make_fluid(G, prim5, Bt3, gam);
  double Tu[4][4];
  stress_tensor(G, F, Tu);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) T16[a * 4 + b] = Tu[a][b];
}

}  // extern "C"
