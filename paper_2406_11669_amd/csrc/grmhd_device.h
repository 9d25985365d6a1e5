// grmhd_device.h -- device-side physics of the Valencia GRMHD right-hand side (gfx950, FP64).
//
// Pointwise building blocks used by the kernels in asterx.hip: 3+1 geometry, ideal-gas
// EOS, prim -> cons, fluxes, characteristic speeds, HLLE, reconstruction and the
// conservative-to-primitive recovery.  Every routine works on one point in registers.
// Section/equation references are to AsterX, arXiv 2406.11669.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DEV __device__ __forceinline__

namespace ax {

// ---------------------------------------------------------------------------------------
// Dual number (value, tangent) for forward-mode directional derivatives of the pointwise
// physics; the adjoint kernels build local Jacobians with it.  Branches (max, min, limiter
// cases) follow the value, i.e. the active branch.
// the double versions stay visible next to the dual overloads below
using ::copysign;
using ::fabs;
using ::fmax;
using ::fmin;
using ::pow;
using ::sqrt;

struct Dual {
  double v, d;
  DEV Dual() = default;
  explicit DEV Dual(double x) : v(x), d(0.0) {}
  DEV Dual(double x, double y) : v(x), d(y) {}
};
DEV Dual mkd(double v, double d = 0.0) { return Dual{v, d}; }
DEV double val(double x) { return x; }
DEV double val(const Dual& x) { return x.v; }
DEV Dual operator+(Dual a, Dual b) { return Dual{a.v + b.v, a.d + b.d}; }
DEV Dual operator-(Dual a, Dual b) { return Dual{a.v - b.v, a.d - b.d}; }
DEV Dual operator-(Dual a) { return Dual{-a.v, -a.d}; }
DEV Dual operator*(Dual a, Dual b) { return Dual{a.v * b.v, a.d * b.v + a.v * b.d}; }
DEV Dual operator/(Dual a, Dual b) {
  double r = 1.0 / b.v, q = a.v * r;
  return Dual{q, (a.d - q * b.d) * r};
}
DEV Dual operator+(Dual a, double b) { return Dual{a.v + b, a.d}; }
DEV Dual operator+(double a, Dual b) { return Dual{a + b.v, b.d}; }
DEV Dual operator-(Dual a, double b) { return Dual{a.v - b, a.d}; }
DEV Dual operator-(double a, Dual b) { return Dual{a - b.v, -b.d}; }
DEV Dual operator*(Dual a, double b) { return Dual{a.v * b, a.d * b}; }
DEV Dual operator*(double a, Dual b) { return Dual{a * b.v, a * b.d}; }
DEV Dual operator/(Dual a, double b) { return Dual{a.v / b, a.d / b}; }
DEV Dual operator/(double a, Dual b) {
  double r = 1.0 / b.v, q = a * r;
  return Dual{q, -q * b.d * r};
}
DEV Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
DEV Dual& operator-=(Dual& a, Dual b) { return a = a - b; }
DEV bool operator<(Dual a, Dual b) { return a.v < b.v; }
DEV bool operator>(Dual a, Dual b) { return a.v > b.v; }
DEV bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
DEV bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
DEV bool operator<(Dual a, double b) { return a.v < b; }
DEV bool operator>(Dual a, double b) { return a.v > b; }
DEV bool operator<=(Dual a, double b) { return a.v <= b; }
DEV bool operator>=(Dual a, double b) { return a.v >= b; }
DEV Dual sqrt(Dual a) {
  double s = ::sqrt(a.v);
  return Dual{s, a.d * 0.5 / s};
}
DEV Dual fabs(Dual a) { return a.v < 0.0 ? -a : a; }
DEV Dual fmax(Dual a, Dual b) { return a.v >= b.v ? a : b; }
DEV Dual fmin(Dual a, Dual b) { return a.v <= b.v ? a : b; }
DEV Dual fmax(Dual a, double b) { return a.v >= b ? a : Dual(b, 0.0); }
DEV Dual fmax(double a, Dual b) { return a >= b.v ? Dual(a, 0.0) : b; }
DEV Dual fmin(Dual a, double b) { return a.v <= b ? a : Dual(b, 0.0); }
DEV Dual fmin(double a, Dual b) { return a <= b.v ? Dual(a, 0.0) : b; }
DEV Dual copysign(Dual m, Dual s) { return (::signbit(m.v) != ::signbit(s.v)) ? -m : m; }
DEV Dual pow(Dual a, double e) {
  // e a^(e-1) da, written without dividing by a (finite at a = 0 for e >= 1)
  return Dual{::pow(a.v, e), a.d != 0.0 ? a.d * e * ::pow(a.v, e - 1.0) : 0.0};
}

// Reciprocal and inverse square root of positive, finite, normal operands from the hardware
// estimates (about 23 correct bits), refined by Newton's iteration -- r <- r + r (1 - b r) for
// 1/b, y <- y (3/2 - x y^2 / 2) for 1/sqrt(x) -- which doubles the correct bits per step: two
// steps reach double precision within a few ulp, in fewer instructions than the correctly
// rounded division and square root.  The dual overloads divide exactly.
DEV double recip(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return fma(r, fma(-b, r, 1.0), r);
}
DEV double quot(double a, double b) {
  const double r = recip(b), q = a * r;
  return fma(r, fma(-b, q, a), q);
}
DEV double inv_sqrt(double x) {
  const double h = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}
DEV Dual recip(Dual b) { return 1.0 / b; }
DEV Dual quot(Dual a, Dual b) { return a / b; }
DEV Dual inv_sqrt(Dual x) { return 1.0 / sqrt(x); }

// Symmetric 3x3 storage: xx, xy, xz, yy, yz, zz.
struct Geo {
  double alp, beta[3];
  double g[6];   // gamma_ij
  double gu[6];  // gamma^ij
  double sqrtg;
};

DEV void geo_from(const double m[10], Geo& G) {
  G.alp = m[0];
  G.beta[0] = m[1];
  G.beta[1] = m[2];
  G.beta[2] = m[3];
#pragma unroll
  for (int c = 0; c < 6; ++c) G.g[c] = m[4 + c];
  const double* g = G.g;
  double c00 = g[3] * g[5] - g[4] * g[4];
  double c01 = g[2] * g[4] - g[1] * g[5];
  double c02 = g[1] * g[4] - g[2] * g[3];
  double c11 = g[0] * g[5] - g[2] * g[2];
  double c12 = g[1] * g[2] - g[0] * g[4];
  double c22 = g[0] * g[3] - g[1] * g[1];
  double det = g[0] * c00 + g[1] * c01 + g[2] * c02;
  double idet = recip(det);
  G.gu[0] = c00 * idet;
  G.gu[1] = c01 * idet;
  G.gu[2] = c02 * idet;
  G.gu[3] = c11 * idet;
  G.gu[4] = c12 * idet;
  G.gu[5] = c22 * idet;
  G.sqrtg = sqrt(det);
}

template <class T>
DEV void lower(const double* g, const T v[3], T vl[3]) {
  vl[0] = g[0] * v[0] + g[1] * v[1] + g[2] * v[2];
  vl[1] = g[1] * v[0] + g[3] * v[1] + g[4] * v[2];
  vl[2] = g[2] * v[0] + g[4] * v[1] + g[5] * v[2];
}

// Component (d, e) of a symmetric 3x3 in the 6-slot storage.
DEV int sym(int d, int e) {
  int a = d < e ? d : e, b = d < e ? e : d;
  return a == 0 ? b : (a == 1 ? 2 + b : 5);
}

// ---------------------------------------------------------------------------------------
// A fluid state with its magnetic field (Sec. 2.2, comoving field from the Eulerian one).
// All quantities needed by fluxes and speeds, expressed through
// W^-2 = 1 - v^2, B.v and B^2 (b^2 = B^2/W^2 + (B.v)^2, alpha b^0 = W B.v).
template <class T>
struct StateT {
  T rho, p, v[3], vl[3], iW2, W, B[3], Bl[3], B2, Bv, bsq, rhoh;
};
using State = StateT<double>;

template <class T>
DEV void state_make(const Geo& G, const T pr[5], const T Bt[3], T gam, StateT<T>& S, T gfac) {
  S.rho = pr[0];
  S.p = pr[1];
  S.v[0] = pr[2];
  S.v[1] = pr[3];
  S.v[2] = pr[4];
  lower(G.g, S.v, S.vl);
  T v2 = S.v[0] * S.vl[0] + S.v[1] * S.vl[1] + S.v[2] * S.vl[2];
  S.iW2 = 1.0 - v2;
  S.W = inv_sqrt(S.iW2);
  double is = recip(G.sqrtg);
  S.B[0] = Bt[0] * is;
  S.B[1] = Bt[1] * is;
  S.B[2] = Bt[2] * is;
  lower(G.g, S.B, S.Bl);
  S.B2 = S.B[0] * S.Bl[0] + S.B[1] * S.Bl[1] + S.B[2] * S.Bl[2];
  S.Bv = S.B[0] * S.vl[0] + S.B[1] * S.vl[1] + S.B[2] * S.vl[2];
  S.bsq = S.B2 * S.iW2 + S.Bv * S.Bv;
  // rho h = rho (1 + eps) + p = rho + Gamma/(Gamma-1) p (ideal gas, Sec. 3.7); gfac = Gamma/(Gamma-1)
  S.rhoh = S.rho + gfac * S.p;
}

DEV void state_make(const Geo& G, const double pr[5], const double Bt[3], double gam, State& S) {
  state_make<double>(G, pr, Bt, gam, S, gam / (gam - 1.0));
}

// Densitized conserved variables, written with z = rho h W^2 (Sec. 3.5 rewriting of the
// definitions): S_j = (z + B^2) v_j - (B.v) B_j, tau = z + B^2 - p - B^2/(2W^2) - (B.v)^2/2 - D.
template <class T>
DEV void cons_of(const Geo& G, const StateT<T>& S, T U[5]) {
  T z = S.rhoh * S.W * S.W;
  T D = S.rho * S.W;
  T zb = z + S.B2;
  U[0] = G.sqrtg * D;
  U[1] = G.sqrtg * (zb * S.vl[0] - S.Bv * S.Bl[0]);
  U[2] = G.sqrtg * (zb * S.vl[1] - S.Bv * S.Bl[1]);
  U[3] = G.sqrtg * (zb * S.vl[2] - S.Bv * S.Bl[2]);
  U[4] = G.sqrtg * (zb - S.p - 0.5 * (S.B2 * S.iW2 + S.Bv * S.Bv) - D);
}

// Conserved vector and flux along D (eq. grmhdeqs times alpha sqrt(gamma)):
// 5 hydro components and the two transverse densitized induction components
// (t1 = (D+1)%3, t2 = (D+2)%3): Btilde^t vt^D - Btilde^D vt^t.
template <int D, class T>
DEV void flux_of(const Geo& G, const StateT<T>& S, T U[7], T F[7]) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  cons_of(G, S, U);
  T vt[3];
  vt[0] = G.alp * S.v[0] - G.beta[0];
  vt[1] = G.alp * S.v[1] - G.beta[1];
  vt[2] = G.alp * S.v[2] - G.beta[2];
  T ptot = S.p + 0.5 * S.bsq;
  double as = G.alp * G.sqrtg;
  // b_j B^D / W = B_j B^D / W^2 + (B.v) v_j B^D ;  alpha b^0 B^D / W = (B.v) B^D
  T BD = S.B[D];
  T m1 = BD * S.iW2, m2 = S.Bv * BD;
  F[0] = U[0] * vt[D];
  F[1] = U[1] * vt[D] - as * (S.Bl[0] * m1 + S.vl[0] * m2);
  F[2] = U[2] * vt[D] - as * (S.Bl[1] * m1 + S.vl[1] * m2);
  F[3] = U[3] * vt[D] - as * (S.Bl[2] * m1 + S.vl[2] * m2);
  F[1 + D] += as * ptot;
  F[4] = U[4] * vt[D] + as * (ptot * S.v[D] - m2);
  T Bt1 = G.sqrtg * S.B[t1], Bt2 = G.sqrtg * S.B[t2], BtD = G.sqrtg * BD;
  F[5] = Bt1 * vt[D] - BtD * vt[t1];
  F[6] = Bt2 * vt[D] - BtD * vt[t2];
  U[5] = Bt1;
  U[6] = Bt2;
}

// ---------------------------------------------------------------------------------------
// Characteristic speeds along D (Sec. 3.3).  The fast-magnetosonic dispersion relation for
// a front with covector (-lambda, e_D):
//   rho h (1 - cs^2) a^4 - (rho h cs^2 + b^2) a^2 G + cs^2 bb^2 G = 0,
// a = -lambda u^0 + u^D, bb = -lambda b^0 + b^D, G = g^00 lambda^2 - 2 g^0D lambda + g^DD,
// expanded into a quartic in lambda and solved by Newton from the outer roots of the
// isotropic bound (1 - w2) a^2 - w2 G = 0, w2 = cs^2 + cA^2 - cs^2 cA^2, inward.
template <class T>
DEV void qroots(T qa, T qb, T qc, T& rp, T& rm) {
  T disc = fmax(qb * qb - 4.0 * qa * qc, 0.0);
  T sd = sqrt(disc);
  T q = -0.5 * (qb + copysign(sd, qb));
  T r1 = q / qa, r2 = qc / q;
  if (val(q) == 0.0) r1 = r2 = q;
  rp = fmax(r1, r2);
  rm = fmin(r1, r2);
}

// Newton on the quartic in Horner form, for both outer roots in one loop (two independent
// dependency chains per iteration).  The step uses the hardware reciprocal estimate of Q':
// an inexact step only scales the Newton correction by (1 + delta), which the next pass
// corrects, so each root is still found to the stopping tolerance.
DEV void quartic_outer_roots(const double c[5], double& xp, double& xm) {
  const double d3 = 4.0 * c[4], d2 = 3.0 * c[3], d1 = 2.0 * c[2];
  const double tol = 8.881784197001252e-16;
  bool dp = false, dm = false;
  for (int it = 0; it < 30; ++it) {
    double qp = (((c[4] * xp + c[3]) * xp + c[2]) * xp + c[1]) * xp + c[0];
    double qm = (((c[4] * xm + c[3]) * xm + c[2]) * xm + c[1]) * xm + c[0];
    double gp = ((d3 * xp + d2) * xp + d1) * xp + c[1];
    double gm = ((d3 * xm + d2) * xm + d1) * xm + c[1];
    double sp = gp != 0.0 ? qp * __builtin_amdgcn_rcp(gp) : 0.0;
    double sm = gm != 0.0 ? qm * __builtin_amdgcn_rcp(gm) : 0.0;
    if (!dp) {
      xp -= sp;
      dp = fabs(sp) <= tol * fmax(1.0, fabs(xp));
    }
    if (!dm) {
      xm -= sm;
      dm = fabs(sm) <= tol * fmax(1.0, fabs(xm));
    }
    if (dp && dm) break;
  }
}

// Root of the quartic found on values; for dual coefficients its tangent follows from the
// implicit function theorem, d lambda = -(sum_k dc_k lambda^k) / Q'(lambda).
DEV double root_tangent(const double c[5], double x) { return x; }
DEV Dual root_tangent(const Dual c[5], double x) {
  double qd = (((c[4].d * x + c[3].d) * x + c[2].d) * x + c[1].d) * x + c[0].d;
  double dq = ((4.0 * c[4].v * x + 3.0 * c[3].v) * x + 2.0 * c[2].v) * x + c[1].v;
  return Dual{x, dq != 0.0 ? -qd / dq : 0.0};
}

template <int D, class T>
DEV void speeds_of(const Geo& G, const StateT<T>& S, T gam, int kind, T& cm, T& cp) {
  double ia = recip(G.alp);
  double bD = G.beta[D];
  T uD = S.W * (S.v[D] - bD * ia);
  T u0 = S.W * ia;
  T b0 = S.W * S.Bv * ia;
  T bDc = (S.B[D] + G.alp * b0 * uD) * (S.iW2 * S.W);  // 1/W = W (1 - v^2)
  T cs2 = quot(gam * S.p, S.rhoh);
  T cA2 = quot(S.bsq, S.rhoh + S.bsq);
  T w2 = cs2 + cA2 - cs2 * cA2;
  double ia2 = ia * ia;
  double G0 = G.gu[sym(D, D)] - bD * bD * ia2, G1 = -2.0 * bD * ia2, G2 = -ia2;
  T a0 = uD, a1 = -u0;
  T om = 1.0 - w2;
  T lp, lm;
  qroots(om * a1 * a1 - w2 * G2, 2.0 * om * a0 * a1 - w2 * G1, om * a0 * a0 - w2 * G0, lp, lm);
  if (kind == 1) {
    cp = lp;
    cm = lm;
    return;
  }
  T A4 = S.rhoh * (1.0 - cs2), Bq = S.rhoh * cs2 + S.bsq, Cq = cs2;
  // a^2 and bb^2 as quadratics, products with G as quartics
  T s0 = a0 * a0, s1 = 2.0 * a0 * a1, s2 = a1 * a1;
  T t0 = bDc * bDc, t1 = -2.0 * bDc * b0, t2 = b0 * b0;
  T c[5];
  // A4 a^4
  c[0] = A4 * s0 * s0;
  c[1] = A4 * 2.0 * s0 * s1;
  c[2] = A4 * (s1 * s1 + 2.0 * s0 * s2);
  c[3] = A4 * 2.0 * s1 * s2;
  c[4] = A4 * s2 * s2;
  // (-Bq a^2 + Cq bb^2) G
  T r0 = -Bq * s0 + Cq * t0, r1 = -Bq * s1 + Cq * t1, r2 = -Bq * s2 + Cq * t2;
  c[0] += r0 * G0;
  c[1] += r0 * G1 + r1 * G0;
  c[2] += r0 * G2 + r1 * G1 + r2 * G0;
  c[3] += r1 * G2 + r2 * G1;
  c[4] += r2 * G2;
  double cv[5] = {val(c[0]), val(c[1]), val(c[2]), val(c[3]), val(c[4])};
  double xp = val(lp), xm = val(lm);
  quartic_outer_roots(cv, xp, xm);
  cp = root_tangent(c, xp);
  cm = root_tangent(c, xm);
}

// Reverse mode of one face side: (X[7] = rho, p, v^i, the two transverse densitized field
// components; Bn, the normal one; Gamma) -> (U[7], F[7], c-, c+) of state_make, flux_of and
// speeds_of, contracted with the cotangents (Ub, Fb, cmb, cpb) in one backward sweep.  The
// speeds are the given outer roots xp, xm of the quartic (kind 0) or of the isotropic bound's
// quadratic (kind 1); their cotangents reach the coefficients through the implicit function
// theorem, d lambda = -(sum_k dc_k lambda^k) / Q'(lambda) (zero where Q' = 0).
template <int D>
DEV void side_vjp(const Geo& G, const double X[7], double Bn, double gam, int kind, double xp, double xm,
                  const double Ub[7], const double Fb[7], double cmb, double cpb, double Xb[7], double& Bnb,
                  double& gb) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  // forward sweep: the state (state_make)
  const double gfac = gam / (gam - 1.0);
  const double rho = X[0], p = X[1], v[3] = {X[2], X[3], X[4]};
  double vl[3];
  lower(G.g, v, vl);
  const double iW2 = 1.0 - (v[0] * vl[0] + v[1] * vl[1] + v[2] * vl[2]);
  const double W = inv_sqrt(iW2);
  const double is = recip(G.sqrtg), sg = G.sqrtg;
  double B[3];
  B[D] = Bn * is;
  B[t1] = X[5] * is;
  B[t2] = X[6] * is;
  double Bl[3];
  lower(G.g, B, Bl);
  const double B2 = B[0] * Bl[0] + B[1] * Bl[1] + B[2] * Bl[2];
  const double Bv = B[0] * vl[0] + B[1] * vl[1] + B[2] * vl[2];
  const double bsq = B2 * iW2 + Bv * Bv;
  const double rhoh = rho + gfac * p;
  // cotangents of the state's quantities
  double rhob = 0.0, pb = 0.0, vb[3] = {0.0, 0.0, 0.0}, vlb[3] = {0.0, 0.0, 0.0}, iW2b = 0.0, Wb = 0.0;
  double Bb[3] = {0.0, 0.0, 0.0}, Blb[3] = {0.0, 0.0, 0.0}, B2b = 0.0, Bvb = 0.0, bsqb = 0.0, rhohb = 0.0;
  double gamb = 0.0;
  // speeds (speeds_of): a = -lambda u^0 + u^D, bb = -lambda b^0 + b^D
  {
    const double alp = G.alp, ia = 1.0 / alp, ia2 = ia * ia, bD = G.beta[D];
    const double uD = W * (v[D] - bD * ia), u0 = W * ia;
    const double cs2 = gam * p / rhoh;
    const double G0 = G.gu[sym(D, D)] - bD * bD * ia2, G1 = -2.0 * bD * ia2, G2 = -ia2;
    const double a0 = uD, a1 = -u0;
    double a0b = 0.0, a1b = 0.0, cs2b = 0.0;
    if (kind == 1) {
      // roots of (1 - w2) a^2 - w2 G = qa l^2 + qb l + qc
      const double ih = 1.0 / (rhoh + bsq), cA2 = bsq * ih;
      const double w2 = cs2 + cA2 - cs2 * cA2, om = 1.0 - w2;
      const double qa = om * a1 * a1 - w2 * G2, qb = 2.0 * om * a0 * a1 - w2 * G1;
      double qab = 0.0, qbb = 0.0, qcb = 0.0;
      const double rr[2] = {xp, xm}, rb[2] = {cpb, cmb};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double dq = 2.0 * qa * rr[k] + qb;
        const double s = dq != 0.0 ? -rb[k] / dq : 0.0;
        qab += s * rr[k] * rr[k];
        qbb += s * rr[k];
        qcb += s;
      }
      const double omb = qab * a1 * a1 + 2.0 * qbb * a0 * a1 + qcb * a0 * a0;
      const double w2b = -(qab * G2 + qbb * G1 + qcb * G0) - omb;
      a1b = 2.0 * om * (qab * a1 + qbb * a0);
      a0b = 2.0 * om * (qbb * a1 + qcb * a0);
      cs2b = w2b * (1.0 - cA2);
      const double cA2b = w2b * (1.0 - cs2);
      bsqb += cA2b * rhoh * ih * ih;
      rhohb -= cA2b * bsq * ih * ih;
    } else {
      // quartic rho h (1 - cs2) a^4 - (rho h cs2 + b^2) a^2 G + cs2 bb^2 G
      const double b0 = W * Bv * ia, iW = 1.0 / W;
      const double bDc = (B[D] + alp * b0 * uD) * iW;
      const double A4 = rhoh * (1.0 - cs2), Bq = rhoh * cs2 + bsq, Cq = cs2;
      const double s0 = a0 * a0, s1 = 2.0 * a0 * a1, s2 = a1 * a1;
      const double q0 = bDc * bDc, q1 = -2.0 * bDc * b0, q2 = b0 * b0;
      const double r0 = -Bq * s0 + Cq * q0, r1 = -Bq * s1 + Cq * q1, r2 = -Bq * s2 + Cq * q2;
      const double c1 = A4 * 2.0 * s0 * s1 + r0 * G1 + r1 * G0;
      const double c2 = A4 * (s1 * s1 + 2.0 * s0 * s2) + r0 * G2 + r1 * G1 + r2 * G0;
      const double c3 = A4 * 2.0 * s1 * s2 + r1 * G2 + r2 * G1;
      const double c4 = A4 * s2 * s2 + r2 * G2;
      double cb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      const double rr[2] = {xp, xm}, rb[2] = {cpb, cmb};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double x = rr[k];
        const double dq = ((4.0 * c4 * x + 3.0 * c3) * x + 2.0 * c2) * x + c1;
        const double s = dq != 0.0 ? -rb[k] / dq : 0.0;
        cb[0] += s;
        cb[1] += s * x;
        cb[2] += s * x * x;
        cb[3] += s * x * x * x;
        cb[4] += s * x * x * x * x;
      }
      const double r0b = cb[0] * G0 + cb[1] * G1 + cb[2] * G2;
      const double r1b = cb[1] * G0 + cb[2] * G1 + cb[3] * G2;
      const double r2b = cb[2] * G0 + cb[3] * G1 + cb[4] * G2;
      const double A4b = cb[0] * s0 * s0 + 2.0 * cb[1] * s0 * s1 + cb[2] * (s1 * s1 + 2.0 * s0 * s2) +
                         2.0 * cb[3] * s1 * s2 + cb[4] * s2 * s2;
      const double s0b = 2.0 * A4 * (s0 * cb[0] + s1 * cb[1] + s2 * cb[2]) - Bq * r0b;
      const double s1b = 2.0 * A4 * (s0 * cb[1] + s1 * cb[2] + s2 * cb[3]) - Bq * r1b;
      const double s2b = 2.0 * A4 * (s0 * cb[2] + s1 * cb[3] + s2 * cb[4]) - Bq * r2b;
      const double Bqb = -(r0b * s0 + r1b * s1 + r2b * s2);
      const double Cqb = r0b * q0 + r1b * q1 + r2b * q2;
      const double q0b = Cq * r0b, q1b = Cq * r1b, q2b = Cq * r2b;
      a0b = 2.0 * (a0 * s0b + a1 * s1b);
      a1b = 2.0 * (a0 * s1b + a1 * s2b);
      const double bDcb = 2.0 * (bDc * q0b - b0 * q1b);
      double b0b = 2.0 * (b0 * q2b - bDc * q1b);
      rhohb += (1.0 - cs2) * A4b + cs2 * Bqb;
      cs2b = rhoh * (Bqb - A4b) + Cqb;
      bsqb += Bqb;
      // bDc = (B^D + alpha b^0 u^D) / W
      Bb[D] += bDcb * iW;
      b0b += bDcb * alp * uD * iW;
      a0b += bDcb * alp * b0 * iW;
      Wb -= bDcb * bDc * iW;
      // b^0 = W (B.v) / alpha
      Wb += b0b * Bv * ia;
      Bvb += b0b * W * ia;
    }
    // cs2 = Gamma p / rho h
    gamb += cs2b * p / rhoh;
    pb += cs2b * gam / rhoh;
    rhohb -= cs2b * cs2 / rhoh;
    // a0 = u^D = W (v^D - beta^D / alpha), a1 = -u^0 = -W / alpha
    Wb += a0b * (v[D] - bD * ia) - a1b * ia;
    vb[D] += a0b * W;
  }
  // conserved variables and fluxes (cons_of, flux_of)
  {
    const double alp = G.alp, as = alp * sg;
    const double vt[3] = {alp * v[0] - G.beta[0], alp * v[1] - G.beta[1], alp * v[2] - G.beta[2]};
    const double vtD = vt[D];
    const double z = rhoh * W * W, Dn = rho * W, zb = z + B2;
    double U[5];
    U[0] = sg * Dn;
#pragma unroll
    for (int j = 0; j < 3; ++j) U[1 + j] = sg * (zb * vl[j] - Bv * Bl[j]);
    U[4] = sg * (zb - p - 0.5 * (B2 * iW2 + Bv * Bv) - Dn);
    const double ptot = p + 0.5 * bsq, BD = B[D], m1 = BD * iW2, m2 = Bv * BD;
    double Ubar[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) Ubar[q] = Ub[q];
    double vtb[3] = {0.0, 0.0, 0.0}, ptotb = 0.0, m1b = 0.0, m2b = 0.0;
    // F0 = U0 vt^D, F_{1+j} = U_{1+j} vt^D - as (B_j m1 + v_j m2) (+ as ptot for j = D),
    // F4 = U4 vt^D + as (ptot v^D - m2)
    Ubar[0] += Fb[0] * vtD;
    vtb[D] += Fb[0] * U[0];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Ubar[1 + j] += Fb[1 + j] * vtD;
      vtb[D] += Fb[1 + j] * U[1 + j];
      Blb[j] -= as * m1 * Fb[1 + j];
      m1b -= as * Bl[j] * Fb[1 + j];
      vlb[j] -= as * m2 * Fb[1 + j];
      m2b -= as * vl[j] * Fb[1 + j];
    }
    ptotb += as * Fb[1 + D];
    Ubar[4] += Fb[4] * vtD;
    vtb[D] += Fb[4] * U[4];
    ptotb += as * v[D] * Fb[4];
    vb[D] += as * ptot * Fb[4];
    m2b -= as * Fb[4];
    // induction: F5 = Bt1 vt^D - BtD vt^t1, F6 = Bt2 vt^D - BtD vt^t2, U5 = Bt1, U6 = Bt2
    const double Bt1 = sg * B[t1], Bt2 = sg * B[t2], BtD = sg * BD;
    const double Bt1b = Fb[5] * vtD + Ubar[5], Bt2b = Fb[6] * vtD + Ubar[6];
    const double BtDb = -(Fb[5] * vt[t1] + Fb[6] * vt[t2]);
    vtb[D] += Fb[5] * Bt1 + Fb[6] * Bt2;
    vtb[t1] -= Fb[5] * BtD;
    vtb[t2] -= Fb[6] * BtD;
    Bb[t1] += sg * Bt1b;
    Bb[t2] += sg * Bt2b;
    Bb[D] += sg * BtDb + iW2 * m1b + Bv * m2b;
    iW2b += BD * m1b;
    Bvb += BD * m2b;
    pb += ptotb;
    bsqb += 0.5 * ptotb;
#pragma unroll
    for (int i = 0; i < 3; ++i) vb[i] += alp * vtb[i];
    // U0 = sg D, U_{1+j} = sg (zb v_j - (B.v) B_j), U4 = sg (zb - p - (B^2/W^2 + (B.v)^2) / 2 - D)
    const double Dnb = sg * (Ubar[0] - Ubar[4]);
    double zbb = sg * Ubar[4];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      zbb += sg * Ubar[1 + j] * vl[j];
      vlb[j] += sg * zb * Ubar[1 + j];
      Bvb -= sg * Ubar[1 + j] * Bl[j];
      Blb[j] -= sg * Bv * Ubar[1 + j];
    }
    pb -= sg * Ubar[4];
    B2b += zbb - 0.5 * sg * iW2 * Ubar[4];
    iW2b -= 0.5 * sg * B2 * Ubar[4];
    Bvb -= sg * Bv * Ubar[4];
    // zb = rho h W^2 + B^2, D = rho W
    rhohb += W * W * zbb;
    Wb += 2.0 * rhoh * W * zbb + rho * Dnb;
    rhob += W * Dnb;
  }
  // back through state_make
  double gfacb = p * rhohb;
  rhob += rhohb;
  pb += gfac * rhohb;
  B2b += iW2 * bsqb;
  iW2b += B2 * bsqb;
  Bvb += 2.0 * Bv * bsqb;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Bb[i] += vl[i] * Bvb + Bl[i] * B2b;
    vlb[i] += B[i] * Bvb;
    Blb[i] += B[i] * B2b;
  }
  double t[3];
  lower(G.g, Blb, t);
#pragma unroll
  for (int i = 0; i < 3; ++i) Bb[i] += t[i];
  iW2b -= 0.5 * W * W * W * Wb;
  // iW2 = 1 - v.vl
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    vb[i] -= vl[i] * iW2b;
    vlb[i] -= v[i] * iW2b;
  }
  lower(G.g, vlb, t);
  Xb[0] = rhob;
  Xb[1] = pb;
#pragma unroll
  for (int i = 0; i < 3; ++i) Xb[2 + i] = vb[i] + t[i];
  Xb[5] = Bb[t1] * is;
  Xb[6] = Bb[t2] * is;
  Bnb = Bb[D] * is;
  const double gm1 = gam - 1.0;
  gb = gamb - gfacb / (gm1 * gm1);
}

// ---------------------------------------------------------------------------------------
// Reconstruction (Sec. 3.3) at the face between cells i-1 and i from a[0..5] = a_{i-3..i+2}:
// L = right-face value of cell i-1, R = left-face value of cell i.
template <class T>
DEV T mm(T x, T y) {
  return (val(x) * val(y) > 0.0) ? copysign(fmin(fabs(x), fabs(y)), x) : T(0.0 * val(x));
}

// Monotonized-central slope of PPM (Colella-Woodward).
template <class T>
DEV T mc_slope(T am, T a0, T ap) {
  // both outcomes evaluated and selected: no branch, so a face kernel's stencil loads can all
  // be in flight before the first limiter runs
  T dl = a0 - am, dr = ap - a0;
  T dc = 0.5 * (ap - am);
  T lim = copysign(fmin(fabs(dc), 2.0 * fmin(fabs(dl), fabs(dr))), dc);
  return val(dl) * val(dr) > 0.0 ? lim : T(0.0 * val(dl));
}

// PPM cell parabola limited per Colella-Woodward; returns (left, right) face values of
// the cell with neighbour face values fl (c-1/2) and fr (c+1/2).
// The limiter's cases: local extremum (flat), or the parabola overshooting on the left or the right.
DEV void ppm_cases(double ac, double fl, double fr, bool& flat, bool& over_l, bool& over_r) {
  flat = (fr - ac) * (ac - fl) <= 0.0;
  const double dd = fr - fl;
  const double a6 = dd * (ac - 0.5 * (fl + fr));
  const double d2 = dd * dd * (1.0 / 6.0);
  over_l = a6 > d2;
  over_r = !over_l && -d2 > a6;
}

template <class T>
DEV void ppm_limit(T ac, T& fl, T& fr) {
  // branch-free form of: local extremum -> flat; else steepen the side the parabola overshoots
  bool flat, over_l, over_r;
  ppm_cases(val(ac), val(fl), val(fr), flat, over_l, over_r);
  T nl = 3.0 * ac - 2.0 * fr, nr = 3.0 * ac - 2.0 * fl;
  fl = flat ? ac : (over_l ? nl : fl);
  fr = flat ? ac : (over_r ? nr : fr);
}

// Transposes of the reconstructions' active branches (the adjoint's reverse sweep): each adds
// xb times the derivative of the face value with respect to each stencil value into ab.
// MC slope: the centred difference, twice the smaller one-sided difference, or zero at an extremum.
DEV void mc_slope_vjp(double am, double a0, double ap, double sb, double& gm, double& g0, double& gp) {
  const double dl = a0 - am, dr = ap - a0, dc = 0.5 * (ap - am);
  if (!(dl * dr > 0.0)) return;
  const double adl = fabs(dl), adr = fabs(dr);
  if (fabs(dc) <= 2.0 * fmin(adl, adr)) {
    gp += 0.5 * sb;
    gm -= 0.5 * sb;
  } else if (adl <= adr) {
    g0 += 2.0 * sb;
    gm -= 2.0 * sb;
  } else {
    gp += 2.0 * sb;
    g0 -= 2.0 * sb;
  }
}

// PPM value at the right face of the middle cell of a[0..4].
DEV void ppm_right_vjp(const double a[5], double xb, double ab[5]) {
  const double sixth = 1.0 / 6.0;
  const double s1 = mc_slope(a[0], a[1], a[2]), s2 = mc_slope(a[1], a[2], a[3]), s3 = mc_slope(a[2], a[3], a[4]);
  const double fl = 0.5 * (a[1] + a[2]) - (s2 - s1) * sixth;
  const double fr = 0.5 * (a[2] + a[3]) - (s3 - s2) * sixth;
  bool flat, over_l, over_r;
  ppm_cases(a[2], fl, fr, flat, over_l, over_r);
  double flb = 0.0, frb = 0.0;
  if (flat) ab[2] += xb;
  else if (over_r) {
    ab[2] += 3.0 * xb;
    flb = -2.0 * xb;
  } else frb = xb;
  ab[1] += 0.5 * flb;
  ab[2] += 0.5 * (flb + frb);
  ab[3] += 0.5 * frb;
  mc_slope_vjp(a[0], a[1], a[2], flb * sixth, ab[0], ab[1], ab[2]);
  mc_slope_vjp(a[1], a[2], a[3], (frb - flb) * sixth, ab[1], ab[2], ab[3]);
  mc_slope_vjp(a[2], a[3], a[4], -frb * sixth, ab[2], ab[3], ab[4]);
}

// WENO-Z (Borges et al. 2008) value at the right face of the middle cell of (m2..p2).
template <class T>
DEV T wenoz_face(T m2, T m1, T c0, T p1, T p2, double eps, double q) {
  const double t13 = 13.0 / 12.0;
  T e0 = m2 - 2.0 * m1 + c0, f0 = m2 - 4.0 * m1 + 3.0 * c0;
  T e1 = m1 - 2.0 * c0 + p1, f1 = m1 - p1;
  T e2 = c0 - 2.0 * p1 + p2, f2 = 3.0 * c0 - 4.0 * p1 + p2;
  T b0 = t13 * e0 * e0 + 0.25 * f0 * f0;
  T b1 = t13 * e1 * e1 + 0.25 * f1 * f1;
  T b2 = t13 * e2 * e2 + 0.25 * f2 * f2;
  T tau = fabs(b0 - b2);
  T r0 = tau / (b0 + eps), r1 = tau / (b1 + eps), r2 = tau / (b2 + eps);
  if (q != 1.0) {
    r0 = pow(r0, q);
    r1 = pow(r1, q);
    r2 = pow(r2, q);
  }
  T w0 = 0.1 * (1.0 + r0), w1 = 0.6 * (1.0 + r1), w2 = 0.3 * (1.0 + r2);
  T q0 = (2.0 * m2 - 7.0 * m1 + 11.0 * c0), q1 = (-m1 + 5.0 * c0 + 2.0 * p1), q2 = (2.0 * c0 + 5.0 * p1 - p2);
  return (w0 * q0 + w1 * q1 + w2 * q2) / (6.0 * (w0 + w1 + w2));
}

// A linear form sum_q c_q a_q over a 5-point stencil, with its value: the piecewise-linear
// reconstructions evaluated on it (selections follow the value) give their gradient exactly.
struct Lin5 {
  double v, c[5];
  DEV Lin5() = default;
  explicit DEV Lin5(double x) : v(x), c{0.0, 0.0, 0.0, 0.0, 0.0} {}
};
DEV double val(const Lin5& x) { return x.v; }
DEV Lin5 operator+(Lin5 a, const Lin5& b) {
  a.v += b.v;
#pragma unroll
  for (int q = 0; q < 5; ++q) a.c[q] += b.c[q];
  return a;
}
DEV Lin5 operator*(double s, Lin5 a) {
  a.v *= s;
#pragma unroll
  for (int q = 0; q < 5; ++q) a.c[q] *= s;
  return a;
}
DEV Lin5 operator*(Lin5 a, double s) { return s * a; }
DEV Lin5 operator-(const Lin5& a) { return -1.0 * a; }
DEV Lin5 operator-(const Lin5& a, const Lin5& b) { return a + (-1.0 * b); }
DEV Lin5 fabs(const Lin5& a) { return a.v < 0.0 ? -a : a; }
DEV Lin5 fmin(const Lin5& a, const Lin5& b) { return a.v <= b.v ? a : b; }
DEV Lin5 copysign(const Lin5& m, const Lin5& s) { return (::signbit(m.v) != ::signbit(s.v)) ? -m : m; }

// MP5 (Suresh & Huynh 1997; cited in Sec. 3.3) value at the right face of the middle cell of
// (m2..p2): the fifth-order interpolant, or, when it leaves the monotonicity-preserving range
// between c0 and c0 + minmod(p1 - c0, 4 (c0 - m1)), its median with the accuracy-preserving
// bounds built from the M4 curvatures.  The median is continuous across that test, so a
// rounding-level change of the interpolant never switches the result between branches.
template <class T>
DEV T tmin(T x, T y) { return val(y) < val(x) ? y : x; }
template <class T>
DEV T tmax(T x, T y) { return val(y) > val(x) ? y : x; }
template <class T>
DEV T minmod4(T w, T x, T y, T z) {
  const bool pos = val(w) > 0.0 && val(x) > 0.0 && val(y) > 0.0 && val(z) > 0.0;
  const bool neg = val(w) < 0.0 && val(x) < 0.0 && val(y) < 0.0 && val(z) < 0.0;
  T lo = tmin(tmin(w, x), tmin(y, z)), hi = tmax(tmax(w, x), tmax(y, z));
  return pos ? lo : (neg ? hi : T(0.0 * val(w)));
}

template <class T>
DEV T mp5_face(T m2, T m1, T c0, T p1, T p2) {
  const double alpha = 4.0;
  T f_or = (2.0 * m2 - 13.0 * m1 + 47.0 * c0 + 27.0 * p1 - 3.0 * p2) * (1.0 / 60.0);
  T f_mp = c0 + mm(p1 - c0, alpha * (c0 - m1));
  T d_m = m2 - 2.0 * m1 + c0, d_0 = m1 - 2.0 * c0 + p1, d_p = c0 - 2.0 * p1 + p2;
  T dr = minmod4(4.0 * d_0 - d_p, 4.0 * d_p - d_0, d_0, d_p);
  T dl = minmod4(4.0 * d_0 - d_m, 4.0 * d_m - d_0, d_0, d_m);
  T f_ul = c0 + alpha * (c0 - m1);
  T f_md = 0.5 * (c0 + p1) - 0.5 * dr;
  T f_lc = c0 + 0.5 * (c0 - m1) + (4.0 / 3.0) * dl;
  T f_min = tmax(tmin(tmin(c0, p1), f_md), tmin(tmin(c0, f_ul), f_lc));
  T f_max = tmin(tmax(tmax(c0, p1), f_md), tmax(tmax(c0, f_ul), f_lc));
  T lim = f_or + mm(f_min - f_or, f_max - f_or);
  return val(f_or - c0) * val(f_or - f_mp) <= 0.0 ? f_or : lim;
}

// ---------------------------------------------------------------------------------------
// Conservative-to-primitive recovery (Sec. 3.5) and atmosphere (Sec. 3.6).
struct C2PParams {
  double gam, rho_atm, k_atm, tol, wmax;
  int maxit, brent_maxit, method;
};

struct C2PIn {
  double D, S[3], tau, B[3], S2, B2, BS;
};

// Noble residuals (eqs. Noble2D momentum, Noble2D energy) with p(z, w) of the ideal gas
// and their Jacobian; solved by Newton with the 2x2 inverse.
DEV bool noble(const Geo& G, const C2PIn& c, const C2PParams& P, double z, double w, double out[5], int& iters) {
  const double gm = (P.gam - 1.0) / P.gam;
  const double wcap = 1.0 - 1.0 / (P.wmax * P.wmax);
  const double BS2 = c.BS * c.BS;
  bool ok = false;
  iters = 0;
  for (int it = 1; it <= P.maxit; ++it) {
    iters = it;
    double sw = sqrt(1.0 - w);
    double iz = 1.0 / z;
    double iz2 = iz * iz;
    double Bz = c.B2 + z;
    double p = gm * (z * (1.0 - w) - c.D * sw);
    double R1 = w * Bz * Bz - BS2 * (c.B2 + 2.0 * z) * iz2 - c.S2;
    double R2 = c.tau + c.D - 0.5 * c.B2 * (1.0 + w) + 0.5 * BS2 * iz2 - z + p;
    double J11 = 2.0 * Bz * (w + BS2 * iz2 * iz);
    double J12 = Bz * Bz;
    double J21 = -BS2 * iz2 * iz - 1.0 + gm * (1.0 - w);
    double J22 = -0.5 * c.B2 + gm * (-z + 0.5 * c.D / sw);
    double idet = 1.0 / (J11 * J22 - J12 * J21);
    double dz = (J12 * R2 - J22 * R1) * idet;
    double dw = (J21 * R1 - J11 * R2) * idet;
    z += dz;
    w = fmin(fmax(w + dw, 0.0), wcap);
    if (!(z > 0.0) || !isfinite(z) || !isfinite(w)) return false;
    if (fmax(fabs(dz) / z, fabs(dw)) < P.tol) {
      ok = true;
      break;
    }
  }
  if (!ok) return false;
  double W2 = 1.0 / (1.0 - w);
  double W = sqrt(W2);
  double rho = c.D / W;
  double eps = (z / (rho * W2) - 1.0) / P.gam;
  double p = (P.gam - 1.0) * rho * eps;
  if (!(eps >= 0.0) || !isfinite(p)) return false;
  double izb = 1.0 / (z + c.B2), fB = c.BS * izb / z;
  out[0] = rho;
  out[1] = p;
  out[2] = (G.gu[0] * c.S[0] + G.gu[1] * c.S[1] + G.gu[2] * c.S[2]) * izb + fB * c.B[0];
  out[3] = (G.gu[1] * c.S[0] + G.gu[3] * c.S[1] + G.gu[4] * c.S[2]) * izb + fB * c.B[1];
  out[4] = (G.gu[2] * c.S[0] + G.gu[4] * c.S[1] + G.gu[5] * c.S[2]) * izb + fB * c.B[2];
  return true;
}

// Palenzuela et al. master function in x = h W (eqs. Palenzuela qrst, Palenzuela Brent;
// the eps expression with t^2/x^2, see the oracle and design notes).
struct Palen {
  double q, r, s, t2, D, gam, iw2min;
};

DEV double palen_f(const Palen& P, double x, double& W, double& rho, double& eps, double& p) {
  double xs = x + P.s;
  double v2 = (P.r * x * x + P.t2 * (2.0 * x + P.s)) / (x * x * xs * xs);
  double iW2 = fmax(1.0 - v2, P.iw2min);
  W = 1.0 / sqrt(iW2);
  rho = P.D / W;
  eps = -1.0 + (x / W) * (1.0 - W * W) + W * (1.0 + P.q - P.s + 0.5 * (P.t2 / (x * x) + P.s * iW2));
  p = (P.gam - 1.0) * rho * eps;
  return x - (1.0 + eps + p / rho) * W;
}

// Brent's method (1973): bracketing with inverse quadratic / secant steps and bisection.
DEV bool palenzuela(const Geo& G, const C2PIn& c, const C2PParams& CP, double out[5]) {
  Palen P;
  P.D = c.D;
  P.q = c.tau / c.D;
  P.r = c.S2 / (c.D * c.D);
  P.s = c.B2 / c.D;
  P.t2 = c.BS * c.BS / (c.D * c.D * c.D);
  P.gam = CP.gam;
  P.iw2min = 1.0 / (CP.wmax * CP.wmax);
  double lo = fmax(1.0 + P.q - P.s, 1.0), hi = 2.0 + 2.0 * P.q - P.s;
  if (!(hi > lo)) return false;
  double W, rho, eps, p;
  double a = lo, b = hi;
  double fa = palen_f(P, a, W, rho, eps, p);
  double fb = palen_f(P, b, W, rho, eps, p);
  if (!isfinite(fa) || !isfinite(fb)) return false;
  if ((fa > 0.0 && fb > 0.0) || (fa < 0.0 && fb < 0.0)) return false;
  double cc = a, fc = fa, d = b - a, e = d;
  bool conv = false;
  for (int it = 0; it < CP.brent_maxit; ++it) {
    if ((fb > 0.0 && fc > 0.0) || (fb < 0.0 && fc < 0.0)) {
      cc = a;
      fc = fa;
      d = e = b - a;
    }
    if (fabs(fc) < fabs(fb)) {
      a = b; fa = fb;
      b = cc; fb = fc;
      cc = a; fc = fa;
    }
    double tol = 4.440892098500626e-16 * fabs(b);
    double m = 0.5 * (cc - b);
    if (fabs(m) <= tol || fb == 0.0) {
      conv = true;
      break;
    }
    if (fabs(e) >= tol && fabs(fa) > fabs(fb)) {
      double s = fb / fa, pp, qq;
      if (a == cc) {
        pp = 2.0 * m * s;
        qq = 1.0 - s;
      } else {
        double qa = fa / fc, r = fb / fc;
        pp = s * (2.0 * m * qa * (qa - r) - (b - a) * (r - 1.0));
        qq = (qa - 1.0) * (r - 1.0) * (s - 1.0);
      }
      if (pp > 0.0) qq = -qq; else pp = -pp;
      if (2.0 * pp < fmin(3.0 * m * qq - fabs(tol * qq), fabs(e * qq))) {
        e = d;
        d = pp / qq;
      } else {
        d = m;
        e = m;
      }
    } else {
      d = m;
      e = m;
    }
    a = b;
    fa = fb;
    b += (fabs(d) > tol) ? d : copysign(tol, m);
    fb = palen_f(P, b, W, rho, eps, p);
    if (!isfinite(fb)) return false;
  }
  if (!conv) return false;
  palen_f(P, b, W, rho, eps, p);
  if (!(eps >= 0.0) || !isfinite(p)) return false;
  double z = c.D * b;
  double izb = 1.0 / (z + c.B2), fB = c.BS * izb / z;
  out[0] = rho;
  out[1] = p;
  out[2] = (G.gu[0] * c.S[0] + G.gu[1] * c.S[1] + G.gu[2] * c.S[2]) * izb + fB * c.B[0];
  out[3] = (G.gu[1] * c.S[0] + G.gu[3] * c.S[1] + G.gu[4] * c.S[2]) * izb + fB * c.B[1];
  out[4] = (G.gu[2] * c.S[0] + G.gu[4] * c.S[1] + G.gu[5] * c.S[2]) * izb + fB * c.B[2];
  return true;
}

// Atmosphere state and its conserved variables (field kept).
DEV void atmo(const Geo& G, const double Bt[3], const C2PParams& P, double pr[5], double U[5]) {
  pr[0] = P.rho_atm;
  pr[1] = P.k_atm * pow(P.rho_atm, P.gam);
  pr[2] = pr[3] = pr[4] = 0.0;
  State S;
  state_make(G, pr, Bt, P.gam, S);
  cons_of(G, S, U);
}

// Undensitized c2p input (D, S_i, tau, B^i and the invariants) from densitized U and Btilde.
DEV void c2p_input(const Geo& G, const double U[5], const double Bt[3], C2PIn& c) {
  double is = 1.0 / G.sqrtg;
  c.D = U[0] * is;
  c.S[0] = U[1] * is;
  c.S[1] = U[2] * is;
  c.S[2] = U[3] * is;
  c.tau = U[4] * is;
  c.B[0] = Bt[0] * is;
  c.B[1] = Bt[1] * is;
  c.B[2] = Bt[2] * is;
  double Su[3];
  Su[0] = G.gu[0] * c.S[0] + G.gu[1] * c.S[1] + G.gu[2] * c.S[2];
  Su[1] = G.gu[1] * c.S[0] + G.gu[3] * c.S[1] + G.gu[4] * c.S[2];
  Su[2] = G.gu[2] * c.S[0] + G.gu[4] * c.S[1] + G.gu[5] * c.S[2];
  c.S2 = Su[0] * c.S[0] + Su[1] * c.S[1] + Su[2] * c.S[2];
  double Bl[3];
  lower(G.g, c.B, Bl);
  c.B2 = c.B[0] * Bl[0] + c.B[1] * Bl[1] + c.B[2] * Bl[2];
  c.BS = c.B[0] * c.S[0] + c.B[1] * c.S[1] + c.B[2] * c.S[2];
}

// Full recovery at a point.  U: densitized conserved (in/out), prev: warm start.
// zw_guess (optional): an initial (z, w) tried first by Noble's Newton iteration; if it does
// not converge, flag 32 is set and the plain warm/cold start follows.  iters: total Newton
// iterations.
// Whether previous primitives make a warm start for Noble's iteration: positive density,
// non-negative pressure, a speed below the cap, all finite.
DEV bool warm_usable(const Geo& G, const double prev[5], const C2PParams& P) {
  double vl[3], v[3] = {prev[2], prev[3], prev[4]};
  lower(G.g, v, vl);
  const double v2 = v[0] * vl[0] + v[1] * vl[1] + v[2] * vl[2];
  const double wcap = 1.0 - 1.0 / (P.wmax * P.wmax);
  return prev[0] > 0.0 && prev[1] >= 0.0 && v2 < wcap && isfinite(v2) && isfinite(prev[1]);
}

DEV uint32_t c2p_point(const Geo& G, double U[5], const double Bt[3], const double prev[5], const C2PParams& P,
                       double out[5], int& iters, const double* zw_guess = nullptr) {
  uint32_t fl = 0;
  iters = 0;
  bool nan_in = !(isfinite(U[0]) && isfinite(U[1]) && isfinite(U[2]) && isfinite(U[3]) && isfinite(U[4]));
  if (nan_in || !(U[0] >= G.sqrtg * P.rho_atm)) {
    fl = 4u | (nan_in ? 16u : 0u);
    atmo(G, Bt, P, out, U);
    return fl;
  }
  C2PIn c;
  c2p_input(G, U, Bt, c);
  // no field and Gamma <= 2: a state with tau <= 0 or S^2 beyond tau (tau + 2D) (by a relative 1e-10) is
  // not a physical state of the ideal gas (E^2 > S^2 + D^2 for every one); the solvers cannot succeed, so the
  // cell takes the failure branch at once, with the flags they would have set (Sec. 3.6)
  if (c.B2 <= 0.0 && P.gam <= 2.0 && (!(c.tau > 0.0) || c.S2 > (1.0 + 1e-10) * c.tau * (c.tau + 2.0 * c.D))) {
    fl = (P.method != 2 ? 1u | (zw_guess ? 32u : 0u) : 0u) | 8u | 4u;
    atmo(G, Bt, P, out, U);
    return fl;
  }
  bool ok = false;
  const double wcap = 1.0 - 1.0 / (P.wmax * P.wmax);
  if (P.method != 2) {
    if (zw_guess) {
      ok = noble(G, c, P, zw_guess[0], zw_guess[1], out, iters);
      if (!ok) fl |= 32u;
    }
    if (!ok) {
      // warm start from the previous primitives, cold start if they are unusable
      double vl[3], v[3] = {prev[2], prev[3], prev[4]};
      lower(G.g, v, vl);
      double v2 = v[0] * vl[0] + v[1] * vl[1] + v[2] * vl[2];
      double z0, w0;
      if (prev[0] > 0.0 && prev[1] >= 0.0 && v2 < wcap && isfinite(v2) && isfinite(prev[1])) {
        double rhoh = prev[0] + P.gam / (P.gam - 1.0) * prev[1];
        z0 = rhoh / (1.0 - v2);
        w0 = v2;
      } else {
        z0 = c.tau + c.D;
        double den = z0 + c.B2;
        w0 = fmin(c.S2 / (den * den), wcap);
      }
      int it2 = 0;
      ok = noble(G, c, P, z0, w0, out, it2);
      iters += it2;
      if (!ok) fl |= 1u;
    }
  }
  if (!ok && P.method != 1) {
    ok = palenzuela(G, c, P, out);
    if (ok && P.method == 0) fl |= 2u;
  }
  if (!ok) {
    fl |= 8u | 4u;
    atmo(G, Bt, P, out, U);
    return fl;
  }
  if (out[0] < P.rho_atm) {
    fl |= 4u;
    atmo(G, Bt, P, out, U);
  }
  return fl;
}

}  // namespace ax
