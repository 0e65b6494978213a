/*
 * mhd_oracle.cpp -- FP64 CPU oracle for the per-patch ideal-MHD update
 * (unsplit MUSCL-Hancock predictor, HLLD face fluxes, constrained transport with
 * edge EMFs from a four-state upwind composition).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct loops over whole padded
 * patches, one pass per step of the method, in the paper's order (§2.1: primitives,
 * slopes, half-step prediction, Riemann solvers, EMFs, conservative + CT update).
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg load it.  It shares
 * no source with the GPU library.
 *
 * The scalar type is a template parameter so the same passes run in
 *   double -- the reference result,
 *   Dual   -- forward-mode derivative at fixed dt (reference gradients),
 *   Cnt    -- counts the arithmetic of one update (algorithmic flops per cell),
 *   TrcT   -- double or x87 extended precision, plus a hash of every branch outcome
 *             (the branch signature; extended precision serves finite differences).
 *
 * Where the paper leaves a point open (limiter, predictor, EMF solver, CFL rule, floors,
 * guard width), the function that needs it states the reading it takes; each function
 * cites what it follows.
 */
#include "mhd_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

namespace {

/* ------------------------------------------------------------------ scalars */

struct Dual {
  double v, d;
  Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline Dual ssqrt(Dual a) {
  const double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}

struct OpCount { int64_t add, mul, div, sqrt, cmp; };
thread_local OpCount g_ops;
struct Cnt {
  double v;
  Cnt(double a = 0.0) : v(a) {}
};
inline Cnt operator+(Cnt a, Cnt b) { g_ops.add++; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { g_ops.add++; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { g_ops.mul++; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { g_ops.div++; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline bool operator<(Cnt a, Cnt b) { g_ops.cmp++; return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { g_ops.cmp++; return a.v > b.v; }
inline bool operator<=(Cnt a, Cnt b) { g_ops.cmp++; return a.v <= b.v; }
inline bool operator>=(Cnt a, Cnt b) { g_ops.cmp++; return a.v >= b.v; }
inline Cnt ssqrt(Cnt a) { g_ops.sqrt++; return Cnt(std::sqrt(a.v)); }

/* Traced value: plain arithmetic in R (double, or x87 extended long double), and every
 * comparison folds its outcome into a running hash, so two runs that take the same
 * branches everywhere (limiter cases, min/max and |.| choices, HLLD regions and
 * degeneracy switch, floors) end with the same hash.  Used to check that the two ends of
 * a finite difference sit on one smooth branch of the update. */
thread_local uint64_t g_sig;
inline bool note(bool b) {
  g_sig = (g_sig ^ (b ? 0x9e3779b97f4a7c15ull : 0x6a09e667f3bcc909ull)) * 0x100000001b3ull;
  return b;
}
template <class R>
struct TrcT {
  R v;
  TrcT(R a = R(0)) : v(a) {}
  friend TrcT operator+(TrcT a, TrcT b) { return TrcT(a.v + b.v); }
  friend TrcT operator-(TrcT a, TrcT b) { return TrcT(a.v - b.v); }
  friend TrcT operator*(TrcT a, TrcT b) { return TrcT(a.v * b.v); }
  friend TrcT operator/(TrcT a, TrcT b) { return TrcT(a.v / b.v); }
  friend TrcT operator-(TrcT a) { return TrcT(-a.v); }
  friend bool operator<(TrcT a, TrcT b) { return note(a.v < b.v); }
  friend bool operator>(TrcT a, TrcT b) { return note(a.v > b.v); }
  friend bool operator<=(TrcT a, TrcT b) { return note(a.v <= b.v); }
  friend bool operator>=(TrcT a, TrcT b) { return note(a.v >= b.v); }
  friend TrcT ssqrt(TrcT a) { return TrcT(std::sqrt(a.v)); }
  friend double val(const TrcT& x) { return double(x.v); }
};

inline double ssqrt(double a) { return std::sqrt(a); }
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double val(const Cnt& x) { return x.v; }

template <class S> inline S smin(S a, S b) { return (b < a) ? b : a; }
template <class S> inline S smax(S a, S b) { return (a < b) ? b : a; }
template <class S> inline S sabs(S a) { return (a < S(0.0)) ? -a : a; }

/* --------------------------------------------------------------- building blocks */

/* Fast magnetosonic speed along a direction whose field component is bn (ideal MHD,
 * mu_0 = 1 as in the energy relation of §2.1).  The radicand is written as
 * (a^2-b^2)^2 + 4 a^2 b_perp^2, equal to (a^2+b^2)^2 - 4 a^2 b_n^2 without cancellation. */
template <class S>
S cfast(S r, S p, S bn, S bt1, S bt2, double gam) {
  const S a2 = gam * p / r;
  const S bt = bt1 * bt1 + bt2 * bt2;
  const S b2 = (bn * bn + bt) / r;
  const S bp2 = bt / r;
  const S d = a2 - b2;
  const S rad = d * d + 4.0 * a2 * bp2;
  return ssqrt(0.5 * (a2 + b2 + ssqrt(rad)));
}

/* Slope limiter of the MUSCL reconstruction (§2.1, "The MUSCL Scheme": the choice of
 * slope estimate suppresses oscillations).  0 = monotonised central, 1 = minmod. */
template <class S>
S limiter(S dl, S dr, int type) {
  if (dl * dr <= S(0.0)) return S(0.0);
  const S al = sabs(dl), ar = sabs(dr);
  S m;
  if (type == 1)
    m = smin(al, ar);
  else
    m = smin(2.0 * smin(al, ar), 0.5 * sabs(dl + dr));
  return (dl > S(0.0)) ? m : -m;
}

/* HLLD flux (§2.1 "HLLD Solver", Fig. 1: six regions separated by S_L, S*_L, S_M, S*_R,
 * S_R, after Miyoshi & Kusano 2005).  Face-normal frame: (rho, u_n, u_t1, u_t2, p, B_n,
 * B_t1, B_t2); B_n is shared by both sides.  Returns (rho, m_n, m_t1, m_t2, E) fluxes of
 * the x-flux vector of eq:MHD_vector written in the face frame. */
template <class S>
void hlld(const S L[8], const S R[8], const mhd_oracle_params& P, S F[5], int* region,
          double* fan_speeds = nullptr, double (*fan_states)[8] = nullptr) {
  const double gam = P.gamma;
  const S bn = L[5];
  const S rl = L[0], ul = L[1], vl = L[2], wl = L[3], pl = L[4], byl = L[6], bzl = L[7];
  const S rr = R[0], ur = R[1], vr = R[2], wr = R[3], pr = R[4], byr = R[6], bzr = R[7];

  const S b2l = bn * bn + byl * byl + bzl * bzl;
  const S b2r = bn * bn + byr * byr + bzr * bzr;
  const S ptl = pl + 0.5 * b2l, ptr = pr + 0.5 * b2r;  // total pressure P_gas + P_mag
  const S el = pl / (gam - 1.0) + 0.5 * rl * (ul * ul + vl * vl + wl * wl) + 0.5 * b2l;
  const S er = pr / (gam - 1.0) + 0.5 * rr * (ur * ur + vr * vr + wr * wr) + 0.5 * b2r;

  // outer wave-speed estimates
  const S cfl = cfast(rl, pl, bn, byl, bzl, gam);
  const S cfr = cfast(rr, pr, bn, byr, bzr, gam);
  const S cmx = smax(cfl, cfr);
  const S sl = smin(ul, ur) - cmx;
  const S sr = smax(ul, ur) + cmx;

  // fluxes of the outer states (eq:MHD_vector with P = total pressure)
  const S ubl = ul * bn + vl * byl + wl * bzl;
  const S ubr = ur * bn + vr * byr + wr * bzr;
  const S FL[5] = {rl * ul, rl * ul * ul + ptl - bn * bn, rl * vl * ul - byl * bn,
                   rl * wl * ul - bzl * bn, ul * (el + ptl) - bn * ubl};
  const S FR[5] = {rr * ur, rr * ur * ur + ptr - bn * bn, rr * vr * ur - byr * bn,
                   rr * wr * ur - bzr * bn, ur * (er + ptr) - bn * ubr};

  // middle (contact) speed and total pressure of the star regions
  const S sdl = sl - ul, sdr = sr - ur;
  const S den = sdr * rr - sdl * rl;
  const S sm = (sdr * rr * ur - sdl * rl * ul - ptr + ptl) / den;
  const S pts = (sdr * rr * ptl - sdl * rl * ptr + rl * rr * sdr * sdl * (ur - ul)) / den;

  // single-star states on each side; tangential components switch to the outer
  // values where the star-state denominator degenerates
  struct Star { S r, v, w, by, bz, e, ub; };
  auto star = [&](S r, S u, S v, S w, S by, S bz, S e, S pt, S ub, S s, S sd) {
    Star o;
    o.r = r * sd / (s - sm);
    const S dd = r * sd * (s - sm) - bn * bn;
    const S ref = r * sd * sd + bn * bn;
    if (sabs(dd) > P.eps_deg * ref) {
      const S tv = bn * (sm - u) / dd;
      const S tb = (r * sd * sd - bn * bn) / dd;
      o.v = v - by * tv;
      o.w = w - bz * tv;
      o.by = by * tb;
      o.bz = bz * tb;
    } else {
      o.v = v; o.w = w; o.by = by; o.bz = bz;
    }
    o.ub = sm * bn + o.v * o.by + o.w * o.bz;
    o.e = (sd * e - pt * u + pts * sm + bn * (ub - o.ub)) / (s - sm);
    return o;
  };
  const Star stl = star(rl, ul, vl, wl, byl, bzl, el, ptl, ubl, sl, sdl);
  const Star str = star(rr, ur, vr, wr, byr, bzr, er, ptr, ubr, sr, sdr);

  // Alfven waves and the double-star state
  const S srl = ssqrt(stl.r), srr = ssqrt(str.r);
  const S ssl = sm - sabs(bn) / srl;
  const S ssr = sm + sabs(bn) / srr;
  const S sgn = (bn < S(0.0)) ? S(-1.0) : S(1.0);
  const S ssum = srl + srr;
  const S vss = (srl * stl.v + srr * str.v + (str.by - stl.by) * sgn) / ssum;
  const S wss = (srl * stl.w + srr * str.w + (str.bz - stl.bz) * sgn) / ssum;
  const S byss = (srl * str.by + srr * stl.by + srl * srr * (str.v - stl.v) * sgn) / ssum;
  const S bzss = (srl * str.bz + srr * stl.bz + srl * srr * (str.w - stl.w) * sgn) / ssum;
  const S ubss = sm * bn + vss * byss + wss * bzss;
  const S essl = stl.e - srl * (stl.ub - ubss) * sgn;
  const S essr = str.e + srr * (str.ub - ubss) * sgn;

  // conserved states of each region and the region fluxes F* = F + S (U* - U), etc.
  const S UL[5] = {rl, rl * ul, rl * vl, rl * wl, el};
  const S UR[5] = {rr, rr * ur, rr * vr, rr * wr, er};
  const S UsL[5] = {stl.r, stl.r * sm, stl.r * stl.v, stl.r * stl.w, stl.e};
  const S UsR[5] = {str.r, str.r * sm, str.r * str.v, str.r * str.w, str.e};
  const S UssL[5] = {stl.r, stl.r * sm, stl.r * vss, stl.r * wss, essl};
  const S UssR[5] = {str.r, str.r * sm, str.r * vss, str.r * wss, essr};
  S FsL[5], FsR[5], FssL[5], FssR[5];
  for (int m = 0; m < 5; ++m) {
    FsL[m] = FL[m] + sl * (UsL[m] - UL[m]);
    FsR[m] = FR[m] + sr * (UsR[m] - UR[m]);
    FssL[m] = FsL[m] + ssl * (UssL[m] - UsL[m]);
    FssR[m] = FsR[m] + ssr * (UssR[m] - UsR[m]);
  }

  // region containing the face (first test that holds wins)
  const S* sel;
  int reg;
  if (sl > S(0.0)) { sel = FL; reg = 0; }
  else if (ssl >= S(0.0)) { sel = FsL; reg = 1; }
  else if (sm >= S(0.0)) { sel = FssL; reg = 2; }
  else if (ssr >= S(0.0)) { sel = FssR; reg = 3; }
  else if (sr >= S(0.0)) { sel = FsR; reg = 4; }
  else { sel = FR; reg = 5; }
  for (int m = 0; m < 5; ++m) F[m] = sel[m];
  if (region) *region = reg;
  // optional record of the wave fan (speeds S_L, S*_L, S_M, S*_R, S_R, the total pressure
  // of the four intermediate states, and the states U*_L, U**_L, U**_R, U*_R as (rho, m_n,
  // m_t1, m_t2, E, B_n, B_t1, B_t2))
  if (fan_speeds) {
    const S sp[6] = {sl, ssl, sm, ssr, sr, pts};
    for (int k = 0; k < 6; ++k) fan_speeds[k] = val(sp[k]);
  }
  if (fan_states) {
    const S* U4[4] = {UsL, UssL, UssR, UsR};
    const S bt[4][2] = {{stl.by, stl.bz}, {byss, bzss}, {byss, bzss}, {str.by, str.bz}};
    for (int k = 0; k < 4; ++k) {
      for (int m = 0; m < 5; ++m) fan_states[k][m] = val(U4[k][m]);
      fan_states[k][5] = val(bn);
      fan_states[k][6] = val(bt[k][0]);
      fan_states[k][7] = val(bt[k][1]);
    }
  }
}

/* Edge EMF from the four predicted corner states around an edge along e (§2.1,
 * "Constrained transport and 2D-extension": corner values LB/RB/LT/RT regrouped as
 * SW/SE/NW/NE, Fig. 3).  Composition of two one-dimensional HLL fluxes of the
 * transverse field with outer speeds bounded over the four states.  (a,b,e) cyclic;
 * W = low a, E = high a, S = low b, N = high b.  EMF_e = u_a B_b - u_b B_a. */
template <class S>
S uct(const S SW[8], const S SE[8], const S NW[8], const S NE[8], int e,
      const mhd_oracle_params& P) {
  const int a = (e + 1) % 3, b = (e + 2) % 3;
  const S* st[4] = {SW, SE, NW, NE};
  S em[4];
  S apa = S(0.0), ama = S(0.0), apb = S(0.0), amb = S(0.0);
  for (int s = 0; s < 4; ++s) {
    const S* W = st[s];
    em[s] = W[1 + a] * W[5 + b] - W[1 + b] * W[5 + a];
    const S cfa = cfast(W[0], W[4], W[5 + a], W[5 + b], W[5 + e], P.gamma);
    const S cfb = cfast(W[0], W[4], W[5 + b], W[5 + e], W[5 + a], P.gamma);
    apa = smax(apa, W[1 + a] + cfa);
    ama = smax(ama, cfa - W[1 + a]);
    apb = smax(apb, W[1 + b] + cfb);
    amb = smax(amb, cfb - W[1 + b]);
  }
  const double tiny = 1e-300;
  const S da = smax(apa + ama, S(tiny));
  const S db = smax(apb + amb, S(tiny));
  const S avg = (apa * apb * em[0] + apa * amb * em[2] + ama * apb * em[1] + ama * amb * em[3]) /
                (da * db);
  const S difa = apa * ama / da * (SE[5 + b] - SW[5 + b]);  // B_b^E - B_b^W
  const S difb = apb * amb / db * (NW[5 + a] - SW[5 + a]);  // B_a^N - B_a^S
  return avg - difa + difb;
}

/* Wave fan of the one-dimensional HLLD problem at a face (§2.1 "HLLD Solver", Fig. 1; Miyoshi
 * & Kusano 2005), as the edge EMF below needs it: the five wave speeds, and per side the
 * single-star density, its square root and the two factors of the single-star relations
 * B*_t = B_t tb and u*_t = u_t - B_t tv, which hold for either transverse component (1 and 0
 * where the star denominator degenerates, the switch of reading R6).  Each side is given as
 * (rho, u_n, p, B_t1, B_t2) with the shared normal field bn.  The same formulas as in hlld(). */
template <class S>
struct Fan {
  S bn, sgn, sl, sr, sm, ssl, ssr;
  S un[2], rs[2], sq[2], tb[2], tv[2];
};

template <class S>
Fan<S> hlld_fan(S bn, const S lo[5], const S hi[5], const mhd_oracle_params& P) {
  const double gam = P.gamma;
  Fan<S> f;
  f.bn = bn;
  const S* side[2] = {lo, hi};
  S pt[2], cf[2];
  for (int k = 0; k < 2; ++k) {
    const S* q = side[k];
    f.un[k] = q[1];
    pt[k] = q[2] + 0.5 * (bn * bn + q[3] * q[3] + q[4] * q[4]);
    cf[k] = cfast(q[0], q[2], bn, q[3], q[4], gam);
  }
  const S cmx = smax(cf[0], cf[1]);
  f.sl = smin(lo[1], hi[1]) - cmx;
  f.sr = smax(lo[1], hi[1]) + cmx;
  const S sdl = f.sl - lo[1], sdr = f.sr - hi[1];
  const S den = sdr * hi[0] - sdl * lo[0];
  f.sm = (sdr * hi[0] * hi[1] - sdl * lo[0] * lo[1] - pt[1] + pt[0]) / den;
  const S spd[2] = {f.sl, f.sr}, sd[2] = {sdl, sdr};
  for (int k = 0; k < 2; ++k) {
    const S r = side[k][0], u = side[k][1];
    f.rs[k] = r * sd[k] / (spd[k] - f.sm);
    const S dd = r * sd[k] * (spd[k] - f.sm) - bn * bn;
    const S ref = r * sd[k] * sd[k] + bn * bn;
    if (sabs(dd) > P.eps_deg * ref) {
      f.tv[k] = bn * (f.sm - u) / dd;
      f.tb[k] = (r * sd[k] * sd[k] - bn * bn) / dd;
    } else {
      f.tv[k] = S(0.0);
      f.tb[k] = S(1.0);
    }
    f.sq[k] = ssqrt(f.rs[k]);
  }
  f.ssl = f.sm - sabs(bn) / f.sq[0];
  f.ssr = f.sm + sabs(bn) / f.sq[1];
  f.sgn = (bn < S(0.0)) ? S(-1.0) : S(1.0);
  return f;
}

/* HLLD flux along the face normal of one transverse field component B_t, from the pair
 * (u_t, B_t) of that component on each side: u_n B_t - B_n u_t in the outer regions; across
 * each wave the flux jumps by the wave speed times the jump of B_t (F* = F + S (B*_t - B_t),
 * F** = F* + S* (B**_t - B*_t)), with the single-star values of the fan's relations and the
 * double-star field of Miyoshi & Kusano (both sides' star values weighted by the square
 * roots of the star densities, plus the velocity jump).  Region order of hlld(). */
template <class S>
S hlld_bt_flux(const Fan<S>& f, S vl, S bl, S vr, S br) {
  const S Fl = f.un[0] * bl - f.bn * vl;
  const S Fr = f.un[1] * br - f.bn * vr;
  const S bsl = bl * f.tb[0], bsr = br * f.tb[1];
  const S vsl = vl - bl * f.tv[0], vsr = vr - br * f.tv[1];
  const S bss = (f.sq[0] * bsr + f.sq[1] * bsl + f.sq[0] * f.sq[1] * (vsr - vsl) * f.sgn) /
                (f.sq[0] + f.sq[1]);
  const S Fsl = Fl + f.sl * (bsl - bl);
  const S Fsr = Fr + f.sr * (bsr - br);
  if (f.sl > S(0.0)) return Fl;
  if (f.ssl >= S(0.0)) return Fsl;
  if (f.sm >= S(0.0)) return Fsl + f.ssl * (bss - bsl);
  if (f.ssr >= S(0.0)) return Fsr + f.ssr * (bss - bsr);
  if (f.sr >= S(0.0)) return Fsr;
  return Fr;
}

/* The transverse-field flux of a fan is linear in the four values (u_t, B_t) of the two
 * sides (the fan's speeds and factors do not depend on them once the states are given), so
 * it equals A_lo B_t,lo + A_hi B_t,hi + C_lo u_t,lo + C_hi u_t,hi.  The coefficients are
 * read off by evaluating the flux on unit values.  The velocity coefficients carry the
 * factor -B_n: w_k = -C_k / B_n are the weights with which the fan advects the transverse
 * velocity (w_lo + w_hi = 1; for B_n = 0 the side of the contact: (1, 0) if S_M >= 0). */
template <class S>
void hlld_bt_coefs(const Fan<S>& f, S A[2], S w[2]) {
  const S z = S(0.0), one = S(1.0);
  A[0] = hlld_bt_flux(f, z, one, z, z);
  A[1] = hlld_bt_flux(f, z, z, z, one);
  if (sabs(f.bn) > S(0.0)) {
    w[0] = -hlld_bt_flux(f, one, z, z, z) / f.bn;
    w[1] = -hlld_bt_flux(f, z, z, one, z) / f.bn;
  } else {
    w[0] = (f.sm >= S(0.0)) ? one : z;
    w[1] = one - w[0];
  }
}

/* Edge EMF with the HLLD wave fan (UCT-HLLD, reading R21; §2.1 "Constrained transport and
 * 2D-extension of the HLLD solver", Fig. 3).  The four corner states around an edge along e
 * pose four one-dimensional HLLD problems: along a on the rows S (SW|SE) and N (NW|NE), whose
 * normal field is that row's B_a, and along b on the columns W (SW|NW) and E (SE|NE), whose
 * normal field is that column's B_b.  EMF_e = u_a B_b - u_b B_a is the a-flux of B_b and minus
 * the b-flux of B_a.  The EMF takes the field part (the B_b terms) of the a-problems' fluxes
 * and minus the field part (the B_a terms) of the b-problems' fluxes, the velocity part of
 * each being carried by the other direction's problems:
 *   - the velocity weights of the two rows (a-problems) averaged over the rows, and those of
 *     the two columns averaged over the columns, give a first upwind weight per column and
 *     per row;
 *   - the rows' field parts are combined with the columns' velocity weights for those rows,
 *     averaged over the columns with the first weights per column; the columns' field parts
 *     likewise with the rows' velocity weights, averaged over the rows.
 * With data that vary only along a this is exactly the HLLD a-flux of B_b (the b-problems
 * then have equal sides, whose field coefficients add up to u_b, so their part becomes the
 * a-problem's velocity terms), symmetrically along b; with flow supersonic along +a (or -a) it
 * is exactly minus the HLLD b-flux of B_a of the column W (or E), symmetrically along b. */
template <class S>
S uct_hlld(const S SW[8], const S SE[8], const S NW[8], const S NE[8], int e,
           const mhd_oracle_params& P) {
  const int a = (e + 1) % 3, b = (e + 2) % 3;
  // one-dimensional problem along n between corner states lo and hi: (rho, u_n, p, B_t1,
  // B_t2) with (n, t1, t2) cyclic, normal field from lo (it is shared by the two sides)
  auto coefs = [&](const S* lo, const S* hi, int n, S A[2], S w[2]) {
    const int t1 = (n + 1) % 3, t2 = (n + 2) % 3;
    const S ql[5] = {lo[0], lo[1 + n], lo[4], lo[5 + t1], lo[5 + t2]};
    const S qh[5] = {hi[0], hi[1 + n], hi[4], hi[5 + t1], hi[5 + t2]};
    hlld_bt_coefs(hlld_fan(lo[5 + n], ql, qh, P), A, w);
  };
  S Ar[2][2], wr[2][2], Ac[2][2], wc[2][2];  // [row S, N] along a; [column W, E] along b
  coefs(SW, SE, a, Ar[0], wr[0]);
  coefs(NW, NE, a, Ar[1], wr[1]);
  coefs(SW, NW, b, Ac[0], wc[0]);
  coefs(SE, NE, b, Ac[1], wc[1]);
  // first upwind weights: per column from the rows, per row from the columns
  S col1[2], row1[2];
  for (int k = 0; k < 2; ++k) {
    col1[k] = 0.5 * (wr[0][k] + wr[1][k]);
    row1[k] = 0.5 * (wc[0][k] + wc[1][k]);
  }
  // weight of each row's field part (the columns' velocity weights for that row) and of each
  // column's field part (the rows' velocity weights for that column)
  S wrow[2], wcol[2];
  for (int k = 0; k < 2; ++k) {
    wrow[k] = col1[0] * wc[0][k] + col1[1] * wc[1][k];
    wcol[k] = row1[0] * wr[0][k] + row1[1] * wr[1][k];
  }
  const S BbW = SW[5 + b], BbE = SE[5 + b], BaS = SW[5 + a], BaN = NW[5 + a];
  S fa = S(0.0), fb = S(0.0);
  for (int k = 0; k < 2; ++k) {
    fa = fa + wrow[k] * (Ar[k][0] * BbW + Ar[k][1] * BbE);
    fb = fb + wcol[k] * (Ac[k][0] * BaS + Ac[k][1] * BaN);
  }
  return fa - fb;
}

/* Time derivative of the primitive variables (rho, u, p, B) of ideal MHD, used for the
 * forward-Euler half-step of the MUSCL predictor (§2.1 "The MUSCL Scheme").  The
 * u(div B) term of the induction equation is dropped (div B = 0 form). */
template <class S>
void dqdt_prim(const S q[8], const S D[3][8], const int act[3], double gam, S out[8]) {
  const S rho = q[0], p = q[4];
  const S u[3] = {q[1], q[2], q[3]};
  const S B[3] = {q[5], q[6], q[7]};
  S divu = S(0.0), adr = S(0.0), adp = S(0.0);
  for (int d = 0; d < 3; ++d) {
    if (!act[d]) continue;
    divu = divu + D[d][1 + d];
    adr = adr + u[d] * D[d][0];
    adp = adp + u[d] * D[d][4];
  }
  out[0] = -(adr + rho * divu);
  out[4] = -(adp + gam * p * divu);
  for (int i = 0; i < 3; ++i) {
    S adv = S(0.0), tens = S(0.0), strt = S(0.0), advb = S(0.0), grad = S(0.0);
    for (int d = 0; d < 3; ++d) {
      if (!act[d]) continue;
      adv = adv + u[d] * D[d][1 + i];
      tens = tens + B[d] * D[d][5 + i];
      strt = strt + B[d] * D[d][1 + i];
      advb = advb + u[d] * D[d][5 + i];
    }
    if (act[i]) grad = D[i][4] + (B[0] * D[i][5] + B[1] * D[i][6] + B[2] * D[i][7]);
    out[1 + i] = -adv - (grad - tens) / rho;
    out[5 + i] = strt - advb - B[i] * divu;
  }
}

/* ------------------------------------------------------------------ patch geometry */

struct Geom {
  int n[3], N[3], g, act[3];
  long st[3], off[3], Nc;
  bool init(const int32_t nn[3], int gg) {
    if (gg < 3) return false;  // the stencil reaches 2 cells down and 3 faces up
    g = gg;
    for (int d = 0; d < 3; ++d) {
      if (nn[d] < 1) return false;
      n[d] = nn[d];
      act[d] = nn[d] > 1;
      if (act[d] && nn[d] < gg) return false;  // guards come from one neighbour deep
      N[d] = act[d] ? nn[d] + 2 * gg : 1;
    }
    st[0] = 1;
    st[1] = N[0];
    st[2] = (long)N[0] * N[1];
    Nc = st[2] * N[2];
    for (int d = 0; d < 3; ++d) off[d] = act[d] ? st[d] : 0;
    return true;
  }
};

/* index box: active direction [lo, N + hi), collapsed direction [0, 1) */
struct Box { int lo[3], hi[3]; };
inline Box mkbox(const Geom& G, const int lo[3], const int hi[3]) {
  Box b;
  for (int d = 0; d < 3; ++d) {
    b.lo[d] = G.act[d] ? lo[d] : 0;
    b.hi[d] = G.act[d] ? G.N[d] + hi[d] : 1;
  }
  return b;
}
inline Box mkbox(const Geom& G, int lo, int hi) {
  const int l[3] = {lo, lo, lo}, h[3] = {hi, hi, hi};
  return mkbox(G, l, h);
}
/* optional record of the arithmetic of every box pass (op-counting runs only):
 * accumulates sum over passes of ops / items, i.e. the work per item of each pass */
thread_local bool g_rec = false;
thread_local double g_per_item[5];

template <class F>
inline void each(const Geom& G, const Box& b, F f) {
  const OpCount o0 = g_ops;
  long items = 0;
  for (int k = b.lo[2]; k < b.hi[2]; ++k)
    for (int j = b.lo[1]; j < b.hi[1]; ++j)
      for (int i = b.lo[0]; i < b.hi[0]; ++i) {
        f((long)i + G.st[1] * j + G.st[2] * k);
        ++items;
      }
  if (g_rec && items > 0) {
    g_per_item[0] += double(g_ops.add - o0.add) / items;
    g_per_item[1] += double(g_ops.mul - o0.mul) / items;
    g_per_item[2] += double(g_ops.div - o0.div) / items;
    g_per_item[3] += double(g_ops.sqrt - o0.sqrt) / items;
    g_per_item[4] += double(g_ops.cmp - o0.cmp) / items;
  }
}

/* ------------------------------------------------------------------ one patch update */

template <class S>
struct Stepper {
  const Geom& G;
  const mhd_oracle_params& P;
  const double dt;
  double dx[3];
  int64_t nfloor[3] = {0, 0, 0};   // activations in cell primitives, face states, corner states
  int site = 0;
  std::vector<S> q[8], dq[3][8], dbf[3][3], en[3], bh[3], qt[8], fl[3][5], emf[3];

  Stepper(const Geom& g, const mhd_oracle_params& p, double dt_, const double dx_[3])
      : G(g), P(p), dt(dt_) {
    for (int d = 0; d < 3; ++d) dx[d] = dx_[d];
    const S nan = S(std::numeric_limits<double>::quiet_NaN());
    auto alloc = [&](std::vector<S>& v) { v.assign(G.Nc, nan); };
    for (int m = 0; m < 8; ++m) { alloc(q[m]); alloc(qt[m]); }
    for (int d = 0; d < 3; ++d) {
      for (int m = 0; m < 8; ++m) alloc(dq[d][m]);
      for (int e = 0; e < 3; ++e) alloc(dbf[d][e]);
      for (int m = 0; m < 5; ++m) alloc(fl[d][m]);
      alloc(en[d]); alloc(bh[d]); alloc(emf[d]);
    }
  }

  S floor_rho(S r) {
    if (r < S(P.rho_floor)) { ++nfloor[site]; return S(P.rho_floor); }
    return r;
  }
  S floor_p(S p) {
    if (p < S(P.p_floor)) { ++nfloor[site]; return S(P.p_floor); }
    return p;
  }
  const S* fld(const S* U, int m) const { return U + (long)m * G.Nc; }

  /* 1. conserved -> primitive (§2.1 "The MUSCL Scheme": density, velocities, pressure,
   * magnetic field); cell-centred B is the mean of the two face values (Fig. 2); the
   * pressure follows the adiabatic energy relation of §2.1. */
  void prims(const S* U) {
    const double gm1 = P.gamma - 1.0;
    site = 0;
    each(G, mkbox(G, 0, -1), [&](long c) {
      const S rho = floor_rho(fld(U, 0)[c]);
      const S u = fld(U, 1)[c] / rho, v = fld(U, 2)[c] / rho, w = fld(U, 3)[c] / rho;
      const S bx = 0.5 * (fld(U, 5)[c] + fld(U, 5)[c + G.off[0]]);
      const S by = 0.5 * (fld(U, 6)[c] + fld(U, 6)[c + G.off[1]]);
      const S bz = 0.5 * (fld(U, 7)[c] + fld(U, 7)[c + G.off[2]]);
      const S ke = 0.5 * rho * (u * u + v * v + w * w);
      const S me = 0.5 * (bx * bx + by * by + bz * bz);
      const S p = floor_p(gm1 * (fld(U, 4)[c] - ke - me));
      q[0][c] = rho; q[1][c] = u; q[2][c] = v; q[3][c] = w;
      q[4][c] = p; q[5][c] = bx; q[6][c] = by; q[7][c] = bz;
    });
  }

  /* 2. limited slopes of every primitive per active direction; the slope of the
   * cell-centred normal field is the exact face difference.  Transverse slopes of the
   * face-centred field, limited among faces, serve the corner values of Fig. 3. */
  void slopes(const S* U) {
    for (int d = 0; d < 3; ++d) {
      if (!G.act[d]) {
        for (int m = 0; m < 8; ++m) std::fill(dq[d][m].begin(), dq[d][m].end(), S(0.0));
        continue;
      }
      const long o = G.off[d];
      each(G, mkbox(G, 1, -2), [&](long c) {
        for (int m = 0; m < 8; ++m) {
          if (m == 5 + d)
            dq[d][m][c] = fld(U, 5 + d)[c + o] - fld(U, 5 + d)[c];
          else
            dq[d][m][c] = limiter(q[m][c] - q[m][c - o], q[m][c + o] - q[m][c], P.limiter);
        }
      });
    }
    for (int d = 0; d < 3; ++d)
      for (int e = 0; e < 3; ++e) {
        if (e == d) continue;
        if (!G.act[e]) {
          std::fill(dbf[d][e].begin(), dbf[d][e].end(), S(0.0));
          continue;
        }
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        lo[e] = 1; hi[e] = -1;
        const long o = G.off[e];
        const S* B = fld(U, 5 + d);
        each(G, mkbox(G, lo, hi), [&](long f) {
          dbf[d][e][f] = limiter(B[f] - B[f - o], B[f + o] - B[f], P.limiter);
        });
      }
  }

  /* 3. edge EMF at time n from arithmetic averages (§2.1 constrained transport: E_z =
   * vx_bar By_bar - vy_bar Bx_bar with 4-cell velocity and 2-face field averages; E_x,
   * E_y by cyclic permutation), then the half-step face field B^{n+1/2} = B^n +
   * (dt/2) curl E^n with the stencil of eq:EMF_to_B and per-direction spacing. */
  void emf_n_and_half_b(const S* U) {
    for (int e = 0; e < 3; ++e) {
      const int a = (e + 1) % 3, b = (e + 2) % 3;
      const long oa = G.off[a], ob = G.off[b];
      int lo[3], hi[3];
      lo[a] = lo[b] = 1; hi[a] = hi[b] = -1; lo[e] = 0; hi[e] = -1;
      const S* Ba = fld(U, 5 + a);
      const S* Bb = fld(U, 5 + b);
      each(G, mkbox(G, lo, hi), [&](long c) {
        const S ua = 0.25 * (q[1 + a][c] + q[1 + a][c - oa] + q[1 + a][c - ob] + q[1 + a][c - oa - ob]);
        const S ub = 0.25 * (q[1 + b][c] + q[1 + b][c - oa] + q[1 + b][c - ob] + q[1 + b][c - oa - ob]);
        const S ba = 0.5 * (Ba[c] + Ba[c - ob]);
        const S bb = 0.5 * (Bb[c] + Bb[c - oa]);
        en[e][c] = ua * bb - ub * ba;
      });
    }
    const double hdt = 0.5 * dt;
    for (int d = 0; d < 3; ++d) {
      const int a = (d + 1) % 3, b = (d + 2) % 3;
      int lo[3], hi[3];
      lo[d] = 1; hi[d] = -1; lo[a] = lo[b] = 1; hi[a] = hi[b] = -2;
      const S* B = fld(U, 5 + d);
      each(G, mkbox(G, lo, hi), [&](long c) {
        S v = B[c];
        if (G.act[a]) v = v + (hdt / dx[a]) * (en[b][c + G.off[a]] - en[b][c]);
        if (G.act[b]) v = v - (hdt / dx[b]) * (en[a][c + G.off[b]] - en[a][c]);
        bh[d][c] = v;
      });
    }
  }

  /* 4. forward-Euler half-step of the primitives from the slopes (§2.1 "The MUSCL
   * Scheme": predictions for t + dt/2 from existing values and gradients). */
  void predictor() {
    each(G, mkbox(G, 1, -2), [&](long c) {
      S qq[8], D[3][8], r[8];
      for (int m = 0; m < 8; ++m) qq[m] = q[m][c];
      for (int d = 0; d < 3; ++d)
        for (int m = 0; m < 8; ++m) D[d][m] = G.act[d] ? dq[d][m][c] / dx[d] : S(0.0);
      dqdt_prim(qq, D, G.act, P.gamma, r);
      for (int m = 0; m < 8; ++m) qt[m][c] = qq[m] + (0.5 * dt) * r[m];
    });
  }

  /* predicted state on the face of cell c in direction d, side s = -1 (lower) / +1
   * (upper); the normal field is the face-centred half-step value. */
  void face_state(long c, int d, int s, S W[8]) {
    for (int m = 0; m < 8; ++m)
      W[m] = (s > 0) ? qt[m][c] + 0.5 * dq[d][m][c] : qt[m][c] - 0.5 * dq[d][m][c];
    W[5 + d] = bh[d][(s > 0) ? c + G.off[d] : c];
    site = 1;
    W[0] = floor_rho(W[0]);
    W[4] = floor_p(W[4]);
  }

  /* predicted state at the corner (sa, sb) of cell c for an edge along e (Fig. 3): cell
   * quantities extrapolated along both transverse directions; the two transverse field
   * components come from the adjacent faces and their transverse slopes. */
  void corner_state(long c, int e, int sa, int sb, S W[8]) {
    const int a = (e + 1) % 3, b = (e + 2) % 3;
    for (int m = 0; m < 8; ++m) {
      const S ta = (sa > 0) ? 0.5 * dq[a][m][c] : -(0.5 * dq[a][m][c]);
      const S tb = (sb > 0) ? 0.5 * dq[b][m][c] : -(0.5 * dq[b][m][c]);
      W[m] = qt[m][c] + (ta + tb);
    }
    const long fa = (sa > 0) ? c + G.off[a] : c;
    const long fb = (sb > 0) ? c + G.off[b] : c;
    W[5 + a] = (sb > 0) ? bh[a][fa] + 0.5 * dbf[a][b][fa] : bh[a][fa] - 0.5 * dbf[a][b][fa];
    W[5 + b] = (sa > 0) ? bh[b][fb] + 0.5 * dbf[b][a][fb] : bh[b][fb] - 0.5 * dbf[b][a][fb];
    site = 2;
    W[0] = floor_rho(W[0]);
    W[4] = floor_p(W[4]);
  }

  /* 5. HLLD fluxes at the faces of every active direction. */
  void face_fluxes() {
    for (int d = 0; d < 3; ++d) {
      if (!G.act[d]) continue;
      const int a = (d + 1) % 3, b = (d + 2) % 3;
      int lo[3] = {1, 1, 1}, hi[3] = {-2, -2, -2};
      lo[d] = 2;
      each(G, mkbox(G, lo, hi), [&](long f) {
        S WL[8], WR[8];
        face_state(f - G.off[d], d, +1, WL);
        face_state(f, d, -1, WR);
        const S L[8] = {WL[0], WL[1 + d], WL[1 + a], WL[1 + b], WL[4], WL[5 + d], WL[5 + a], WL[5 + b]};
        const S R[8] = {WR[0], WR[1 + d], WR[1 + a], WR[1 + b], WR[4], WR[5 + d], WR[5 + a], WR[5 + b]};
        S F[5];
        hlld(L, R, P, F, nullptr);
        fl[d][0][f] = F[0];
        fl[d][1 + d][f] = F[1];
        fl[d][1 + a][f] = F[2];
        fl[d][1 + b][f] = F[3];
        fl[d][4][f] = F[4];
      });
    }
  }

  /* 6. half-step EMF at every edge from the four corner states around it. */
  void edge_emfs() {
    for (int e = 0; e < 3; ++e) {
      const int a = (e + 1) % 3, b = (e + 2) % 3;
      const long oa = G.off[a], ob = G.off[b];
      int lo[3], hi[3];
      lo[a] = lo[b] = 2; hi[a] = hi[b] = -2; lo[e] = 1; hi[e] = -2;
      each(G, mkbox(G, lo, hi), [&](long c) {
        S SW[8], SE[8], NW[8], NE[8];
        corner_state(c - oa - ob, e, +1, +1, SW);
        corner_state(c - ob, e, -1, +1, SE);
        corner_state(c - oa, e, +1, -1, NW);
        corner_state(c, e, -1, -1, NE);
        emf[e][c] = P.emf_solver == 1 ? uct_hlld(SW, SE, NW, NE, e, P)
                                       : uct(SW, SE, NW, NE, e, P);
      });
    }
  }

  /* 7. conservative update of rho, rho u, E from face-flux differences (§2.1 flux-based
   * finite volume) and constrained-transport update of the face field, eq:EMF_to_B with
   * each difference divided by its own spacing (§2.3 per-direction dx lesson). */
  void update(const S* U, S* Uo) {
    for (long i = 0; i < 8 * G.Nc; ++i) Uo[i] = U[i];
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) { lo[d] = G.g; hi[d] = -G.g; }
    each(G, mkbox(G, lo, hi), [&](long c) {
      for (int m = 0; m < 5; ++m) {
        S v = fld(U, m)[c];
        for (int d = 0; d < 3; ++d)
          if (G.act[d]) v = v - (dt / dx[d]) * (fl[d][m][c + G.off[d]] - fl[d][m][c]);
        Uo[(long)m * G.Nc + c] = v;
      }
      for (int d = 0; d < 3; ++d) {
        const int a = (d + 1) % 3, b = (d + 2) % 3;
        S v = fld(U, 5 + d)[c];
        if (G.act[a]) v = v + (dt / dx[a]) * (emf[b][c + G.off[a]] - emf[b][c]);
        if (G.act[b]) v = v - (dt / dx[b]) * (emf[a][c + G.off[b]] - emf[a][c]);
        Uo[(long)(5 + d) * G.Nc + c] = v;
      }
    });
  }

  void run(const S* U, S* Uo) {
    prims(U);
    slopes(U);
    emf_n_and_half_b(U);
    predictor();
    face_fluxes();
    edge_emfs();
    update(U, Uo);
  }
};

/* time-step rule: C min over interior cells of 1 / sum_d (|u_d| + c_f,d) / dx_d */
double cfl_patch(const Geom& G, const double* U, const double dx[3], const mhd_oracle_params& P) {
  const double gm1 = P.gamma - 1.0;
  const long Nc = G.Nc;
  double smx = 0.0;
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) { lo[d] = G.g; hi[d] = -G.g; }
  each(G, mkbox(G, lo, hi), [&](long c) {
    const double rho = std::max(U[c], P.rho_floor);
    const double u[3] = {U[Nc + c] / rho, U[2 * Nc + c] / rho, U[3 * Nc + c] / rho};
    double B[3];
    for (int d = 0; d < 3; ++d) B[d] = 0.5 * (U[(5 + d) * Nc + c] + U[(5 + d) * Nc + c + G.off[d]]);
    const double ke = 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const double me = 0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    const double p = std::max(gm1 * (U[4 * Nc + c] - ke - me), P.p_floor);
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
      if (!G.act[d]) continue;
      const double cf = cfast(rho, p, B[d], B[(d + 1) % 3], B[(d + 2) % 3], P.gamma);
      s += (std::fabs(u[d]) + cf) / dx[d];
    }
    smx = std::max(smx, s);
  });
  return P.cfl / smx;
}

bool check_params(const mhd_oracle_params* p) {
  return p && p->gamma > 1.0 && p->cfl > 0.0 && p->rho_floor > 0.0 && p->p_floor > 0.0 &&
         p->eps_deg >= 0.0 && (p->limiter == 0 || p->limiter == 1) &&
         (p->emf_solver == 0 || p->emf_solver == 1);
}

long patch_elems(const int32_t n[3], int g) {
  long e = 8;
  for (int d = 0; d < 3; ++d) e *= (n[d] > 1) ? n[d] + 2 * g : 1;
  return e;
}

}  // namespace

/* ------------------------------------------------------------------ C interface */

/* Every guard cell of every patch with its owner (the framework's guard exchange, §2.2):
 * f(p, cd, src, cs, Nc_p, Nc_src, base_p, base_src) for destination cell cd of patch p and
 * source cell cs of patch src.  A direction whose face neighbour is the domain boundary
 * takes the zero-gradient copy of the nearest owned cell. */
template <class F>
int for_each_guard(int32_t npatch, const int32_t* dims, int32_t g, const int32_t* nbr, F f) {
  if (npatch < 0 || !nbr) return -1;
  std::vector<Geom> Gs(npatch);
  std::vector<long> base(npatch + 1, 0);
  for (int p = 0; p < npatch; ++p) {
    if (!Gs[p].init(dims + 3 * p, g)) return -1;
    base[p + 1] = base[p] + 8 * Gs[p].Nc;
  }
  for (int p = 0; p < npatch; ++p) {
    const Geom& G = Gs[p];
    for (int k = 0; k < G.N[2]; ++k)
      for (int j = 0; j < G.N[1]; ++j)
        for (int i = 0; i < G.N[0]; ++i) {
          int idx[3] = {i, j, k}, o[3];
          bool guard = false;
          for (int d = 0; d < 3; ++d) {
            o[d] = 0;
            if (!G.act[d]) continue;
            if (idx[d] < g) o[d] = -1;
            else if (idx[d] >= g + G.n[d]) o[d] = +1;
            if (o[d]) guard = true;
          }
          if (!guard) continue;
          for (int d = 0; d < 3; ++d) {
            if (!o[d]) continue;
            int fo[3] = {0, 0, 0};
            fo[d] = o[d];
            if (nbr[27 * p + (fo[0] + 1) + 3 * (fo[1] + 1) + 9 * (fo[2] + 1)] < 0) {
              idx[d] = std::min(std::max(idx[d], g), g + G.n[d] - 1);
              o[d] = 0;
            }
          }
          int src = p;
          if (o[0] || o[1] || o[2]) src = nbr[27 * p + (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)];
          if (src < 0 || src >= npatch) return -1;
          const Geom& H = Gs[src];
          if (H.n[0] != G.n[0] || H.n[1] != G.n[1] || H.n[2] != G.n[2]) return -1;
          const long cs = (idx[0] - o[0] * G.n[0]) + H.st[1] * (idx[1] - o[1] * G.n[1]) +
                          H.st[2] * (idx[2] - o[2] * G.n[2]);
          const long cd = (long)i + G.st[1] * j + G.st[2] * k;
          f(p, cd, src, cs, G.Nc, H.Nc, base[p], base[src]);
        }
  }
  return 0;
}

template <class E>
int fill_guards_t(int32_t npatch, const int32_t* dims, int32_t g, E* U, const int32_t* nbr) {
  if (!U) return -1;
  return for_each_guard(npatch, dims, g, nbr,
                        [&](int, long cd, int, long cs, long Nc, long Ns, long bp, long bs) {
                          for (int m = 0; m < 8; ++m) U[bp + m * Nc + cd] = U[bs + m * Ns + cs];
                        });
}

/* one update in arithmetic R with the branch signature (sig may be NULL) */
template <class R>
int step_traced(const int32_t n[3], int32_t g, const R* U_in, R* U_out, double dt,
                const double dx[3], const mhd_oracle_params* prm, uint64_t* sig) {
  Geom G;
  if (!G.init(n, g) || !check_params(prm) || !U_in || !U_out || !(dt >= 0.0)) return -1;
  const long ne = 8 * G.Nc;
  std::vector<TrcT<R>> a(ne), b(ne);
  for (long i = 0; i < ne; ++i) a[i] = TrcT<R>(U_in[i]);
  Stepper<TrcT<R>> s(G, *prm, dt, dx);
  g_sig = 0xcbf29ce484222325ull;
  s.run(a.data(), b.data());
  if (sig) *sig = g_sig;
  for (long i = 0; i < ne; ++i) U_out[i] = b[i].v;
  return 0;
}

template <class R>
int step_traced_many(int32_t npatch, const int32_t* dims, int32_t g, const R* U_in, R* U_out,
                     const double* dt, const double* dx, const mhd_oracle_params* prm,
                     uint64_t* sig) {
  if (npatch < 0 || !check_params(prm)) return -1;
  std::vector<long> base(npatch + 1, 0);
  for (int p = 0; p < npatch; ++p) base[p + 1] = base[p] + patch_elems(dims + 3 * p, g);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
  for (int p = 0; p < npatch; ++p)
    if (step_traced(dims + 3 * p, g, U_in + base[p], U_out + base[p], dt[p], dx + 3 * p, prm,
                    sig ? sig + p : nullptr))
      bad += 1;
  return bad ? -1 : 0;
}

extern "C" {

int mhd_oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void mhd_oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int mhd_oracle_step(const int32_t n[3], int32_t g, const double* U_in, double* U_out, double dt,
                    const double dx[3], const mhd_oracle_params* prm, int64_t* nfloor) {
  Geom G;
  if (!G.init(n, g) || !check_params(prm) || !U_in || !U_out || !(dt >= 0.0)) return -1;
  Stepper<double> s(G, *prm, dt, dx);
  s.run(U_in, U_out);
  if (nfloor)
    for (int i = 0; i < 3; ++i) nfloor[i] += s.nfloor[i];
  return 0;
}

int mhd_oracle_step_many(int32_t npatch, const int32_t* dims, int32_t g, const double* U_in,
                         double* U_out, const double* dt, const double* dx,
                         const mhd_oracle_params* prm, int64_t* nfloor) {
  if (npatch < 0 || !check_params(prm)) return -1;
  std::vector<long> base(npatch + 1, 0);
  for (int p = 0; p < npatch; ++p) base[p + 1] = base[p] + patch_elems(dims + 3 * p, g);
  int bad = 0;
  int64_t nf0 = 0, nf1 = 0, nf2 = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad, nf0, nf1, nf2)
  for (int p = 0; p < npatch; ++p) {
    int64_t f[3] = {0, 0, 0};
    if (mhd_oracle_step(dims + 3 * p, g, U_in + base[p], U_out + base[p], dt[p], dx + 3 * p, prm, f))
      bad += 1;
    nf0 += f[0]; nf1 += f[1]; nf2 += f[2];
  }
  if (nfloor) { nfloor[0] += nf0; nfloor[1] += nf1; nfloor[2] += nf2; }
  return bad ? -1 : 0;
}

double mhd_oracle_cfl(const int32_t n[3], int32_t g, const double* U, const double dx[3],
                      const mhd_oracle_params* prm) {
  Geom G;
  if (!G.init(n, g) || !check_params(prm) || !U) return -1.0;
  return cfl_patch(G, U, dx, *prm);
}

int mhd_oracle_cfl_many(int32_t npatch, const int32_t* dims, int32_t g, const double* U,
                        const double* dx, const mhd_oracle_params* prm, double* dt_out) {
  if (npatch < 0 || !check_params(prm)) return -1;
  std::vector<long> base(npatch + 1, 0);
  for (int p = 0; p < npatch; ++p) base[p + 1] = base[p] + patch_elems(dims + 3 * p, g);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
  for (int p = 0; p < npatch; ++p) {
    dt_out[p] = mhd_oracle_cfl(dims + 3 * p, g, U + base[p], dx + 3 * p, prm);
    if (!(dt_out[p] > 0.0)) bad += 1;
  }
  return bad ? -1 : 0;
}

int mhd_oracle_fill_guards(int32_t npatch, const int32_t* dims, int32_t g, double* U,
                           const int32_t* nbr) {
  return fill_guards_t(npatch, dims, g, U, nbr);
}

int mhd_oracle_fill_guards_ext(int32_t npatch, const int32_t* dims, int32_t g, long double* U,
                               const int32_t* nbr) {
  return fill_guards_t(npatch, dims, g, U, nbr);
}

/* Guard fill at each patch's own time (local time stepping: §2.2 "DISPATCH", patches carry
 * several time slices; §3.1 "DISPATCH Validation", guard zones interpolated between
 * asynchronous patch times).  A guard cell of patch p whose owner is q receives q's value
 * at time t[p], interpolated linearly between q's slices (t_prev[q], U_prev) and (t[q], U):
 * (1 - th) U_prev + th U with th = (t[p] - t_prev[q]) / (t[q] - t_prev[q]); q's current
 * value when t[q] == t_prev[q].  Patches with mask[p] == 0 are left alone (mask NULL: all). */
int mhd_oracle_fill_guards_at(int32_t npatch, const int32_t* dims, int32_t g, double* U,
                              const double* U_prev, const double* t, const double* t_prev,
                              const int32_t* nbr, const int32_t* mask) {
  if (!U || !U_prev || !t || !t_prev) return -1;
  return for_each_guard(
      npatch, dims, g, nbr, [&](int p, long cd, int q, long cs, long Nc, long Ns, long bp, long bs) {
        if (mask && !mask[p]) return;
        const bool two = t[q] > t_prev[q];
        const double th = two ? (t[p] - t_prev[q]) / (t[q] - t_prev[q]) : 1.0;
        for (int m = 0; m < 8; ++m) {
          const double a = U_prev[bs + m * Ns + cs], b = U[bs + m * Ns + cs];
          U[bp + m * Nc + cd] = two ? (1.0 - th) * a + th * b : b;
        }
      });
}

int mhd_oracle_step_jvp(const int32_t n[3], int32_t g, const double* U_in, const double* dU_in,
                        double* U_out, double* dU_out, double dt, const double dx[3],
                        const mhd_oracle_params* prm) {
  Geom G;
  if (!G.init(n, g) || !check_params(prm)) return -1;
  const long ne = 8 * G.Nc;
  std::vector<Dual> a(ne), b(ne);
  for (long i = 0; i < ne; ++i) a[i] = Dual(U_in[i], dU_in[i]);
  Stepper<Dual> s(G, *prm, dt, dx);
  s.run(a.data(), b.data());
  for (long i = 0; i < ne; ++i) { U_out[i] = b[i].v; dU_out[i] = b[i].d; }
  return 0;
}

int mhd_oracle_step_jvp_many(int32_t npatch, const int32_t* dims, int32_t g, const double* U_in,
                             const double* dU_in, double* U_out, double* dU_out, const double* dt,
                             const double* dx, const mhd_oracle_params* prm) {
  if (npatch < 0 || !check_params(prm)) return -1;
  std::vector<long> base(npatch + 1, 0);
  for (int p = 0; p < npatch; ++p) base[p + 1] = base[p] + patch_elems(dims + 3 * p, g);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
  for (int p = 0; p < npatch; ++p)
    if (mhd_oracle_step_jvp(dims + 3 * p, g, U_in + base[p], dU_in + base[p], U_out + base[p],
                            dU_out + base[p], dt[p], dx + 3 * p, prm))
      bad += 1;
  return bad ? -1 : 0;
}

int mhd_oracle_step_sig(const int32_t n[3], int32_t g, const double* U_in, double* U_out,
                        double dt, const double dx[3], const mhd_oracle_params* prm,
                        uint64_t* sig) {
  if (!sig) return -1;
  return step_traced(n, g, U_in, U_out, dt, dx, prm, sig);
}

int mhd_oracle_step_sig_many(int32_t npatch, const int32_t* dims, int32_t g, const double* U_in,
                             double* U_out, const double* dt, const double* dx,
                             const mhd_oracle_params* prm, uint64_t* sig) {
  if (!sig) return -1;
  return step_traced_many(npatch, dims, g, U_in, U_out, dt, dx, prm, sig);
}

int mhd_oracle_step_ext_many(int32_t npatch, const int32_t* dims, int32_t g,
                             const long double* U_in, long double* U_out, const double* dt,
                             const double* dx, const mhd_oracle_params* prm, uint64_t* sig) {
  return step_traced_many(npatch, dims, g, U_in, U_out, dt, dx, prm, sig);
}

int mhd_oracle_count_ops(const int32_t n[3], int32_t g, const double* U_in, double dt,
                         const double dx[3], const mhd_oracle_params* prm, int64_t counts[5]) {
  Geom G;
  if (!G.init(n, g) || !check_params(prm)) return -1;
  const long ne = 8 * G.Nc;
  std::vector<Cnt> a(ne), b(ne);
  for (long i = 0; i < ne; ++i) a[i] = Cnt(U_in[i]);
  Stepper<Cnt> s(G, *prm, dt, dx);
  g_ops = OpCount{0, 0, 0, 0, 0};
  s.run(a.data(), b.data());
  counts[0] = g_ops.add; counts[1] = g_ops.mul; counts[2] = g_ops.div;
  counts[3] = g_ops.sqrt; counts[4] = g_ops.cmp;
  return 0;
}

int mhd_oracle_ops_per_cell(const int32_t n[3], int32_t g, const double* U_in, double dt,
                            const double dx[3], const mhd_oracle_params* prm, double out[5]) {
  Geom G;
  if (!G.init(n, g) || !check_params(prm)) return -1;
  const long ne = 8 * G.Nc;
  std::vector<Cnt> a(ne), b(ne);
  for (long i = 0; i < ne; ++i) a[i] = Cnt(U_in[i]);
  Stepper<Cnt> s(G, *prm, dt, dx);
  g_ops = OpCount{0, 0, 0, 0, 0};
  for (int i = 0; i < 5; ++i) g_per_item[i] = 0.0;
  g_rec = true;
  s.run(a.data(), b.data());
  g_rec = false;
  for (int i = 0; i < 5; ++i) out[i] = g_per_item[i];
  return 0;
}

void mhd_oracle_hlld(const double L[8], const double R[8], const mhd_oracle_params* prm,
                     double F[5], int32_t* region) {
  int reg = -1;
  hlld(L, R, *prm, F, &reg);
  if (region) *region = reg;
}

void mhd_oracle_hlld_fan(const double L[8], const double R[8], const mhd_oracle_params* prm,
                         double F[5], int32_t* region, double speeds[6], double states[4][8]) {
  int reg = -1;
  hlld(L, R, *prm, F, &reg, speeds, states);
  if (region) *region = reg;
}

double mhd_oracle_cfast(double rho, double p, double bn, double bt1, double bt2, double gamma) {
  return cfast(rho, p, bn, bt1, bt2, gamma);
}

double mhd_oracle_limiter(double dl, double dr, int32_t lim) { return limiter(dl, dr, lim); }

double mhd_oracle_uct(const double W[4][8], const mhd_oracle_params* prm) {
  return prm->emf_solver == 1 ? uct_hlld(W[0], W[1], W[2], W[3], 2, *prm)
                              : uct(W[0], W[1], W[2], W[3], 2, *prm);
}

void mhd_oracle_dqdt(const double q[8], const double D[3][8], const int32_t act[3], double gamma,
                     double dqdt[8]) {
  const int a[3] = {act[0] != 0, act[1] != 0, act[2] != 0};
  dqdt_prim(q, D, a, gamma, dqdt);
}

}  // extern "C"
