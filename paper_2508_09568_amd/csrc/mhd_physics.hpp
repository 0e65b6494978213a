// mhd_physics.hpp -- pointwise building blocks of the ideal-MHD update, device side.
//
// Templated on the element type (float or double).  Everything here is a pure function
// of its arguments: slope limiter, fast magnetosonic speed, the primitive-variable time
// derivative used by the half-step predictor, the HLLD Riemann flux and the four-state
// edge EMF.  Code units with mu_0 = 1 (the energy relation of the paper's §2.1).
#pragma once

namespace mhd {

// type-exact elementary functions (no silent promotion of float arguments to double)
__host__ __device__ __forceinline__ float m_abs(float x) { return fabsf(x); }
__host__ __device__ __forceinline__ double m_abs(double x) { return fabs(x); }
__host__ __device__ __forceinline__ float m_min(float a, float b) { return fminf(a, b); }
__host__ __device__ __forceinline__ double m_min(double a, double b) { return fmin(a, b); }
__host__ __device__ __forceinline__ float m_max(float a, float b) { return fmaxf(a, b); }
__host__ __device__ __forceinline__ double m_max(double a, double b) { return fmax(a, b); }

// Reciprocal, square root and reciprocal square root.  The update takes them of nonzero
// finite numbers (densities and pressures after the floors, wave-speed sums bounded below)
// and of zero only in m_sqrt.  On the device they are built on the CDNA hardware
// approximations instead of the IEEE-exact library sequences (which spend 10-17
// instructions on scaling and special cases):
//  float : v_rcp_f32 / v_sqrt_f32 / v_rsq_f32 as they are (about 1 ulp);
//  double: v_rcp_f64 / v_rsq_f64 seeds refined by Newton-Raphson (reciprocal: two
//          iterations of r <- r + r (1 - x r); square root: the coupled iteration for
//          g ~ sqrt(x), h ~ 1 / (2 sqrt(x)) with one residual correction), within about
//          1 ulp of the exact result.
// The host versions (CPU builds of this header) are the plain operations, and so are the
// device versions of a build with MHD_STRICT_IEEE defined (correctly rounded division and
// square root): with contraction off as well, that build rounds every operation as a plain
// CPU evaluation of the same expressions does.
#if defined(__HIP_DEVICE_COMPILE__) && !defined(MHD_STRICT_IEEE)
#define MHD_HW_MATH 1
#else
#define MHD_HW_MATH 0
#endif
__host__ __device__ __forceinline__ float m_rcp(float x) {
#if MHD_HW_MATH
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ double m_rcp(double x) {
#if MHD_HW_MATH
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}
__host__ __device__ __forceinline__ float m_sqrt(float x) {
#if MHD_HW_MATH
  return __builtin_amdgcn_sqrtf(x);
#else
  return sqrtf(x);
#endif
}
__host__ __device__ __forceinline__ double m_sqrt(double x) {
#if MHD_HW_MATH
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  g = fma(h, d, g);
  return x > 0.0 ? g : 0.0;
#else
  return sqrt(x);
#endif
}
// square root of a strictly positive finite argument (no zero guard)
__host__ __device__ __forceinline__ float m_sqrt_pos(float x) { return m_sqrt(x); }
__host__ __device__ __forceinline__ double m_sqrt_pos(double x) {
#if MHD_HW_MATH
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(h, d, g);
#else
  return sqrt(x);
#endif
}
__host__ __device__ __forceinline__ float m_rsqrt(float x) {
#if MHD_HW_MATH
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}
__host__ __device__ __forceinline__ double m_rsqrt(double x) {
#if MHD_HW_MATH
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
#else
  return 1.0 / sqrt(x);
#endif
}

// Forward-mode dual number (value, derivative along one seeded input).  The pointwise
// functions below are templates on the scalar, so the same code yields derivatives when
// instantiated with Dual<T>; the adjoint kernels use this to differentiate every stage.
template <typename T>
struct Dual {
  T v, d;
  __host__ __device__ __forceinline__ Dual() : v(T(0)), d(T(0)) {}
  __host__ __device__ __forceinline__ Dual(T a) : v(a), d(T(0)) {}
  __host__ __device__ __forceinline__ Dual(T a, T b) : v(a), d(b) {}
  __host__ __device__ __forceinline__ Dual& operator+=(const Dual& o) { v += o.v; d += o.d; return *this; }
};
template <typename T>
__host__ __device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return Dual<T>(a.v + b.v, a.d + b.d); }
template <typename T>
__host__ __device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return Dual<T>(a.v - b.v, a.d - b.d); }
template <typename T>
__host__ __device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return Dual<T>(-a.v, -a.d); }
template <typename T>
__host__ __device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) {
  return Dual<T>(a.v * b.v, a.d * b.v + a.v * b.d);
}
template <typename T>
__host__ __device__ __forceinline__ Dual<T> m_rcp(Dual<T> x) {
  const T r = m_rcp(x.v);
  return Dual<T>(r, -(x.d * r) * r);
}
template <typename T>
__host__ __device__ __forceinline__ bool operator<(Dual<T> a, Dual<T> b) { return a.v < b.v; }
template <typename T>
__host__ __device__ __forceinline__ bool operator>(Dual<T> a, Dual<T> b) { return a.v > b.v; }
template <typename T>
__host__ __device__ __forceinline__ bool operator<=(Dual<T> a, Dual<T> b) { return a.v <= b.v; }
template <typename T>
__host__ __device__ __forceinline__ bool operator>=(Dual<T> a, Dual<T> b) { return a.v >= b.v; }
template <typename T>
__host__ __device__ __forceinline__ Dual<T> m_abs(Dual<T> x) { return x.v < T(0) ? -x : x; }
template <typename T>
__host__ __device__ __forceinline__ Dual<T> m_min(Dual<T> a, Dual<T> b) { return b.v < a.v ? b : a; }
template <typename T>
__host__ __device__ __forceinline__ Dual<T> m_max(Dual<T> a, Dual<T> b) { return a.v < b.v ? b : a; }
template <typename T>
__host__ __device__ __forceinline__ Dual<T> m_sqrt(Dual<T> x) {
  const T s = m_sqrt(x.v);
  return Dual<T>(s, x.d * (T(0.5) * m_rcp(s)));
}
template <typename T>
__host__ __device__ __forceinline__ Dual<T> m_sqrt_pos(Dual<T> x) {
  const T s = m_sqrt_pos(x.v);
  return Dual<T>(s, x.d * (T(0.5) * m_rcp(s)));
}
template <typename T>
__host__ __device__ __forceinline__ Dual<T> m_rsqrt(Dual<T> x) {
  const T y = m_rsqrt(x.v);
  return Dual<T>(y, (T(-0.5) * x.d) * (y * y * y));
}

template <typename T>
struct Consts {
  T gamma;      // adiabatic index
  T gm1;        // gamma - 1
  T inv_gm1;    // 1 / (gamma - 1)
  T rho_floor;  // floors applied to every reconstructed state
  T p_floor;
  T eps_deg;    // relative threshold of the HLLD degeneracy switch
  T tiny;       // guard of the EMF denominators
  int limiter;  // 0 monotonised central, 1 minmod
  int emf;      // edge EMF: 0 UCT-HLL, 1 UCT-HLLD (kernels take it as a template parameter;
                // the adjoint's dual-number gather reads it here)
};

// constants of one scalar type converted to another (e.g. T -> Dual<T>)
template <typename S, typename T>
__host__ __device__ __forceinline__ Consts<S> lift(const Consts<T>& c) {
  Consts<S> o;
  o.gamma = S(c.gamma);
  o.gm1 = S(c.gm1);
  o.inv_gm1 = S(c.inv_gm1);
  o.rho_floor = S(c.rho_floor);
  o.p_floor = S(c.p_floor);
  o.eps_deg = S(c.eps_deg);
  o.tiny = S(c.tiny);
  o.limiter = c.limiter;
  o.emf = c.emf;
  return o;
}

// Limited slope from the backward and forward differences (§2.1 "The MUSCL Scheme": the
// slope estimate must suppress oscillations).  Zero unless both differences share a
// strict sign; MC = min(2|dm|, 2|dp|, |dm+dp|/2), minmod = min(|dm|, |dp|).
template <typename T>
__host__ __device__ __forceinline__ T limited_slope(T dm, T dp, int kind) {
  if (!(dm * dp > T(0))) return T(0);
  const T am = m_abs(dm), ap = m_abs(dp);
  T mag = m_min(am, ap);
  if (kind == 0) mag = m_min(T(2) * mag, T(0.5) * m_abs(dm + dp));
  return dm > T(0) ? mag : -mag;
}

// Fast magnetosonic speed along a direction with normal field bn; the radicand is the
// cancellation-free (a^2 - b^2)^2 + 4 a^2 b_t^2 / rho.  The direction-independent part
// (1/rho, a^2, b^2 = |B|^2/rho) is split off so that the two directions of one state
// share it.
template <typename T>
struct WaveBase {
  T ir, a2, b2, d2;
};
template <typename T>
__host__ __device__ __forceinline__ WaveBase<T> wave_base(T rho, T p, T bsq, T gamma) {
  WaveBase<T> w;
  w.ir = m_rcp(rho);
  w.a2 = gamma * p * w.ir;
  w.b2 = bsq * w.ir;
  const T d = w.a2 - w.b2;
  w.d2 = d * d;
  return w;
}
// (the outer argument is at least a^2 > 0: pressure and density are floored positive)
template <typename T>
__host__ __device__ __forceinline__ T fast_speed_t(const WaveBase<T>& w, T bt) {
  const T rad = w.d2 + T(4) * w.a2 * (bt * w.ir);
  return m_sqrt_pos(T(0.5) * (w.a2 + w.b2 + m_sqrt(rad)));
}
template <typename T>
__host__ __device__ __forceinline__ T fast_speed(T rho, T p, T bn, T bt1, T bt2, T gamma) {
  const T bt = bt1 * bt1 + bt2 * bt2;
  return fast_speed_t(wave_base(rho, p, bn * bn + bt, gamma), bt);
}

// d(q)/dt of ideal MHD in primitive variables q = (rho, u, v, w, p, Bx, By, Bz) from
// slopes D[d][m] and inverse cell sizes ix[d] (rows of collapsed directions are zero).  The induction
// equation is taken in its div B = 0 form.  Forward-Euler half step of the predictor.
template <typename T>
__host__ __device__ __forceinline__ void prim_rate(const T q[8], const T D[3][8], const T ix[3],
                                                   T gamma, T r[8]) {
  // spatial derivative of primitive m along d: the slope over the cell size
#define MHD_G(d, m) (D[d][m] * ix[d])
  const T rho = q[0], p = q[4];
  const T ir = m_rcp(rho);
  const T div = MHD_G(0, 1) + MHD_G(1, 2) + MHD_G(2, 3);
  T ar = T(0), ap = T(0);
  for (int d = 0; d < 3; ++d) {
    ar += q[1 + d] * MHD_G(d, 0);
    ap += q[1 + d] * MHD_G(d, 4);
  }
  r[0] = -(ar + rho * div);
  r[4] = -(ap + gamma * p * div);
  for (int i = 0; i < 3; ++i) {
    T adv = T(0), ten = T(0), str = T(0), advb = T(0);
    for (int d = 0; d < 3; ++d) {
      adv += q[1 + d] * MHD_G(d, 1 + i);
      ten += q[5 + d] * MHD_G(d, 5 + i);
      str += q[5 + d] * MHD_G(d, 1 + i);
      advb += q[1 + d] * MHD_G(d, 5 + i);
    }
    const T grad = MHD_G(i, 4) + (q[5] * MHD_G(i, 5) + q[6] * MHD_G(i, 6) + q[7] * MHD_G(i, 7));
    r[1 + i] = -adv - (grad - ten) * ir;
    r[5 + i] = str - advb - q[5 + i] * div;
  }
#undef MHD_G
}

// HLLD flux through a face (§2.1 "HLLD Solver", Fig. 1; Miyoshi & Kusano 2005).
// s[0] = left, s[1] = right state in the face frame: (rho, u_n, u_t1, u_t2, p, B_t1, B_t2);
// bn = shared normal field.  F = (rho, m_n, m_t1, m_t2, E) flux.  The region containing the
// face is found from the wave fan S_L < S*_L < S_M < S*_R < S_R; its flux is accumulated as
// F_a + S_a (U*_a - U_a) [+ S*_a (U**_a - U*_a)] on the side a of the contact.
template <typename T>
__host__ __device__ __forceinline__ void hlld_flux(const T s[2][7], T bn, const Consts<T>& c,
                                                   T F[5]) {
  const T bn2 = bn * bn;
  T pt[2], en[2], ub[2], cf[2];
  for (int k = 0; k < 2; ++k) {
    const T r = s[k][0], u = s[k][1], v = s[k][2], w = s[k][3], p = s[k][4];
    const T by = s[k][5], bz = s[k][6];
    const T b2 = bn2 + by * by + bz * bz;
    pt[k] = p + T(0.5) * b2;
    en[k] = p * c.inv_gm1 + T(0.5) * r * (u * u + v * v + w * w) + T(0.5) * b2;
    ub[k] = u * bn + v * by + w * bz;
    cf[k] = fast_speed(r, p, bn, by, bz, c.gamma);
  }
  const T cmx = m_max(cf[0], cf[1]);
  const T S[2] = {m_min(s[0][1], s[1][1]) - cmx, m_max(s[0][1], s[1][1]) + cmx};
  const T sd[2] = {S[0] - s[0][1], S[1] - s[1][1]};     // S_a - u_a
  const T mf[2] = {sd[0] * s[0][0], sd[1] * s[1][0]};   // rho_a (S_a - u_a)
  const T iden = m_rcp(mf[1] - mf[0]);
  const T sm = (mf[1] * s[1][1] - mf[0] * s[0][1] - pt[1] + pt[0]) * iden;
  const T pts = (mf[1] * pt[0] - mf[0] * pt[1] + mf[0] * mf[1] * (s[1][1] - s[0][1])) * iden;

  // single-star states
  T rs[2], vs[2], ws[2], bys[2], bzs[2], es[2], ubs[2];
  for (int k = 0; k < 2; ++k) {
    const T isd = m_rcp(S[k] - sm);
    rs[k] = mf[k] * isd;
    const T dd = mf[k] * (S[k] - sm) - bn2;
    const T qq = mf[k] * sd[k] - bn2;
    if (m_abs(dd) > c.eps_deg * (mf[k] * sd[k] + bn2)) {
      const T idd = m_rcp(dd);
      const T tv = bn * (sm - s[k][1]) * idd;
      const T tb = qq * idd;
      vs[k] = s[k][2] - s[k][5] * tv;
      ws[k] = s[k][3] - s[k][6] * tv;
      bys[k] = s[k][5] * tb;
      bzs[k] = s[k][6] * tb;
    } else {
      vs[k] = s[k][2];
      ws[k] = s[k][3];
      bys[k] = s[k][5];
      bzs[k] = s[k][6];
    }
    ubs[k] = sm * bn + vs[k] * bys[k] + ws[k] * bzs[k];
    es[k] = (sd[k] * en[k] - pt[k] * s[k][1] + pts * sm + bn * (ub[k] - ubs[k])) * isd;
  }

  // rotational (Alfven) discontinuities and the double-star state
  const T isq[2] = {m_rsqrt(rs[0]), m_rsqrt(rs[1])};
  const T sq[2] = {rs[0] * isq[0], rs[1] * isq[1]};
  const T abn = m_abs(bn);
  const T Ss[2] = {sm - abn * isq[0], sm + abn * isq[1]};
  const T sg = bn < T(0) ? T(-1) : T(1);
  const T isum = m_rcp(sq[0] + sq[1]);
  const T vss = (sq[0] * vs[0] + sq[1] * vs[1] + (bys[1] - bys[0]) * sg) * isum;
  const T wss = (sq[0] * ws[0] + sq[1] * ws[1] + (bzs[1] - bzs[0]) * sg) * isum;
  const T byss = (sq[0] * bys[1] + sq[1] * bys[0] + sq[0] * sq[1] * (vs[1] - vs[0]) * sg) * isum;
  const T bzss = (sq[0] * bzs[1] + sq[1] * bzs[0] + sq[0] * sq[1] * (ws[1] - ws[0]) * sg) * isum;
  const T ubss = sm * bn + vss * byss + wss * bzss;

  // region of the face and the side it belongs to
  int reg;
  if (S[0] > T(0)) reg = 0;
  else if (Ss[0] >= T(0)) reg = 1;
  else if (sm >= T(0)) reg = 2;
  else if (Ss[1] >= T(0)) reg = 3;
  else if (S[1] >= T(0)) reg = 4;
  else reg = 5;
  // the side of the contact: every per-side quantity is picked by a two-way select (a run-time
  // index into the 2 x 7 state array would become a select chain over all 14 entries)
  const bool lft = reg <= 2;
  const auto pick = [lft](T a, T b) { return lft ? a : b; };
  const T r = pick(s[0][0], s[1][0]), u = pick(s[0][1], s[1][1]), v = pick(s[0][2], s[1][2]),
          w = pick(s[0][3], s[1][3]);
  const T by = pick(s[0][5], s[1][5]), bz = pick(s[0][6], s[1][6]);
  const T ptk = pick(pt[0], pt[1]), enk = pick(en[0], en[1]), ubk = pick(ub[0], ub[1]);
  F[0] = r * u;
  F[1] = r * u * u + ptk - bn2;
  F[2] = r * v * u - by * bn;
  F[3] = r * w * u - bz * bn;
  F[4] = u * (enk + ptk) - bn * ubk;
  if (reg >= 1 && reg <= 4) {
    const T rsk = pick(rs[0], rs[1]), esk = pick(es[0], es[1]);
    const T Us[5] = {rsk, rsk * sm, rsk * pick(vs[0], vs[1]), rsk * pick(ws[0], ws[1]), esk};
    const T Uo[5] = {r, r * u, r * v, r * w, enk};
    const T Sk = pick(S[0], S[1]);
    T Fs[5];
    for (int m = 0; m < 5; ++m) Fs[m] = F[m] + Sk * (Us[m] - Uo[m]);
    if (reg == 2 || reg == 3) {
      const T ess = lft ? es[0] - sq[0] * (ubs[0] - ubss) * sg
                        : es[1] + sq[1] * (ubs[1] - ubss) * sg;
      const T Uss[5] = {rsk, rsk * sm, rsk * vss, rsk * wss, ess};
      const T Ssk = pick(Ss[0], Ss[1]);
      for (int m = 0; m < 5; ++m) Fs[m] = Fs[m] + Ssk * (Uss[m] - Us[m]);
    }
    for (int m = 0; m < 5; ++m) F[m] = Fs[m];
  }
}

// Edge EMF from the four predicted corner states around an edge (§2.1 "Constrained
// transport and 2D-extension", Fig. 3: SW/SE/NW/NE).  Each corner C = (rho, u_a, u_b, p,
// B_e, B_a, B_b) for the edge direction e and its cyclic transverse pair (a, b); W/E are
// the low/high a sides, S/N the low/high b sides.  Two one-dimensional HLL fluxes of the
// transverse field, composed, with outer speeds bounded over the four corners.  The corners
// are taken one at a time (0 SW, 1 SE, 2 NW, 3 NE), so a caller need not hold all four
// states; the speed bounds are maxima, exact in any order.
template <typename T>
struct UctAcc {
  T emf[4];
  T apa, ama, apb, amb;
  T ba0, bb0, bb1, ba2;  // B_a, B_b of SW; B_b of SE; B_a of NW
  __host__ __device__ __forceinline__ UctAcc() : apa(T(0)), ama(T(0)), apb(T(0)), amb(T(0)) {}
  __host__ __device__ __forceinline__ void add(int k, const T C[7], const Consts<T>& c) {
    const T r = C[0], ua = C[1], ubb = C[2], p = C[3];
    const T be = C[4], ba = C[5], bb = C[6];
    emf[k] = ua * bb - ubb * ba;
    const T ba2_ = ba * ba, bb2 = bb * bb, be2 = be * be;
    const WaveBase<T> wb = wave_base(r, p, ba2_ + bb2 + be2, c.gamma);
    const T cfa = fast_speed_t(wb, bb2 + be2);
    const T cfb = fast_speed_t(wb, be2 + ba2_);
    apa = m_max(apa, ua + cfa);
    ama = m_max(ama, cfa - ua);
    apb = m_max(apb, ubb + cfb);
    amb = m_max(amb, cfb - ubb);
    if (k == 0) { ba0 = ba; bb0 = bb; }
    if (k == 1) bb1 = bb;
    if (k == 2) ba2 = ba;
  }
  __host__ __device__ __forceinline__ T finish(const Consts<T>& c) const {
    const T da = m_max(apa + ama, c.tiny);
    const T db = m_max(apb + amb, c.tiny);
    const T ida = m_rcp(da), idb = m_rcp(db);
    const T avg = (apa * apb * emf[0] + apa * amb * emf[2] + ama * apb * emf[1] + ama * amb * emf[3]) *
                  (ida * idb);
    return avg - apa * ama * ida * (bb1 - bb0) + apb * amb * idb * (ba2 - ba0);
  }
};
template <typename T>
__host__ __device__ __forceinline__ T uct_emf(const T C[4][7], const Consts<T>& c) {
  UctAcc<T> u;
  #pragma unroll
  for (int k = 0; k < 4; ++k) u.add(k, C[k], c);
  return u.finish(c);
}


// ---------------------------------------------------------------- UCT-HLLD edge EMF
// The HLLD flux of one transverse field component B_t through a face, for given outer
// states, is linear in that component's pair (u_t, B_t) on the two sides: the wave fan (its
// speeds, single-star densities and the star relations B*_t = phi B_t, u*_t = u_t - kap B_t)
// depends on the states but not on which transverse component is followed.  Written as
//   F_t = A_lo B_t,lo + A_hi B_t,hi - B_n (w_lo u_t,lo + w_hi u_t,hi),  w_lo + w_hi = 1,
// the coefficients are, region by region of the fan (S_L < S*_L < S_M < S*_R < S_R), with
// r = sqrt(rho*) per side, q = 1 / (r_lo + r_hi), sg = sign(B_n):
//   left of S_L:   A = (u_lo, 0),                      w = (1, 0)
//   S_L..S*_L:     A = (u_lo + S_L (phi_lo - 1), 0),   w = (1, 0)
//   S*_L..S_M:     A_lo = u_lo + S_L (phi_lo - 1) + S*_L ((r_hi phi_lo + r_lo r_hi sg kap_lo) q - phi_lo)
//                  A_hi = S*_L (r_lo phi_hi - r_lo r_hi sg kap_hi) q,  w_hi = -S*_L r_lo r_hi q / |B_n|
// and mirrored right of the contact (the jump of the flux across a wave is the wave speed times
// the jump of B_t; the double-star field is Miyoshi & Kusano's r-weighted average of the two
// single-star fields plus sg r_lo r_hi q times the velocity jump).  In the double-star regions
// |B_n| > 0 (S*_L < 0 <= S_M needs |B_n| / r_lo > S_M >= 0), so the division is safe.
template <typename T>
struct BtCoef {
  T A0, A1, w0, w1;
};
// lo, hi: (rho, u_n, p, B_t1, B_t2); bn: the shared normal field
template <typename T>
__host__ __device__ __forceinline__ BtCoef<T> hlld_bt_coef(const T lo[5], const T hi[5], T bn,
                                                           const Consts<T>& c) {
  const T bn2 = bn * bn;
  const T* sd_[2] = {lo, hi};
  T pt[2], cf[2];
  #pragma unroll
  for (int k = 0; k < 2; ++k) {
    const T* q = sd_[k];
    const T bt = q[3] * q[3] + q[4] * q[4];
    pt[k] = q[2] + T(0.5) * (bn2 + bt);
    cf[k] = fast_speed_t(wave_base(q[0], q[2], bn2 + bt, c.gamma), bt);
  }
  const T cmx = m_max(cf[0], cf[1]);
  const T S0 = m_min(lo[1], hi[1]) - cmx, S1 = m_max(lo[1], hi[1]) + cmx;
  const T mf0 = (S0 - lo[1]) * lo[0], mf1 = (S1 - hi[1]) * hi[0];  // rho (S - u) per side
  const T sm = (mf1 * hi[1] - mf0 * lo[1] - pt[1] + pt[0]) * m_rcp(mf1 - mf0);
  // star relations per side
  T phi[2], kap[2], rs[2];
  #pragma unroll
  for (int k = 0; k < 2; ++k) {
    const T Sk = k ? S1 : S0, mfk = k ? mf1 : mf0, uk = sd_[k][1];
    const T sdk = Sk - uk;
    rs[k] = mfk * m_rcp(Sk - sm);
    const T dd = mfk * (Sk - sm) - bn2;
    if (m_abs(dd) > c.eps_deg * (mfk * sdk + bn2)) {
      const T idd = m_rcp(dd);
      phi[k] = (mfk * sdk - bn2) * idd;
      kap[k] = bn * (sm - uk) * idd;
    } else {
      phi[k] = T(1);
      kap[k] = T(0);
    }
  }
  const T isq0 = m_rsqrt(rs[0]), isq1 = m_rsqrt(rs[1]);
  const T abn = m_abs(bn);
  const T Ss0 = sm - abn * isq0, Ss1 = sm + abn * isq1;
  // region of the face, in the order of the face solver (first test that holds)
  const int reg = S0 > T(0) ? 0 : Ss0 >= T(0) ? 1 : sm >= T(0) ? 2 : Ss1 >= T(0) ? 3
                : S1 >= T(0) ? 4 : 5;
  BtCoef<T> o;
  if (reg == 0) {
    o.A0 = lo[1]; o.A1 = T(0); o.w0 = T(1); o.w1 = T(0);
  } else if (reg == 1) {
    o.A0 = lo[1] + S0 * (phi[0] - T(1)); o.A1 = T(0); o.w0 = T(1); o.w1 = T(0);
  } else if (reg == 5) {
    o.A0 = T(0); o.A1 = hi[1]; o.w0 = T(0); o.w1 = T(1);
  } else if (reg == 4) {
    o.A0 = T(0); o.A1 = hi[1] + S1 * (phi[1] - T(1)); o.w0 = T(0); o.w1 = T(1);
  } else {
    // double-star regions: r_lo r_hi q = 1 / (1/r_lo + 1/r_hi)
    const T rq = m_rcp(isq0 + isq1);
    const T sg = bn < T(0) ? T(-1) : T(1);
    const T cl = isq0 * rq, ch = isq1 * rq;           // r_hi q and r_lo q
    const T Blo = phi[0] * cl + sg * rq * kap[0];      // d B** / d B_lo
    const T Bhi = phi[1] * ch - sg * rq * kap[1];      // d B** / d B_hi
    const T wv = rq * m_rcp(abn);                      // r_lo r_hi q / |B_n|
    if (reg == 2) {
      o.A0 = lo[1] + S0 * (phi[0] - T(1)) + Ss0 * (Blo - phi[0]);
      o.A1 = Ss0 * Bhi;
      o.w1 = -Ss0 * wv;
      o.w0 = T(1) - o.w1;
    } else {
      o.A1 = hi[1] + S1 * (phi[1] - T(1)) + Ss1 * (Bhi - phi[1]);
      o.A0 = Ss1 * Blo;
      o.w0 = Ss1 * wv;
      o.w1 = T(1) - o.w0;
    }
  }
  return o;
}

// Edge EMF from the four corner states (same layout and corner order as UctAcc: 0 SW, 1 SE,
// 2 NW, 3 NE; C = (rho, u_a, u_b, p, B_e, B_a, B_b)) with the HLLD fan (the UCT-HLLD
// composition).  Four one-dimensional problems: along a on the rows SW|SE and NW|NE (normal
// field B_a of the row, transverse pair (B_b, B_e)), along b on the columns SW|NW and SE|NE
// (normal field B_b of the column, transverse pair (B_e, B_a)).  EMF_e = u_a B_b - u_b B_a is
// assembled from the B_b parts of the rows and minus the B_a parts of the columns; the row
// parts are weighted by the columns' velocity weights, taken per column with the rows'
// upwind weight of that column, and the column parts symmetrically.  Data varying along one
// direction only give that direction's one-dimensional HLLD flux.
template <typename T>
__host__ __device__ __forceinline__ T uct_hlld_emf(const T C[4][7], const Consts<T>& c) {
  BtCoef<T> row[2], col[2];
  #pragma unroll
  for (int k = 0; k < 2; ++k) {
    const T* l = C[2 * k];
    const T* h = C[2 * k + 1];
    const T ql[5] = {l[0], l[1], l[3], l[6], l[4]};
    const T qh[5] = {h[0], h[1], h[3], h[6], h[4]};
    row[k] = hlld_bt_coef(ql, qh, l[5], c);
  }
  #pragma unroll
  for (int k = 0; k < 2; ++k) {
    const T* l = C[k];
    const T* h = C[k + 2];
    const T ql[5] = {l[0], l[2], l[3], l[4], l[5]};
    const T qh[5] = {h[0], h[2], h[3], h[4], h[5]};
    col[k] = hlld_bt_coef(ql, qh, l[6], c);
  }
  // rows' upwind weight of each column, columns' upwind weight of each row
  const T cw0 = T(0.5) * (row[0].w0 + row[1].w0), cw1 = T(0.5) * (row[0].w1 + row[1].w1);
  const T rw0 = T(0.5) * (col[0].w0 + col[1].w0), rw1 = T(0.5) * (col[0].w1 + col[1].w1);
  const T wS = cw0 * col[0].w0 + cw1 * col[1].w0, wN = cw0 * col[0].w1 + cw1 * col[1].w1;
  const T wW = rw0 * row[0].w0 + rw1 * row[1].w0, wE = rw0 * row[0].w1 + rw1 * row[1].w1;
  const T BbW = C[0][6], BbE = C[1][6], BaS = C[0][5], BaN = C[2][5];
  const T fa = wS * (row[0].A0 * BbW + row[0].A1 * BbE) + wN * (row[1].A0 * BbW + row[1].A1 * BbE);
  const T fb = wW * (col[0].A0 * BaS + col[0].A1 * BaN) + wE * (col[1].A0 * BaS + col[1].A1 * BaN);
  return fa - fb;
}

}  // namespace mhd
