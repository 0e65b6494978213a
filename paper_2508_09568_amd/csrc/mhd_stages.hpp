// mhd_stages.hpp -- per-item stages of the patch update and the patch/launch tables.
//
// Every stage is a function of one item (a cell, a face or an edge of one patch) that
// reads and writes plain arrays; the kernels in mhd_bunch.hip map threads to items.
//
// Per patch, scratch of one update holds
//   Q  (8 x Nc): primitives rho, u, v, w, p, Bx, By, Bz (cell-centred field = mean of the
//                two face values) on cells [0, N-1) of each active direction,
//   En (3 x Nc): edge EMFs at time n from arithmetic averages (eq. of E_z in §2.1 and its
//                cyclic permutations) on cells [1, N-1),
//   W  (38 x Nw): predictor data on the cells [g-1, g+n+1) around the interior:
//                 0..7   q + dt/2 dq/dt                                  (half-step state)
//                 8..28  limited slopes, 7 per direction (all primitives but the normal
//                        field of that direction)
//                 29..31 half-step face field on the cell's lower x, y, z faces
//                 32..37 limited transverse slopes of those face fields:
//                        dBx/dy, dBx/dz, dBy/dz, dBy/dx, dBz/dx, dBz/dy.
#pragma once

#include <stdint.h>

#include "mhd_physics.hpp"

namespace mhd {

constexpr int NW = 38;       // predictor values per cell
constexpr int W_QT = 0, W_SL = 8, W_BH = 29, W_DB = 32;

struct PatchDev {
  int64_t ubase;    // element offset of the patch in the state buffers
  int64_t sbase;    // element offset of its Q and En scratch in the chunk scratch
  int64_t wbase;    // element offset of its W scratch in the chunk scratch
  int64_t Nc;       // padded cells per field
  int64_t off[3];   // neighbour offset per direction (0 for a collapsed direction)
  int64_t Nwc;      // cells of the predictor box
  int64_t woff[3];  // neighbour offset inside the predictor box
  int32_t n[3];     // interior cells
  int32_t N[3];     // padded cells
  int32_t act;      // bit d set for an active direction
  int32_t chunk;    // chunk of patches it belongs to
};

struct BoxBlock {   // one work-group: BLK consecutive items of one patch's box
  int32_t patch;
  int32_t first;
};

struct TileDev {    // one work-group of the solver: tile origin inside the interior
  int32_t patch;
  int32_t x0, y0, z0;
};

enum BoxKind { BOX_PRIM = 0, BOX_EN = 1, BOX_PRED = 2, BOX_INTERIOR = 3, BOX_ALL = 4, BOX_GUARD = 5,
               BOX_LINE = 6, NBOX = 7 };

__host__ __device__ __forceinline__ bool active(const PatchDev& P, int d) { return (P.act >> d) & 1; }

// index box of each stage, per direction: lo and size (collapsed direction: [0, 1))
__host__ __device__ __forceinline__ void box_of(const PatchDev& P, int kind, int g, int lo[3],
                                                int sz[3]) {
  for (int d = 0; d < 3; ++d) {
    if (!active(P, d)) { lo[d] = 0; sz[d] = 1; continue; }
    switch (kind) {
      case BOX_PRIM: lo[d] = 0; sz[d] = P.N[d] - 1; break;
      case BOX_EN: lo[d] = 1; sz[d] = P.N[d] - 2; break;
      case BOX_PRED: lo[d] = g - 1; sz[d] = P.n[d] + 2; break;
      case BOX_INTERIOR: lo[d] = g; sz[d] = P.n[d]; break;
      default: lo[d] = 0; sz[d] = P.N[d]; break;
    }
  }
}

// Guard cells of a patch (padded box minus interior) as one index range: first the guard
// layers normal to z (whole planes), then those normal to y inside the interior z range, then
// those normal to x inside the interior y and z ranges.
__host__ __device__ __forceinline__ int guard_count(const PatchDev& P) {
  int in[3];
  for (int d = 0; d < 3; ++d) in[d] = active(P, d) ? P.n[d] : 1;
  return P.N[0] * P.N[1] * P.N[2] - in[0] * in[1] * in[2];
}
__host__ __device__ __forceinline__ void guard_cell(const PatchDev& P, int g, int t, int& i, int& j,
                                                    int& k) {
  const int Nx = P.N[0], Ny = P.N[1], Nz = P.N[2];
  const int lo[3] = {active(P, 0) ? g : 0, active(P, 1) ? g : 0, active(P, 2) ? g : 0};
  const int in[3] = {active(P, 0) ? P.n[0] : 1, active(P, 1) ? P.n[1] : 1, active(P, 2) ? P.n[2] : 1};
  const int nz = Nz - in[2], ny = Ny - in[1], nx = Nx - in[0];  // guard layers per direction
  const int rz = nz * Ny * Nx, ry = in[2] * ny * Nx;
  if (t < rz) {
    const int q = t / (Ny * Nx), r = t - q * (Ny * Nx);
    k = q < lo[2] ? q : q + in[2];
    j = r / Nx;
    i = r - j * Nx;
  } else if (t < rz + ry) {
    t -= rz;
    const int q = t / (ny * Nx), r = t - q * (ny * Nx);
    k = lo[2] + q;
    const int jj = r / Nx;
    j = jj < lo[1] ? jj : jj + in[1];
    i = r - jj * Nx;
  } else {
    t -= rz + ry;
    const int q = t / (in[1] * nx), r = t - q * (in[1] * nx);
    k = lo[2] + q;
    const int jj = r / nx, ii = r - jj * nx;
    j = lo[1] + jj;
    i = ii < lo[0] ? ii : ii + in[0];
  }
}

__host__ __device__ __forceinline__ int64_t cell_of(const PatchDev& P, int i, int j, int k) {
  return (int64_t)i + (int64_t)P.N[0] * ((int64_t)j + (int64_t)P.N[1] * k);
}

// predictor-box index of the padded cell (i, j, k)
__host__ __device__ __forceinline__ int64_t wcell_of(const PatchDev& P, int g, int i, int j, int k) {
  const int a = active(P, 0) ? i - (g - 1) : 0;
  const int b = active(P, 1) ? j - (g - 1) : 0;
  const int c = active(P, 2) ? k - (g - 1) : 0;
  return a + P.woff[1] * b + P.woff[2] * c;
}

__host__ __device__ __forceinline__ int slope_slot(int d, int m) {
  return W_SL + 7 * d + (m < 5 + d ? m : m - 1);
}
__host__ __device__ __forceinline__ int dbf_slot(int d, int e) {
  return W_DB + 2 * d + (e == (d + 1) % 3 ? 0 : 1);
}

// Loads: every stage reads its inputs through an accessor taking the absolute element
// index of the array, so the same code runs on plain values (Ld) or on dual numbers with one
// seeded input element (LdSeed, used by the adjoint).
template <typename T>
struct Ld {
  const T* p;
  __host__ __device__ __forceinline__ T operator()(int64_t i) const { return p[i]; }
};

// Loads from one patch's block of an array (base pointer of the block) by 32-bit element
// index: a block is smaller than 4 GiB, so the address is the uniform base plus a 32-bit
// byte offset and no 64-bit index arithmetic is spent per load.
template <typename T>
struct LdRel {
  const T* p;
  uint32_t Nw;  // elements per slot of the block (slot v of cell c at v Nw + c)
  __host__ __device__ __forceinline__ T operator()(uint32_t i) const {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) +
                                       (uint32_t)(i * (uint32_t)sizeof(T)));
  }
  // elements i and i + 1 (x neighbours in a predictor block) by one memory instruction: the
  // vector units fetch 16 bytes per lane at the cost of 8 (the address only needs the
  // element's own alignment)
  __host__ __device__ __forceinline__ void pair(uint32_t i, T& a, T& b) const {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef T v2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
    const v2 v = *reinterpret_cast<const v2*>(reinterpret_cast<const char*>(p) +
                                              (uint32_t)(i * (uint32_t)sizeof(T)));
    a = v.x;
    b = v.y;
#else
    a = (*this)(i);
    b = (*this)(i + 1);
#endif
  }
  // slot v of cell c (and of cell c + 1)
  __host__ __device__ __forceinline__ T at(uint32_t c, int v) const { return (*this)(c + (uint32_t)v * Nw); }
  __host__ __device__ __forceinline__ void pair_at(uint32_t c, int v, T& a, T& b) const {
    pair(c + (uint32_t)v * Nw, a, b);
  }
};

// The same loads with the slot's base formed apart from the cell: the base is uniform across
// the wavefront (scalar registers) and the cell's byte offset is shared by every slot read at
// that cell, so a load spends no vector instruction on its address beyond the offset of its
// cell.  Used by the FP32 edge lines (3 % faster there; no gain measured in FP64 or in the
// solver tile's faces, whose scalar registers are tight).
template <bool C, class A, class B>
struct Pick {
  typedef A type;
};
template <class A, class B>
struct Pick<false, A, B> {
  typedef B type;
};

template <typename T>
struct LdSlot {
  const T* p;
  uint32_t Nw;
  __host__ __device__ __forceinline__ const char* slot(int v) const {
    return reinterpret_cast<const char*>(p) + (size_t)((uint32_t)v * Nw) * sizeof(T);
  }
  __host__ __device__ __forceinline__ T at(uint32_t c, int v) const {
    return *reinterpret_cast<const T*>(slot(v) + (uint32_t)(c * (uint32_t)sizeof(T)));
  }
  __host__ __device__ __forceinline__ void pair_at(uint32_t c, int v, T& a, T& b) const {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef T v2 __attribute__((ext_vector_type(2), aligned(sizeof(T))));
    const v2 x = *reinterpret_cast<const v2*>(slot(v) + (uint32_t)(c * (uint32_t)sizeof(T)));
    a = x.x;
    b = x.y;
#else
    a = at(c, v);
    b = at(c + 1u, v);
#endif
  }
};

template <typename T>
struct LdSeed {
  const T* p;
  int64_t seed;  // element whose derivative is taken (-1: none)
  int64_t Nw;    // elements per slot where the block holds predictor values
  __host__ __device__ __forceinline__ Dual<T> operator()(int64_t i) const {
    return Dual<T>(p[i], i == seed ? T(1) : T(0));
  }
  __host__ __device__ __forceinline__ Dual<T> at(int64_t c, int v) const { return (*this)(v * Nw + c); }
  __host__ __device__ __forceinline__ void pair_at(int64_t c, int v, Dual<T>& a, Dual<T>& b) const {
    a = at(c, v);
    b = at(c + 1, v);
  }
};

// ---------------------------------------------------------------- stage 1: primitives
// Primitives of padded cell `cell` from U (absolute indices through u).  Returns 1 if the
// conserved state is not physical (rho <= 0, p <= 0 or NaN).
template <typename S, class AU>
__host__ __device__ __forceinline__ int prim_point(const PatchDev& P, int64_t cell, const AU& u,
                                                   const Consts<S>& c, S q[8]) {
  const int64_t Nc = P.Nc, b = P.ubase + cell;
  S rho = u(b);
  const S mx = u(b + Nc), my = u(b + 2 * Nc), mz = u(b + 3 * Nc), en = u(b + 4 * Nc);
  const S bx = S(0.5) * (u(b + 5 * Nc) + u(b + 5 * Nc + P.off[0]));
  const S by = S(0.5) * (u(b + 6 * Nc) + u(b + 6 * Nc + P.off[1]));
  const S bz = S(0.5) * (u(b + 7 * Nc) + u(b + 7 * Nc + P.off[2]));
  int bad = !(rho > S(0));
  if (rho < c.rho_floor) rho = c.rho_floor;
  const S ir = m_rcp(rho);
  const S vx = mx * ir, vy = my * ir, vz = mz * ir;
  S p = c.gm1 * (en - S(0.5) * rho * (vx * vx + vy * vy + vz * vz) -
                 S(0.5) * (bx * bx + by * by + bz * bz));
  bad |= !(p > S(0));
  if (p < c.p_floor) p = c.p_floor;
  q[0] = rho; q[1] = vx; q[2] = vy; q[3] = vz;
  q[4] = p; q[5] = bx; q[6] = by; q[7] = bz;
  return bad;
}

// ------------------------------------------------- stage 2: edge EMFs at time n
// E_e at the edge along e of padded cell `cell` (corner (-1/2, -1/2) in the cyclic (a, b)
// plane): 4-cell average velocities, 2-face average fields.  q reads primitives (absolute
// index P.sbase + m Nc + cell), u reads U.
template <typename S, class AQ, class AU>
__host__ __device__ __forceinline__ S en_comp(const PatchDev& P, int64_t cell, int e, const AQ& q,
                                              const AU& u) {
  const int64_t Nc = P.Nc, qb = P.sbase + cell, ub = P.ubase + cell;
  const int a = (e + 1) % 3, b = (e + 2) % 3;
  const int64_t oa = P.off[a], ob = P.off[b];
  const int64_t qa = qb + (1 + a) * Nc, qbb = qb + (1 + b) * Nc;
  const S va = S(0.25) * (q(qa) + q(qa - oa) + q(qa - ob) + q(qa - oa - ob));
  const S vb = S(0.25) * (q(qbb) + q(qbb - oa) + q(qbb - ob) + q(qbb - oa - ob));
  const S ba = S(0.5) * (u(ub + (5 + a) * Nc) + u(ub + (5 + a) * Nc - ob));
  const S bb = S(0.5) * (u(ub + (5 + b) * Nc) + u(ub + (5 + b) * Nc - oa));
  return va * bb - vb * ba;
}
template <typename S, class AQ, class AU>
__host__ __device__ __forceinline__ void en_point(const PatchDev& P, int64_t cell, const AQ& q,
                                                  const AU& u, S E[3]) {
  for (int e = 0; e < 3; ++e) E[e] = en_comp<S>(P, cell, e, q, u);
}

// Edge EMFs at time n evaluated where they are read: the predictor reads E_e of cell c + o
// through e_at(e, comp, eb, Nc, o) with eb = P.sbase + 8 Nc + c; an ordinary accessor loads
// element eb + comp Nc + o, EnOnTheFly computes the value from the primitives and face fields
// instead (the fused predictor keeps only those in shared memory).
template <typename S, class AQ, class AU>
struct EnOnTheFly {
  const PatchDev& P;
  const AQ& q;
  const AU& u;
};
template <class AE>
__host__ __device__ __forceinline__ auto e_at(const AE& e, int comp, int64_t eb, int64_t Nc,
                                              int64_t o) -> decltype(e(eb)) {
  return e(eb + comp * Nc + o);
}
template <typename S, class AQ, class AU>
__host__ __device__ __forceinline__ S e_at(const EnOnTheFly<S, AQ, AU>& e, int comp, int64_t eb,
                                           int64_t Nc, int64_t o) {
  return en_comp<S>(e.P, eb - e.P.sbase - 8 * Nc + o, comp, e.q, e.u);
}

// ------------------------------------------------------ stage 3: predictor data
// The 38 predictor values of padded cell (i, j, k): q + dt/2 dq/dt, limited slopes, half-step
// field on the three lower faces, transverse slopes of those face fields.  q reads the
// primitives, e the edge EMFs (absolute index P.sbase + 8 Nc + e Nc + cell), u reads U.
// w receives value v by `w[v] = x`: an array of NW, or a WStore that writes it to the W block
// at once (no value is read back).
template <typename S, class AU, class AQ, class AE, class WO>
__host__ __device__ __forceinline__ void pred_point(const PatchDev& P, int i, int j, int k,
                                                    const AU& u, const AQ& q, const AE& e,
                                                    double dt, const double* dxp,
                                                    const Consts<S>& c, WO&& w) {
  const int64_t Nc = P.Nc;
  const int64_t cell = cell_of(P, i, j, k);
  const int64_t qb = P.sbase + cell, ub = P.ubase + cell, eb = P.sbase + 8 * Nc + cell;
  S qc[8];
  #pragma unroll
  for (int m = 0; m < 8; ++m) qc[m] = q(qb + m * Nc);
  S D[3][8];
  S ix[3];
  #pragma unroll
  for (int d = 0; d < 3; ++d) {
    ix[d] = S(1.0 / dxp[d]);
    if (!active(P, d)) {
      #pragma unroll
      for (int m = 0; m < 8; ++m) D[d][m] = S(0);
      continue;
    }
    const int64_t o = P.off[d];
    #pragma unroll
    for (int m = 0; m < 8; ++m) {
      if (m == 5 + d)
        D[d][m] = u(ub + (5 + d) * Nc + o) - u(ub + (5 + d) * Nc);
      else
        D[d][m] = limited_slope(qc[m] - q(qb + m * Nc - o), q(qb + m * Nc + o) - qc[m], c.limiter);
    }
  }
  S r[8];
  prim_rate(qc, D, ix, c.gamma, r);
  const S hdt = S(0.5 * dt);
  #pragma unroll
  for (int m = 0; m < 8; ++m) w[W_QT + m] = qc[m] + hdt * r[m];
  #pragma unroll
  for (int d = 0; d < 3; ++d)
    #pragma unroll
    for (int m = 0; m < 8; ++m)
      if (m != 5 + d) w[slope_slot(d, m)] = D[d][m];
  // half-step face field B^{n+1/2} = B^n + dt/2 curl E^n on the three lower faces
  #pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int a = (d + 1) % 3, b = (d + 2) % 3;
    S v = u(ub + (5 + d) * Nc);
    if (active(P, a))
      v = v + S(0.5 * dt / dxp[a]) * (e_at(e, b, eb, Nc, P.off[a]) - e_at(e, b, eb, Nc, 0));
    if (active(P, b))
      v = v - S(0.5 * dt / dxp[b]) * (e_at(e, a, eb, Nc, P.off[b]) - e_at(e, a, eb, Nc, 0));
    w[W_BH + d] = v;
  }
  // transverse slopes of the face fields (used by the corner states of the edges)
  #pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t B = ub + (5 + d) * Nc;
    #pragma unroll
    for (int f = 0; f < 3; ++f) {
      if (f == d) continue;
      S sl = S(0);
      if (active(P, f)) {
        const int64_t o = P.off[f];
        sl = limited_slope(u(B) - u(B - o), u(B + o) - u(B), c.limiter);
      }
      w[dbf_slot(d, f)] = sl;
    }
  }
}

// ---------------------------------------------------- stage 4a: HLLD face flux
// Face of direction d on the lower side of padded cell (i, j, k).  Returns the flux in
// the face frame (rho, m_n, m_t1, m_t2, E) with (d, t1, t2) cyclic.  w reads the predictor
// data of the patch by index v Nwc + wcell relative to its block (P.wbase).
template <typename S, class AW>
__host__ __device__ __forceinline__ void face_point(const PatchDev& P, int g, int d, int i, int j,
                                                    int k, const AW& w, const Consts<S>& c,
                                                    S F[5]) {
  const uint32_t wr = (uint32_t)wcell_of(P, g, i, j, k);
  const uint32_t wl = wr - (uint32_t)P.woff[d];
  const int a = (d + 1) % 3, b = (d + 2) % 3;
  const int comp[7] = {0, 1 + d, 1 + a, 1 + b, 4, 5 + a, 5 + b};
  S s[2][7];
  for (int t = 0; t < 7; ++t) {
    const int m = comp[t];
    const int sl = slope_slot(d, m);
    s[0][t] = w.at(wl, m) + S(0.5) * w.at(wl, sl);
    s[1][t] = w.at(wr, m) - S(0.5) * w.at(wr, sl);
  }
  for (int k2 = 0; k2 < 2; ++k2) {
    if (s[k2][0] < c.rho_floor) s[k2][0] = c.rho_floor;
    if (s[k2][4] < c.p_floor) s[k2][4] = c.p_floor;
  }
  const S bn = w.at(wr, W_BH + d);
  hlld_flux(s, bn, c, F);
}

// predicted corner state at corner (sa, sb) of a cell for an edge along e, from the cell's
// values v and slopes along a and b (sla, slb) of the components (rho, u_a, u_b, p, B_e), and
// the face fields BA, BB with their transverse slopes tA, tB on the faces the corner touches:
// (rho, u_a, u_b, p, B_e, B_a, B_b)
template <typename S>
__host__ __device__ __forceinline__ void corner_from(const S v[5], const S sla[5], const S slb[5],
                                                     S BA, S tA, S BB, S tB, int sa, int sb,
                                                     const Consts<S>& c, S C[7]) {
  for (int t = 0; t < 5; ++t) {
    const S ha = S(0.5) * sla[t];
    const S hb = S(0.5) * slb[t];
    C[t] = v[t] + ((sa > 0 ? ha : -ha) + (sb > 0 ? hb : -hb));
  }
  const S ta = S(0.5) * tA;
  const S tb = S(0.5) * tB;
  C[5] = BA + (sb > 0 ? ta : -ta);
  C[6] = BB + (sa > 0 ? tb : -tb);
  if (C[0] < c.rho_floor) C[0] = c.rho_floor;
  if (C[3] < c.p_floor) C[3] = c.p_floor;
}

// predicted corner state of predictor cell wc (index in the patch's predictor box) at corner
// (sa, sb) for an edge along e: (rho, u_a, u_b, p, B_e, B_a, B_b)
template <typename S, class AW>
__host__ __device__ __forceinline__ void corner_state(const PatchDev& P, const AW& w, uint32_t wc,
                                                      int e, int sa, int sb, const Consts<S>& c,
                                                      S C[7]) {
  const int a = (e + 1) % 3, b = (e + 2) % 3;
  const int comp[5] = {0, 1 + a, 1 + b, 4, 5 + e};
  S v[5], sla[5], slb[5];
  for (int t = 0; t < 5; ++t) {
    const int m = comp[t];
    v[t] = w.at(wc, m);
    sla[t] = w.at(wc, slope_slot(a, m));
    slb[t] = w.at(wc, slope_slot(b, m));
  }
  const uint32_t fa = wc + (sa > 0 ? (uint32_t)P.woff[a] : 0u);
  const uint32_t fb = wc + (sb > 0 ? (uint32_t)P.woff[b] : 0u);
  corner_from(v, sla, slb, w.at(fa, W_BH + a), w.at(fa, dbf_slot(a, b)),
              w.at(fb, W_BH + b), w.at(fb, dbf_slot(b, a)), sa, sb, c, C);
}

// -------------------------------------------------------- stage 4b: edge EMF
// Edge along e at the (a, b) = (-1/2, -1/2) corner of padded cell (i, j, k).  EMF: 0 the
// UCT-HLL composition, 1 UCT-HLLD.
template <int EMF, typename S, class AW>
__host__ __device__ __forceinline__ S edge_point(const PatchDev& P, int g, int e, int i, int j, int k,
                                                 const AW& w, const Consts<S>& c) {
  const int a = (e + 1) % 3, b = (e + 2) % 3;
  const uint32_t wc = (uint32_t)wcell_of(P, g, i, j, k);
  const uint32_t oa = (uint32_t)P.woff[a], ob = (uint32_t)P.woff[b];
  S C[4][7];
  corner_state(P, w, wc - oa - ob, e, +1, +1, c, C[0]);  // SW
  corner_state(P, w, wc - ob, e, -1, +1, c, C[1]);       // SE
  corner_state(P, w, wc - oa, e, +1, -1, c, C[2]);       // NW
  corner_state(P, w, wc, e, -1, -1, c, C[3]);            // NE
  if constexpr (EMF == 1)
    return uct_hlld_emf(C, c);
  else
    return uct_emf(C, c);
}

// Scheduling fence (device code): instructions are not moved across it, which bounds how many
// paired loads the compiler issues ahead of the arithmetic that consumes them (each holds four
// registers in FP64) and so the register count of the kernels that use them.
#if defined(__HIP_DEVICE_COMPILE__)
#define MHD_SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)
#else
#define MHD_SCHED_FENCE() ((void)0)
#endif

// ----------------------------------- paired forms (x neighbours by one memory access)
// The same items as face_point and edge_point, with the same arithmetic, for a patch whose x
// direction is active: the values of x-neighbour cells come in pairs (LdRel::pair).
//  - face_x_point: one x face (its two sides are x neighbours);
//  - edge_px_point<E>: one edge along E = 1 or 2 (two of its corners are x neighbours of the
//    other two).
// (Taking the y/z faces and x edges two per lane to pair them as well measured slower in FP64:
// the extra live state spills at the occupancy the shared memory allows.)
// Slot values of the 5 corner components and their slopes along a and b of cell wc and of
// wc + 1 (for one edge direction E).
template <int E, typename S, class AW>
__host__ __device__ __forceinline__ void corner_vals_pair(const AW& w, uint32_t wc, S v[2][5],
                                                          S sla[2][5], S slb[2][5]) {
  constexpr int a = (E + 1) % 3, b = (E + 2) % 3;
  constexpr int comp[5] = {0, 1 + a, 1 + b, 4, 5 + E};
  #pragma unroll
  for (int t = 0; t < 5; ++t) {
    const int m = comp[t];
    w.pair_at(wc, m, v[0][t], v[1][t]);
    w.pair_at(wc, slope_slot(a, m), sla[0][t], sla[1][t]);
    w.pair_at(wc, slope_slot(b, m), slb[0][t], slb[1][t]);
  }
}

template <typename S, class AW>
__host__ __device__ __forceinline__ void face_x_point(const PatchDev& P, int g, int i, int j, int k,
                                                      const AW& w, const Consts<S>& c, S F[5]) {
  const uint32_t wl = (uint32_t)wcell_of(P, g, i, j, k) - 1u;
  constexpr int comp[7] = {0, 1, 2, 3, 4, 6, 7};
  S s[2][7];
  #pragma unroll
  for (int t = 0; t < 7; ++t) {
    const int m = comp[t];
    S vl, vr, ql, qr;
    w.pair_at(wl, m, vl, vr);
    w.pair_at(wl, slope_slot(0, m), ql, qr);
    s[0][t] = vl + S(0.5) * ql;
    s[1][t] = vr - S(0.5) * qr;
  }
  #pragma unroll
  for (int k2 = 0; k2 < 2; ++k2) {
    if (s[k2][0] < c.rho_floor) s[k2][0] = c.rho_floor;
    if (s[k2][4] < c.p_floor) s[k2][4] = c.p_floor;
  }
  hlld_flux(s, w.at(wl + 1u, W_BH), c, F);
}

template <int E, int EMF, typename S, class AW>
__host__ __device__ __forceinline__ S edge_px_point(const PatchDev& P, int g, int i, int j, int k,
                                                    const AW& w, const Consts<S>& c) {
  static_assert(E == 1 || E == 2, "edges along y or z");
  constexpr int a = (E + 1) % 3, b = (E + 2) % 3;
  const uint32_t wc = (uint32_t)wcell_of(P, g, i, j, k);
  // the transverse direction that is not x: corners one cell apart along it
  constexpr int t = E == 2 ? b : a;  // E = z: (a, b) = (x, y); E = y: (a, b) = (z, x)
  const uint32_t ot = (uint32_t)P.woff[t];
  UctAcc<S> u;
  S Call[EMF == 1 ? 4 : 1][7];  // UCT-HLLD: all four corners at once
  #pragma unroll
  for (int row = 0; row < 2; ++row) {
    // cells (x - 1, row) and (x, row) along t: row 0 at t - 1, row 1 at t
    const uint32_t c0 = wc - 1u - (row == 0 ? ot : 0u);
    S v[2][5], sla[2][5], slb[2][5];
    corner_vals_pair<E>(w, c0, v, sla, slb);
    // corner signs (sa, sb) and corner index of the x - 1 and x cells of this row
    int sa[2], sb[2], kk[2];
    if (E == 2) {  // a = x, b = y: row 0 = (SW, SE), row 1 = (NW, NE)
      sa[0] = +1; sa[1] = -1;
      sb[0] = sb[1] = row == 0 ? +1 : -1;
      kk[0] = row == 0 ? 0 : 2;
      kk[1] = row == 0 ? 1 : 3;
    } else {       // a = z, b = x: row 0 (z - 1) = (SW, NW), row 1 (z) = (SE, NE)
      sa[0] = sa[1] = row == 0 ? +1 : -1;
      sb[0] = +1; sb[1] = -1;
      kk[0] = row == 0 ? 0 : 1;
      kk[1] = row == 0 ? 2 : 3;
    }
    S BA[2], tA[2], BB[2], tB[2];
    #pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t cell = c0 + (uint32_t)h;
      const uint32_t fa = cell + (sa[h] > 0 ? (uint32_t)P.woff[a] : 0u);
      const uint32_t fb = cell + (sb[h] > 0 ? (uint32_t)P.woff[b] : 0u);
      if (h == 0) {
        // the face values of both corners of the row, paired where they are x neighbours
        if (E == 2) {  // a = x: both corners read B_x on the face at x (cell c0 + 1)
          BA[0] = BA[1] = w.at(c0 + 1u, W_BH + a);
          tA[0] = tA[1] = w.at(c0 + 1u, dbf_slot(a, b));
          w.pair_at(fb, W_BH + b, BB[0], BB[1]);
          w.pair_at(fb, dbf_slot(b, a), tB[0], tB[1]);
        } else {       // b = x: both corners read B_x on the face at x (cell c0 + 1)
          w.pair_at(fa, W_BH + a, BA[0], BA[1]);
          w.pair_at(fa, dbf_slot(a, b), tA[0], tA[1]);
          BB[0] = BB[1] = w.at(c0 + 1u, W_BH + b);
          tB[0] = tB[1] = w.at(c0 + 1u, dbf_slot(b, a));
        }
      }
    }
    S C[2][7];
    #pragma unroll
    for (int h = 0; h < 2; ++h)
      corner_from(v[h], sla[h], slb[h], BA[h], tA[h], BB[h], tB[h], sa[h], sb[h], c, C[h]);
    if constexpr (EMF == 1) {
      #pragma unroll
      for (int h = 0; h < 2; ++h)
        #pragma unroll
        for (int t = 0; t < 7; ++t) Call[kk[h]][t] = C[h][t];
    } else {
      u.add(kk[0], C[0], c);
      u.add(kk[1], C[1], c);
    }
    MHD_SCHED_FENCE();
  }
  if constexpr (EMF == 1)
    return uct_hlld_emf(Call, c);
  else
    return u.finish(c);
}

// value of lane 0 of the wavefront (the caller guarantees it is the same on every lane)
__host__ __device__ __forceinline__ int wave_uniform(int v) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_readfirstlane(v);
#else
  return v;
#endif
}

// ------------------------------------------------------------------ edge lines
// The edges a patch owns, taken as lines of consecutive edges, one line per thread: edges
// along x and along y stepped in z, edges along z stepped in y.  Two of an edge's four corner
// cells lie in the line's current plane (row) and two in the previous one, so each step loads
// the values of one new plane and keeps the previous plane's in registers: about half the
// loads per edge of edge_point / edge_px_point, with the same arithmetic on the same values
// (corner_from, then the same UCT combination), so the EMFs are bitwise theirs.  For patches
// with all three directions active.
// Per patch the lines are numbered in three segments, each padded to whole wavefronts:
//   x edges: (lx, ly) in [0, n_x) x [0, n_y], lz = 0 .. n_z
//   y edges: (lx, ly) in [0, n_x] x [0, n_y), lz = 0 .. n_z
//   z edges: (lx, lz) in [0, n_x] x [0, n_z), ly = 0 .. n_y
// i.e. the lower edges of the patch's cells plus the upper layers: each edge of the patch once.
__host__ __device__ __forceinline__ int pad_wave(int n) { return (n + 63) / 64 * 64; }
__host__ __device__ __forceinline__ void edge_line_segments(const PatchDev& P, int L[3]) {
  const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
  L[0] = pad_wave(nx * (ny + 1));
  L[1] = pad_wave((nx + 1) * ny);
  L[2] = pad_wave((nx + 1) * nz);
}
__host__ __device__ __forceinline__ int edge_line_count(const PatchDev& P) {
  int L[3];
  edge_line_segments(P, L);
  return L[0] + L[1] + L[2];
}

// the 5 corner components of predictor cell wc and their slopes along a and b (edge along E)
template <int E, typename S, class AW>
__host__ __device__ __forceinline__ void corner_vals(const AW& w, uint32_t wc, S v[5], S sla[5],
                                                     S slb[5]) {
  constexpr int a = (E + 1) % 3, b = (E + 2) % 3;
  constexpr int comp[5] = {0, 1 + a, 1 + b, 4, 5 + E};
  #pragma unroll
  for (int t = 0; t < 5; ++t) {
    const int m = comp[t];
    v[t] = w.at(wc, m);
    sla[t] = w.at(wc, slope_slot(a, m));
    slb[t] = w.at(wc, slope_slot(b, m));
  }
}

// one corner into the EMF: UCT-HLL accumulates it, UCT-HLLD keeps it for the end
template <int EMF, typename S>
struct EdgeAcc {
  UctAcc<S> u;
  S C[EMF == 1 ? 4 : 1][7];
  __host__ __device__ __forceinline__ void corner(int k, const S v[5], const S sla[5], const S slb[5],
                                                  S BA, S tA, S BB, S tB, int sa, int sb,
                                                  const Consts<S>& c) {
    if constexpr (EMF == 1) {
      corner_from(v, sla, slb, BA, tA, BB, tB, sa, sb, c, C[k]);
    } else {
      S Ck[7];
      corner_from(v, sla, slb, BA, tA, BB, tB, sa, sb, c, Ck);
      u.add(k, Ck, c);
    }
  }
  __host__ __device__ __forceinline__ S finish(const Consts<S>& c) const {
    if constexpr (EMF == 1)
      return uct_hlld_emf(C, c);
    else
      return u.finish(c);
  }
};

template <typename S>
__host__ __device__ __forceinline__ void keep5(S d[5], const S s[5]) {
  #pragma unroll
  for (int t = 0; t < 5; ++t) d[t] = s[t];
}

// Edges along x at (i, j, k0 .. k0 + nk - 1) (padded indices), written to out[s * ostride].
// a = y, b = z.  Corner cells of the edge at plane k: A = (j - 1, k), B = (j, k) and A', B'
// one plane below; SW = A', SE = B', NW = A, NE = B.  The faces the corners read: B_y on the
// lower y face of B' (SW, SE) or B (NW, NE), B_z on the lower z face of A (SW, NW) or B (SE, NE).
template <int EMF, typename S, class AW>
__host__ __device__ __forceinline__ void edge_line_x(const PatchDev& P, int g, int i, int j, int k0,
                                                     int nk, const AW& w, S* out, int64_t ostride,
                                                     const Consts<S>& c) {
  const uint32_t oa = (uint32_t)P.woff[1], ob = (uint32_t)P.woff[2];
  uint32_t wb = (uint32_t)wcell_of(P, g, i, j, k0) - ob;  // B of the plane below the first edge
  S pv[2][5], psa[2][5], psb[2][5];
  corner_vals<0>(w, wb - oa, pv[0], psa[0], psb[0]);
  corner_vals<0>(w, wb, pv[1], psa[1], psb[1]);
  S pBA = w.at(wb, W_BH + 1), ptA = w.at(wb, dbf_slot(1, 2));
  for (int s = 0; s < nk; ++s) {
    wb += ob;
    S v[2][5], sla[2][5], slb[2][5];
    corner_vals<0>(w, wb - oa, v[0], sla[0], slb[0]);
    corner_vals<0>(w, wb, v[1], sla[1], slb[1]);
    const S BA = w.at(wb, W_BH + 1), tA = w.at(wb, dbf_slot(1, 2));
    const S BBa = w.at(wb - oa, W_BH + 2), tBa = w.at(wb - oa, dbf_slot(2, 1));
    const S BBb = w.at(wb, W_BH + 2), tBb = w.at(wb, dbf_slot(2, 1));
    EdgeAcc<EMF, S> acc;
    acc.corner(0, pv[0], psa[0], psb[0], pBA, ptA, BBa, tBa, +1, +1, c);  // SW
    acc.corner(1, pv[1], psa[1], psb[1], pBA, ptA, BBb, tBb, -1, +1, c);  // SE
    acc.corner(2, v[0], sla[0], slb[0], BA, tA, BBa, tBa, +1, -1, c);     // NW
    acc.corner(3, v[1], sla[1], slb[1], BA, tA, BBb, tBb, -1, -1, c);     // NE
    out[s * ostride] = acc.finish(c);
    #pragma unroll
    for (int h = 0; h < 2; ++h) {
      keep5(pv[h], v[h]);
      keep5(psa[h], sla[h]);
      keep5(psb[h], slb[h]);
    }
    pBA = BA;
    ptA = tA;
    MHD_SCHED_FENCE();
  }
}

// Edges along y at (i, j, k0 .. k0 + nk - 1): a = z, b = x.  A row is the x-neighbour pair
// (i - 1, i) of one plane (values loaded in pairs); the row below has sa = +1 (corners SW at
// i - 1, NW at i), the current row sa = -1 (SE, NE).  B_z on the lower z faces of the current
// row's pair (both rows), B_x on the lower x face of cell i of each row.
template <int EMF, typename S, class AW>
__host__ __device__ __forceinline__ void edge_line_y(const PatchDev& P, int g, int i, int j, int k0,
                                                     int nk, const AW& w, S* out, int64_t ostride,
                                                     const Consts<S>& c) {
  const uint32_t oz = (uint32_t)P.woff[2];
  uint32_t c0 = (uint32_t)wcell_of(P, g, i, j, k0) - 1u - oz;
  S pv[2][5], psa[2][5], psb[2][5];
  corner_vals_pair<1>(w, c0, pv, psa, psb);
  S pBB = w.at(c0 + 1u, W_BH), ptB = w.at(c0 + 1u, dbf_slot(0, 2));
  for (int s = 0; s < nk; ++s) {
    c0 += oz;
    S v[2][5], sla[2][5], slb[2][5];
    corner_vals_pair<1>(w, c0, v, sla, slb);
    S BA[2], tA[2];
    w.pair_at(c0, W_BH + 2, BA[0], BA[1]);
    w.pair_at(c0, dbf_slot(2, 0), tA[0], tA[1]);
    const S BB = w.at(c0 + 1u, W_BH), tB = w.at(c0 + 1u, dbf_slot(0, 2));
    EdgeAcc<EMF, S> acc;
    acc.corner(0, pv[0], psa[0], psb[0], BA[0], tA[0], pBB, ptB, +1, +1, c);
    acc.corner(2, pv[1], psa[1], psb[1], BA[1], tA[1], pBB, ptB, +1, -1, c);
    acc.corner(1, v[0], sla[0], slb[0], BA[0], tA[0], BB, tB, -1, +1, c);
    acc.corner(3, v[1], sla[1], slb[1], BA[1], tA[1], BB, tB, -1, -1, c);
    out[s * ostride] = acc.finish(c);
    #pragma unroll
    for (int h = 0; h < 2; ++h) {
      keep5(pv[h], v[h]);
      keep5(psa[h], sla[h]);
      keep5(psb[h], slb[h]);
    }
    pBB = BB;
    ptB = tB;
    MHD_SCHED_FENCE();
  }
}

// Edges along z at (i, j0 .. j0 + nj - 1, k): a = x, b = y.  A row is the x-neighbour pair
// (i - 1, i) of one y row; the row below has sb = +1 (SW at i - 1, SE at i), the current row
// sb = -1 (NW, NE).  B_x on the lower x face of cell i of each row, B_y on the lower y faces of
// the current row's pair (both rows).
template <int EMF, typename S, class AW>
__host__ __device__ __forceinline__ void edge_line_z(const PatchDev& P, int g, int i, int j0, int k,
                                                     int nj, const AW& w, S* out, int64_t ostride,
                                                     const Consts<S>& c) {
  const uint32_t oy = (uint32_t)P.woff[1];
  uint32_t c0 = (uint32_t)wcell_of(P, g, i, j0, k) - 1u - oy;
  S pv[2][5], psa[2][5], psb[2][5];
  corner_vals_pair<2>(w, c0, pv, psa, psb);
  S pBA = w.at(c0 + 1u, W_BH), ptA = w.at(c0 + 1u, dbf_slot(0, 1));
  for (int s = 0; s < nj; ++s) {
    c0 += oy;
    S v[2][5], sla[2][5], slb[2][5];
    corner_vals_pair<2>(w, c0, v, sla, slb);
    S BB[2], tB[2];
    w.pair_at(c0, W_BH + 1, BB[0], BB[1]);
    w.pair_at(c0, dbf_slot(1, 0), tB[0], tB[1]);
    const S BA = w.at(c0 + 1u, W_BH), tA = w.at(c0 + 1u, dbf_slot(0, 1));
    EdgeAcc<EMF, S> acc;
    acc.corner(0, pv[0], psa[0], psb[0], pBA, ptA, BB[0], tB[0], +1, +1, c);
    acc.corner(1, pv[1], psa[1], psb[1], pBA, ptA, BB[1], tB[1], -1, +1, c);
    acc.corner(2, v[0], sla[0], slb[0], BA, tA, BB[0], tB[0], +1, -1, c);
    acc.corner(3, v[1], sla[1], slb[1], BA, tA, BB[1], tB[1], -1, -1, c);
    out[s * ostride] = acc.finish(c);
    #pragma unroll
    for (int h = 0; h < 2; ++h) {
      keep5(pv[h], v[h]);
      keep5(psa[h], sla[h]);
      keep5(psb[h], slb[h]);
    }
    pBA = BA;
    ptA = tA;
    MHD_SCHED_FENCE();
  }
}

// Line `item` of a patch's edge lines (numbering above): its half-step EMFs into the scratch
// slots of the time-n EMFs, E_e of padded cell (i, j, k) at S[P.sbase + (8 + e) Nc + cell].
template <int EMF, typename T>
__host__ __device__ __forceinline__ void edge_line_item(const PatchDev& P, int g, int item, T* S,
                                                        const Consts<T>& c) {
  int L[3];
  edge_line_segments(P, L);
  const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
  // FP32: slot-based loads (3 % faster); FP64: the combined index (no gain measured)
  typedef typename Pick<sizeof(T) == 4, LdSlot<T>, LdRel<T>>::type Acc;
  const Acc w{S + P.wbase, (uint32_t)P.Nwc};
  T* eb = S + P.sbase + 8 * P.Nc;
  const int seg = wave_uniform(item < L[0] ? 0 : item < L[0] + L[1] ? 1 : 2);
  if (seg == 0) {
    const int lx = item % nx, ly = item / nx;
    if (ly > ny) return;
    edge_line_x<EMF>(P, g, g + lx, g + ly, g, nz + 1, w, eb + cell_of(P, g + lx, g + ly, g),
                     P.off[2], c);
  } else if (seg == 1) {
    const int r = item - L[0];
    const int lx = r % (nx + 1), ly = r / (nx + 1);
    if (ly >= ny) return;
    edge_line_y<EMF>(P, g, g + lx, g + ly, g, nz + 1, w,
                     eb + P.Nc + cell_of(P, g + lx, g + ly, g), P.off[2], c);
  } else {
    const int r = item - L[0] - L[1];
    const int lx = r % (nx + 1), lz = r / (nx + 1);
    if (lz >= nz) return;
    edge_line_z<EMF>(P, g, g + lx, g, g + lz, ny + 1, w,
                     eb + 2 * P.Nc + cell_of(P, g + lx, g, g + lz), P.off[1], c);
  }
}

// ------------------------------------------------ forward writers of stages 1-3
// Writes predictor value v of one cell straight into the patch's predictor block (base of the
// block, 32-bit offsets), so a value's registers are free once it is computed.
template <typename T>
struct WStore {
  char* b;
  uint32_t wcell, Nw;
  struct Ref {
    T* p;
    __host__ __device__ __forceinline__ void operator=(T x) const { *p = x; }
  };
  __host__ __device__ __forceinline__ Ref operator[](int v) const {
    return Ref{reinterpret_cast<T*>(b + (uint32_t)((wcell + (uint32_t)v * Nw) * (uint32_t)sizeof(T)))};
  }
};
template <typename T>
__host__ __device__ __forceinline__ WStore<T> w_store(T* base, uint32_t wcell, uint32_t Nw) {
  return WStore<T>{reinterpret_cast<char*>(base), wcell, Nw};
}

template <typename T>
__host__ __device__ __forceinline__ int prim_item(const PatchDev& P, int64_t cell, const T* U, T* S,
                                                  const Consts<T>& c) {
  T q[8];
  const int bad = prim_point(P, cell, Ld<T>{U}, c, q);
  T* o = S + P.sbase + cell;
  for (int m = 0; m < 8; ++m) o[m * P.Nc] = q[m];
  return bad;
}

template <typename T>
__host__ __device__ __forceinline__ void en_item(const PatchDev& P, int64_t cell, const T* U, T* S) {
  T E[3];
  en_point(P, cell, Ld<T>{S}, Ld<T>{U}, E);
  T* o = S + P.sbase + 8 * P.Nc + cell;
  for (int e = 0; e < 3; ++e) o[e * P.Nc] = E[e];
}

template <typename T>
__host__ __device__ __forceinline__ void pred_item(const PatchDev& P, int g, int i, int j, int k,
                                                   const T* U, const T* S, T* Wout, double dt,
                                                   const double* dxp, const Consts<T>& c) {
  pred_point(P, i, j, k, Ld<T>{U}, Ld<T>{S}, Ld<T>{S}, dt, dxp, c,
             w_store(Wout + P.wbase, (uint32_t)wcell_of(P, g, i, j, k), (uint32_t)P.Nwc));
}

template <typename T>
__host__ __device__ __forceinline__ void face_flux_item(const PatchDev& P, int g, int d, int i, int j,
                                                        int k, const T* Win, const Consts<T>& c,
                                                        T F[5]) {
  face_point(P, g, d, i, j, k, LdRel<T>{Win + P.wbase, (uint32_t)P.Nwc}, c, F);
}

template <int EMF, typename T>
__host__ __device__ __forceinline__ T edge_emf_item(const PatchDev& P, int g, int e, int i, int j, int k,
                                                    const T* Win, const Consts<T>& c) {
  return edge_point<EMF>(P, g, e, i, j, k, LdRel<T>{Win + P.wbase, (uint32_t)P.Nwc}, c);
}

// -------------------------------------------------------------- time step
// sum over active directions of (|u_d| + c_f,d) / dx_d of a cell with density r, momentum
// m, energy e and the face fields bl (lower faces) and bu (upper faces)
template <typename T>
__host__ __device__ __forceinline__ double cfl_point(const PatchDev& P, T r, const T m[3], T e,
                                                     const T bl[3], const T bu[3],
                                                     const double* dxp, const Consts<T>& c) {
  T rho = r;
  if (rho < c.rho_floor) rho = c.rho_floor;
  const T ir = m_rcp(rho);
  const T v[3] = {m[0] * ir, m[1] * ir, m[2] * ir};
  T B[3];
  for (int d = 0; d < 3; ++d) B[d] = T(0.5) * (bl[d] + bu[d]);
  T p = c.gm1 * (e - T(0.5) * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) -
                 T(0.5) * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]));
  if (p < c.p_floor) p = c.p_floor;
  double s = 0.0;
  for (int d = 0; d < 3; ++d) {
    if (!active(P, d)) continue;
    const T cf = fast_speed(rho, p, B[d], B[(d + 1) % 3], B[(d + 2) % 3], c.gamma);
    s += (double)(m_abs(v[d]) + cf) / dxp[d];
  }
  return s;
}

// the same at interior cell `cell` of the state U
template <typename T>
__host__ __device__ __forceinline__ double cfl_item(const PatchDev& P, int64_t cell, const T* U,
                                                    const double* dxp, const Consts<T>& c) {
  const int64_t Nc = P.Nc;
  const T* u = U + P.ubase;
  const T m[3] = {u[Nc + cell], u[2 * Nc + cell], u[3 * Nc + cell]};
  T bl[3], bu[3];
  for (int d = 0; d < 3; ++d) {
    bl[d] = u[(5 + d) * Nc + cell];
    bu[d] = u[(5 + d) * Nc + cell + P.off[d]];
  }
  return cfl_point(P, u[cell], m, u[4 * Nc + cell], bl, bu, dxp, c);
}

// ------------------------------------------------------------------ guard fill
// Owner of padded cell (i, j, k) of patch p under a 27-entry neighbour table (-1 = domain
// boundary: zero-gradient copy of the nearest owned cell).  Returns 0 if the cell is owned
// (src = p, scell = its own cell), 1 if it is a guard with owner (src, scell), -1 if the
// table is inconsistent.
__host__ __device__ __forceinline__ int guard_source(const PatchDev* PT, int p, int g, int i, int j,
                                                     int k, const int32_t* nbr, int npatch, int& src,
                                                     int64_t& scell) {
  const PatchDev& P = PT[p];
  int idx[3] = {i, j, k};
  int o[3] = {0, 0, 0};
  bool guard = false;
  for (int d = 0; d < 3; ++d) {
    if (!active(P, d)) continue;
    if (idx[d] < g) o[d] = -1;
    else if (idx[d] >= g + P.n[d]) o[d] = 1;
    guard |= o[d] != 0;
  }
  src = p;
  if (!guard) {
    scell = cell_of(P, i, j, k);
    return 0;
  }
  for (int d = 0; d < 3; ++d) {
    if (!o[d]) continue;
    int f[3] = {0, 0, 0};
    f[d] = o[d];
    if (nbr[27 * p + (f[0] + 1) + 3 * (f[1] + 1) + 9 * (f[2] + 1)] < 0) {
      idx[d] = idx[d] < g ? g : (idx[d] > g + P.n[d] - 1 ? g + P.n[d] - 1 : idx[d]);
      o[d] = 0;
    }
  }
  if (o[0] || o[1] || o[2]) src = nbr[27 * p + (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)];
  if (src < 0 || src >= npatch) return -1;
  const PatchDev& Q = PT[src];
  if (Q.n[0] != P.n[0] || Q.n[1] != P.n[1] || Q.n[2] != P.n[2]) return -1;
  scell = cell_of(Q, idx[0] - o[0] * P.n[0], idx[1] - o[1] * P.n[1], idx[2] - o[2] * P.n[2]);
  return 1;
}

// Copies one guard cell of patch p (all 8 fields) from its owner.  Returns 0 if (i, j, k)
// is owned or was filled, 1 if the table is inconsistent.
template <typename T>
__host__ __device__ __forceinline__ int guard_item(const PatchDev* PT, int p, int g, int i, int j,
                                                   int k, T* U, const int32_t* nbr, int npatch) {
  int src;
  int64_t cs;
  const int r = guard_source(PT, p, g, i, j, k, nbr, npatch, src, cs);
  if (r == 0) return 0;
  if (r < 0) return 1;
  const PatchDev& P = PT[p];
  const PatchDev& Q = PT[src];
  const int64_t cd = cell_of(P, i, j, k);
  for (int m = 0; m < 8; ++m) U[P.ubase + m * P.Nc + cd] = U[Q.ubase + m * Q.Nc + cs];
  return 0;
}

// Local time stepping: patch p fills its guards at its own time t[p] from two time slices
// of each owner q, (t_prev[q], U_prev) and (t[q], U).  The weight and the blend are taken in
// double without contraction (the same two roundings for every value), then rounded to T;
// an owner with a single slice (t[q] == t_prev[q]) gives its current value.
__host__ __device__ inline double time_blend(double th, double a, double b) {
#pragma clang fp contract(off)
  return (1.0 - th) * a + th * b;
}
template <typename T>
__host__ __device__ __forceinline__ int guard_item_at(const PatchDev* PT, int p, int g, int i, int j,
                                                      int k, T* U, const T* Uprev, const double* t,
                                                      const double* tprev, const int32_t* nbr,
                                                      int npatch) {
  int src;
  int64_t cs;
  const int r = guard_source(PT, p, g, i, j, k, nbr, npatch, src, cs);
  if (r == 0) return 0;
  if (r < 0) return 1;
  const PatchDev& P = PT[p];
  const PatchDev& Q = PT[src];
  const int64_t cd = cell_of(P, i, j, k);
  const bool two = t[src] > tprev[src];
  const double th = two ? (t[p] - tprev[src]) / (t[src] - tprev[src]) : 1.0;
  for (int m = 0; m < 8; ++m) {
    const int64_t e = Q.ubase + m * Q.Nc + cs;
    const double b = (double)U[e];
    U[P.ubase + m * P.Nc + cd] = (T)(two ? time_blend(th, (double)Uprev[e], b) : b);
  }
  return 0;
}

// ================================================================ adjoint stages
// The adjoint of one update at fixed dt is assembled stage by stage in reverse order.  Each
// adjoint element is a gather over the forward items that read the corresponding input:
// lambda_x = sum over items I reading x of  sum_o lambda_o(I) d o(I) / d x, where the
// derivative is the forward item evaluated in dual numbers with x seeded.  Every sum runs in a
// fixed order, so the result is deterministic; no atomics.

__host__ __device__ __forceinline__ bool owned(const PatchDev& P, int g, const int x[3]) {
  for (int d = 0; d < 3; ++d)
    if (active(P, d) && (x[d] < g || x[d] >= g + P.n[d])) return false;
  return true;
}

// adjoint of the update outputs: owned cells and faces only
template <typename T>
__host__ __device__ __forceinline__ T lam_out_at(const PatchDev& P, int g, const T* lam, int m,
                                                 const int x[3]) {
  if (!owned(P, g, x)) return T(0);
  return lam[P.ubase + m * P.Nc + cell_of(P, x[0], x[1], x[2])];
}

// forward face set of direction d: normal index in [g, g+n], transverse in [g, g+n)
__host__ __device__ __forceinline__ bool face_computed(const PatchDev& P, int g, int d, const int x[3]) {
  for (int f = 0; f < 3; ++f) {
    if (!active(P, f)) continue;
    const int hi = g + P.n[f] + (f == d ? 1 : 0);
    if (x[f] < g || x[f] >= hi) return false;
  }
  return true;
}

// forward edge set of direction e: transverse indices in [g, g+n], along e in [g, g+n)
__host__ __device__ __forceinline__ bool edge_computed(const PatchDev& P, int g, int e, const int x[3]) {
  for (int f = 0; f < 3; ++f) {
    if (!active(P, f)) continue;
    const int hi = g + P.n[f] + (f != e ? 1 : 0);
    if (x[f] < g || x[f] >= hi) return false;
  }
  return true;
}

__host__ __device__ __forceinline__ bool in_box(const PatchDev& P, int kind, int g, const int x[3]) {
  int lo[3], sz[3];
  box_of(P, kind, g, lo, sz);
  for (int d = 0; d < 3; ++d)
    if (x[d] < lo[d] || x[d] >= lo[d] + sz[d]) return false;
  return true;
}

// lambda of the face flux component m (global frame) of direction d at face x
template <typename T>
__host__ __device__ __forceinline__ T lam_flux(const PatchDev& P, int g, const T* lam, int d, int m,
                                               const int x[3], T dtdx) {
  int y[3] = {x[0], x[1], x[2]};
  y[d] -= 1;
  return dtdx * (lam_out_at(P, g, lam, m, x) - lam_out_at(P, g, lam, m, y));
}

// lambda of the edge EMF along e at edge x (constrained-transport update, per-direction dx)
template <typename T>
__host__ __device__ __forceinline__ T lam_emf(const PatchDev& P, int g, const T* lam, int e,
                                              const int x[3], const T dtdx[3]) {
  T r = T(0);
  const int d1 = (e + 1) % 3, a1 = (e + 2) % 3;  // B_d1 += dtdx_a1 (E_e[c + a1] - E_e[c])
  if (active(P, a1)) {
    int y[3] = {x[0], x[1], x[2]};
    y[a1] -= 1;
    r = r + dtdx[a1] * (lam_out_at(P, g, lam, 5 + d1, y) - lam_out_at(P, g, lam, 5 + d1, x));
  }
  const int d2 = (e + 2) % 3, b2 = (e + 1) % 3;  // B_d2 -= dtdx_b2 (E_e[c + b2] - E_e[c])
  if (active(P, b2)) {
    int y[3] = {x[0], x[1], x[2]};
    y[b2] -= 1;
    r = r + dtdx[b2] * (lam_out_at(P, g, lam, 5 + d2, x) - lam_out_at(P, g, lam, 5 + d2, y));
  }
  return r;
}

// Predictor slots a face normal to d reads (face_point): the half-step state of every
// component but the normal field, the slopes along d, the half-step normal field.
__host__ __device__ __forceinline__ bool face_reads_slot(int d, int v) {
  if (v < 8) return v != 5 + d;
  if (v < W_BH) return (v - W_SL) / 7 == d;
  return v == W_BH + d;
}
// Predictor slots an edge along e reads (corner_state, at any of its corner cells): the
// corner components, their slopes along the two transverse directions, the two transverse
// half-step face fields and their transverse slopes.
__host__ __device__ __forceinline__ bool edge_reads_slot(int e, int v) {
  const int a = (e + 1) % 3, b = (e + 2) % 3;
  const int comp[5] = {0, 1 + a, 1 + b, 4, 5 + e};
  for (int t = 0; t < 5; ++t)
    if (v == comp[t] || v == slope_slot(a, comp[t]) || v == slope_slot(b, comp[t])) return true;
  return v == W_BH + a || v == W_BH + b || v == dbf_slot(a, b) || v == dbf_slot(b, a);
}

// lambda_W[v] at predictor cell x: faces and edges that read it (those that do not read slot
// v have a zero derivative and are skipped).  PART 0: the faces' terms; PART 1: the edges'
// terms added to sum0 (the faces' sum), in the order of one pass over both -- two launches
// hold fewer registers than one (EMF: the edge solver, 0 UCT-HLL, 1 UCT-HLLD).
template <int EMF, int PART, typename T>
__host__ __device__ __forceinline__ T adj_w_item(const PatchDev& P, int g, const int x[3], int v,
                                                 const T* W, const T* lam, double dt,
                                                 const double* dxp, const Consts<T>& c,
                                                 T sum0 = T(0)) {
  typedef Dual<T> S;
  const Consts<S> cd = lift<S>(c);
  const LdSeed<T> acc{W + P.wbase, (int64_t)v * P.Nwc + wcell_of(P, g, x[0], x[1], x[2]), P.Nwc};
  const T dtdx[3] = {T(dt / dxp[0]), T(dt / dxp[1]), T(dt / dxp[2])};
  T sum = sum0;
  for (int d = 0; d < 3 && PART == 0; ++d) {
    if (!active(P, d) || !face_reads_slot(d, v)) continue;
    const int a = (d + 1) % 3, b = (d + 2) % 3;
    const int map[5] = {0, 1 + d, 1 + a, 1 + b, 4};
    for (int s = 0; s < 2; ++s) {
      int f[3] = {x[0], x[1], x[2]};
      f[d] += s;
      if (!face_computed(P, g, d, f)) continue;
      S F[5];
      face_point(P, g, d, f[0], f[1], f[2], acc, cd, F);
      for (int t = 0; t < 5; ++t) sum = sum + lam_flux(P, g, lam, d, map[t], f, dtdx[d]) * F[t].d;
    }
  }
  for (int e = 0; e < 3 && PART == 1; ++e) {
    if (!edge_reads_slot(e, v)) continue;
    const int a = (e + 1) % 3, b = (e + 2) % 3;
    for (int sb = 0; sb <= (active(P, b) ? 1 : 0); ++sb)
      for (int sa = 0; sa <= (active(P, a) ? 1 : 0); ++sa) {
        int y[3] = {x[0], x[1], x[2]};
        y[a] += sa;
        y[b] += sb;
        if (!edge_computed(P, g, e, y)) continue;
        const S em = edge_point<EMF>(P, g, e, y[0], y[1], y[2], acc, cd);
        sum = sum + lam_emf(P, g, lam, e, y, dtdx) * em.d;
      }
  }
  return sum;
}

// sum over the predictor cells y that read the seeded input of lambda_W(y) . dW(y)/d(seed),
// the seed given by the accessors.  pred_point at y reads the primitives and the face fields
// at y and y +- e_d (slopes), and the time-n edge EMFs at y and y + e_d: with a seed at x the
// cells that can read it are x and x -+ e_d (STENCIL 1, primitive or face-field seed) or x
// and x - e_d (STENCIL 2, edge-EMF seed); the others have a zero derivative and are skipped.
template <int STENCIL, typename T, class AU, class AQ, class AE>
__host__ __device__ __forceinline__ T pred_gather(const PatchDev& P, int g, const int x[3],
                                                  const AU& u, const AQ& q, const AE& e,
                                                  const T* LW, double dt, const double* dxp,
                                                  const Consts<Dual<T>>& cd) {
  T sum = T(0);
  const int r0 = active(P, 0), r1 = active(P, 1), r2 = active(P, 2);
  for (int dz = -r2; dz <= r2; ++dz)
    for (int dy = -r1; dy <= r1; ++dy)
      for (int dx = -r0; dx <= r0; ++dx) {
        if ((dx != 0) + (dy != 0) + (dz != 0) > 1) continue;  // only one direction off x
        if (STENCIL == 2 && (dx > 0 || dy > 0 || dz > 0)) continue;
        const int y[3] = {x[0] + dx, x[1] + dy, x[2] + dz};
        if (!in_box(P, BOX_PRED, g, y)) continue;
        Dual<T> w[NW];
        pred_point(P, y[0], y[1], y[2], u, q, e, dt, dxp, cd, w);
        const T* lw = LW + P.wbase + wcell_of(P, g, y[0], y[1], y[2]);
        for (int v = 0; v < NW; ++v) sum = sum + lw[(int64_t)v * P.Nwc] * w[v].d;
      }
  return sum;
}

// sum over the edge-EMF cells y that read the seeded input of lambda_E(y) . dE(y)/d(seed): the
// EMFs of cell y read the primitives of y, y - e_a, y - e_b, y - e_a - e_b and the face fields
// of y, y - e_a, y - e_b (a, b transverse), so a seed at x is read from y = x + o with o in
// {0, 1}^3 and not all three directions set
template <typename T, class AQ, class AU>
__host__ __device__ __forceinline__ T en_gather(const PatchDev& P, int g, const int x[3], const AQ& q,
                                                const AU& u, const T* LS) {
  T sum = T(0);
  const int r0 = active(P, 0), r1 = active(P, 1), r2 = active(P, 2);
  for (int dz = 0; dz <= r2; ++dz)
    for (int dy = 0; dy <= r1; ++dy)
      for (int dx = 0; dx <= r0; ++dx) {
        if (dx + dy + dz == 3) continue;
        const int y[3] = {x[0] + dx, x[1] + dy, x[2] + dz};
        if (!in_box(P, BOX_EN, g, y)) continue;
        Dual<T> E[3];
        const int64_t cy = cell_of(P, y[0], y[1], y[2]);
        en_point(P, cy, q, u, E);
        const T* le = LS + P.sbase + 8 * P.Nc + cy;
        for (int k = 0; k < 3; ++k) sum = sum + le[k * P.Nc] * E[k].d;
      }
  return sum;
}

// lambda_E[k] at edge-EMF cell x (only the predictor reads E)
template <typename T>
__host__ __device__ __forceinline__ T adj_e_item(const PatchDev& P, int g, const int x[3], int k,
                                                 const T* U, const T* S, const T* LW, double dt,
                                                 const double* dxp, const Consts<T>& c) {
  const Consts<Dual<T>> cd = lift<Dual<T>>(c);
  const int64_t seed = P.sbase + 8 * P.Nc + (int64_t)k * P.Nc + cell_of(P, x[0], x[1], x[2]);
  return pred_gather<2>(P, g, x, LdSeed<T>{U, -1}, LdSeed<T>{S, -1}, LdSeed<T>{S, seed}, LW, dt, dxp, cd);
}

// lambda_Q[m] at primitive cell x (read by the predictor and the edge EMFs at time n)
template <typename T>
__host__ __device__ __forceinline__ T adj_q_item(const PatchDev& P, int g, const int x[3], int m,
                                                 const T* U, const T* S, const T* LW, const T* LS,
                                                 double dt, const double* dxp, const Consts<T>& c) {
  const Consts<Dual<T>> cd = lift<Dual<T>>(c);
  const int64_t seed = P.sbase + (int64_t)m * P.Nc + cell_of(P, x[0], x[1], x[2]);
  const LdSeed<T> qs{S, seed}, plainU{U, -1}, plainS{S, -1};
  T sum = pred_gather<1>(P, g, x, plainU, qs, plainS, LW, dt, dxp, cd);
  if (m >= 1 && m <= 3) sum = sum + en_gather(P, g, x, qs, plainU, LS);
  return sum;
}

// lambda_U[m] at padded cell x: direct term of the update, predictor (face fields), edge EMFs
// at time n (face fields) and primitives
template <typename T>
__host__ __device__ __forceinline__ T adj_u_item(const PatchDev& P, int g, const int x[3], int m,
                                                 const T* U, const T* S, const T* LW, const T* LS,
                                                 const T* lam, double dt, const double* dxp,
                                                 const Consts<T>& c) {
  const Consts<Dual<T>> cd = lift<Dual<T>>(c);
  const int64_t seed = P.ubase + (int64_t)m * P.Nc + cell_of(P, x[0], x[1], x[2]);
  const LdSeed<T> us{U, seed}, plainS{S, -1};
  T sum = lam_out_at(P, g, lam, m, x);
  if (m >= 5) {
    sum = sum + pred_gather<1>(P, g, x, us, plainS, plainS, LW, dt, dxp, cd);
    sum = sum + en_gather(P, g, x, plainS, us, LS);
  }
  // primitives of x and of the cell below in direction m-5 (cell-centred field average; the
  // primitives of y read the fields of y and the face fields of y + e_d)
  const int r0 = active(P, 0), r1 = active(P, 1), r2 = active(P, 2);
  for (int dz = -r2; dz <= 0; ++dz)
    for (int dy = -r1; dy <= 0; ++dy)
      for (int dx = -r0; dx <= 0; ++dx) {
        if ((dx != 0) + (dy != 0) + (dz != 0) > 1) continue;
        const int y[3] = {x[0] + dx, x[1] + dy, x[2] + dz};
        if (!in_box(P, BOX_PRIM, g, y)) continue;
        Dual<T> q[8];
        const int64_t cy = cell_of(P, y[0], y[1], y[2]);
        prim_point(P, cy, us, cd, q);
        const T* lq = LS + P.sbase + cy;
        for (int k = 0; k < 8; ++k) sum = sum + lq[k * P.Nc] * q[k].d;
      }
  return sum;
}

// ------------------------------------------------ fused predictor tile (stages 1-3)
// One tile of the predictor box [g-1, g+n+1): primitives and face fields of the tile plus one
// cell around it go to shared memory L, then the 38 predictor values of the tile's cells ->
// W, with the edge EMFs at time n evaluated from L where the predictor reads them.  Stages
// 1-3 read shared memory through a patch description F of the local box (Q fields at
// [0, 8 Nl), face fields at [8 Nl, 11 Nl) with F.ubase = 3 Nl), so the point functions are
// the ones of the staged kernels.  Returns 1 if a non-physical state was met.
template <int PX, int PY, int PZ>
struct PredShape {
  static constexpr int LX = PX > 1 ? PX + 2 : 1, LY = PY > 1 ? PY + 2 : 1, LZ = PZ > 1 ? PZ + 2 : 1;
  static constexpr int NL = LX * LY * LZ;
  static constexpr int LDS_ELEMS = 11 * NL;
  static constexpr int THREADS = PX * PY * PZ < 64 ? 64 : PX * PY * PZ;
};

// The tile shape follows the bunch's activity pattern (direction d is active exactly when the
// tile extent along d exceeds 1), so the local box and its strides are compile-time constants
// (shared-memory offsets fold into the instructions); a ragged tile at the end of the box uses
// the leading part of the local box.
template <typename T, int PX, int PY, int PZ, class X>
__host__ __device__ __forceinline__ int predict_tile(X& ex, T* L, const PatchDev& P, int g,
                                                     const TileDev& tl, const T* U, T* W,
                                                     double dt, const double* dxp,
                                                     const Consts<T>& c) {
  using SH = PredShape<PX, PY, PZ>;
  constexpr int PT[3] = {PX, PY, PZ}, LB[3] = {SH::LX, SH::LY, SH::LZ};
  constexpr int64_t Nl = SH::NL;
  const int t0[3] = {tl.x0, tl.y0, tl.z0};
  int e3[3], o3[3], l3[3];  // tile extent, padded index of its first cell, local box extent
  #pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (PT[d] > 1) {
      e3[d] = P.n[d] + 2 - t0[d] < PT[d] ? P.n[d] + 2 - t0[d] : PT[d];
      o3[d] = g - 1 + t0[d];
      l3[d] = e3[d] + 2;
    } else {
      e3[d] = 1;
      o3[d] = 0;
      l3[d] = 1;
    }
  }
  PatchDev F = {};
  F.act = (PX > 1) | (PY > 1) << 1 | (PZ > 1) << 2;
  #pragma unroll
  for (int d = 0; d < 3; ++d) F.N[d] = LB[d];
  F.Nc = Nl;
  F.off[0] = PX > 1 ? 1 : 0;
  F.off[1] = PY > 1 ? LB[0] : 0;
  F.off[2] = PZ > 1 ? LB[0] * LB[1] : 0;
  F.sbase = 0;
  F.ubase = 3 * Nl;
  const int tid = ex.tid(), nth = ex.nthr();
  int bad = 0;
  // A full tile splits its item index by constants; a ragged tile numbers only its actual
  // items, so no wavefront runs with most lanes masked.
  const bool full = e3[0] == PT[0] && e3[1] == PT[1] && e3[2] == PT[2];
  // 1. primitives and face fields of the local box (local index 0 = one cell below the tile)
  const int nl = full ? (int)Nl : l3[0] * l3[1] * l3[2];
  for (int it0 = tid; it0 < nl; it0 += nth) {
    int li, lj, lk;
    if (full) {
      li = it0 % LB[0]; lj = (it0 / LB[0]) % LB[1]; lk = it0 / (LB[0] * LB[1]);
    } else {
      li = it0 % l3[0]; lj = (it0 / l3[0]) % l3[1]; lk = it0 / (l3[0] * l3[1]);
    }
    const int it = li + LB[0] * (lj + LB[1] * lk);
    const int gi = PX > 1 ? o3[0] - 1 + li : 0;
    const int gj = PY > 1 ? o3[1] - 1 + lj : 0;
    const int gk = PZ > 1 ? o3[2] - 1 + lk : 0;
    const int64_t gc = cell_of(P, gi, gj, gk);
    T q[8];
    bad |= prim_point(P, gc, Ld<T>{U}, c, q);
    for (int m = 0; m < 8; ++m) L[m * Nl + it] = q[m];
    for (int d = 0; d < 3; ++d) L[(8 + d) * Nl + it] = U[P.ubase + (5 + d) * P.Nc + gc];
  }
  ex.sync();
  // 2. predictor values of the tile's cells (local [1, e + 1) in active directions)
  constexpr int lo3[3] = {PX > 1, PY > 1, PZ > 1};
  const Ld<T> lq{L};
  const EnOnTheFly<T, Ld<T>, Ld<T>> le{F, lq, lq};
  const int nt = full ? PX * PY * PZ : e3[0] * e3[1] * e3[2];
  for (int it = tid; it < nt; it += nth) {
    int ti, tj, tk;
    if (full) {
      ti = it % PX; tj = (it / PX) % PY; tk = it / (PX * PY);
    } else {
      ti = it % e3[0]; tj = (it / e3[0]) % e3[1]; tk = it / (e3[0] * e3[1]);
    }
    const int gi = PX > 1 ? o3[0] + ti : 0;
    const int gj = PY > 1 ? o3[1] + tj : 0;
    const int gk = PZ > 1 ? o3[2] + tk : 0;
    pred_point(F, lo3[0] + ti, lo3[1] + tj, lo3[2] + tk, lq, lq, le, dt, dxp, c,
               w_store(W + P.wbase, (uint32_t)wcell_of(P, g, gi, gj, gk), (uint32_t)P.Nwc));
  }
  return bad;
}

// ---------------------------------------------------- solver tile (fluxes + update)
// One tile of TX x TY x TZ interior cells: HLLD fluxes on its faces, edge EMFs on its
// edges (shared memory), then the conservative + constrained-transport update of its
// cells.  X provides tid(), nthr() and sync() of the work-group.

template <int TX, int TY, int TZ>
struct TileShape {
  static constexpr int NFX = (TX + 1) * TY * TZ, NFY = TX * (TY + 1) * TZ, NFZ = TX * TY * (TZ + 1);
  static constexpr int NEZ = (TX + 1) * (TY + 1) * TZ, NEX = TX * (TY + 1) * (TZ + 1),
                       NEY = (TX + 1) * TY * (TZ + 1);
  static constexpr int LDS_ELEMS = 5 * (NFX + NFY + NFZ) + NEZ + NEX + NEY;
  // two-phase tile (faces and hydro update, then edges and field update): the flux and EMF
  // arrays take turns in the same shared memory
  static constexpr int NFLUX = 5 * (NFX + NFY + NFZ), NEMF = NEZ + NEX + NEY;
  static constexpr int LDS_SPLIT = NFLUX > NEMF ? NFLUX : NEMF;
  template <int FORM>
  struct Lds {
    static constexpr int value = FORM == 0 ? LDS_ELEMS : (FORM == 1 ? LDS_SPLIT : NFLUX);
  };
  static constexpr int THREADS = TX * TY * TZ < 64 ? 64 : TX * TY * TZ;
  static_assert(THREADS % 64 == 0, "solver work-groups are whole wavefronts");
};

// A tile of a patch whose time step is zero (at rest in a local-time-stepping run): the update
// is the identity, so its cells' 8 values (cell fields and owned lower faces) are copied.
template <int TX, int TY, int TZ, typename T, class X>
__host__ __device__ __forceinline__ void copy_tile(X& ex, const PatchDev& P, int g,
                                                   const TileDev& tl, const T* Uin, T* Uout) {
  constexpr int ax = TX > 1, ay = TY > 1, az = TZ > 1;
  const int tx = ax ? (P.n[0] - tl.x0 < TX ? P.n[0] - tl.x0 : TX) : 1;
  const int ty = ay ? (P.n[1] - tl.y0 < TY ? P.n[1] - tl.y0 : TY) : 1;
  const int tz = az ? (P.n[2] - tl.z0 < TZ ? P.n[2] - tl.z0 : TZ) : 1;
  const int i0 = ax ? g + tl.x0 : 0, j0 = ay ? g + tl.y0 : 0, k0 = az ? g + tl.z0 : 0;
  const T* u = Uin + P.ubase;
  T* uo = Uout + P.ubase;
  for (int it = ex.tid(); it < tx * ty * tz; it += ex.nthr()) {
    const int64_t cell = cell_of(P, i0 + it % tx, j0 + (it / tx) % ty, k0 + it / (tx * ty));
    for (int m = 0; m < 8; ++m) uo[m * P.Nc + cell] = u[m * P.Nc + cell];
  }
}

// FORM 0: face fluxes and edge EMFs of the tile in shared memory together, then the update;
// FORM 1: two phases (faces and hydro update, then edges and field update) sharing the
// shared memory; FORM 2: faces only, the half-step edge EMFs having been computed once per
// edge by a FORM 3 pass into the scratch slots of the time-n EMFs (P.sbase + (8 + e) Nc);
// FORM 3: that pass -- the edges the tile owns (its cells' lower edges, plus the upper layer
// where the tile ends the patch), written to the scratch, no update.
// With nbr != nullptr the tile also returns the largest sum over directions of
// (|u_d| + c_f,d) / dx_d of its updated cells (the time-step rule) as the state will be after
// the guard exchange with the neighbour table nbr: the upper face of a cell is the face the
// next cell's update writes, which the tile computes from its edge EMFs -- at a face shared
// with a neighbour patch it is the value that patch's update writes there (the same EMFs,
// the same dt); at a domain boundary (nbr entry -1) the exchange copies the last owned face.
// Otherwise it returns 0.
// KEEP: each cell's state is read before any of it is written and no other cell of Uin is
// read (nbr must be nullptr), so the update may run in place (Uout == Uin), and the cell's
// state before the update is also written to keep (the previous time slice of local time
// stepping: owned cells and faces).
template <typename T, int TX, int TY, int TZ, int FORM, int EMF, bool KEEP = false, class X>
__host__ __device__ __forceinline__ double solve_tile(X& ex, T* lds, const PatchDev& P, int g,
                                                    const TileDev& tl, const T* Uin, T* Uout,
                                                    const T* Win, double dt, const double* dxp,
                                                    const Consts<T>& c,
                                                    const int32_t* nbr = nullptr, int patch = 0,
                                                    T* keep = nullptr) {
  using SH = TileShape<TX, TY, TZ>;
  T* fx = lds;
  T* fy = fx + 5 * SH::NFX;
  T* fz = fy + 5 * SH::NFY;
  constexpr int SPLIT = FORM == 1, EXT = FORM == 2, EDGES = FORM == 3;
  T* ez = SPLIT ? lds : fz + 5 * SH::NFZ;
  T* exx = ez + SH::NEZ;
  T* ey = exx + SH::NEX;
  // the tile shape follows the bunch's activity pattern: direction d is active exactly when
  // the tile extent along d exceeds 1
  constexpr int ax = TX > 1, ay = TY > 1, az = TZ > 1;
  const int tx = ax ? (P.n[0] - tl.x0 < TX ? P.n[0] - tl.x0 : TX) : 1;
  const int ty = ay ? (P.n[1] - tl.y0 < TY ? P.n[1] - tl.y0 : TY) : 1;
  const int tz = az ? (P.n[2] - tl.z0 < TZ ? P.n[2] - tl.z0 : TZ) : 1;
  // padded index of local (0, 0, 0)
  const int i0 = ax ? g + tl.x0 : 0, j0 = ay ? g + tl.y0 : 0, k0 = az ? g + tl.z0 : 0;
  const int tid = ex.tid(), nth = ex.nthr();

  // Work list of the tile: six segments (faces normal to x, y, z; edges along x, y, z),
  // each padded to whole wavefronts.  The work-group size is a multiple of the wavefront,
  // so every wavefront works on one segment per round: the face/edge branch and the
  // direction-dependent offsets stay uniform across its lanes, and the rounds are shared
  // by all segments instead of each direction leaving a ragged last round.  Segment k has
  // the compile-time extent of a full tile (so the item index splits by constants); items
  // beyond the tile's actual extent (ragged tiles, collapsed directions) are skipped.
  // SPLIT: faces first (then the hydro update), edges after (then the field update), so
  // flux and EMF arrays share the shared memory.
  // With x active, the x faces and the y and z edges read the values of x-neighbour cells in
  // pairs (one memory instruction for two values).
  constexpr int WAVE = 64;
  constexpr bool PR = TX > 1;
  constexpr int X1 = TX > 1 ? TX + 1 : 1, Y1 = TY > 1 ? TY + 1 : 1, Z1 = TZ > 1 ? TZ + 1 : 1;
  constexpr int NS[6] = {X1 * TY * TZ, TX * Y1 * TZ, TX * TY * Z1,
                         TX * Y1 * Z1, X1 * TY * Z1, X1 * Y1 * TZ};
  constexpr int B1 = (NS[0] + WAVE - 1) / WAVE * WAVE, B2 = B1 + (NS[1] + WAVE - 1) / WAVE * WAVE,
                B3 = B2 + (NS[2] + WAVE - 1) / WAVE * WAVE, B4 = B3 + (NS[3] + WAVE - 1) / WAVE * WAVE,
                B5 = B4 + (NS[4] + WAVE - 1) / WAVE * WAVE, B6 = B5 + (NS[5] + WAVE - 1) / WAVE * WAVE;
  const int fact[3] = {ax, ay, az};
  const T dtdx[3] = {T(dt / dxp[0]), T(dt / dxp[1]), T(dt / dxp[2])};
  // external EMFs: E_e of padded cell (i, j, k) at Win[P.sbase + (8 + e) Nc + cell]
  const T* eg = Win + P.sbase + 8 * P.Nc;
  const int ncell = tx * ty * tz;
  const int64_t Nc = P.Nc;
  const T* u = Uin + P.ubase;
  T* uo = Uout + P.ubase;
  T* kp = KEEP ? keep + P.ubase : nullptr;
  const LdRel<T> wa{Win + P.wbase, (uint32_t)P.Nwc};
  // time step of the next step: per direction, whether the tile's last cells sit at a domain
  // boundary (their upper face is then the exchange's copy of the last owned face)
  const bool cfl = nbr != nullptr;
  bool obnd[3] = {false, false, false};
  if (cfl) {
    obnd[0] = ax && tl.x0 + tx == P.n[0] && nbr[27 * patch + 14] < 0;
    obnd[1] = ay && tl.y0 + ty == P.n[1] && nbr[27 * patch + 16] < 0;
    obnd[2] = az && tl.z0 + tz == P.n[2] && nbr[27 * patch + 22] < 0;
  }
  double smx = 0.0;

  for (int phase = 0; phase < (SPLIT ? 2 : 1); ++phase) {
    if (EDGES) {
      // the owned edges only; no shared memory, no update
      for (int it = B3 + tid; it < B6; it += nth) {
        const int k = wave_uniform(it < B4 ? 3 : it < B5 ? 4 : 5);
        int lx, ly, lz;
        switch (k) {
          case 3: { const int r = it - B3; lx = r % TX; ly = (r / TX) % Y1; lz = r / (TX * Y1); break; }
          case 4: { const int r = it - B4; lx = r % X1; ly = (r / X1) % TY; lz = r / (X1 * TY); break; }
          default: { const int r = it - B5; lx = r % X1; ly = (r / X1) % Y1; lz = r / (X1 * Y1); break; }
        }
        const int e = k - 3;
        const int e0 = tx + (e != 0 && ax && tl.x0 + tx == P.n[0]);
        const int e1 = ty + (e != 1 && ay && tl.y0 + ty == P.n[1]);
        const int e2 = tz + (e != 2 && az && tl.z0 + tz == P.n[2]);
        if (lx >= e0 || ly >= e1 || lz >= e2) continue;
        const int64_t cg = cell_of(P, i0 + lx, j0 + ly, k0 + lz);
        T* eo = const_cast<T*>(eg) + e * Nc + cg;
        if (PR && e == 1)
          eo[0] = edge_px_point<1, EMF>(P, g, i0 + lx, j0 + ly, k0 + lz, wa, c);
        else if (PR && e == 2)
          eo[0] = edge_px_point<2, EMF>(P, g, i0 + lx, j0 + ly, k0 + lz, wa, c);
        else
          eo[0] = edge_emf_item<EMF>(P, g, e, i0 + lx, j0 + ly, k0 + lz, Win, c);
      }
      return 0.0;
    }
    const int ibeg = SPLIT && phase == 1 ? B3 : 0;
    const int iend = (SPLIT && phase == 0) || EXT ? B3 : B6;
    for (int it = ibeg + tid; it < iend; it += nth) {
      const int k = wave_uniform(it < B1 ? 0 : it < B2 ? 1 : it < B3 ? 2 : it < B4 ? 3 : it < B5 ? 4 : 5);
      int lx, ly, lz, e0, e1, e2;
      switch (k) {
        case 0: { const int r = it;      lx = r % X1; ly = (r / X1) % TY; lz = r / (X1 * TY); break; }
        case 1: { const int r = it - B1; lx = r % TX; ly = (r / TX) % Y1; lz = r / (TX * Y1); break; }
        case 2: { const int r = it - B2; lx = r % TX; ly = (r / TX) % TY; lz = r / (TX * TY); break; }
        case 3: { const int r = it - B3; lx = r % TX; ly = (r / TX) % Y1; lz = r / (TX * Y1); break; }
        case 4: { const int r = it - B4; lx = r % X1; ly = (r / X1) % TY; lz = r / (X1 * TY); break; }
        default: { const int r = it - B5; lx = r % X1; ly = (r / X1) % Y1; lz = r / (X1 * Y1); break; }
      }
      if (k < 3) {
        // face normal to d: actual extents t + 1 along d; none for a collapsed d
        const int d = k;
        if (!fact[d]) continue;
        e0 = tx + (d == 0);
        e1 = ty + (d == 1);
        e2 = tz + (d == 2);
        if (lx >= e0 || ly >= e1 || lz >= e2) continue;
        const int LX = TX + (d == 0), LY = TY + (d == 1);
        T* fd = d == 0 ? fx : (d == 1 ? fy : fz);
        const int NF = d == 0 ? SH::NFX : (d == 1 ? SH::NFY : SH::NFZ);
        const int a = (d + 1) % 3, b = (d + 2) % 3;
        T F[5];
        if (PR && d == 0)
          face_x_point(P, g, i0 + lx, j0 + ly, k0 + lz, wa, c, F);
        else
          face_flux_item(P, g, d, i0 + lx, j0 + ly, k0 + lz, Win, c, F);
        const int li = lx + LX * (ly + LY * lz);
        fd[0 * NF + li] = F[0];
        fd[(1 + d) * NF + li] = F[1];
        fd[(1 + a) * NF + li] = F[2];
        fd[(1 + b) * NF + li] = F[3];
        fd[4 * NF + li] = F[4];
      } else if (!EXT) {
        // edge along e: extents t + 1 along the two transverse directions when active
        const int e = k - 3;
        e0 = tx + (e != 0 && ax);
        e1 = ty + (e != 1 && ay);
        e2 = tz + (e != 2 && az);
        if (lx >= e0 || ly >= e1 || lz >= e2) continue;
        const int LX = TX + (e != 0), LY = TY + (e != 1);
        T* ed = e == 0 ? exx : (e == 1 ? ey : ez);
        const int li = lx + LX * (ly + LY * lz);
        if (PR && e == 1)
          ed[li] = edge_px_point<1, EMF>(P, g, i0 + lx, j0 + ly, k0 + lz, wa, c);
        else if (PR && e == 2)
          ed[li] = edge_px_point<2, EMF>(P, g, i0 + lx, j0 + ly, k0 + lz, wa, c);
        else
          ed[li] = edge_emf_item<EMF>(P, g, e, i0 + lx, j0 + ly, k0 + lz, Win, c);
      }
    }
    ex.sync();

    for (int it = tid; it < ncell; it += nth) {
      const int lx = it % tx, ly = (it / tx) % ty, lz = it / (tx * ty);
      const int64_t cell = cell_of(P, i0 + lx, j0 + ly, k0 + lz);
      T hn[5];  // the cell's new density, momentum, energy
      const bool hyd = !SPLIT || phase == 0, mag = !SPLIT || phase == 1;
      T u0[8];  // KEEP: the fields this phase updates, all read before any write
      if constexpr (KEEP) {
        if (hyd)
          for (int m = 0; m < 5; ++m) u0[m] = u[m * Nc + cell];
        if (mag)
          for (int m = 5; m < 8; ++m) u0[m] = u[m * Nc + cell];
        if (hyd)
          for (int m = 0; m < 5; ++m) kp[m * Nc + cell] = u0[m];
        if (mag)
          for (int m = 5; m < 8; ++m) kp[m * Nc + cell] = u0[m];
      }
      if (hyd) {
        const int fxl = lx + (TX + 1) * (ly + TY * lz), fyl = lx + TX * (ly + (TY + 1) * lz),
                  fzl = lx + TX * (ly + TY * lz);
        for (int m = 0; m < 5; ++m) {
          T v = KEEP ? u0[m] : u[m * Nc + cell];
          if (ax) v = v - dtdx[0] * (fx[m * SH::NFX + fxl + 1] - fx[m * SH::NFX + fxl]);
          if (ay) v = v - dtdx[1] * (fy[m * SH::NFY + fyl + TX] - fy[m * SH::NFY + fyl]);
          if (az) v = v - dtdx[2] * (fz[m * SH::NFZ + fzl + TX * TY] - fz[m * SH::NFZ + fzl]);
          uo[m * Nc + cell] = v;
          hn[m] = v;
        }
      } else if (cfl) {
        for (int m = 0; m < 5; ++m) hn[m] = uo[m * Nc + cell];  // written by this thread in phase 0
      }
      T bl[3], bu[3];  // new lower and upper faces (time step of the next step)
      if (EXT) {
        const int64_t ox = P.off[0], oy = P.off[1], oz = P.off[2];
        const T* E0 = eg;
        const T* E1 = eg + Nc;
        const T* E2 = eg + 2 * Nc;
        T bx = KEEP ? u0[5] : u[5 * Nc + cell], by = KEEP ? u0[6] : u[6 * Nc + cell],
          bz = KEEP ? u0[7] : u[7 * Nc + cell];
        if (ay) bx = bx + dtdx[1] * (E2[cell + oy] - E2[cell]);
        if (az) bx = bx - dtdx[2] * (E1[cell + oz] - E1[cell]);
        if (az) by = by + dtdx[2] * (E0[cell + oz] - E0[cell]);
        if (ax) by = by - dtdx[0] * (E2[cell + ox] - E2[cell]);
        if (ax) bz = bz + dtdx[0] * (E1[cell + ox] - E1[cell]);
        if (ay) bz = bz - dtdx[1] * (E0[cell + oy] - E0[cell]);
        uo[5 * Nc + cell] = bx;
        uo[6 * Nc + cell] = by;
        uo[7 * Nc + cell] = bz;
        if (cfl) {
          bl[0] = bx; bl[1] = by; bl[2] = bz;
          const int64_t cx = cell + ox, cy = cell + oy, cz = cell + oz;
          T ux = u[5 * Nc + cx], uy = u[6 * Nc + cy], uz = u[7 * Nc + cz];
          if (ay) ux = ux + dtdx[1] * (E2[cx + oy] - E2[cx]);
          if (az) ux = ux - dtdx[2] * (E1[cx + oz] - E1[cx]);
          if (az) uy = uy + dtdx[2] * (E0[cy + oz] - E0[cy]);
          if (ax) uy = uy - dtdx[0] * (E2[cy + ox] - E2[cy]);
          if (ax) uz = uz + dtdx[0] * (E1[cz + ox] - E1[cz]);
          if (ay) uz = uz - dtdx[1] * (E0[cz + oy] - E0[cz]);
          bu[0] = ux; bu[1] = uy; bu[2] = uz;
        }
      } else if (!SPLIT || phase == 1) {
        // edge arrays: ez (TX+1)x(TY+1)xTZ, ex TXx(TY+1)x(TZ+1), ey (TX+1)xTYx(TZ+1)
        const int zl = lx + (TX + 1) * (ly + (TY + 1) * lz);
        const int xl = lx + TX * (ly + (TY + 1) * lz);
        const int yl = lx + (TX + 1) * (ly + TY * lz);
        T bx = KEEP ? u0[5] : u[5 * Nc + cell], by = KEEP ? u0[6] : u[6 * Nc + cell],
          bz = KEEP ? u0[7] : u[7 * Nc + cell];
        if (ay) bx = bx + dtdx[1] * (ez[zl + (TX + 1)] - ez[zl]);
        if (az) bx = bx - dtdx[2] * (ey[yl + (TX + 1) * TY] - ey[yl]);
        if (az) by = by + dtdx[2] * (exx[xl + TX * (TY + 1)] - exx[xl]);
        if (ax) by = by - dtdx[0] * (ez[zl + 1] - ez[zl]);
        if (ax) bz = bz + dtdx[0] * (ey[yl + 1] - ey[yl]);
        if (ay) bz = bz - dtdx[1] * (exx[xl + TX] - exx[xl]);
        uo[5 * Nc + cell] = bx;
        uo[6 * Nc + cell] = by;
        uo[7 * Nc + cell] = bz;
        if (cfl) {
          bl[0] = bx; bl[1] = by; bl[2] = bz;
          // the same formulas one face up: x at (lx + 1), y at (ly + 1), z at (lz + 1)
          const int zx = zl + 1, yx = yl + 1;
          const int xy = xl + TX, zy = zl + (TX + 1);
          const int yz = yl + (TX + 1) * TY, xz = xl + TX * (TY + 1);
          T ux = u[5 * Nc + cell + P.off[0]], uy = u[6 * Nc + cell + P.off[1]],
            uz = u[7 * Nc + cell + P.off[2]];
          if (ay) ux = ux + dtdx[1] * (ez[zx + (TX + 1)] - ez[zx]);
          if (az) ux = ux - dtdx[2] * (ey[yx + (TX + 1) * TY] - ey[yx]);
          if (az) uy = uy + dtdx[2] * (exx[xy + TX * (TY + 1)] - exx[xy]);
          if (ax) uy = uy - dtdx[0] * (ez[zy + 1] - ez[zy]);
          if (ax) uz = uz + dtdx[0] * (ey[yz + 1] - ey[yz]);
          if (ay) uz = uz - dtdx[1] * (exx[xz + TX] - exx[xz]);
          bu[0] = ux; bu[1] = uy; bu[2] = uz;
        }
      }
      if (cfl && (!SPLIT || phase == 1)) {
        const bool last[3] = {lx == tx - 1, ly == ty - 1, lz == tz - 1};
        for (int d = 0; d < 3; ++d) {
          if (!fact[d]) bu[d] = bl[d];                     // collapsed: one face
          else if (obnd[d] && last[d]) bu[d] = bl[d];      // exchange copies the last owned face
        }
        const T mn[3] = {hn[1], hn[2], hn[3]};
        const double sc = cfl_point(P, hn[0], mn, hn[4], bl, bu, dxp, c);
        smx = smx > sc ? smx : sc;
      }
    }
    if (SPLIT && phase == 0) ex.sync();  // the edge phase overwrites the fluxes
  }
  return smx;
}

}  // namespace mhd
