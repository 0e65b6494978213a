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

enum BoxKind { BOX_PRIM = 0, BOX_EN = 1, BOX_PRED = 2, BOX_INTERIOR = 3, BOX_ALL = 4, NBOX = 5 };

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

// ---------------------------------------------------------------- stage 1: primitives
// Returns 1 if the conserved state is not physical (rho <= 0, p <= 0 or NaN).
template <typename T>
__host__ __device__ __forceinline__ int prim_item(const PatchDev& P, int64_t cell, const T* U,
                                                  T* S, const Consts<T>& c) {
  const int64_t Nc = P.Nc;
  const T* u = U + P.ubase;
  T rho = u[cell];
  const T mx = u[Nc + cell], my = u[2 * Nc + cell], mz = u[3 * Nc + cell], en = u[4 * Nc + cell];
  const T bx = T(0.5) * (u[5 * Nc + cell] + u[5 * Nc + cell + P.off[0]]);
  const T by = T(0.5) * (u[6 * Nc + cell] + u[6 * Nc + cell + P.off[1]]);
  const T bz = T(0.5) * (u[7 * Nc + cell] + u[7 * Nc + cell + P.off[2]]);
  int bad = !(rho > T(0));
  if (rho < c.rho_floor) rho = c.rho_floor;
  const T ir = T(1) / rho;
  const T vx = mx * ir, vy = my * ir, vz = mz * ir;
  T p = c.gm1 * (en - T(0.5) * rho * (vx * vx + vy * vy + vz * vz) -
                 T(0.5) * (bx * bx + by * by + bz * bz));
  bad |= !(p > T(0));
  if (p < c.p_floor) p = c.p_floor;
  T* q = S + P.sbase;
  q[cell] = rho;
  q[Nc + cell] = vx;
  q[2 * Nc + cell] = vy;
  q[3 * Nc + cell] = vz;
  q[4 * Nc + cell] = p;
  q[5 * Nc + cell] = bx;
  q[6 * Nc + cell] = by;
  q[7 * Nc + cell] = bz;
  return bad;
}

// ------------------------------------------------- stage 2: edge EMFs at time n
template <typename T>
__host__ __device__ __forceinline__ void en_item(const PatchDev& P, int64_t cell, const T* U, T* S) {
  const int64_t Nc = P.Nc;
  const T* u = U + P.ubase;
  const T* q = S + P.sbase;
  T* E = S + P.sbase + 8 * Nc;
  for (int e = 0; e < 3; ++e) {
    const int a = (e + 1) % 3, b = (e + 2) % 3;
    const int64_t oa = P.off[a], ob = P.off[b];
    const T* qa = q + (1 + a) * Nc;
    const T* qb = q + (1 + b) * Nc;
    const T va = T(0.25) * (qa[cell] + qa[cell - oa] + qa[cell - ob] + qa[cell - oa - ob]);
    const T vb = T(0.25) * (qb[cell] + qb[cell - oa] + qb[cell - ob] + qb[cell - oa - ob]);
    const T ba = T(0.5) * (u[(5 + a) * Nc + cell] + u[(5 + a) * Nc + cell - ob]);
    const T bb = T(0.5) * (u[(5 + b) * Nc + cell] + u[(5 + b) * Nc + cell - oa]);
    E[e * Nc + cell] = va * bb - vb * ba;
  }
}

// ------------------------------------------------------ stage 3: predictor data
template <typename T>
__host__ __device__ __forceinline__ void pred_item(const PatchDev& P, int g, int i, int j, int k,
                                                   const T* U, const T* S, T* Wout, double dt,
                                                   const double* dxp, const Consts<T>& c) {
  const int64_t Nc = P.Nc;
  const int64_t cell = cell_of(P, i, j, k);
  const T* u = U + P.ubase;
  const T* q = S + P.sbase;
  const T* E = S + P.sbase + 8 * Nc;
  T qc[8];
  for (int m = 0; m < 8; ++m) qc[m] = q[m * Nc + cell];
  T D[3][8];
  T G[3][8];
  for (int d = 0; d < 3; ++d) {
    if (!active(P, d)) {
      for (int m = 0; m < 8; ++m) { D[d][m] = T(0); G[d][m] = T(0); }
      continue;
    }
    const int64_t o = P.off[d];
    const T idx = T(1.0 / dxp[d]);
    for (int m = 0; m < 8; ++m) {
      if (m == 5 + d)
        D[d][m] = u[(5 + d) * Nc + cell + o] - u[(5 + d) * Nc + cell];
      else
        D[d][m] = limited_slope(qc[m] - q[m * Nc + cell - o], q[m * Nc + cell + o] - qc[m], c.limiter);
      G[d][m] = D[d][m] * idx;
    }
  }
  T r[8];
  prim_rate(qc, G, c.gamma, r);
  const T hdt = T(0.5 * dt);
  T* w = Wout + P.wbase;
  const int64_t wc = wcell_of(P, g, i, j, k);
  const int64_t Nw = P.Nwc;
  for (int m = 0; m < 8; ++m) w[(W_QT + m) * Nw + wc] = qc[m] + hdt * r[m];
  for (int d = 0; d < 3; ++d)
    for (int m = 0; m < 8; ++m)
      if (m != 5 + d) w[slope_slot(d, m) * Nw + wc] = D[d][m];
  // half-step face field B^{n+1/2} = B^n + dt/2 curl E^n on the three lower faces
  for (int d = 0; d < 3; ++d) {
    const int a = (d + 1) % 3, b = (d + 2) % 3;
    T v = u[(5 + d) * Nc + cell];
    if (active(P, a)) v = v + T(0.5 * dt / dxp[a]) * (E[b * Nc + cell + P.off[a]] - E[b * Nc + cell]);
    if (active(P, b)) v = v - T(0.5 * dt / dxp[b]) * (E[a * Nc + cell + P.off[b]] - E[a * Nc + cell]);
    w[(W_BH + d) * Nw + wc] = v;
  }
  // transverse slopes of the face fields (used by the corner states of the edges)
  for (int d = 0; d < 3; ++d) {
    const T* B = u + (5 + d) * Nc;
    for (int e = 0; e < 3; ++e) {
      if (e == d) continue;
      T s = T(0);
      if (active(P, e)) {
        const int64_t o = P.off[e];
        s = limited_slope(B[cell] - B[cell - o], B[cell + o] - B[cell], c.limiter);
      }
      w[dbf_slot(d, e) * Nw + wc] = s;
    }
  }
}

// ---------------------------------------------------- stage 4a: HLLD face flux
// Face of direction d on the lower side of padded cell (i, j, k).  Returns the flux in
// the face frame (rho, m_n, m_t1, m_t2, E) with (d, t1, t2) cyclic.
template <typename T>
__host__ __device__ __forceinline__ void face_flux_item(const PatchDev& P, int g, int d, int i, int j,
                                                        int k, const T* Win, const Consts<T>& c,
                                                        T F[5]) {
  const T* w = Win + P.wbase;
  const int64_t Nw = P.Nwc;
  const int64_t wr = wcell_of(P, g, i, j, k);
  const int64_t wl = wr - P.woff[d];
  const int a = (d + 1) % 3, b = (d + 2) % 3;
  const int comp[7] = {0, 1 + d, 1 + a, 1 + b, 4, 5 + a, 5 + b};
  T s[2][7];
  for (int t = 0; t < 7; ++t) {
    const int m = comp[t];
    const int sl = slope_slot(d, m);
    s[0][t] = w[m * Nw + wl] + T(0.5) * w[sl * Nw + wl];
    s[1][t] = w[m * Nw + wr] - T(0.5) * w[sl * Nw + wr];
  }
  for (int k2 = 0; k2 < 2; ++k2) {
    if (s[k2][0] < c.rho_floor) s[k2][0] = c.rho_floor;
    if (s[k2][4] < c.p_floor) s[k2][4] = c.p_floor;
  }
  const T bn = w[(W_BH + d) * Nw + wr];
  hlld_flux(s, bn, c, F);
}

// predicted corner state of predictor cell wc at corner (sa, sb) for an edge along e:
// (rho, u_a, u_b, p, B_e, B_a, B_b)
template <typename T>
__host__ __device__ __forceinline__ void corner_state(const PatchDev& P, const T* w, int64_t wc, int e,
                                                      int sa, int sb, const Consts<T>& c, T C[7]) {
  const int64_t Nw = P.Nwc;
  const int a = (e + 1) % 3, b = (e + 2) % 3;
  const int comp[5] = {0, 1 + a, 1 + b, 4, 5 + e};
  for (int t = 0; t < 5; ++t) {
    const int m = comp[t];
    const T ha = T(0.5) * w[slope_slot(a, m) * Nw + wc];
    const T hb = T(0.5) * w[slope_slot(b, m) * Nw + wc];
    C[t] = w[m * Nw + wc] + ((sa > 0 ? ha : -ha) + (sb > 0 ? hb : -hb));
  }
  const int64_t fa = wc + (sa > 0 ? P.woff[a] : 0);
  const int64_t fb = wc + (sb > 0 ? P.woff[b] : 0);
  const T ta = T(0.5) * w[dbf_slot(a, b) * Nw + fa];
  const T tb = T(0.5) * w[dbf_slot(b, a) * Nw + fb];
  C[5] = w[(W_BH + a) * Nw + fa] + (sb > 0 ? ta : -ta);
  C[6] = w[(W_BH + b) * Nw + fb] + (sa > 0 ? tb : -tb);
  if (C[0] < c.rho_floor) C[0] = c.rho_floor;
  if (C[3] < c.p_floor) C[3] = c.p_floor;
}

// -------------------------------------------------------- stage 4b: edge EMF
// Edge along e at the (a, b) = (-1/2, -1/2) corner of padded cell (i, j, k).
template <typename T>
__host__ __device__ __forceinline__ T edge_emf_item(const PatchDev& P, int g, int e, int i, int j, int k,
                                                    const T* Win, const Consts<T>& c) {
  const T* w = Win + P.wbase;
  const int a = (e + 1) % 3, b = (e + 2) % 3;
  const int64_t wc = wcell_of(P, g, i, j, k);
  const int64_t oa = P.woff[a], ob = P.woff[b];
  T C[4][7];
  corner_state(P, w, wc - oa - ob, e, +1, +1, c, C[0]);  // SW
  corner_state(P, w, wc - ob, e, -1, +1, c, C[1]);       // SE
  corner_state(P, w, wc - oa, e, +1, -1, c, C[2]);       // NW
  corner_state(P, w, wc, e, -1, -1, c, C[3]);            // NE
  return uct_emf(C, c);
}

// -------------------------------------------------------------- time step
// sum over active directions of (|u_d| + c_f,d) / dx_d at interior cell `cell`
template <typename T>
__host__ __device__ __forceinline__ double cfl_item(const PatchDev& P, int64_t cell, const T* U,
                                                    const double* dxp, const Consts<T>& c) {
  const int64_t Nc = P.Nc;
  const T* u = U + P.ubase;
  T rho = u[cell];
  if (rho < c.rho_floor) rho = c.rho_floor;
  const T ir = T(1) / rho;
  const T v[3] = {u[Nc + cell] * ir, u[2 * Nc + cell] * ir, u[3 * Nc + cell] * ir};
  T B[3];
  for (int d = 0; d < 3; ++d) B[d] = T(0.5) * (u[(5 + d) * Nc + cell] + u[(5 + d) * Nc + cell + P.off[d]]);
  T p = c.gm1 * (u[4 * Nc + cell] - T(0.5) * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) -
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

// ------------------------------------------------------------------ guard fill
// Copies one guard element of patch p from its owner (neighbour table, 27 entries per
// patch; -1 = domain boundary: zero-gradient copy).  Returns 0 if (i, j, k) is owned or
// was filled, 1 if the table is inconsistent.
template <typename T>
__host__ __device__ __forceinline__ int guard_item(const PatchDev* PT, int p, int g, int i, int j,
                                                   int k, T* U, const int32_t* nbr, int npatch) {
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
  if (!guard) return 0;
  for (int d = 0; d < 3; ++d) {
    if (!o[d]) continue;
    int f[3] = {0, 0, 0};
    f[d] = o[d];
    if (nbr[27 * p + (f[0] + 1) + 3 * (f[1] + 1) + 9 * (f[2] + 1)] < 0) {
      idx[d] = idx[d] < g ? g : (idx[d] > g + P.n[d] - 1 ? g + P.n[d] - 1 : idx[d]);
      o[d] = 0;
    }
  }
  int src = p;
  if (o[0] || o[1] || o[2]) src = nbr[27 * p + (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)];
  if (src < 0 || src >= npatch) return 1;
  const PatchDev& Q = PT[src];
  if (Q.n[0] != P.n[0] || Q.n[1] != P.n[1] || Q.n[2] != P.n[2]) return 1;
  const int64_t cs = cell_of(Q, idx[0] - o[0] * P.n[0], idx[1] - o[1] * P.n[1], idx[2] - o[2] * P.n[2]);
  const int64_t cd = cell_of(P, i, j, k);
  for (int m = 0; m < 8; ++m) U[P.ubase + m * P.Nc + cd] = U[Q.ubase + m * Q.Nc + cs];
  return 0;
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
  static constexpr int THREADS = TX * TY * TZ < 64 ? 64 : TX * TY * TZ;
};

template <typename T, int TX, int TY, int TZ, class X>
__host__ __device__ __forceinline__ void solve_tile(X& ex, T* lds, const PatchDev& P, int g,
                                                    const TileDev& tl, const T* Uin, T* Uout,
                                                    const T* Win, double dt, const double* dxp,
                                                    const Consts<T>& c) {
  using SH = TileShape<TX, TY, TZ>;
  T* fx = lds;
  T* fy = fx + 5 * SH::NFX;
  T* fz = fy + 5 * SH::NFY;
  T* ez = fz + 5 * SH::NFZ;
  T* exx = ez + SH::NEZ;
  T* ey = exx + SH::NEX;
  const int ax = active(P, 0), ay = active(P, 1), az = active(P, 2);
  const int tx = ax ? (P.n[0] - tl.x0 < TX ? P.n[0] - tl.x0 : TX) : 1;
  const int ty = ay ? (P.n[1] - tl.y0 < TY ? P.n[1] - tl.y0 : TY) : 1;
  const int tz = az ? (P.n[2] - tl.z0 < TZ ? P.n[2] - tl.z0 : TZ) : 1;
  // padded index of local (0, 0, 0)
  const int i0 = ax ? g + tl.x0 : 0, j0 = ay ? g + tl.y0 : 0, k0 = az ? g + tl.z0 : 0;
  const int tid = ex.tid(), nth = ex.nthr();

  // faces: local extents (t + 1 along the face normal)
  for (int d = 0; d < 3; ++d) {
    if (!active(P, d)) continue;
    const int ex_[3] = {tx + (d == 0), ty + (d == 1), tz + (d == 2)};
    const int LX = TX + (d == 0), LY = TY + (d == 1);
    T* fd = d == 0 ? fx : (d == 1 ? fy : fz);
    const int NF = d == 0 ? SH::NFX : (d == 1 ? SH::NFY : SH::NFZ);
    const int nitem = ex_[0] * ex_[1] * ex_[2];
    const int a = (d + 1) % 3, b = (d + 2) % 3;
    for (int it = tid; it < nitem; it += nth) {
      const int lx = it % ex_[0], ly = (it / ex_[0]) % ex_[1], lz = it / (ex_[0] * ex_[1]);
      T F[5];
      face_flux_item(P, g, d, i0 + lx, j0 + ly, k0 + lz, Win, c, F);
      const int li = lx + LX * (ly + LY * lz);
      fd[0 * NF + li] = F[0];
      fd[(1 + d) * NF + li] = F[1];
      fd[(1 + a) * NF + li] = F[2];
      fd[(1 + b) * NF + li] = F[3];
      fd[4 * NF + li] = F[4];
    }
  }
  // edges: extents t + 1 along the two transverse directions when active
  for (int e = 0; e < 3; ++e) {
    const int ex_[3] = {tx + (e != 0 && ax), ty + (e != 1 && ay), tz + (e != 2 && az)};
    const int LX = TX + (e != 0), LY = TY + (e != 1);
    T* ed = e == 0 ? exx : (e == 1 ? ey : ez);
    const int nitem = ex_[0] * ex_[1] * ex_[2];
    for (int it = tid; it < nitem; it += nth) {
      const int lx = it % ex_[0], ly = (it / ex_[0]) % ex_[1], lz = it / (ex_[0] * ex_[1]);
      ed[lx + LX * (ly + LY * lz)] = edge_emf_item(P, g, e, i0 + lx, j0 + ly, k0 + lz, Win, c);
    }
  }
  ex.sync();

  const T dtdx[3] = {T(dt / dxp[0]), T(dt / dxp[1]), T(dt / dxp[2])};
  const int ncell = tx * ty * tz;
  const int64_t Nc = P.Nc;
  for (int it = tid; it < ncell; it += nth) {
    const int lx = it % tx, ly = (it / tx) % ty, lz = it / (tx * ty);
    const int64_t cell = cell_of(P, i0 + lx, j0 + ly, k0 + lz);
    const T* u = Uin + P.ubase;
    T* uo = Uout + P.ubase;
    const int fxl = lx + (TX + 1) * (ly + TY * lz), fyl = lx + TX * (ly + (TY + 1) * lz),
              fzl = lx + TX * (ly + TY * lz);
    for (int m = 0; m < 5; ++m) {
      T v = u[m * Nc + cell];
      if (ax) v = v - dtdx[0] * (fx[m * SH::NFX + fxl + 1] - fx[m * SH::NFX + fxl]);
      if (ay) v = v - dtdx[1] * (fy[m * SH::NFY + fyl + TX] - fy[m * SH::NFY + fyl]);
      if (az) v = v - dtdx[2] * (fz[m * SH::NFZ + fzl + TX * TY] - fz[m * SH::NFZ + fzl]);
      uo[m * Nc + cell] = v;
    }
    // edge arrays: ez (TX+1)x(TY+1)xTZ, ex TXx(TY+1)x(TZ+1), ey (TX+1)xTYx(TZ+1)
    const int zl = lx + (TX + 1) * (ly + (TY + 1) * lz);
    const int xl = lx + TX * (ly + (TY + 1) * lz);
    const int yl = lx + (TX + 1) * (ly + TY * lz);
    T bx = u[5 * Nc + cell], by = u[6 * Nc + cell], bz = u[7 * Nc + cell];
    if (ay) bx = bx + dtdx[1] * (ez[zl + (TX + 1)] - ez[zl]);
    if (az) bx = bx - dtdx[2] * (ey[yl + (TX + 1) * TY] - ey[yl]);
    if (az) by = by + dtdx[2] * (exx[xl + TX * (TY + 1)] - exx[xl]);
    if (ax) by = by - dtdx[0] * (ez[zl + 1] - ez[zl]);
    if (ax) bz = bz + dtdx[0] * (ey[yl + 1] - ey[yl]);
    if (ay) bz = bz - dtdx[1] * (exx[xl + TX] - exx[xl]);
    uo[5 * Nc + cell] = bx;
    uo[6 * Nc + cell] = by;
    uo[7 * Nc + cell] = bz;
  }
}

}  // namespace mhd
