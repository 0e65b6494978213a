// mhd_bunch.hip -- kernels and C ABI of the ideal-MHD bunch update for gfx950.
//
// One update of a chunk of patches runs four kernels on the caller's stream:
//   k_prim  : primitives on every padded cell                      (box [0, N-1))
//   k_en    : edge EMFs at time n from 4-cell / 2-face averages      (box [1, N-1))
//   k_pred  : limited slopes, half-step state, half-step face field,
//             transverse face-field slopes on the cells around the interior
//   k_solve : per 3D tile, HLLD on every face and the four-state EMF on every edge into
//             shared memory, then the conservative + constrained-transport update.
// Side kernels: k_cfl (per-patch time step, wavefront max-reduction + one 64-bit atomic
// per work-group), k_guards (guard fill from a neighbour table).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "mhd_bunch.h"
#include "mhd_stages.hpp"

using namespace mhd;

namespace {

constexpr int BLK = 256;

struct DevX {
  __device__ int tid() const { return threadIdx.x; }
  __device__ int nthr() const { return blockDim.x; }
  __device__ void sync() const { __syncthreads(); }
};

__device__ __forceinline__ bool decode(const PatchDev& P, int kind, int g, int first, int& i, int& j,
                                       int& k) {
  int lo[3], sz[3];
  box_of(P, kind, g, lo, sz);
  const int it = first + (int)threadIdx.x;
  if (it >= sz[0] * sz[1] * sz[2]) return false;
  i = lo[0] + it % sz[0];
  j = lo[1] + (it / sz[0]) % sz[1];
  k = lo[2] + it / (sz[0] * sz[1]);
  return true;
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_prim(const PatchDev* __restrict__ pt,
                                              const BoxBlock* __restrict__ blk,
                                              const T* __restrict__ U, T* __restrict__ S,
                                              Consts<T> c, int g, int* status) {
  const BoxBlock b = blk[blockIdx.x];
  const PatchDev P = pt[b.patch];
  int i, j, k;
  if (!decode(P, BOX_PRIM, g, b.first, i, j, k)) return;
  if (prim_item(P, cell_of(P, i, j, k), U, S, c)) atomicOr(status, 1);
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_en(const PatchDev* __restrict__ pt,
                                            const BoxBlock* __restrict__ blk,
                                            const T* __restrict__ U, T* __restrict__ S, int g) {
  const BoxBlock b = blk[blockIdx.x];
  const PatchDev P = pt[b.patch];
  int i, j, k;
  if (!decode(P, BOX_EN, g, b.first, i, j, k)) return;
  en_item(P, cell_of(P, i, j, k), U, S);
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_pred(const PatchDev* __restrict__ pt,
                                              const BoxBlock* __restrict__ blk,
                                              const T* __restrict__ U, T* __restrict__ S,
                                              const double* __restrict__ dt,
                                              const double* __restrict__ dx, Consts<T> c, int g) {
  const BoxBlock b = blk[blockIdx.x];
  const PatchDev P = pt[b.patch];
  int i, j, k;
  if (!decode(P, BOX_PRED, g, b.first, i, j, k)) return;
  pred_item(P, g, i, j, k, U, S, S, dt[b.patch], dx + 3 * b.patch, c);
}

template <typename T, int TX, int TY, int TZ>
__global__ __launch_bounds__((TileShape<TX, TY, TZ>::THREADS)) void k_solve(
    const PatchDev* __restrict__ pt, const TileDev* __restrict__ tiles, const T* __restrict__ Uin,
    T* __restrict__ Uout, const T* __restrict__ S, const double* __restrict__ dt,
    const double* __restrict__ dx, Consts<T> c, int g) {
  __shared__ T lds[TileShape<TX, TY, TZ>::LDS_ELEMS];
  const TileDev tl = tiles[blockIdx.x];
  const PatchDev P = pt[tl.patch];
  DevX ex;
  solve_tile<T, TX, TY, TZ>(ex, lds, P, g, tl, Uin, Uout, S, dt[tl.patch], dx + 3 * tl.patch, c);
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_cfl(const PatchDev* __restrict__ pt,
                                             const BoxBlock* __restrict__ blk,
                                             const T* __restrict__ U, const double* __restrict__ dx,
                                             Consts<T> c, int g, unsigned long long* smax) {
  const BoxBlock b = blk[blockIdx.x];
  const PatchDev P = pt[b.patch];
  int i, j, k;
  double s = 0.0;
  if (decode(P, BOX_INTERIOR, g, b.first, i, j, k))
    s = cfl_item(P, cell_of(P, i, j, k), U, dx + 3 * b.patch, c);
  for (int o = 32; o > 0; o >>= 1) s = fmax(s, __shfl_xor(s, o));
  __shared__ double red[BLK / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < BLK / 64; ++w) m = fmax(m, red[w]);
    // s >= 0, so its IEEE bit pattern orders like the value
    atomicMax(smax + b.patch, (unsigned long long)__double_as_longlong(m));
  }
}

__global__ __launch_bounds__(BLK) void k_cfl_final(int np, const unsigned long long* __restrict__ smax,
                                                   double C, double* __restrict__ dt, int global) {
  __shared__ double red[BLK / 64];
  double mn = 1e300;
  for (int p = threadIdx.x; p < np; p += BLK) {
    const double v = C / __longlong_as_double((long long)smax[p]);
    dt[p] = v;
    mn = fmin(mn, v);
  }
  if (!global) return;
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mn;
  __syncthreads();
  double m = red[0];
  for (int w = 1; w < BLK / 64; ++w) m = fmin(m, red[w]);
  for (int p = threadIdx.x; p < np; p += BLK) dt[p] = m;
}

__global__ void k_zero_u64(unsigned long long* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0ull;
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_guards(const PatchDev* __restrict__ pt,
                                                const BoxBlock* __restrict__ blk, T* U,
                                                const int32_t* __restrict__ nbr, int g, int np,
                                                int* status) {
  const BoxBlock b = blk[blockIdx.x];
  const PatchDev P = pt[b.patch];
  int i, j, k;
  if (!decode(P, BOX_ALL, g, b.first, i, j, k)) return;
  if (guard_item(pt, b.patch, g, i, j, k, U, nbr, np)) atomicOr(status, 2);
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// ------------------------------------------------------------------------ handle

struct mhd_bunch {
  int P = 0, g = 3, prec = 8, limiter = 0;
  double gamma = 5.0 / 3.0, cfl = 0.4, rho_floor = 1e-12, p_floor = 1e-12, eps_deg = 1e-10;
  int64_t max_scratch = 0;
  std::vector<PatchDev> pt;
  int64_t state_elems = 0;
  int act = 0;  // active-direction pattern shared by all patches
  struct Chunk {
    int p0 = 0, p1 = 0;
    int blk0[NBOX] = {0}, nblk[NBOX] = {0};
    int tile0 = 0, ntile = 0;
  };
  std::vector<Chunk> chunks;
  std::vector<BoxBlock> blocks[NBOX];
  std::vector<TileDev> tiles;
  int TX = 8, TY = 8, TZ = 4;
  int64_t scratch_elems = 0;
  size_t o_pt = 0, o_blk[NBOX] = {0}, o_tiles = 0, o_smax = 0, o_status = 0, o_scratch = 0;
  size_t ws_bytes = 0;
  char* ws = nullptr;
  bool bound = false;
  char last_error[256] = {0};
  // record the first failing HIP call of an API call; returns true on success
  bool hip_ok(hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    snprintf(last_error, sizeof(last_error), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    return false;
  }
  // optional HIP-event timing of every kernel launch (mhd_bunch_profile)
  struct Mark { int kid; hipEvent_t a, b; };
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<Mark> marks;
  ~mhd_bunch() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }
  hipEvent_t ev_get() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }
  hipEvent_t tic(hipStream_t s) {
    if (!prof) return nullptr;
    hipEvent_t e = ev_get();
    if (e) (void)hipEventRecord(e, s);
    return e;
  }
  void toc(hipStream_t s, int kid, hipEvent_t a) {
    if (!prof || !a) return;
    hipEvent_t e = ev_get();
    if (!e) return;
    (void)hipEventRecord(e, s);
    marks.push_back(Mark{kid, a, e});
  }

  template <typename T>
  Consts<T> consts() const {
    Consts<T> c;
    c.gamma = T(gamma);
    c.gm1 = T(gamma - 1.0);
    c.inv_gm1 = T(1.0 / (gamma - 1.0));
    c.rho_floor = T(rho_floor);
    c.p_floor = T(p_floor);
    c.eps_deg = T(eps_deg);
    c.tiny = sizeof(T) == 8 ? T(1e-300) : T(1e-37);
    c.limiter = limiter;
    return c;
  }
  const PatchDev* d_pt() const { return (const PatchDev*)(ws + o_pt); }
  const BoxBlock* d_blk(int k) const { return (const BoxBlock*)(ws + o_blk[k]); }
  const TileDev* d_tiles() const { return (const TileDev*)(ws + o_tiles); }
  unsigned long long* d_smax() const { return (unsigned long long*)(ws + o_smax); }
  int* d_status() const { return (int*)(ws + o_status); }
  void* d_scratch() const { return ws + o_scratch; }
};

namespace {

void add_blocks(std::vector<BoxBlock>& out, const PatchDev& P, int p, int kind, int g) {
  int lo[3], sz[3];
  box_of(P, kind, g, lo, sz);
  const int n = sz[0] * sz[1] * sz[2];
  for (int f = 0; f < n; f += BLK) out.push_back(BoxBlock{p, f});
}

void pick_tile(mhd_bunch* h) {
  switch (h->act) {
    case 7: h->TX = 8; h->TY = 8; h->TZ = 4; break;
    case 3: h->TX = 16; h->TY = 16; h->TZ = 1; break;
    case 6: h->TX = 1; h->TY = 16; h->TZ = 16; break;
    case 5: h->TX = 16; h->TY = 1; h->TZ = 16; break;
    case 1: h->TX = 64; h->TY = 1; h->TZ = 1; break;
    case 2: h->TX = 1; h->TY = 64; h->TZ = 1; break;
    default: h->TX = 1; h->TY = 1; h->TZ = 64; break;
  }
}

template <typename T>
mhd_status launch_update(mhd_bunch* h, const T* Uin, T* Uout, const double* dt, const double* dx,
                         hipStream_t s) {
  const Consts<T> c = h->consts<T>();
  T* S = (T*)h->d_scratch();
  for (const auto& ch : h->chunks) {
    hipEvent_t t0;
    if (ch.nblk[BOX_PRIM]) {
      t0 = h->tic(s);
      hipLaunchKernelGGL(k_prim<T>, dim3(ch.nblk[BOX_PRIM]), dim3(BLK), 0, s, h->d_pt(),
                         h->d_blk(BOX_PRIM) + ch.blk0[BOX_PRIM], Uin, S, c, h->g, h->d_status());
      h->toc(s, MHD_KERNEL_PRIM, t0);
    }
    if (ch.nblk[BOX_EN]) {
      t0 = h->tic(s);
      hipLaunchKernelGGL(k_en<T>, dim3(ch.nblk[BOX_EN]), dim3(BLK), 0, s, h->d_pt(),
                         h->d_blk(BOX_EN) + ch.blk0[BOX_EN], Uin, S, h->g);
      h->toc(s, MHD_KERNEL_EDGE_EMF_N, t0);
    }
    if (ch.nblk[BOX_PRED]) {
      t0 = h->tic(s);
      hipLaunchKernelGGL(k_pred<T>, dim3(ch.nblk[BOX_PRED]), dim3(BLK), 0, s, h->d_pt(),
                         h->d_blk(BOX_PRED) + ch.blk0[BOX_PRED], Uin, S, dt, dx, c, h->g);
      h->toc(s, MHD_KERNEL_PREDICT, t0);
    }
    if (ch.ntile) {
      t0 = h->tic(s);
      const TileDev* tl = h->d_tiles() + ch.tile0;
#define MHD_SOLVE(X, Y, Z)                                                                    \
  hipLaunchKernelGGL((k_solve<T, X, Y, Z>), dim3(ch.ntile), dim3(TileShape<X, Y, Z>::THREADS), 0, \
                     s, h->d_pt(), tl, Uin, Uout, (const T*)S, dt, dx, c, h->g)
      switch (h->act) {
        case 7: MHD_SOLVE(8, 8, 4); break;
        case 3: MHD_SOLVE(16, 16, 1); break;
        case 6: MHD_SOLVE(1, 16, 16); break;
        case 5: MHD_SOLVE(16, 1, 16); break;
        case 1: MHD_SOLVE(64, 1, 1); break;
        case 2: MHD_SOLVE(1, 64, 1); break;
        default: MHD_SOLVE(1, 1, 64); break;
      }
#undef MHD_SOLVE
      h->toc(s, MHD_KERNEL_SOLVE, t0);
    }
  }
  return h->hip_ok(hipGetLastError(), "launch update kernels") ? MHD_OK : MHD_EDEVICE;
}

template <typename T>
mhd_status launch_cfl(mhd_bunch* h, const T* U, const double* dx, double* dt, int global,
                      hipStream_t s) {
  const Consts<T> c = h->consts<T>();
  hipEvent_t t0 = h->tic(s);
  hipLaunchKernelGGL(k_zero_u64, dim3((h->P + 255) / 256), dim3(256), 0, s, h->d_smax(), h->P);
  const int nb = (int)h->blocks[BOX_INTERIOR].size();
  hipLaunchKernelGGL(k_cfl<T>, dim3(nb), dim3(BLK), 0, s, h->d_pt(), h->d_blk(BOX_INTERIOR), U, dx, c,
                     h->g, h->d_smax());
  hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(BLK), 0, s, h->P, (const unsigned long long*)h->d_smax(),
                     h->cfl, dt, global);
  h->toc(s, MHD_KERNEL_CFL, t0);
  return h->hip_ok(hipGetLastError(), "launch cfl kernels") ? MHD_OK : MHD_EDEVICE;
}

template <typename T>
mhd_status launch_guards(mhd_bunch* h, T* U, const int32_t* nbr, hipStream_t s) {
  const int nb = (int)h->blocks[BOX_ALL].size();
  hipEvent_t t0 = h->tic(s);
  hipLaunchKernelGGL(k_guards<T>, dim3(nb), dim3(BLK), 0, s, h->d_pt(), h->d_blk(BOX_ALL), U, nbr, h->g,
                     h->P, h->d_status());
  h->toc(s, MHD_KERNEL_GUARDS, t0);
  return h->hip_ok(hipGetLastError(), "launch guard kernel") ? MHD_OK : MHD_EDEVICE;
}

}  // namespace

// ------------------------------------------------------------------------ C ABI

extern "C" {

mhd_status mhd_bunch_profile(mhd_bunch* h, int32_t enable) {
  if (!h) return MHD_EINVAL;
  h->prof = enable != 0;
  h->ev_used = 0;
  h->marks.clear();
  return MHD_OK;
}

mhd_status mhd_bunch_profile_read(mhd_bunch* h, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!h || !total_ms || !launches || kernel < 0 || kernel >= MHD_KERNEL_COUNT) return MHD_EINVAL;
  double tot = 0.0;
  int64_t n = 0;
  for (const auto& m : h->marks) {
    if (m.kid != kernel) continue;
    if (hipEventSynchronize(m.b) != hipSuccess) return MHD_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, m.a, m.b) != hipSuccess) return MHD_EDEVICE;
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *launches = n;
  return MHD_OK;
}

const char* mhd_status_string(mhd_status s) {
  switch (s) {
    case MHD_OK: return "ok";
    case MHD_EINVAL: return "invalid argument";
    case MHD_ENOMEM: return "out of host memory";
    case MHD_EDEVICE: return "HIP error";
    case MHD_ESTATE: return "call out of order";
    case MHD_ENONPHYS: return "non-physical state met on the device";
    case MHD_EUNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

mhd_status mhd_bunch_create(mhd_bunch** out, const mhd_bunch_desc* d) {
  if (!out || !d || !d->dims || d->n_patches < 1) return MHD_EINVAL;
  if (d->guard < 3 || (d->precision != 4 && d->precision != 8)) return MHD_EINVAL;
  if (!(d->gamma > 1.0) || !(d->cfl > 0.0) || !(d->rho_floor > 0.0) || !(d->p_floor > 0.0) ||
      !(d->eps_deg >= 0.0) || (d->limiter != 0 && d->limiter != 1) || d->max_scratch_bytes < 0)
    return MHD_EINVAL;
  mhd_bunch* h = new (std::nothrow) mhd_bunch;
  if (!h) return MHD_ENOMEM;
  h->P = d->n_patches;
  h->g = d->guard;
  h->prec = d->precision;
  h->gamma = d->gamma;
  h->cfl = d->cfl;
  h->limiter = d->limiter;
  h->rho_floor = d->rho_floor;
  h->p_floor = d->p_floor;
  h->eps_deg = d->eps_deg;
  h->max_scratch = d->max_scratch_bytes;
  const int g = h->g;
  h->pt.resize(h->P);
  int64_t base = 0;
  for (int p = 0; p < h->P; ++p) {
    PatchDev& P = h->pt[p];
    std::memset(&P, 0, sizeof(P));
    int act = 0;
    for (int dd = 0; dd < 3; ++dd) {
      const int n = d->dims[3 * p + dd];
      if (n < 1 || n > 4096) { delete h; return MHD_EINVAL; }
      P.n[dd] = n;
      if (n > 1) {
        if (n < g) { delete h; return MHD_EINVAL; }
        act |= 1 << dd;
      }
      P.N[dd] = n > 1 ? n + 2 * g : 1;
    }
    if (p == 0) h->act = act;
    if (act != h->act || act == 0) { delete h; return MHD_EUNSUPPORTED; }
    P.act = act;
    P.Nc = (int64_t)P.N[0] * P.N[1] * P.N[2];
    const int64_t st[3] = {1, P.N[0], (int64_t)P.N[0] * P.N[1]};
    int Nw[3];
    for (int dd = 0; dd < 3; ++dd) {
      P.off[dd] = (act >> dd & 1) ? st[dd] : 0;
      Nw[dd] = (act >> dd & 1) ? P.n[dd] + 2 : 1;
    }
    P.woff[0] = (act & 1) ? 1 : 0;
    P.woff[1] = (act & 2) ? Nw[0] : 0;
    P.woff[2] = (act & 4) ? (int64_t)Nw[0] * Nw[1] : 0;
    P.Nwc = (int64_t)Nw[0] * Nw[1] * Nw[2];
    P.ubase = base;
    base += 8 * P.Nc;
  }
  h->state_elems = base;
  pick_tile(h);

  // chunks of consecutive patches whose scratch fits the cap
  const int64_t esz = h->prec;
  {
    int chunk = 0;
    int64_t used = 0;
    for (int p = 0; p < h->P; ++p) {
      PatchDev& P = h->pt[p];
      const int64_t need = 11 * P.Nc + NW * P.Nwc;
      if (h->max_scratch > 0 && used > 0 && (used + need) * esz > h->max_scratch) {
        ++chunk;
        used = 0;
      }
      P.sbase = used;
      P.wbase = used + 11 * P.Nc;
      P.chunk = chunk;
      used += need;
      h->scratch_elems = std::max(h->scratch_elems, used);
    }
    for (int p = 0; p < h->P; ++p)
      if (p == 0 || h->pt[p].chunk != h->pt[p - 1].chunk) {
        mhd_bunch::Chunk ch;
        ch.p0 = p;
        h->chunks.push_back(ch);
      }
    for (size_t c = 0; c < h->chunks.size(); ++c)
      h->chunks[c].p1 = c + 1 < h->chunks.size() ? h->chunks[c + 1].p0 : h->P;
  }
  for (auto& ch : h->chunks) {
    for (int kind : {BOX_PRIM, BOX_EN, BOX_PRED}) {
      ch.blk0[kind] = (int)h->blocks[kind].size();
      for (int p = ch.p0; p < ch.p1; ++p) add_blocks(h->blocks[kind], h->pt[p], p, kind, g);
      ch.nblk[kind] = (int)h->blocks[kind].size() - ch.blk0[kind];
    }
    ch.tile0 = (int)h->tiles.size();
    for (int p = ch.p0; p < ch.p1; ++p) {
      const PatchDev& P = h->pt[p];
      const int T3[3] = {h->TX, h->TY, h->TZ};
      int nt[3];
      for (int dd = 0; dd < 3; ++dd) nt[dd] = (P.act >> dd & 1) ? (P.n[dd] + T3[dd] - 1) / T3[dd] : 1;
      for (int z = 0; z < nt[2]; ++z)
        for (int y = 0; y < nt[1]; ++y)
          for (int x = 0; x < nt[0]; ++x) h->tiles.push_back(TileDev{p, x * h->TX, y * h->TY, z * h->TZ});
    }
    ch.ntile = (int)h->tiles.size() - ch.tile0;
  }
  for (int p = 0; p < h->P; ++p) {
    add_blocks(h->blocks[BOX_INTERIOR], h->pt[p], p, BOX_INTERIOR, g);
    add_blocks(h->blocks[BOX_ALL], h->pt[p], p, BOX_ALL, g);
  }
  // workspace layout
  size_t o = 0;
  h->o_pt = o;
  o = align256(o + sizeof(PatchDev) * h->P);
  for (int k = 0; k < NBOX; ++k) {
    h->o_blk[k] = o;
    o = align256(o + sizeof(BoxBlock) * std::max<size_t>(1, h->blocks[k].size()));
  }
  h->o_tiles = o;
  o = align256(o + sizeof(TileDev) * std::max<size_t>(1, h->tiles.size()));
  h->o_smax = o;
  o = align256(o + sizeof(unsigned long long) * h->P);
  h->o_status = o;
  o = align256(o + sizeof(unsigned long long));
  h->o_scratch = o;
  o = align256(o + (size_t)h->scratch_elems * esz);
  h->ws_bytes = o;
  *out = h;
  return MHD_OK;
}

void mhd_bunch_destroy(mhd_bunch* h) { delete h; }

int64_t mhd_bunch_state_elems(const mhd_bunch* h) { return h ? h->state_elems : -1; }
int64_t mhd_bunch_state_bytes(const mhd_bunch* h) { return h ? h->state_elems * h->prec : -1; }
int64_t mhd_bunch_patch_offset(const mhd_bunch* h, int32_t p) {
  if (!h || p < 0 || p >= h->P) return -1;
  return h->pt[p].ubase;
}
int64_t mhd_bunch_workspace_bytes(const mhd_bunch* h) { return h ? (int64_t)h->ws_bytes : -1; }

mhd_status mhd_bunch_bind(mhd_bunch* h, void* ws, hipStream_t s) {
  if (!h || !ws || ((uintptr_t)ws & 255)) return MHD_EINVAL;
  h->ws = (char*)ws;
  h->last_error[0] = 0;
  bool ok = h->hip_ok(hipMemcpyAsync(h->ws + h->o_pt, h->pt.data(), sizeof(PatchDev) * h->P,
                                     hipMemcpyHostToDevice, s), "upload patch table");
  for (int k = 0; k < NBOX && ok; ++k)
    if (!h->blocks[k].empty())
      ok = h->hip_ok(hipMemcpyAsync(h->ws + h->o_blk[k], h->blocks[k].data(),
                                    sizeof(BoxBlock) * h->blocks[k].size(), hipMemcpyHostToDevice, s),
                     "upload block table");
  if (ok && !h->tiles.empty())
    ok = h->hip_ok(hipMemcpyAsync(h->ws + h->o_tiles, h->tiles.data(), sizeof(TileDev) * h->tiles.size(),
                                  hipMemcpyHostToDevice, s), "upload tile table");
  if (ok) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, (unsigned long long*)(h->ws + h->o_status), 1);
    ok = h->hip_ok(hipGetLastError(), "clear status word");
  }
  // the tables live in host memory owned by the handle; make the uploads complete
  if (ok) ok = h->hip_ok(hipStreamSynchronize(s), "synchronise after upload");
  if (!ok) return MHD_EDEVICE;
  h->bound = true;
  return MHD_OK;
}

const char* mhd_bunch_last_error(const mhd_bunch* h) { return h ? h->last_error : "null handle"; }

mhd_status mhd_bunch_load(mhd_bunch* h, void* U, int32_t p, const void* src, int32_t src_dev,
                          hipStream_t s) {
  if (!h || !U || !src || p < 0 || p >= h->P) return MHD_EINVAL;
  const size_t bytes = (size_t)(8 * h->pt[p].Nc) * h->prec;
  char* dst = (char*)U + (size_t)h->pt[p].ubase * h->prec;
  const hipError_t e = hipMemcpyAsync(dst, src, bytes, src_dev ? hipMemcpyDeviceToDevice
                                                               : hipMemcpyHostToDevice, s);
  return e == hipSuccess ? MHD_OK : MHD_EDEVICE;
}

mhd_status mhd_bunch_store(const mhd_bunch* h, const void* U, int32_t p, void* dst, int32_t dst_dev,
                           hipStream_t s) {
  if (!h || !U || !dst || p < 0 || p >= h->P) return MHD_EINVAL;
  const size_t bytes = (size_t)(8 * h->pt[p].Nc) * h->prec;
  const char* src = (const char*)U + (size_t)h->pt[p].ubase * h->prec;
  const hipError_t e = hipMemcpyAsync(dst, src, bytes, dst_dev ? hipMemcpyDeviceToDevice
                                                               : hipMemcpyDeviceToHost, s);
  return e == hipSuccess ? MHD_OK : MHD_EDEVICE;
}

mhd_status mhd_bunch_fill_guards(mhd_bunch* h, void* U, const int32_t* nbr, hipStream_t s) {
  if (!h || !U || !nbr) return MHD_EINVAL;
  if (!h->bound) return MHD_ESTATE;
  return h->prec == 8 ? launch_guards<double>(h, (double*)U, nbr, s)
                      : launch_guards<float>(h, (float*)U, nbr, s);
}

mhd_status mhd_bunch_cfl(mhd_bunch* h, const void* U, const double* dx, double* dt, int32_t global,
                         hipStream_t s) {
  if (!h || !U || !dx || !dt) return MHD_EINVAL;
  if (!h->bound) return MHD_ESTATE;
  return h->prec == 8 ? launch_cfl<double>(h, (const double*)U, dx, dt, global, s)
                      : launch_cfl<float>(h, (const float*)U, dx, dt, global, s);
}

mhd_status mhd_bunch_update(mhd_bunch* h, const void* Uin, void* Uout, const double* dt,
                            const double* dx, hipStream_t s) {
  if (!h || !Uin || !Uout || !dt || !dx || Uin == Uout) return MHD_EINVAL;
  if (!h->bound) return MHD_ESTATE;
  const size_t bytes = (size_t)h->state_elems * h->prec;
  const char *a = (const char*)Uin, *b = (const char*)Uout;
  if (a < b + bytes && b < a + bytes) return MHD_EINVAL;
  return h->prec == 8 ? launch_update<double>(h, (const double*)Uin, (double*)Uout, dt, dx, s)
                      : launch_update<float>(h, (const float*)Uin, (float*)Uout, dt, dx, s);
}

mhd_status mhd_bunch_check(mhd_bunch* h, hipStream_t s) {
  if (!h) return MHD_EINVAL;
  if (!h->bound) return MHD_ESTATE;
  int st = 0;
  if (hipStreamSynchronize(s) != hipSuccess) return MHD_EDEVICE;
  if (hipMemcpy(&st, h->ws + h->o_status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return MHD_EDEVICE;
  if (st) {
    const int zero = 0;
    if (hipMemcpy(h->ws + h->o_status, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
      return MHD_EDEVICE;
    return (st & 2) ? MHD_EINVAL : MHD_ENONPHYS;
  }
  return MHD_OK;
}

}  // extern "C"
