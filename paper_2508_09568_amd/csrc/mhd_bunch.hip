// mhd_bunch.hip -- kernels and C ABI of the ideal-MHD bunch update for gfx950.
//
// One update of a chunk of patches runs on the caller's stream:
//   predictor, staged (predictor mode 0), three kernels over flat block tables:
//     k_prim    : primitives on every padded cell                    (box [0, N-1))
//     k_en      : edge EMFs at time n from 4-cell / 2-face averages    (box [1, N-1))
//     k_pred    : limited slopes, half-step state, half-step face field,
//                 transverse face-field slopes on the cells around the interior
//   predictor, fused (modes >= 1): k_predict does the three steps per 3D tile, with the
//               tile's primitives and face fields in shared memory and the edge EMFs at
//               time n evaluated from them where they are read
//   k_edges   : (solver form 2) half-step edge EMFs, each edge once, into scratch
//   k_edge_lines: (solver form 3, 3D bunches) the same EMFs as lines of edges, one thread
//               stepping along each line
//   k_solve   : per 3D tile, HLLD on every face and the four-state EMF on every edge (or
//               the EMFs the edge pass left) into shared memory, then the conservative +
//               constrained-transport update.
// Side kernels: k_cfl / k_cfl_final (per-patch time step, wavefront max-reduction + one
// 64-bit atomic per work-group), k_guards (guard fill from a neighbour table), the local
// time stepping step (k_lts_ready, k_guards_at, k_lts_dt and k_lts_time around the update,
// which runs in place and writes the previous slice), and the k_adj_* reverse sweep of the adjoint, which re-runs the staged
// predictor kernels first.  Patches with dt = 0 are copied by the update, not computed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
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

// Work-groups are handed to the 8 XCDs round-robin (block b runs on XCD b % 8), and each
// XCD has its own L2.  With remap on, block b takes logical block remap_xcd(b, nb), which
// gives every XCD one contiguous range of the block table: neighbouring tiles of a patch,
// whose halos overlap, then share one L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int remap_xcd(int b, int nb) {
  const int per = nb / NXCD, rem = nb % NXCD, x = b % NXCD, i = b / NXCD;
  return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}
// Kernels over a block (or tile) table of nb entries loop over virtual blocks
// vb = blockIdx.x, blockIdx.x + gridDim.x, ...: one virtual block per work-group when the
// grid is nb (plain launch), several when the grid is a persistent one sized to the machine.
// A persistent grid is a multiple of NXCD, so every virtual block of a work-group runs on
// that work-group's XCD and remap_xcd keeps its meaning.
__device__ __forceinline__ int logical_block(int vb, int nb, int remap) {
  return remap ? remap_xcd(vb, nb) : vb;
}
// Table length of a launch: the host's count, or (tables compacted on the device, see
// k_compact_scan) the count the device wrote; the grid is then a persistent one.
__device__ __forceinline__ int table_count(int nb, const int* __restrict__ dcount) {
  return dcount ? *dcount : nb;
}

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
                                              const double* __restrict__ zdt, Consts<T> c, int g,
                                              int* status, int nb0, int remap,
                                              const int* __restrict__ dcount) {
  const int nb = table_count(nb0, dcount);
  for (int vb = blockIdx.x; vb < nb; vb += gridDim.x) {
    const BoxBlock b = blk[logical_block(vb, nb, remap)];
    if (zdt && zdt[b.patch] == 0.0) continue;
    const PatchDev& P = pt[b.patch];
    int i, j, k;
    if (!decode(P, BOX_PRIM, g, b.first, i, j, k)) continue;
    if (prim_item(P, cell_of(P, i, j, k), U, S, c)) atomicOr(status, 1);
  }
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_en(const PatchDev* __restrict__ pt,
                                            const BoxBlock* __restrict__ blk,
                                            const T* __restrict__ U, T* __restrict__ S,
                                            const double* __restrict__ zdt, int g, int nb0,
                                            int remap, const int* __restrict__ dcount) {
  const int nb = table_count(nb0, dcount);
  for (int vb = blockIdx.x; vb < nb; vb += gridDim.x) {
    const BoxBlock b = blk[logical_block(vb, nb, remap)];
    if (zdt && zdt[b.patch] == 0.0) continue;
    const PatchDev& P = pt[b.patch];
    int i, j, k;
    if (!decode(P, BOX_EN, g, b.first, i, j, k)) continue;
    en_item(P, cell_of(P, i, j, k), U, S);
  }
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_pred(const PatchDev* __restrict__ pt,
                                              const BoxBlock* __restrict__ blk,
                                              const T* __restrict__ U, T* __restrict__ S,
                                              const double* __restrict__ dt,
                                              const double* __restrict__ dx,
                                              const double* __restrict__ zdt, Consts<T> c, int g,
                                              int nb0, int remap, const int* __restrict__ dcount) {
  const int nb = table_count(nb0, dcount);
  for (int vb = blockIdx.x; vb < nb; vb += gridDim.x) {
    const BoxBlock b = blk[logical_block(vb, nb, remap)];
    if (zdt && zdt[b.patch] == 0.0) continue;
    const PatchDev& P = pt[b.patch];
    int i, j, k;
    if (!decode(P, BOX_PRED, g, b.first, i, j, k)) continue;
    pred_item(P, g, i, j, k, U, S, S, dt[b.patch], dx + 3 * b.patch, c);
  }
}

// Waves per SIMD that the shared memory of a solver work-group allows (160 KB per compute
// unit), capped at 3 in FP64 and 4 in FP32, in whole work-groups (a 512-thread work-group
// puts 2 waves on each SIMD); the hint makes the register allocation fit them (paired loads
// hold four registers each in FP64).
template <typename T, int TX, int TY, int TZ, int FORM>
struct SolveWaves {
  static constexpr int WG = TileShape<TX, TY, TZ>::THREADS / 64;  // waves per work-group
  static constexpr int PER = WG >= 4 ? WG / 4 : 1;                 // waves per SIMD per work-group
  static constexpr int LDSB = TileShape<TX, TY, TZ>::template Lds<FORM>::value * (int)sizeof(T);
  static constexpr int BY_LDS = (LDSB > 0 ? (160 * 1024) / LDSB : 8) * WG / 4;
  static constexpr int CAP = sizeof(T) == 8 ? (PER == 2 ? 4 : 3) : 4;
  static constexpr int RAW = BY_LDS < CAP ? BY_LDS : CAP;
  static constexpr int value = RAW / PER * PER < 1 ? 1 : RAW / PER * PER;
};
template <typename T, int TX, int TY, int TZ, int FORM, int EMF>
__global__ __launch_bounds__((TileShape<TX, TY, TZ>::THREADS))
__attribute__((amdgpu_waves_per_eu(SolveWaves<T, TX, TY, TZ, FORM>::value))) void k_solve(
    const PatchDev* __restrict__ pt, const TileDev* __restrict__ tiles, const T* __restrict__ Uin,
    T* __restrict__ Uout, const T* __restrict__ S, const double* __restrict__ dt,
    const double* __restrict__ dx, Consts<T> c, int g, int ntile0, int remap, int copy_rest,
    const int* __restrict__ dcount, unsigned long long* cfl_max, const int32_t* __restrict__ nbr) {
  __shared__ T lds[TileShape<TX, TY, TZ>::template Lds<FORM>::value];
  __shared__ double red[TileShape<TX, TY, TZ>::THREADS / 64];
  DevX ex;
  const int ntile = table_count(ntile0, dcount);
  for (int vb = blockIdx.x; vb < ntile; vb += gridDim.x) {
    const TileDev tl = tiles[logical_block(vb, ntile, remap)];
    const PatchDev& P = pt[tl.patch];
    if (dt[tl.patch] == 0.0) {  // a patch at rest this step: its owned values are copied
      if (copy_rest) copy_tile<TX, TY, TZ>(ex, P, g, tl, Uin, Uout);
      continue;
    }
    double s = solve_tile<T, TX, TY, TZ, FORM, EMF>(ex, lds, P, g, tl, Uin, Uout, S, dt[tl.patch],
                                                    dx + 3 * tl.patch, c, cfl_max ? nbr : nullptr,
                                                    tl.patch);
    if (cfl_max) {  // the tile's largest time-step sum -> the patch's slot (one atomic)
      for (int o = 32; o > 0; o >>= 1) s = fmax(s, __shfl_xor(s, o));
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
      __syncthreads();
      if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < TileShape<TX, TY, TZ>::THREADS / 64; ++w) m = fmax(m, red[w]);
        atomicMax(cfl_max + tl.patch, (unsigned long long)__double_as_longlong(m));
      }
    }
    ex.sync();  // the next tile reuses the shared memory
  }
}

// The update of local time stepping: in place (U is read and written; each cell's state is
// read before it is written and no tile reads another's cells) with the previous state of
// every updated cell written to keep; patches at rest (dt = 0) are skipped.
template <typename T, int TX, int TY, int TZ, int FORM, int EMF>
__global__ __launch_bounds__((TileShape<TX, TY, TZ>::THREADS))
__attribute__((amdgpu_waves_per_eu(SolveWaves<T, TX, TY, TZ, FORM>::value))) void k_solve_keep(
    const PatchDev* __restrict__ pt, const TileDev* __restrict__ tiles, T* U,
    T* __restrict__ keep, const T* __restrict__ S, const double* __restrict__ dt,
    const double* __restrict__ dx, Consts<T> c, int g, int ntile0, int remap,
    const int* __restrict__ dcount) {
  __shared__ T lds[TileShape<TX, TY, TZ>::template Lds<FORM>::value];
  DevX ex;
  const int ntile = table_count(ntile0, dcount);
  for (int vb = blockIdx.x; vb < ntile; vb += gridDim.x) {
    const TileDev tl = tiles[logical_block(vb, ntile, remap)];
    if (dt[tl.patch] == 0.0) continue;
    solve_tile<T, TX, TY, TZ, FORM, EMF, true>(ex, lds, pt[tl.patch], g, tl, U, U, S, dt[tl.patch],
                                               dx + 3 * tl.patch, c, nullptr, tl.patch, keep);
    ex.sync();  // the next tile reuses the shared memory
  }
}

// Waves per SIMD that the shared memory of a predictor work-group allows, capped at 3 in
// FP64 and 5 in FP32; the hint keeps the registers within them.
template <typename T, int PX, int PY, int PZ>
struct PredWaves {
  static constexpr int WG = (PredShape<PX, PY, PZ>::THREADS + 63) / 64;
  static constexpr int PER_CU = (160 * 1024) / (PredShape<PX, PY, PZ>::LDS_ELEMS * (int)sizeof(T));
  static constexpr int BY_LDS = (PER_CU * WG + 3) / 4;
  static constexpr int CAP = sizeof(T) == 8 ? 3 : 5;
  static constexpr int value = BY_LDS < 1 ? 1 : (BY_LDS < CAP ? BY_LDS : CAP);
};
template <typename T, int PX, int PY, int PZ>
__global__ __launch_bounds__((PredShape<PX, PY, PZ>::THREADS))
__attribute__((amdgpu_waves_per_eu(PredWaves<T, PX, PY, PZ>::value))) void k_predict(
    const PatchDev* __restrict__ pt, const TileDev* __restrict__ tiles, const T* __restrict__ U,
    T* __restrict__ W, const double* __restrict__ dt, const double* __restrict__ dx, Consts<T> c,
    int g, int* status, int ntile0, int remap, const int* __restrict__ dcount) {
  __shared__ T lds[PredShape<PX, PY, PZ>::LDS_ELEMS];
  DevX ex;
  int bad = 0;
  const int ntile = table_count(ntile0, dcount);
  for (int vb = blockIdx.x; vb < ntile; vb += gridDim.x) {
    const TileDev tl = tiles[logical_block(vb, ntile, remap)];
    if (dt[tl.patch] == 0.0) continue;  // patch at rest: no predictor values needed
    const PatchDev& P = pt[tl.patch];
    bad |= predict_tile<T, PX, PY, PZ>(ex, lds, P, g, tl, U, W, dt[tl.patch], dx + 3 * tl.patch, c);
    ex.sync();  // the next tile reuses the shared memory
  }
  if (bad) atomicOr(status, 1);
}

// half-step edge EMFs, each edge once, by the solver tiles that own them (solver form 2); no
// shared memory: registers alone set the occupancy, three waves per SIMD (<= 168 VGPRs)
template <typename T, int TX, int TY, int TZ, int EMF>
__global__ __launch_bounds__((TileShape<TX, TY, TZ>::THREADS)) __attribute__((amdgpu_waves_per_eu(3)))
void k_edges(
    const PatchDev* __restrict__ pt, const TileDev* __restrict__ tiles, T* __restrict__ S,
    const double* __restrict__ dt, const double* __restrict__ dx, Consts<T> c, int g, int ntile0,
    int remap, const int* __restrict__ dcount) {
  DevX ex;
  const int ntile = table_count(ntile0, dcount);
  for (int vb = blockIdx.x; vb < ntile; vb += gridDim.x) {
    const TileDev tl = tiles[logical_block(vb, ntile, remap)];
    if (dt[tl.patch] == 0.0) continue;  // patch at rest: no EMFs needed
    const PatchDev& P = pt[tl.patch];
    solve_tile<T, TX, TY, TZ, 3, EMF>(ex, (T*)nullptr, P, g, tl, (const T*)S, S, S, 1.0, dx + 3 * tl.patch,
                                 c);
  }
}

// the same half-step edge EMFs as edge lines (solver form 3, patches with all three
// directions active): BLK consecutive lines of one patch per work-group, each line marched by
// one thread; registers alone set the occupancy: three waves per SIMD (<= 168 VGPRs), two
// for the FP64 UCT-HLLD lines, which hold four corner states and spill within 168
template <typename T, int EMF>
struct EdgeLineWaves {
  static constexpr int value = EMF == 1 && sizeof(T) == 8 ? 2 : 3;
};
template <typename T, int EMF>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(EdgeLineWaves<T, EMF>::value))) void k_edge_lines(
    const PatchDev* __restrict__ pt, const BoxBlock* __restrict__ blk, T* __restrict__ S,
    const double* __restrict__ dt, Consts<T> c, int g, int nb0, int remap,
    const int* __restrict__ dcount) {
  const int nb = table_count(nb0, dcount);
  for (int vb = blockIdx.x; vb < nb; vb += gridDim.x) {
    const BoxBlock b = blk[logical_block(vb, nb, remap)];
    if (dt[b.patch] == 0.0) continue;  // patch at rest: no EMFs needed
    const PatchDev& P = pt[b.patch];
    const int item = b.first + (int)threadIdx.x;
    if (item < edge_line_count(P)) edge_line_item<EMF>(P, g, item, S, c);
  }
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_cfl(const PatchDev* __restrict__ pt,
                                             const BoxBlock* __restrict__ blk,
                                             const T* __restrict__ U, const double* __restrict__ dx,
                                             const int32_t* __restrict__ mask, Consts<T> c, int g,
                                             unsigned long long* smax, int nb0,
                                             const int* __restrict__ dcount) {
  __shared__ double red[BLK / 64];
  const int nb = table_count(nb0, dcount);
  for (int vb = blockIdx.x; vb < nb; vb += gridDim.x) {
    const BoxBlock b = blk[vb];
    if (mask && !mask[b.patch]) continue;  // whole work-group: patch not asked for (dt: inf)
    const PatchDev& P = pt[b.patch];
    int i, j, k;
    double s = 0.0;
    if (decode(P, BOX_INTERIOR, g, b.first, i, j, k))
      s = cfl_item(P, cell_of(P, i, j, k), U, dx + 3 * b.patch, c);
    for (int o = 32; o > 0; o >>= 1) s = fmax(s, __shfl_xor(s, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = red[0];
      for (int w = 1; w < BLK / 64; ++w) m = fmax(m, red[w]);
      // s >= 0, so its IEEE bit pattern orders like the value
      atomicMax(smax + b.patch, (unsigned long long)__double_as_longlong(m));
    }
    __syncthreads();  // red is rewritten by the next block
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
  const PatchDev& P = pt[b.patch];
  const int t = b.first + (int)threadIdx.x;
  if (t >= guard_count(P)) return;
  int i, j, k;
  guard_cell(P, g, t, i, j, k);
  if (guard_item(pt, b.patch, g, i, j, k, U, nbr, np)) atomicOr(status, 2);
}

// ------------------------------------------------------- local time stepping kernels
// A patch is ready when it is below t_end and none of its neighbours (26 directions) is
// behind it: every guard value it needs then lies between an owner's two slices.
__global__ __launch_bounds__(BLK) void k_lts_ready(const int32_t* __restrict__ nbr,
                                                   const double* __restrict__ t, double t_end,
                                                   int32_t* __restrict__ ready, int np) {
  const int p = blockIdx.x * BLK + threadIdx.x;
  if (p >= np) return;
  const double tp = t[p];
  int r = tp < t_end;
  for (int o = 0; o < 27 && r; ++o) {
    const int q = nbr[27 * p + o];
    if (q >= 0 && q < np && q != p && t[q] < tp) r = 0;
  }
  ready[p] = r;
}

// guard cells of the ready patches at their own time
template <typename T>
__global__ __launch_bounds__(BLK) void k_guards_at(const PatchDev* __restrict__ pt,
                                                   const BoxBlock* __restrict__ blk, T* U,
                                                   const T* __restrict__ Uprev,
                                                   const double* __restrict__ t,
                                                   const double* __restrict__ tprev,
                                                   const int32_t* __restrict__ nbr,
                                                   const int32_t* __restrict__ ready, int g,
                                                   int np, int* status, int nb0,
                                                   const int* __restrict__ dcount) {
  const int nb = table_count(nb0, dcount);
  for (int vb = blockIdx.x; vb < nb; vb += gridDim.x) {
    const BoxBlock b = blk[vb];
    if (!ready[b.patch]) continue;
    const PatchDev& P = pt[b.patch];
    const int q = b.first + (int)threadIdx.x;
    if (q >= guard_count(P)) continue;
    int i, j, k;
    guard_cell(P, g, q, i, j, k);
    if (guard_item_at(pt, b.patch, g, i, j, k, U, Uprev, t, tprev, nbr, np)) atomicOr(status, 2);
  }
}

// step of each patch: its own (or the given) step, rounded down to quantum x 2^k when a
// quantum is given (time levels: exact powers of two, frexp is exact), clipped to t_end when
// ready, else zero
// A ready patch whose step is not finite and positive (a non-finite state, or a bad given
// step) does not advance: its step is 0, it leaves the ready set (so the slice bookkeeping
// after the update leaves its state and time alone) and status bit 4 is raised.
__global__ __launch_bounds__(BLK) void k_lts_dt(int32_t* __restrict__ ready,
                                                const double* __restrict__ t, double t_end,
                                                double quantum, const double* src, double* dt,
                                                int np, int* status) {
  const int p = blockIdx.x * BLK + threadIdx.x;
  if (p >= np) return;
  double d = src[p];
  const bool good = d > 0.0 && d <= 1.7976931348623157e308;
  if (quantum > 0.0 && good) {
    int e;
    (void)frexp(d / quantum, &e);  // d / quantum in [2^(e-1), 2^e)
    d = ldexp(quantum, e - 1);
  }
  const double rest = t_end - t[p];
  const int r = ready[p];
  if (r && !good) {
    atomicOr(status, 4);
    ready[p] = 0;
  }
  dt[p] = r && good ? (d < rest ? d : rest) : 0.0;
}

// time of every ready patch advances by its step; a step clipped to t_end ends exactly there
__global__ __launch_bounds__(BLK) void k_lts_time(const int32_t* __restrict__ ready,
                                                  double* __restrict__ t,
                                                  double* __restrict__ tprev,
                                                  const double* __restrict__ dt, double t_end,
                                                  int np) {
  const int p = blockIdx.x * BLK + threadIdx.x;
  if (p >= np || !ready[p]) return;
  const double tp = t[p];
  tprev[p] = tp;
  t[p] = dt[p] >= t_end - tp ? t_end : tp + dt[p];
}

// ------------------------------------------------- compaction of the launch tables
// In a local time step only the ready patches work.  Every launch table (blocks or tiles)
// lists its entries patch by patch, so first[p] .. first[p + 1] are patch p's entries; the
// step copies the entries of the ready patches, in patch order, into compacted tables whose
// lengths the device writes, and the kernels run persistent grids over them.
constexpr int MAXKIND = 8;
struct CompactArgs {
  int nk;                              // tables compacted this step (<= MAXKIND)
  const int32_t* first[MAXKIND];       // per table: first entry of every patch, [P + 1]
  const uint64_t* src[MAXKIND];        // the full tables
  uint64_t* dst[MAXKIND];              // their compacted copies
  int words[MAXKIND];                  // 64-bit words per entry (BoxBlock 1, TileDev 2)
  int32_t* pref;                       // [MAXKIND][P + 1]: first compacted entry per ready patch
  int32_t* total;                      // [MAXKIND + 1]: entries per table, then the ready count
  int32_t* list;                       // ready patches in order, [P]
  int np;
};

// exclusive prefix sum over the work-group (a multiple of 64 threads, at most 1024); *total
// receives the sum
__device__ __forceinline__ int block_scan_excl(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int k = 0; k < nw; ++k) {
      const int t = sh[k];
      sh[k] = acc;
      acc += t;
    }
    sh[nw] = acc;
  }
  __syncthreads();
  const int r = sh[w] + x - v;
  *total = sh[nw];
  __syncthreads();  // sh is reused by the next call
  return r;
}

// one work-group of 1024 threads: the ready list, then per table the prefix of the ready
// patches' entry counts
__global__ __launch_bounds__(1024) void k_compact_scan(const int32_t* __restrict__ ready,
                                                       CompactArgs a) {
  __shared__ int sh[17];
  int nr = 0;
  for (int p0 = 0; p0 < a.np; p0 += 1024) {
    const int p = p0 + (int)threadIdx.x;
    const int f = p < a.np ? (ready[p] != 0) : 0;
    int tot;
    const int r = nr + block_scan_excl(f, sh, &tot);
    if (f) a.list[r] = p;
    nr += tot;
  }
  #pragma unroll
  for (int k = 0; k < MAXKIND; ++k) {
    if (k >= a.nk) break;
    const int32_t* first = a.first[k];
    int32_t* pref = a.pref + (int64_t)k * (a.np + 1);
    int acc = 0;
    for (int r0 = 0; r0 < nr; r0 += 1024) {
      const int r = r0 + (int)threadIdx.x;
      int c = 0;
      if (r < nr) {
        const int p = a.list[r];
        c = first[p + 1] - first[p];
      }
      int tot;
      const int e = acc + block_scan_excl(c, sh, &tot);
      if (r < nr) pref[r] = e;
      acc += tot;
    }
    if (threadIdx.x == 0) a.total[k] = acc;
  }
  if (threadIdx.x == 0) a.total[MAXKIND] = nr;
}

// work-groups take ready patches in turn and copy their entries of every table
__global__ __launch_bounds__(BLK) void k_compact_copy(CompactArgs a) {
  const int nr = a.total[MAXKIND];
  #pragma unroll
  for (int k = 0; k < MAXKIND; ++k) {
    if (k >= a.nk) break;
    const int32_t* first = a.first[k];
    const int32_t* pref = a.pref + (int64_t)k * (a.np + 1);
    const uint64_t* src = a.src[k];
    uint64_t* dst = a.dst[k];
    const int w = a.words[k];
    for (int r = blockIdx.x; r < nr; r += gridDim.x) {
      const int p = a.list[r];
      const int f0 = first[p], n = (first[p + 1] - f0) * w;
      const uint64_t* sp = src + (int64_t)f0 * w;
      uint64_t* dp = dst + (int64_t)pref[r] * w;
      for (int i = threadIdx.x; i < n; i += BLK) dp[i] = sp[i];
    }
  }
}

// ------------------------------------------------------------------- adjoint kernels
// grid.x: block table of the item box, grid.y: component

__device__ __forceinline__ bool decode3(const PatchDev& P, int kind, int g, int first, int x[3]) {
  return decode(P, kind, g, first, x[0], x[1], x[2]);
}

// lambda_W in two launches: PART 0 writes the faces' terms, PART 1 adds the edges' terms;
// two waves per SIMD (the dual-number items spill at three)
template <typename T, int EMF, int PART>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(2))) void k_adj_w(const PatchDev* __restrict__ pt,
                                               const BoxBlock* __restrict__ blk, const T* __restrict__ S,
                                               T* __restrict__ LS, const T* __restrict__ lam,
                                               const double* __restrict__ dt,
                                               const double* __restrict__ dx, Consts<T> c, int g,
                                              int remap) {
  const BoxBlock b = blk[logical_block(blockIdx.x, gridDim.x, remap)];
  const PatchDev& P = pt[b.patch];
  int x[3];
  if (!decode3(P, BOX_PRED, g, b.first, x)) return;
  const int v = blockIdx.y;
  T& out = LS[P.wbase + (int64_t)v * P.Nwc + wcell_of(P, g, x[0], x[1], x[2])];
  out = adj_w_item<EMF, PART>(P, g, x, v, S, lam, dt[b.patch], dx + 3 * b.patch, c,
                              PART == 1 ? out : T(0));
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_adj_e(const PatchDev* __restrict__ pt,
                                               const BoxBlock* __restrict__ blk, const T* __restrict__ U,
                                               const T* __restrict__ S, T* __restrict__ LS,
                                               const double* __restrict__ dt,
                                               const double* __restrict__ dx, Consts<T> c, int g,
                                              int remap) {
  const BoxBlock b = blk[logical_block(blockIdx.x, gridDim.x, remap)];
  const PatchDev& P = pt[b.patch];
  int x[3];
  if (!decode3(P, BOX_EN, g, b.first, x)) return;
  const int k = blockIdx.y;
  LS[P.sbase + 8 * P.Nc + (int64_t)k * P.Nc + cell_of(P, x[0], x[1], x[2])] =
      adj_e_item(P, g, x, k, U, S, (const T*)LS, dt[b.patch], dx + 3 * b.patch, c);
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_adj_q(const PatchDev* __restrict__ pt,
                                               const BoxBlock* __restrict__ blk, const T* __restrict__ U,
                                               const T* __restrict__ S, T* __restrict__ LS,
                                               const double* __restrict__ dt,
                                               const double* __restrict__ dx, Consts<T> c, int g,
                                              int remap) {
  const BoxBlock b = blk[logical_block(blockIdx.x, gridDim.x, remap)];
  const PatchDev& P = pt[b.patch];
  int x[3];
  if (!decode3(P, BOX_PRIM, g, b.first, x)) return;
  const int m = blockIdx.y;
  LS[P.sbase + (int64_t)m * P.Nc + cell_of(P, x[0], x[1], x[2])] =
      adj_q_item(P, g, x, m, U, S, (const T*)LS, (const T*)LS, dt[b.patch], dx + 3 * b.patch, c);
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_adj_u(const PatchDev* __restrict__ pt,
                                               const BoxBlock* __restrict__ blk, const T* __restrict__ U,
                                               const T* __restrict__ S, const T* __restrict__ LS,
                                               const T* __restrict__ lam, T* __restrict__ LU,
                                               const double* __restrict__ dt,
                                               const double* __restrict__ dx, Consts<T> c, int g,
                                              int remap) {
  const BoxBlock b = blk[logical_block(blockIdx.x, gridDim.x, remap)];
  const PatchDev& P = pt[b.patch];
  int x[3];
  if (!decode3(P, BOX_ALL, g, b.first, x)) return;
  const int m = blockIdx.y;
  LU[P.ubase + (int64_t)m * P.Nc + cell_of(P, x[0], x[1], x[2])] =
      adj_u_item(P, g, x, m, U, S, LS, LS, lam, dt[b.patch], dx + 3 * b.patch, c);
}

// guard copies are functions of their owners: owners collect the adjoints of their copies
// (deterministic order of the owner -> copies map built on the host); guards get zero
template <typename T>
__global__ __launch_bounds__(BLK) void k_adj_fold(const PatchDev* __restrict__ pt,
                                                  const BoxBlock* __restrict__ blk,
                                                  const T* __restrict__ LU, T* __restrict__ lam_in,
                                                  const int32_t* __restrict__ row,
                                                  const int32_t* __restrict__ col_patch,
                                                  const int32_t* __restrict__ col_cell, int g, int fold) {
  const BoxBlock b = blk[blockIdx.x];
  const PatchDev& P = pt[b.patch];
  int x[3];
  if (!decode3(P, BOX_ALL, g, b.first, x)) return;
  const int m = blockIdx.y;
  const int64_t cell = cell_of(P, x[0], x[1], x[2]);
  const int64_t o = P.ubase + (int64_t)m * P.Nc + cell;
  if (!fold) {
    lam_in[o] = LU[o];
    return;
  }
  if (!owned(P, g, x)) {
    lam_in[o] = T(0);
    return;
  }
  T s = LU[o];
  const int64_t id = P.ubase / 8 + cell;
  for (int32_t r = row[id]; r < row[id + 1]; ++r) {
    const PatchDev& Q = pt[col_patch[r]];
    s = s + LU[Q.ubase + (int64_t)m * Q.Nc + col_cell[r]];
  }
  lam_in[o] = s;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }



// Solver tile shapes per activity pattern (bit d set = direction d active), the first one
// the default.  The lists drive both the host-side tables and the kernel instantiations.
#define MHD_SHAPES_7(F) \
  F(8, 8, 4) F(16, 4, 4) F(8, 4, 8) F(16, 8, 2) F(32, 4, 2) F(8, 8, 2) F(32, 8, 2) F(32, 4, 4)
#define MHD_SHAPES_3(F) F(16, 16, 1) F(32, 8, 1) F(64, 4, 1) F(8, 8, 1)
#define MHD_SHAPES_1(F) F(64, 1, 1) F(128, 1, 1)
#define MHD_SHAPES_6(F) F(1, 16, 16)
#define MHD_SHAPES_5(F) F(16, 1, 16)
#define MHD_SHAPES_2(F) F(1, 64, 1)
#define MHD_SHAPES_4(F) F(1, 1, 64)
// fused predictor tile shapes per activity pattern, the first the default.  A tile as wide
// as the predictor box of a 32-cell patch (34) stores whole rows, so each wavefront writes
// one contiguous run of a predictor slot (the compact 8 x 8 x 4 tile has the smaller halo)
#define MHD_PSHAPES_7(F) F(8, 8, 4) F(34, 4, 2)
#define MHD_PSHAPES_3(F) F(16, 16, 1) F(34, 8, 1)
#define MHD_PSHAPES_6(F) F(1, 16, 16)
#define MHD_PSHAPES_5(F) F(16, 1, 16)
#define MHD_PSHAPES_1(F) F(128, 1, 1)
#define MHD_PSHAPES_2(F) F(1, 128, 1)
#define MHD_PSHAPES_4(F) F(1, 1, 128)
#define MHD_PRED_SHAPES(act, F)               \
  switch (act) {                               \
    case 7: MHD_PSHAPES_7(F) break;            \
    case 3: MHD_PSHAPES_3(F) break;            \
    case 6: MHD_PSHAPES_6(F) break;            \
    case 5: MHD_PSHAPES_5(F) break;            \
    case 1: MHD_PSHAPES_1(F) break;            \
    case 2: MHD_PSHAPES_2(F) break;            \
    default: MHD_PSHAPES_4(F) break;           \
  }
constexpr int MAXPSHAPE = 4;
constexpr int MAXSHAPE = 8;
// every shape list fits the fixed-size tables of the handle
#define MHD_COUNT_SHAPE(X, Y, Z) +1
static_assert(0 MHD_PSHAPES_7(MHD_COUNT_SHAPE) <= MAXPSHAPE &&
              0 MHD_PSHAPES_3(MHD_COUNT_SHAPE) <= MAXPSHAPE &&
              0 MHD_PSHAPES_6(MHD_COUNT_SHAPE) <= MAXPSHAPE &&
              0 MHD_PSHAPES_5(MHD_COUNT_SHAPE) <= MAXPSHAPE &&
              0 MHD_PSHAPES_1(MHD_COUNT_SHAPE) <= MAXPSHAPE &&
              0 MHD_PSHAPES_2(MHD_COUNT_SHAPE) <= MAXPSHAPE &&
              0 MHD_PSHAPES_4(MHD_COUNT_SHAPE) <= MAXPSHAPE,
              "a predictor shape list exceeds MAXPSHAPE");
static_assert(0 MHD_SHAPES_7(MHD_COUNT_SHAPE) <= MAXSHAPE &&
              0 MHD_SHAPES_3(MHD_COUNT_SHAPE) <= MAXSHAPE &&
              0 MHD_SHAPES_6(MHD_COUNT_SHAPE) <= MAXSHAPE &&
              0 MHD_SHAPES_5(MHD_COUNT_SHAPE) <= MAXSHAPE &&
              0 MHD_SHAPES_1(MHD_COUNT_SHAPE) <= MAXSHAPE &&
              0 MHD_SHAPES_2(MHD_COUNT_SHAPE) <= MAXSHAPE &&
              0 MHD_SHAPES_4(MHD_COUNT_SHAPE) <= MAXSHAPE,
              "a solver shape list exceeds MAXSHAPE");
#undef MHD_COUNT_SHAPE
constexpr int NMODE = 3;  // launch modes per tile shape: plain grid, XCD remap, persistent
struct TileCand {
  int x, y, z;
};

}  // namespace

// ------------------------------------------------------------------ static scratch
// Predictor scratch of mhd_bunch_update_static: one array per device in the library's code
// object, held by every device the library runs on until the process ends.  Its host-side
// name is not a device address: host code never passes `scratch` itself to a kernel or a
// copy.  mhd_bunch_bind resolves the device address once per device (with that device
// current) and keeps it in static_scratch_ptr; the entry point passes that pointer.
__device__ __align__(256) unsigned char scratch[MHD_STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex static_scratch_mu;
void* static_scratch_ptr[MAX_DEVICES] = {nullptr};

// device address of `scratch` on device `dev` (the current device), resolved on first use
hipError_t static_scratch_of(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(static_scratch_mu);
  if (!static_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    static_scratch_ptr[dev] = p;
  }
  *out = static_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

// ------------------------------------------------------------------------ handle

struct mhd_bunch {
  int P = 0, g = 3, prec = 8, limiter = 0, emf = 0;
  double gamma = 5.0 / 3.0, cfl = 0.4, rho_floor = 1e-12, p_floor = 1e-12, eps_deg = 1e-10;
  int64_t max_scratch = 0;
  std::vector<PatchDev> pt;
  int64_t state_elems = 0;
  int act = 0;  // active-direction pattern shared by all patches
  struct Chunk {
    int p0 = 0, p1 = 0;
    int blk0[NBOX] = {0}, nblk[NBOX] = {0};
    int tile0[MAXSHAPE] = {0}, ntile[MAXSHAPE] = {0};
    int ptile0[MAXPSHAPE] = {0}, nptile[MAXPSHAPE] = {0};
    int blk0_all = 0, nblk_all = 0;  // range of the whole-bunch BOX_ALL table
  };
  std::vector<Chunk> chunks;
  std::vector<BoxBlock> blocks[NBOX];
  // solver tile shapes for this bunch's dimensionality (mhd_bunch_tile_*), one tile table
  // per shape; the launch configuration in use is (shape, remap)
  int nshape = 0, shape = 0, mode = 0;  // mode 0 plain grid, 1 XCD remap, 2 persistent + remap
  int ncu = 256;                           // compute units of the bound device
  int dev = -1;                            // device current at bind
  void* static_scratch = nullptr;          // that device's address of `scratch`
  TileCand shapes[MAXSHAPE];
  std::vector<TileDev> tiles[MAXSHAPE];
  // predictor (mhd_bunch_set_predictor): 0 staged kernels, k >= 1 fused with tile shape
  // pshapes[k - 1]; one tile table over the predictor boxes per fused shape
  int fused = 0;
  int split = 0;  // solver form (mhd_bunch_set_solver_split): 0 one-phase, 1 two-phase, 2 edge
                  // pass, 3 edge pass as edge lines
  int npshape = 0;
  TileCand pshapes[MAXPSHAPE];
  std::vector<TileDev> ptiles[MAXPSHAPE];
  size_t o_ptiles[MAXPSHAPE] = {0};
  int64_t scratch_elems = 0;
  size_t o_ready = 0;  // local time stepping: ready flag per patch (int32)
  // Compacted launch tables of a local time step (bunches of one chunk): for every table its
  // per-patch first entries (uploaded) and room for a compacted copy.  Table ids: block kind k
  // -> k, solver tiles of shape k -> NBOX + k, predictor tiles of shape k -> NBOX + MAXSHAPE + k.
  static constexpr int NTAB = NBOX + MAXSHAPE + MAXPSHAPE;
  std::vector<int32_t> first[NTAB];
  size_t o_first[NTAB] = {0}, o_ctab[NTAB] = {0}, o_pref = 0, o_total = 0, o_list = 0;
  bool compact = false;     // launches read the compacted tables (inside a local time step)
  // mhd_bunch_update_cfl: the solver tiles also reduce the next step's time-step sums
  unsigned long long* cfl_next = nullptr;
  const int32_t* cfl_nbr = nullptr;
  int cslot[NTAB];          // slot of each table in the step's compaction, -1 if none
  // table id -> pointer and device count of its compacted copy
  const void* ctab(int id) const { return ws + o_ctab[id]; }
  const int* ccount(int id) const { return (const int*)(ws + o_total) + cslot[id]; }
  bool copy_rest = true;  // update: copy patches at rest (false inside a local time step)
  // inside a local time step: the update runs in place and the solver tiles write each
  // updated cell's previous state here (the previous time slice)
  void* keep = nullptr;
  size_t o_pt = 0, o_blk[NBOX] = {0}, o_tiles[MAXSHAPE] = {0}, o_smax = 0, o_status = 0,
         o_scratch = 0;
  // mhd_bunch_graph_capture: instantiated graph of a multi-step run
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  size_t ws_bytes = 0;
  char* ws = nullptr;
  bool bound = false;
  char last_error[256] = {0};
  // adjoint workspace: lambda scratch (layout of the forward scratch), lambda of the padded
  // input state, and the owner -> guard-copies map (CSR over all padded cells)
  char* aws = nullptr;
  bool adj_bound = false;
  bool adj_fold = false;
  size_t a_ls = 0, a_lu = 0, a_row = 0, a_colp = 0, a_colc = 0, a_bytes = 0;
  std::vector<int32_t> row, colp, colc;
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
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  }
  ~mhd_bunch() {
    drop_graph();
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
    c.emf = emf;
    return c;
  }
  // persistent grid: at most `per_cu` work-groups per compute unit, a multiple of the XCD
  // count when it is smaller than the table (see logical_block)
  int persistent_grid(int nb, int per_cu) const {
    const int cap = ncu * per_cu;
    if (nb <= cap) return nb;
    return std::max(NXCD, cap / NXCD * NXCD);
  }
  int stage_grid(int nb) const { return mode == 2 ? persistent_grid(nb, 2048 / BLK) : nb; }
  const PatchDev* d_pt() const { return (const PatchDev*)(ws + o_pt); }
  const BoxBlock* d_blk(int k) const { return (const BoxBlock*)(ws + o_blk[k]); }
  const TileDev* d_tiles(int k) const { return (const TileDev*)(ws + o_tiles[k]); }
  const TileDev* d_ptiles(int k) const { return (const TileDev*)(ws + o_ptiles[k]); }
  unsigned long long* d_smax() const { return (unsigned long long*)(ws + o_smax); }
  int* d_status() const { return (int*)(ws + o_status); }
  int32_t* d_ready() const { return (int32_t*)(ws + o_ready); }
  // the scratch of a sub-bunch of a host-streamed bunch lives in the stream's shared region
  char* scratch_ext = nullptr;
  void* d_scratch() const { return scratch_ext ? (void*)scratch_ext : (void*)(ws + o_scratch); }
};

namespace {

void add_blocks(std::vector<BoxBlock>& out, const PatchDev& P, int p, int kind, int g) {
  int lo[3], sz[3];
  box_of(P, kind, g, lo, sz);
  const int n = kind == BOX_GUARD ? guard_count(P)
                : kind == BOX_LINE ? (P.act == 7 ? edge_line_count(P) : 0)
                                   : sz[0] * sz[1] * sz[2];
  for (int f = 0; f < n; f += BLK) out.push_back(BoxBlock{p, f});
}

void set_shapes(mhd_bunch* h) {
  h->nshape = 0;
#define MHD_ADD(X, Y, Z) h->shapes[h->nshape++] = TileCand{X, Y, Z};
  switch (h->act) {
    case 7: MHD_SHAPES_7(MHD_ADD) break;
    case 3: MHD_SHAPES_3(MHD_ADD) break;
    case 1: MHD_SHAPES_1(MHD_ADD) break;
    case 6: MHD_SHAPES_6(MHD_ADD) break;
    case 5: MHD_SHAPES_5(MHD_ADD) break;
    case 2: MHD_SHAPES_2(MHD_ADD) break;
    default: MHD_SHAPES_4(MHD_ADD) break;
  }
#undef MHD_ADD
}

template <typename T, int X, int Y, int Z, int FORM, int EMF>
void solve_launch(mhd_bunch* h, int nt, const TileDev* tl, const T* Uin, T* Uout, const T* S,
                  const double* dt, const double* dx, const Consts<T>& c, hipStream_t s,
                  const int* dcount) {
  int grid = nt;
  const void* kern = h->keep ? reinterpret_cast<const void*>(k_solve_keep<T, X, Y, Z, FORM, EMF>)
                             : reinterpret_cast<const void*>(k_solve<T, X, Y, Z, FORM, EMF>);
  if (h->mode == 2 || dcount) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, TileShape<X, Y, Z>::THREADS, 0) !=
            hipSuccess ||
        occ < 1)
      occ = 1;
    grid = h->persistent_grid(nt, occ);
  }
  if (h->keep)  // in place (Uin == Uout), no fused time step, patches at rest skipped
    hipLaunchKernelGGL((k_solve_keep<T, X, Y, Z, FORM, EMF>), dim3(grid),
                       dim3(TileShape<X, Y, Z>::THREADS), 0, s, h->d_pt(), tl, Uout, (T*)h->keep,
                       S, dt, dx, c, h->g, nt, h->mode >= 1 || dcount, dcount);
  else
    hipLaunchKernelGGL((k_solve<T, X, Y, Z, FORM, EMF>), dim3(grid),
                       dim3(TileShape<X, Y, Z>::THREADS), 0, s, h->d_pt(), tl, Uin, Uout, S, dt,
                       dx, c, h->g, nt, h->mode >= 1 || dcount, h->copy_rest ? 1 : 0, dcount,
                       h->cfl_next, h->cfl_nbr);
}

template <typename T, int X, int Y, int Z, int EMF>
void edges_launch(mhd_bunch* h, int nt, const TileDev* tl, T* S, const double* dt,
                  const double* dx, const Consts<T>& c, hipStream_t s, const int* dcount) {
  int grid = nt;
  if (h->mode == 2 || dcount) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, reinterpret_cast<const void*>(k_edges<T, X, Y, Z, EMF>), TileShape<X, Y, Z>::THREADS,
            0) != hipSuccess || occ < 1)
      occ = 1;
    grid = h->persistent_grid(nt, occ);
  }
  hipLaunchKernelGGL((k_edges<T, X, Y, Z, EMF>), dim3(grid), dim3(TileShape<X, Y, Z>::THREADS), 0, s,
                     h->d_pt(), tl, S, dt, dx, c, h->g, nt, h->mode >= 1 || dcount, dcount);
}

// edges = true: the per-tile owned-edge pass (solver form 2, and form 3 outside 3D); else the
// solver tiles
template <typename T>
void launch_solve(mhd_bunch* h, const mhd_bunch::Chunk& ch, const T* Uin, T* Uout, T* S,
                  const double* dt, const double* dx, const Consts<T>& c, hipStream_t s,
                  bool edges) {
  const int k = h->shape;
  const TileCand tc = h->shapes[k];
  const int nt = ch.ntile[k];
  const int id = NBOX + k;
  const bool cmp = h->compact && h->cslot[id] >= 0;
  const TileDev* tl = cmp ? (const TileDev*)h->ctab(id) : h->d_tiles(k) + ch.tile0[k];
  const int* dc = cmp ? h->ccount(id) : nullptr;
#define MHD_TRY_EMF(X, Y, Z, EMF)                                                             \
  if (edges)                                                                                  \
    edges_launch<T, X, Y, Z, EMF>(h, nt, tl, S, dt, dx, c, s, dc);                            \
  else if (h->split >= 2)                                                                     \
    solve_launch<T, X, Y, Z, 2, EMF>(h, nt, tl, Uin, Uout, S, dt, dx, c, s, dc);              \
  else if (h->split == 1)                                                                     \
    solve_launch<T, X, Y, Z, 1, EMF>(h, nt, tl, Uin, Uout, S, dt, dx, c, s, dc);              \
  else                                                                                        \
    solve_launch<T, X, Y, Z, 0, EMF>(h, nt, tl, Uin, Uout, S, dt, dx, c, s, dc);
#define MHD_TRY(X, Y, Z)                                                                      \
  if (tc.x == X && tc.y == Y && tc.z == Z) {                                                  \
    if (h->emf == 1) {                                                                        \
      MHD_TRY_EMF(X, Y, Z, 1)                                                                 \
    } else {                                                                                  \
      MHD_TRY_EMF(X, Y, Z, 0)                                                                 \
    }                                                                                         \
    return;                                                                                   \
  }
  switch (h->act) {
    case 7: MHD_SHAPES_7(MHD_TRY) break;
    case 3: MHD_SHAPES_3(MHD_TRY) break;
    case 1: MHD_SHAPES_1(MHD_TRY) break;
    case 6: MHD_SHAPES_6(MHD_TRY) break;
    case 5: MHD_SHAPES_5(MHD_TRY) break;
    case 2: MHD_SHAPES_2(MHD_TRY) break;
    default: MHD_SHAPES_4(MHD_TRY) break;
  }
#undef MHD_TRY
#undef MHD_TRY_EMF
}

template <typename T, int EMF>
void edge_lines_launch(mhd_bunch* h, int nb, const BoxBlock* tb, T* S, const double* dt,
                       const Consts<T>& c, hipStream_t s, const int* dcount) {
  int grid = nb;
  if (h->mode == 2 || dcount) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, reinterpret_cast<const void*>(k_edge_lines<T, EMF>), BLK, 0) != hipSuccess ||
        occ < 1)
      occ = 1;
    grid = h->persistent_grid(nb, occ);
  }
  hipLaunchKernelGGL((k_edge_lines<T, EMF>), dim3(grid), dim3(BLK), 0, s, h->d_pt(), tb, S, dt, c,
                     h->g, nb, h->mode >= 1 || dcount, dcount);
}

// the edge pass of solver form 3: the chunk's edge lines (or their compacted copy)
template <typename T>
void launch_edge_lines(mhd_bunch* h, const mhd_bunch::Chunk& ch, T* S, const double* dt,
                       const Consts<T>& c, hipStream_t s) {
  const int nb = ch.nblk[BOX_LINE];
  if (!nb) return;
  const bool cmp = h->compact && h->cslot[BOX_LINE] >= 0;
  const BoxBlock* tb = cmp ? (const BoxBlock*)h->ctab(BOX_LINE) : h->d_blk(BOX_LINE) + ch.blk0[BOX_LINE];
  const int* dc = cmp ? h->ccount(BOX_LINE) : nullptr;
  if (h->emf == 1)
    edge_lines_launch<T, 1>(h, nb, tb, S, dt, c, s, dc);
  else
    edge_lines_launch<T, 0>(h, nb, tb, S, dt, c, s, dc);
}

// S: scratch of one chunk of patches
template <typename T>
mhd_status launch_update(mhd_bunch* h, const T* Uin, T* Uout, const double* dt, const double* dx,
                         hipStream_t s, T* S) {
  const Consts<T> c = h->consts<T>();
  const int rm = h->mode >= 1;
  for (const auto& ch : h->chunks) {
    hipEvent_t t0;
    if (h->fused && ch.nptile[h->fused - 1]) {
      t0 = h->tic(s);
      const int pk = h->fused - 1;
      const TileCand pc = h->pshapes[pk];
      const int nt = ch.nptile[pk];
      const int id = NBOX + MAXSHAPE + pk;
      const bool cmp = h->compact && h->cslot[id] >= 0;
      const TileDev* tl = cmp ? (const TileDev*)h->ctab(id) : h->d_ptiles(pk) + ch.ptile0[pk];
      const int* dc = cmp ? h->ccount(id) : nullptr;
#define MHD_PRED_LAUNCH(X, Y, Z)                                                                \
  if (pc.x == X && pc.y == Y && pc.z == Z) {                                                   \
    int grid = nt;                                                                             \
    if (h->mode == 2 || dc) {                                                                  \
      int occ = 0;                                                                             \
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(                                        \
              &occ, reinterpret_cast<const void*>(k_predict<T, X, Y, Z>),                      \
              PredShape<X, Y, Z>::THREADS, 0) != hipSuccess || occ < 1)                        \
        occ = 1;                                                                               \
      grid = h->persistent_grid(nt, occ);                                                      \
    }                                                                                          \
    hipLaunchKernelGGL((k_predict<T, X, Y, Z>), dim3(grid), dim3(PredShape<X, Y, Z>::THREADS), 0, \
                       s, h->d_pt(), tl, Uin, S, dt, dx, c, h->g, h->d_status(), nt, rm || dc, dc);  \
  }
      MHD_PRED_SHAPES(h->act, MHD_PRED_LAUNCH)
#undef MHD_PRED_LAUNCH
      h->toc(s, MHD_KERNEL_PREDICT, t0);
    }
    // staged predictor: the block tables of the chunk, or their compacted copies
    auto stage = [&](int kind, const BoxBlock*& tb, int& grid, const int*& dc) {
      const int nb = ch.nblk[kind];
      const bool cmp = h->compact && h->cslot[kind] >= 0;
      tb = cmp ? (const BoxBlock*)h->ctab(kind) : h->d_blk(kind) + ch.blk0[kind];
      dc = cmp ? h->ccount(kind) : nullptr;
      grid = cmp ? h->persistent_grid(nb, 2048 / BLK) : h->stage_grid(nb);
      return nb;
    };
    if (!h->fused && ch.nblk[BOX_PRIM]) {
      const BoxBlock* tb;
      int grid;
      const int* dc;
      const int nb = stage(BOX_PRIM, tb, grid, dc);
      t0 = h->tic(s);
      hipLaunchKernelGGL(k_prim<T>, dim3(grid), dim3(BLK), 0, s, h->d_pt(), tb, Uin, S, dt, c,
                         h->g, h->d_status(), nb, rm || dc, dc);
      h->toc(s, MHD_KERNEL_PRIM, t0);
    }
    if (!h->fused && ch.nblk[BOX_EN]) {
      const BoxBlock* tb;
      int grid;
      const int* dc;
      const int nb = stage(BOX_EN, tb, grid, dc);
      t0 = h->tic(s);
      hipLaunchKernelGGL(k_en<T>, dim3(grid), dim3(BLK), 0, s, h->d_pt(), tb, Uin, S, dt, h->g,
                         nb, rm || dc, dc);
      h->toc(s, MHD_KERNEL_EDGE_EMF_N, t0);
    }
    if (!h->fused && ch.nblk[BOX_PRED]) {
      const BoxBlock* tb;
      int grid;
      const int* dc;
      const int nb = stage(BOX_PRED, tb, grid, dc);
      t0 = h->tic(s);
      hipLaunchKernelGGL(k_pred<T>, dim3(grid), dim3(BLK), 0, s, h->d_pt(), tb, Uin, S, dt, dx,
                         dt, c, h->g, nb, rm || dc, dc);
      h->toc(s, MHD_KERNEL_PREDICT, t0);
    }
    if (h->split >= 2 && ch.ntile[h->shape]) {
      t0 = h->tic(s);
      if (h->split == 3 && h->act == 7)
        launch_edge_lines<T>(h, ch, S, dt, c, s);
      else
        launch_solve<T>(h, ch, Uin, Uout, S, dt, dx, c, s, true);
      h->toc(s, MHD_KERNEL_EDGE, t0);
    }
    if (ch.ntile[h->shape]) {
      t0 = h->tic(s);
      launch_solve<T>(h, ch, Uin, Uout, S, dt, dx, c, s, false);
      h->toc(s, MHD_KERNEL_SOLVE, t0);
    }
  }
  return h->hip_ok(hipGetLastError(), "launch update kernels") ? MHD_OK : MHD_EDEVICE;
}

template <typename T>
mhd_status launch_cfl(mhd_bunch* h, const T* U, const double* dx, double* dt, int global,
                      hipStream_t s, const int32_t* mask = nullptr) {
  const Consts<T> c = h->consts<T>();
  hipEvent_t t0 = h->tic(s);
  hipLaunchKernelGGL(k_zero_u64, dim3((h->P + 255) / 256), dim3(256), 0, s, h->d_smax(), h->P);
  const int nb = (int)h->blocks[BOX_INTERIOR].size();
  const bool cmp = h->compact && h->cslot[BOX_INTERIOR] >= 0;
  hipLaunchKernelGGL(k_cfl<T>, dim3(cmp ? h->persistent_grid(nb, 2048 / BLK) : nb), dim3(BLK), 0, s,
                     h->d_pt(), cmp ? (const BoxBlock*)h->ctab(BOX_INTERIOR) : h->d_blk(BOX_INTERIOR),
                     U, dx, mask, c, h->g, h->d_smax(), nb,
                     cmp ? h->ccount(BOX_INTERIOR) : nullptr);
  hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(BLK), 0, s, h->P, (const unsigned long long*)h->d_smax(),
                     h->cfl, dt, global);
  h->toc(s, MHD_KERNEL_CFL, t0);
  return h->hip_ok(hipGetLastError(), "launch cfl kernels") ? MHD_OK : MHD_EDEVICE;
}

template <typename T>
mhd_status launch_guards(mhd_bunch* h, T* U, const int32_t* nbr, hipStream_t s) {
  const int nb = (int)h->blocks[BOX_GUARD].size();
  if (nb == 0) return MHD_OK;
  hipEvent_t t0 = h->tic(s);
  hipLaunchKernelGGL(k_guards<T>, dim3(nb), dim3(BLK), 0, s, h->d_pt(), h->d_blk(BOX_GUARD), U, nbr, h->g,
                     h->P, h->d_status());
  h->toc(s, MHD_KERNEL_GUARDS, t0);
  return h->hip_ok(hipGetLastError(), "launch guard kernel") ? MHD_OK : MHD_EDEVICE;
}

// owner -> guard-copies map of the whole bunch (empty when nbr is NULL: frozen guards)
int build_guard_map(mhd_bunch* h, const int32_t* nbr) {
  h->row.clear();
  h->colp.clear();
  h->colc.clear();
  if (!nbr) return 0;
  const int64_t ncell = h->state_elems / 8;
  if (ncell >= INT32_MAX) return -1;
  std::vector<int32_t> cnt(ncell + 1, 0);
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      h->row.assign(ncell + 1, 0);
      for (int64_t i = 0; i < ncell; ++i) h->row[i + 1] = h->row[i] + cnt[i];
      h->colp.assign(h->row[ncell], 0);
      h->colc.assign(h->row[ncell], 0);
      std::fill(cnt.begin(), cnt.end(), 0);
    }
    for (int p = 0; p < h->P; ++p) {
      const PatchDev& P = h->pt[p];
      for (int k = 0; k < P.N[2]; ++k)
        for (int j = 0; j < P.N[1]; ++j)
          for (int i = 0; i < P.N[0]; ++i) {
            int src;
            int64_t sc;
            const int r = guard_source(h->pt.data(), p, h->g, i, j, k, nbr, h->P, src, sc);
            if (r < 0) return -1;
            if (r == 0) continue;
            const int64_t id = h->pt[src].ubase / 8 + sc;
            if (pass == 1) {
              const int32_t at = h->row[id] + cnt[id];
              h->colp[at] = p;
              h->colc[at] = (int32_t)cell_of(P, i, j, k);
            }
            cnt[id]++;
          }
    }
  }
  return 0;
}

template <typename T>
mhd_status launch_adjoint(mhd_bunch* h, const T* U, const T* lam, T* lam_in, const double* dt,
                          const double* dx, hipStream_t s) {
  const Consts<T> c = h->consts<T>();
  T* S = (T*)h->d_scratch();
  T* LS = (T*)(h->aws + h->a_ls);
  T* LU = (T*)(h->aws + h->a_lu);
  for (const auto& ch : h->chunks) {
    // forward intermediates of this update (primitives, EMFs at t^n, predictor data)
    if (ch.nblk[BOX_PRIM])
      hipLaunchKernelGGL(k_prim<T>, dim3(ch.nblk[BOX_PRIM]), dim3(BLK), 0, s, h->d_pt(),
                         h->d_blk(BOX_PRIM) + ch.blk0[BOX_PRIM], U, S, (const double*)nullptr, c,
                         h->g, h->d_status(), ch.nblk[BOX_PRIM], 0, (const int*)nullptr);
    if (ch.nblk[BOX_EN])
      hipLaunchKernelGGL(k_en<T>, dim3(ch.nblk[BOX_EN]), dim3(BLK), 0, s, h->d_pt(),
                         h->d_blk(BOX_EN) + ch.blk0[BOX_EN], U, S, (const double*)nullptr, h->g,
                         ch.nblk[BOX_EN], 0, (const int*)nullptr);
    if (ch.nblk[BOX_PRED])
      hipLaunchKernelGGL(k_pred<T>, dim3(ch.nblk[BOX_PRED]), dim3(BLK), 0, s, h->d_pt(),
                         h->d_blk(BOX_PRED) + ch.blk0[BOX_PRED], U, S, dt, dx,
                         (const double*)nullptr, c, h->g, ch.nblk[BOX_PRED], 0, (const int*)nullptr);
    // reverse sweep: predictor data, EMFs at t^n, primitives, padded input state
    if (ch.nblk[BOX_PRED]) {
      const dim3 grid(ch.nblk[BOX_PRED], NW);
      const BoxBlock* tb = h->d_blk(BOX_PRED) + ch.blk0[BOX_PRED];
      hipLaunchKernelGGL((k_adj_w<T, 0, 0>), grid, dim3(BLK), 0, s, h->d_pt(), tb, (const T*)S, LS,
                         lam, dt, dx, c, h->g, 0);
      if (h->emf == 1)
        hipLaunchKernelGGL((k_adj_w<T, 1, 1>), grid, dim3(BLK), 0, s, h->d_pt(), tb, (const T*)S,
                           LS, lam, dt, dx, c, h->g, 0);
      else
        hipLaunchKernelGGL((k_adj_w<T, 0, 1>), grid, dim3(BLK), 0, s, h->d_pt(), tb, (const T*)S,
                           LS, lam, dt, dx, c, h->g, 0);
    }
    if (ch.nblk[BOX_EN])
      hipLaunchKernelGGL(k_adj_e<T>, dim3(ch.nblk[BOX_EN], 3), dim3(BLK), 0, s, h->d_pt(),
                         h->d_blk(BOX_EN) + ch.blk0[BOX_EN], U, (const T*)S, LS, dt, dx, c, h->g, 0);
    if (ch.nblk[BOX_PRIM])
      hipLaunchKernelGGL(k_adj_q<T>, dim3(ch.nblk[BOX_PRIM], 8), dim3(BLK), 0, s, h->d_pt(),
                         h->d_blk(BOX_PRIM) + ch.blk0[BOX_PRIM], U, (const T*)S, LS, dt, dx, c, h->g, 0);
    const int nb = ch.nblk_all;
    if (nb)
      hipLaunchKernelGGL(k_adj_u<T>, dim3(nb, 8), dim3(BLK), 0, s, h->d_pt(),
                         h->d_blk(BOX_ALL) + ch.blk0_all, U, (const T*)S, (const T*)LS, lam, LU, dt,
                         dx, c, h->g, 0);
  }
  const int nball = (int)h->blocks[BOX_ALL].size();
  hipLaunchKernelGGL(k_adj_fold<T>, dim3(nball, 8), dim3(BLK), 0, s, h->d_pt(), h->d_blk(BOX_ALL),
                     (const T*)LU, lam_in, (const int32_t*)(h->aws + h->a_row),
                     (const int32_t*)(h->aws + h->a_colp), (const int32_t*)(h->aws + h->a_colc), h->g,
                     h->adj_fold ? 1 : 0);
  return h->hip_ok(hipGetLastError(), "launch adjoint kernels") ? MHD_OK : MHD_EDEVICE;
}

template <typename T>
mhd_status launch_lts_step(mhd_bunch* h, T* Ucur, T* Uprev, double* t, double* tprev,
                           double* dt, const double* dt_fixed, const double* dx,
                           const int32_t* nbr, double t_end, double quantum, hipStream_t s) {
  const int pg = (h->P + BLK - 1) / BLK;
  int32_t* ready = h->d_ready();
  hipLaunchKernelGGL(k_lts_ready, dim3(pg), dim3(BLK), 0, s, nbr, (const double*)t, t_end, ready,
                     h->P);
  // With free steps few patches are ready at a time: with one chunk, every launch below then
  // runs over the ready patches' entries only (the tables it reads are compacted on the device
  // first, persistent grids).  With time levels (quantum > 0) patches advance in lock-step
  // groups, most of the bunch at once, where the tuned full-table launches are faster.
  const bool cmp = h->chunks.size() == 1 && !(quantum > 0.0);
  if (cmp) {
    CompactArgs a = {};
    a.np = h->P;
    auto add = [&](int id, int words) {
      h->cslot[id] = a.nk;
      a.first[a.nk] = (const int32_t*)(h->ws + h->o_first[id]);
      a.src[a.nk] = (const uint64_t*)(id < NBOX ? (const void*)h->d_blk(id)
                                     : id < NBOX + MAXSHAPE ? (const void*)h->d_tiles(id - NBOX)
                                                            : (const void*)h->d_ptiles(id - NBOX - MAXSHAPE));
      a.dst[a.nk] = (uint64_t*)(h->ws + h->o_ctab[id]);
      a.words[a.nk] = words;
      ++a.nk;
    };
    for (int id = 0; id < mhd_bunch::NTAB; ++id) h->cslot[id] = -1;
    add(BOX_GUARD, 1);
    if (!dt_fixed) add(BOX_INTERIOR, 1);
    add(NBOX + h->shape, 2);
    if (h->split == 3 && h->act == 7) add(BOX_LINE, 1);
    if (h->fused) {
      add(NBOX + MAXSHAPE + h->fused - 1, 2);
    } else {
      add(BOX_PRIM, 1);
      add(BOX_EN, 1);
      add(BOX_PRED, 1);
    }
    a.pref = (int32_t*)(h->ws + h->o_pref);
    a.total = (int32_t*)(h->ws + h->o_total);
    a.list = (int32_t*)(h->ws + h->o_list);
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, (const int32_t*)ready, a);
    hipLaunchKernelGGL(k_compact_copy, dim3(std::min(h->P, h->ncu * 4)), dim3(BLK), 0, s, a);
    h->compact = true;
  }
  const int ng = (int)h->blocks[BOX_GUARD].size();
  if (ng) {
    hipEvent_t t0 = h->tic(s);
    hipLaunchKernelGGL(k_guards_at<T>, dim3(cmp ? h->persistent_grid(ng, 2048 / BLK) : ng),
                       dim3(BLK), 0, s, h->d_pt(),
                       cmp ? (const BoxBlock*)h->ctab(BOX_GUARD) : h->d_blk(BOX_GUARD), Ucur,
                       (const T*)Uprev, (const double*)t, (const double*)tprev, nbr,
                       (const int32_t*)ready, h->g, h->P, h->d_status(), ng,
                       cmp ? h->ccount(BOX_GUARD) : nullptr);
    h->toc(s, MHD_KERNEL_GUARDS, t0);
  }
  mhd_status st = MHD_OK;
  if (!dt_fixed) st = launch_cfl<T>(h, (const T*)Ucur, dx, dt, 0, s, ready);
  if (st == MHD_OK) {
    hipLaunchKernelGGL(k_lts_dt, dim3(pg), dim3(BLK), 0, s, ready, (const double*)t,
                       t_end, quantum, dt_fixed ? dt_fixed : (const double*)dt, dt, h->P,
                       h->d_status());
    // the ready patches advance in place; their solver tiles write each cell's state before
    // the update to U_prev (owned cells and faces: the previous slice); patches at rest are
    // neither computed nor written
    h->copy_rest = false;
    h->keep = Uprev;
    st = launch_update<T>(h, (const T*)Ucur, Ucur, dt, dx, s, (T*)h->d_scratch());
    h->keep = nullptr;
    h->copy_rest = true;
  }
  if (st == MHD_OK) {
    hipLaunchKernelGGL(k_lts_time, dim3(pg), dim3(BLK), 0, s, (const int32_t*)ready, t, tprev,
                       (const double*)dt, t_end, h->P);
  }
  h->compact = false;
  if (st != MHD_OK) return st;
  return h->hip_ok(hipGetLastError(), "launch local time step") ? MHD_OK : MHD_EDEVICE;
}

}  // namespace

// ------------------------------------------------------------ host-streamed bunches
// A bunch whose state stays in host memory is cut into consecutive sub-bunches; each update
// streams them through `slots` device slots on three streams (copy in, compute, copy out),
// so that the copy of sub-bunch j+1 in, the update of j and the copy of j-1 out overlap.
struct mhd_stream {
  std::vector<mhd_bunch*> sub;       // one handle per sub-bunch (tables in `dev`)
  std::vector<int> p0;               // first patch of each sub-bunch (p0[nsub] = P)
  std::vector<int64_t> base;         // element offset of each sub-bunch in the state
  int P = 0, prec = 8, slots = 3;
  int64_t slot_elems = 0;            // largest sub-bunch state
  size_t o_scratch = 0, o_dt = 0, o_dx = 0, o_slot = 0, bytes = 0;
  std::vector<size_t> o_tab;         // table region of each sub-bunch
  char* dev = nullptr;
  bool bound = false;
  hipStream_t st[3] = {nullptr, nullptr, nullptr};   // copy in, compute, copy out
  std::vector<hipEvent_t> ev;        // per slot: input ready, compute done, output done; + start
  char last_error[256] = {0};
  ~mhd_stream() {
    for (mhd_bunch* b : sub) delete b;
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipStream_t x : st)
      if (x) (void)hipStreamDestroy(x);
  }
  char* slot_in(int k) const { return dev + o_slot + (size_t)(2 * k) * align256((size_t)slot_elems * prec); }
  char* slot_out(int k) const { return slot_in(k) + align256((size_t)slot_elems * prec); }
  bool ok(hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    snprintf(last_error, sizeof(last_error), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    return false;
  }
};

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
      !(d->eps_deg >= 0.0) || (d->limiter != 0 && d->limiter != 1) || d->max_scratch_bytes < 0 ||
      (d->emf_solver != 0 && d->emf_solver != 1))
    return MHD_EINVAL;
  mhd_bunch* h = new (std::nothrow) mhd_bunch;
  if (!h) return MHD_ENOMEM;
  h->P = d->n_patches;
  h->g = d->guard;
  h->prec = d->precision;
  h->gamma = d->gamma;
  h->cfl = d->cfl;
  h->limiter = d->limiter;
  h->emf = d->emf_solver;
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
    // the kernels address a patch's scratch block by 32-bit byte offsets from its base
    if ((11 * P.Nc + NW * P.Nwc) * (int64_t)h->prec > (int64_t)UINT32_MAX) {
      delete h;
      return MHD_EUNSUPPORTED;
    }
    P.ubase = base;
    base += 8 * P.Nc;
  }
  h->state_elems = base;
  set_shapes(h);
  h->npshape = 0;
#define MHD_ADD_PRED(X, Y, Z) h->pshapes[h->npshape++] = TileCand{X, Y, Z};
  MHD_PRED_SHAPES(h->act, MHD_ADD_PRED)
#undef MHD_ADD_PRED

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
    for (int kind : {BOX_PRIM, BOX_EN, BOX_PRED, BOX_LINE}) {
      ch.blk0[kind] = (int)h->blocks[kind].size();
      for (int p = ch.p0; p < ch.p1; ++p) add_blocks(h->blocks[kind], h->pt[p], p, kind, g);
      ch.nblk[kind] = (int)h->blocks[kind].size() - ch.blk0[kind];
    }
    for (int k = 0; k < h->nshape; ++k) {
      const TileCand tc = h->shapes[k];
      const int T3[3] = {tc.x, tc.y, tc.z};
      ch.tile0[k] = (int)h->tiles[k].size();
      for (int p = ch.p0; p < ch.p1; ++p) {
        const PatchDev& P = h->pt[p];
        int nt[3];
        for (int dd = 0; dd < 3; ++dd) nt[dd] = (P.act >> dd & 1) ? (P.n[dd] + T3[dd] - 1) / T3[dd] : 1;
        for (int z = 0; z < nt[2]; ++z)
          for (int y = 0; y < nt[1]; ++y)
            for (int x = 0; x < nt[0]; ++x)
              h->tiles[k].push_back(TileDev{p, x * tc.x, y * tc.y, z * tc.z});
      }
      ch.ntile[k] = (int)h->tiles[k].size() - ch.tile0[k];
    }
    for (int k = 0; k < h->npshape; ++k) {
      const TileCand pc = h->pshapes[k];
      const int T3[3] = {pc.x, pc.y, pc.z};
      ch.ptile0[k] = (int)h->ptiles[k].size();
      for (int p = ch.p0; p < ch.p1; ++p) {
        const PatchDev& P = h->pt[p];
        int nt[3];
        for (int dd = 0; dd < 3; ++dd) nt[dd] = (P.act >> dd & 1) ? (P.n[dd] + 2 + T3[dd] - 1) / T3[dd] : 1;
        for (int z = 0; z < nt[2]; ++z)
          for (int y = 0; y < nt[1]; ++y)
            for (int x = 0; x < nt[0]; ++x)
              h->ptiles[k].push_back(TileDev{p, x * T3[0], y * T3[1], z * T3[2]});
      }
      ch.nptile[k] = (int)h->ptiles[k].size() - ch.ptile0[k];
    }
  }
  for (auto& ch : h->chunks) {
    ch.blk0_all = (int)h->blocks[BOX_ALL].size();
    for (int p = ch.p0; p < ch.p1; ++p) {
      add_blocks(h->blocks[BOX_INTERIOR], h->pt[p], p, BOX_INTERIOR, g);
      add_blocks(h->blocks[BOX_ALL], h->pt[p], p, BOX_ALL, g);
      add_blocks(h->blocks[BOX_GUARD], h->pt[p], p, BOX_GUARD, g);
    }
    ch.nblk_all = (int)h->blocks[BOX_ALL].size() - ch.blk0_all;
  }
  // per-patch first entry of every launch table (each lists its entries patch by patch)
  auto firsts = [&](std::vector<int32_t>& f, auto const& tab) {
    f.assign(h->P + 1, 0);
    std::vector<int32_t> cnt(h->P, 0);
    for (const auto& e : tab) cnt[e.patch]++;
    for (int p = 0; p < h->P; ++p) f[p + 1] = f[p] + cnt[p];
  };
  for (int k = 0; k < NBOX; ++k) firsts(h->first[k], h->blocks[k]);
  for (int k = 0; k < h->nshape; ++k) firsts(h->first[NBOX + k], h->tiles[k]);
  for (int k = 0; k < h->npshape; ++k) firsts(h->first[NBOX + MAXSHAPE + k], h->ptiles[k]);
  for (int id = 0; id < mhd_bunch::NTAB; ++id) h->cslot[id] = -1;
  // workspace layout
  size_t o = 0;
  h->o_pt = o;
  o = align256(o + sizeof(PatchDev) * h->P);
  for (int k = 0; k < NBOX; ++k) {
    h->o_blk[k] = o;
    o = align256(o + sizeof(BoxBlock) * std::max<size_t>(1, h->blocks[k].size()));
  }
  for (int k = 0; k < h->nshape; ++k) {
    h->o_tiles[k] = o;
    o = align256(o + sizeof(TileDev) * std::max<size_t>(1, h->tiles[k].size()));
  }
  for (int k = 0; k < h->npshape; ++k) {
    h->o_ptiles[k] = o;
    o = align256(o + sizeof(TileDev) * std::max<size_t>(1, h->ptiles[k].size()));
  }
  h->o_smax = o;
  o = align256(o + sizeof(unsigned long long) * h->P);
  h->o_status = o;
  o = align256(o + sizeof(unsigned long long));
  h->o_ready = o;
  o = align256(o + sizeof(int32_t) * h->P);
  // compaction of a local time step: first entries, compacted copies, prefix sums, counts
  {
    auto entry_bytes = [&](int id) -> size_t {
      if (id < NBOX) return sizeof(BoxBlock) * h->blocks[id].size();
      if (id < NBOX + MAXSHAPE) return sizeof(TileDev) * h->tiles[id - NBOX].size();
      return sizeof(TileDev) * h->ptiles[id - NBOX - MAXSHAPE].size();
    };
    for (int id = 0; id < mhd_bunch::NTAB; ++id) {
      if (h->first[id].empty()) continue;
      h->o_first[id] = o;
      o = align256(o + sizeof(int32_t) * h->first[id].size());
      h->o_ctab[id] = o;
      o = align256(o + std::max<size_t>(16, entry_bytes(id)));
    }
    h->o_pref = o;
    o = align256(o + sizeof(int32_t) * (size_t)MAXKIND * (h->P + 1));
    h->o_total = o;
    o = align256(o + sizeof(int32_t) * (MAXKIND + 1));
    h->o_list = o;
    o = align256(o + sizeof(int32_t) * h->P);
  }
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
  {
    int dev = 0, n = 0;
    if (!h->hip_ok(hipGetDevice(&dev), "current device")) return MHD_EDEVICE;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      h->ncu = n;
    h->dev = dev;
    // set-up of the allocation-free update: this device's address of the static scratch
    if (!h->hip_ok(static_scratch_of(dev, &h->static_scratch), "resolve static scratch"))
      return MHD_EDEVICE;
  }
  bool ok = h->hip_ok(hipMemcpyAsync(h->ws + h->o_pt, h->pt.data(), sizeof(PatchDev) * h->P,
                                     hipMemcpyHostToDevice, s), "upload patch table");
  for (int k = 0; k < NBOX && ok; ++k)
    if (!h->blocks[k].empty())
      ok = h->hip_ok(hipMemcpyAsync(h->ws + h->o_blk[k], h->blocks[k].data(),
                                    sizeof(BoxBlock) * h->blocks[k].size(), hipMemcpyHostToDevice, s),
                     "upload block table");
  for (int k = 0; k < h->npshape; ++k)
    if (ok && !h->ptiles[k].empty())
      ok = h->hip_ok(hipMemcpyAsync(h->ws + h->o_ptiles[k], h->ptiles[k].data(),
                                    sizeof(TileDev) * h->ptiles[k].size(), hipMemcpyHostToDevice, s),
                   "upload predictor tile table");
  for (int k = 0; k < h->nshape && ok; ++k)
    if (!h->tiles[k].empty())
      ok = h->hip_ok(hipMemcpyAsync(h->ws + h->o_tiles[k], h->tiles[k].data(),
                                    sizeof(TileDev) * h->tiles[k].size(), hipMemcpyHostToDevice, s),
                     "upload tile table");
  for (int id = 0; id < mhd_bunch::NTAB && ok; ++id)
    if (!h->first[id].empty())
      ok = h->hip_ok(hipMemcpyAsync(h->ws + h->o_first[id], h->first[id].data(),
                                    sizeof(int32_t) * h->first[id].size(), hipMemcpyHostToDevice, s),
                     "upload table index");
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

int64_t mhd_bunch_adjoint_workspace_bytes(mhd_bunch* h, const int32_t* nbr_host) {
  if (!h) return -1;
  if (build_guard_map(h, nbr_host) != 0) return -1;
  size_t o = 0;
  h->a_ls = o;
  o = align256(o + (size_t)h->scratch_elems * h->prec);
  h->a_lu = o;
  o = align256(o + (size_t)h->state_elems * h->prec);
  h->a_row = o;
  o = align256(o + sizeof(int32_t) * std::max<size_t>(1, h->row.size()));
  h->a_colp = o;
  o = align256(o + sizeof(int32_t) * std::max<size_t>(1, h->colp.size()));
  h->a_colc = o;
  o = align256(o + sizeof(int32_t) * std::max<size_t>(1, h->colc.size()));
  h->a_bytes = o;
  return (int64_t)o;
}

mhd_status mhd_bunch_adjoint_bind(mhd_bunch* h, const int32_t* nbr_host, void* ws, hipStream_t s) {
  if (!h || !ws || ((uintptr_t)ws & 255)) return MHD_EINVAL;
  if (!h->bound) return MHD_ESTATE;
  if (mhd_bunch_adjoint_workspace_bytes(h, nbr_host) < 0) return MHD_EINVAL;
  h->aws = (char*)ws;
  h->adj_fold = nbr_host != nullptr;
  bool ok = true;
  if (h->adj_fold) {
    ok = h->hip_ok(hipMemcpyAsync(h->aws + h->a_row, h->row.data(), sizeof(int32_t) * h->row.size(),
                                  hipMemcpyHostToDevice, s), "upload guard map");
    if (ok && !h->colp.empty())
      ok = h->hip_ok(hipMemcpyAsync(h->aws + h->a_colp, h->colp.data(), sizeof(int32_t) * h->colp.size(),
                                    hipMemcpyHostToDevice, s), "upload guard map") &&
           h->hip_ok(hipMemcpyAsync(h->aws + h->a_colc, h->colc.data(), sizeof(int32_t) * h->colc.size(),
                                    hipMemcpyHostToDevice, s), "upload guard map");
    if (ok) ok = h->hip_ok(hipStreamSynchronize(s), "synchronise after upload");
  }
  if (!ok) return MHD_EDEVICE;
  h->adj_bound = true;
  return MHD_OK;
}

mhd_status mhd_bunch_adjoint(mhd_bunch* h, const void* U_in, const void* lam_out, void* lam_in,
                             const double* dt, const double* dx, hipStream_t s) {
  if (!h || !U_in || !lam_out || !lam_in || !dt || !dx || lam_in == lam_out) return MHD_EINVAL;
  if (!h->bound || !h->adj_bound) return MHD_ESTATE;
  return h->prec == 8
             ? launch_adjoint<double>(h, (const double*)U_in, (const double*)lam_out, (double*)lam_in, dt, dx, s)
             : launch_adjoint<float>(h, (const float*)U_in, (const float*)lam_out, (float*)lam_in, dt, dx, s);
}

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
  return h->prec == 8 ? launch_update<double>(h, (const double*)Uin, (double*)Uout, dt, dx, s,
                                              (double*)h->d_scratch())
                      : launch_update<float>(h, (const float*)Uin, (float*)Uout, dt, dx, s,
                                             (float*)h->d_scratch());
}

mhd_status mhd_bunch_update_cfl(mhd_bunch* h, const void* Uin, void* Uout, const double* dt,
                                const double* dx, const int32_t* nbr, double* dt_next,
                                hipStream_t s) {
  if (!h || !Uin || !Uout || !dt || !dx || !nbr || !dt_next || Uin == Uout ||
      dt_next == dt)
    return MHD_EINVAL;
  if (!h->bound) return MHD_ESTATE;
  const size_t bytes = (size_t)h->state_elems * h->prec;
  const char *a = (const char*)Uin, *b = (const char*)Uout;
  if (a < b + bytes && b < a + bytes) return MHD_EINVAL;
  hipEvent_t t0 = h->tic(s);
  hipLaunchKernelGGL(k_zero_u64, dim3((h->P + 255) / 256), dim3(256), 0, s, h->d_smax(), h->P);
  h->toc(s, MHD_KERNEL_CFL, t0);
  h->cfl_next = h->d_smax();
  h->cfl_nbr = nbr;
  const mhd_status st =
      h->prec == 8 ? launch_update<double>(h, (const double*)Uin, (double*)Uout, dt, dx, s,
                                           (double*)h->d_scratch())
                   : launch_update<float>(h, (const float*)Uin, (float*)Uout, dt, dx, s,
                                          (float*)h->d_scratch());
  h->cfl_next = nullptr;
  h->cfl_nbr = nullptr;
  if (st != MHD_OK) return st;
  t0 = h->tic(s);
  hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(BLK), 0, s, h->P,
                     (const unsigned long long*)h->d_smax(), h->cfl, dt_next, 1);
  h->toc(s, MHD_KERNEL_CFL, t0);
  return h->hip_ok(hipGetLastError(), "launch update with time step") ? MHD_OK : MHD_EDEVICE;
}

mhd_status mhd_bunch_update_static(mhd_bunch* h, const void* Uin, void* Uout, const double* dt,
                                   const double* dx, hipStream_t s) {
  if (!h || !Uin || !Uout || !dt || !dx || Uin == Uout) return MHD_EINVAL;
  if (!h->bound || !h->static_scratch) return MHD_ESTATE;
  const size_t bytes = (size_t)h->state_elems * h->prec;
  const char *a = (const char*)Uin, *b = (const char*)Uout;
  if (a < b + bytes && b < a + bytes) return MHD_EINVAL;
  const int64_t need = h->scratch_elems * (int64_t)h->prec;
  if (need > (int64_t)MHD_STATIC_SCRATCH_BYTES) {
    snprintf(h->last_error, sizeof(h->last_error),
             "update_static: one chunk needs %lld scratch bytes, the static scratch holds %lld "
             "(create the bunch with max_scratch_bytes <= %lld)",
             (long long)need, (long long)MHD_STATIC_SCRATCH_BYTES,
             (long long)MHD_STATIC_SCRATCH_BYTES);
    return MHD_EINVAL;
  }
  int dev = -1;
  if (!h->hip_ok(hipGetDevice(&dev), "current device")) return MHD_EDEVICE;
  if (dev != h->dev) {
    snprintf(h->last_error, sizeof(h->last_error),
             "update_static: current device %d is not the bound device %d", dev, h->dev);
    return MHD_EINVAL;
  }
  return h->prec == 8 ? launch_update<double>(h, (const double*)Uin, (double*)Uout, dt, dx, s,
                                              (double*)h->static_scratch)
                      : launch_update<float>(h, (const float*)Uin, (float*)Uout, dt, dx, s,
                                             (float*)h->static_scratch);
}

mhd_status mhd_bunch_lts_step(mhd_bunch* h, void* U_cur, void* U_new, void* U_prev, double* t,
                              double* t_prev, double* dt, const double* dt_fixed,
                              const double* dx, const int32_t* nbr, double t_end,
                              double dt_quantum, hipStream_t s) {
  if (!h || !U_cur || !U_prev || !t || !t_prev || !dt || !dx || !nbr) return MHD_EINVAL;
  if (!(t_end == t_end) || t == t_prev || dt == t || dt == t_prev) return MHD_EINVAL;
  if (dt_fixed && (dt_fixed == dt || dt_fixed == t || dt_fixed == t_prev)) return MHD_EINVAL;
  if (!(dt_quantum >= 0.0) || dt_quantum > 1e300) return MHD_EINVAL;
  if (!h->bound) return MHD_ESTATE;
  const size_t bytes = (size_t)h->state_elems * h->prec;
  const char* b[3] = {(const char*)U_cur, (const char*)U_prev, (const char*)U_new};
  for (int x = 0; x < 3; ++x)
    for (int y = x + 1; y < 3; ++y)
      if (b[x] && b[y] && b[x] < b[y] + bytes && b[y] < b[x] + bytes) return MHD_EINVAL;
  return h->prec == 8
             ? launch_lts_step<double>(h, (double*)U_cur, (double*)U_prev, t, t_prev, dt,
                                       dt_fixed, dx, nbr, t_end, dt_quantum, s)
             : launch_lts_step<float>(h, (float*)U_cur, (float*)U_prev, t, t_prev, dt, dt_fixed,
                                      dx, nbr, t_end, dt_quantum, s);
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
    return (st & 6) ? MHD_EINVAL : MHD_ENONPHYS;
  }
  return MHD_OK;
}

int32_t mhd_bunch_tile_count(const mhd_bunch* h) { return h ? NMODE * h->nshape : -1; }

int32_t mhd_bunch_tile_current(const mhd_bunch* h) { return h ? NMODE * h->shape + h->mode : -1; }

mhd_status mhd_bunch_tile_get(const mhd_bunch* h, int32_t idx, int32_t cfg[4]) {
  if (!h || !cfg || idx < 0 || idx >= NMODE * h->nshape) return MHD_EINVAL;
  const TileCand tc = h->shapes[idx / NMODE];
  cfg[0] = tc.x;
  cfg[1] = tc.y;
  cfg[2] = tc.z;
  cfg[3] = idx % NMODE;
  return MHD_OK;
}

mhd_status mhd_bunch_tile_set(mhd_bunch* h, int32_t idx) {
  if (!h || idx < 0 || idx >= NMODE * h->nshape) return MHD_EINVAL;
  h->shape = idx / NMODE;
  h->mode = idx % NMODE;
  return MHD_OK;
}

mhd_status mhd_bunch_set_predictor(mhd_bunch* h, int32_t mode) {
  if (!h || mode < 0 || mode > h->npshape) return MHD_EINVAL;
  h->fused = mode;
  return MHD_OK;
}

int32_t mhd_bunch_predictor(const mhd_bunch* h) { return h ? h->fused : -1; }

int32_t mhd_bunch_predictor_count(const mhd_bunch* h) { return h ? h->npshape + 1 : -1; }

mhd_status mhd_bunch_predictor_shape(const mhd_bunch* h, int32_t mode, int32_t* tile3) {
  if (!h || !tile3 || mode < 0 || mode > h->npshape) return MHD_EINVAL;
  if (mode == 0) {
    tile3[0] = tile3[1] = tile3[2] = 0;
  } else {
    tile3[0] = h->pshapes[mode - 1].x;
    tile3[1] = h->pshapes[mode - 1].y;
    tile3[2] = h->pshapes[mode - 1].z;
  }
  return MHD_OK;
}

mhd_status mhd_bunch_set_solver_split(mhd_bunch* h, int32_t split) {
  if (!h || split < 0 || split > 3) return MHD_EINVAL;
  h->split = split;
  return MHD_OK;
}

int32_t mhd_bunch_solver_split(const mhd_bunch* h) { return h ? h->split : -1; }

mhd_status mhd_bunch_autotune(mhd_bunch* h, const void* Uin, void* Uout, const double* dt,
                              const double* dx, int32_t reps, hipStream_t s, int32_t* best,
                              float* ms) {
  if (!h || !Uin || !Uout || !dt || !dx || reps < 1 || Uin == Uout) return MHD_EINVAL;
  if (!h->bound) return MHD_ESTATE;
  const int n = NMODE * h->nshape;
  const bool prof = h->prof;
  h->prof = false;
  hipEvent_t a = nullptr, b = nullptr;
  bool ok = h->hip_ok(hipEventCreate(&a), "autotune event") && h->hip_ok(hipEventCreate(&b), "autotune event");
  // mean time of `reps` updates after one warm-up, in the current configuration
  auto time_it = [&](float* t) {
    ok = ok && mhd_bunch_update(h, Uin, Uout, dt, dx, s) == MHD_OK;
    ok = ok && h->hip_ok(hipEventRecord(a, s), "autotune event");
    for (int r = 0; r < reps && ok; ++r) ok = mhd_bunch_update(h, Uin, Uout, dt, dx, s) == MHD_OK;
    ok = ok && h->hip_ok(hipEventRecord(b, s), "autotune event") &&
         h->hip_ok(hipEventSynchronize(b), "autotune sync") &&
         h->hip_ok(hipEventElapsedTime(t, a, b), "autotune timing");
    *t /= reps;
  };
  // tile shape x launch mode x solver form, jointly (the two-phase and edge-pass forms are
  // what let the larger tiles fit), then the predictor form with the winner
  const int shape0 = h->shape, mode0 = h->mode, split0 = h->split;
  int bi = 0, bsplit = 0;
  float bms = 0.0f;
  bool first = true;
  for (int k = 0; k < n && ok; ++k) {
    h->shape = k / NMODE;
    h->mode = k % NMODE;
    float kbest = 0.0f;
    for (int sp = 0; sp < (h->act == 7 ? 4 : 3) && ok; ++sp) {
      h->split = sp;
      float t = 0.0f;
      time_it(&t);
      if (!ok) break;
      if (sp == 0 || t < kbest) kbest = t;
      if (first || t < bms) {
        bi = k;
        bsplit = sp;
        bms = t;
        first = false;
      }
    }
    if (ms) ms[k] = kbest;
  }
  h->shape = bi / NMODE;
  h->mode = bi % NMODE;
  h->split = bsplit;
  const int f0 = h->fused;
  int fbest = 0;
  float fbms = 0.0f;
  for (int f = 0; f <= h->npshape && ok; ++f) {
    h->fused = f;
    float t = 0.0f;
    time_it(&t);
    if (f == 0 || t < fbms) {
      fbest = f;
      fbms = t;
    }
  }
  h->fused = ok ? fbest : f0;
  if (!ok) {  // a failed run leaves the configuration the caller had
    h->shape = shape0;
    h->mode = mode0;
    h->split = split0;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  h->prof = prof;
  if (best) *best = bi;
  return ok ? MHD_OK : MHD_EDEVICE;
}

mhd_status mhd_bunch_graph_capture(mhd_bunch* h, int32_t nsteps, void* U_a, void* U_b, double* dt,
                                   const double* dx, const int32_t* nbr, int32_t dt_mode,
                                   hipStream_t s) {
  (void)s;
  if (!h || nsteps < 1 || !U_a || !U_b || !dt || !dx || dt_mode < 0 || dt_mode > 2) return MHD_EINVAL;
  if (dt_mode == 1 && nbr) return MHD_EINVAL;  // neighbours at other times: use mhd_bunch_lts_step
  if (!h->bound) return MHD_ESTATE;
  const size_t bytes = (size_t)h->state_elems * h->prec;
  const char *pa = (const char*)U_a, *pb = (const char*)U_b;
  if (pa < pb + bytes && pb < pa + bytes) return MHD_EINVAL;
  h->drop_graph();
  // captured on a private stream: the caller's may be the null stream, which cannot be
  // captured; the graph is later launched on the caller's stream
  hipStream_t cs = nullptr;
  if (!h->hip_ok(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream"))
    return MHD_EDEVICE;
  const bool prof = h->prof;
  h->prof = false;
  mhd_status st = MHD_OK;
  if (!h->hip_ok(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture")) {
    st = MHD_EDEVICE;
  } else {
    for (int k = 0; k < nsteps && st == MHD_OK; ++k) {
      void* in = (k % 2 == 0) ? U_a : U_b;
      void* out = (k % 2 == 0) ? U_b : U_a;
      if (nbr) st = mhd_bunch_fill_guards(h, in, nbr, cs);
      if (st == MHD_OK && dt_mode) st = mhd_bunch_cfl(h, in, dx, dt, dt_mode == 2, cs);
      if (st == MHD_OK) st = mhd_bunch_update(h, in, out, dt, dx, cs);
    }
    hipGraph_t g = nullptr;
    const bool ended = h->hip_ok(hipStreamEndCapture(cs, &g), "end capture");
    if (st == MHD_OK && !ended) st = MHD_EDEVICE;
    if (st == MHD_OK) {
      h->graph = g;
      if (!h->hip_ok(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0), "instantiate graph")) {
        h->gexec = nullptr;
        st = MHD_EDEVICE;
      }
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  h->prof = prof;
  (void)hipStreamDestroy(cs);
  if (st != MHD_OK) h->drop_graph();
  return st;
}

mhd_status mhd_stream_create(mhd_stream** out, const mhd_bunch_desc* d, int32_t per_bunch,
                             int32_t slots) {
  if (!out || !d || !d->dims || d->n_patches < 1 || per_bunch < 1 || slots < 1 || slots > 8)
    return MHD_EINVAL;
  mhd_stream* S = new (std::nothrow) mhd_stream;
  if (!S) return MHD_ENOMEM;
  S->P = d->n_patches;
  S->prec = d->precision;
  S->slots = slots;
  size_t o = 0, scratch = 0;
  int64_t base = 0;
  for (int p = 0; p < d->n_patches; p += per_bunch) {
    mhd_bunch_desc sd = *d;
    sd.n_patches = std::min(per_bunch, d->n_patches - p);
    sd.dims = d->dims + 3 * p;
    mhd_bunch* h = nullptr;
    const mhd_status st = mhd_bunch_create(&h, &sd);
    if (st != MHD_OK) {
      delete S;
      return st;
    }
    S->sub.push_back(h);
    S->p0.push_back(p);
    S->base.push_back(base);
    base += h->state_elems;
    S->slot_elems = std::max(S->slot_elems, h->state_elems);
    scratch = std::max(scratch, (size_t)h->scratch_elems * h->prec);
    S->o_tab.push_back(o);
    o = align256(o + h->o_scratch);       // the tables only: the scratch is shared
  }
  S->p0.push_back(d->n_patches);
  S->base.push_back(base);
  S->o_scratch = o;
  o = align256(o + scratch);
  S->o_dt = o;
  o = align256(o + sizeof(double) * S->P);
  S->o_dx = o;
  o = align256(o + 3 * sizeof(double) * S->P);
  S->o_slot = o;
  o += (size_t)(2 * slots) * align256((size_t)S->slot_elems * S->prec);
  S->bytes = o;
  *out = S;
  return MHD_OK;
}

void mhd_stream_destroy(mhd_stream* S) { delete S; }

int64_t mhd_stream_device_bytes(const mhd_stream* S) { return S ? (int64_t)S->bytes : -1; }

int32_t mhd_stream_bunch_count(const mhd_stream* S) { return S ? (int32_t)S->sub.size() : -1; }

mhd_status mhd_stream_bind(mhd_stream* S, void* dev, hipStream_t s) {
  if (!S || !dev || ((uintptr_t)dev & 255)) return MHD_EINVAL;
  S->dev = (char*)dev;
  S->last_error[0] = 0;
  for (size_t j = 0; j < S->sub.size(); ++j) {
    mhd_bunch* h = S->sub[j];
    const mhd_status st = mhd_bunch_bind(h, S->dev + S->o_tab[j], s);
    if (st != MHD_OK) {
      snprintf(S->last_error, sizeof(S->last_error), "sub-bunch %zu: %s", j, h->last_error);
      return st;
    }
    h->scratch_ext = S->dev + S->o_scratch;
  }
  if (!S->st[0])
    for (int k = 0; k < 3; ++k)
      if (!S->ok(hipStreamCreateWithFlags(&S->st[k], hipStreamNonBlocking), "create stream"))
        return MHD_EDEVICE;
  if (S->ev.empty()) {
    S->ev.resize(3 * S->slots + 1, nullptr);
    for (hipEvent_t& e : S->ev)
      if (!S->ok(hipEventCreateWithFlags(&e, hipEventDisableTiming), "create event"))
        return MHD_EDEVICE;
  }
  S->bound = true;
  return MHD_OK;
}

mhd_status mhd_stream_configure(mhd_stream* S, int32_t tile, int32_t predictor, int32_t split) {
  if (!S) return MHD_EINVAL;
  for (mhd_bunch* h : S->sub) {
    mhd_status st = mhd_bunch_tile_set(h, tile);
    if (st == MHD_OK) st = mhd_bunch_set_predictor(h, predictor);
    if (st == MHD_OK) st = mhd_bunch_set_solver_split(h, split);
    if (st != MHD_OK) return st;
  }
  return MHD_OK;
}

mhd_status mhd_stream_update(mhd_stream* S, const void* Uin, void* Uout, const double* dt,
                             const double* dx, hipStream_t s) {
  if (!S || !Uin || !Uout || !dt || !dx || Uin == Uout) return MHD_EINVAL;
  if (!S->bound) return MHD_ESTATE;
  const size_t es = S->prec;
  const size_t total = (size_t)S->base.back() * es;
  const char *a = (const char*)Uin, *b = (const char*)Uout;
  if (a < b + total && b < a + total) return MHD_EINVAL;
  const int K = S->slots, nsub = (int)S->sub.size();
  hipEvent_t* ev_in = S->ev.data();
  hipEvent_t* ev_comp = ev_in + K;
  hipEvent_t* ev_out = ev_comp + K;
  hipEvent_t ev_start = ev_out[K];
  hipStream_t up = S->st[0], comp = S->st[1], down = S->st[2];
  double* ddt = (double*)(S->dev + S->o_dt);
  double* ddx = (double*)(S->dev + S->o_dx);
  bool ok = S->ok(hipEventRecord(ev_start, s), "record start");
  for (int k = 0; k < 3 && ok; ++k) ok = S->ok(hipStreamWaitEvent(S->st[k], ev_start, 0), "wait start");
  ok = ok && S->ok(hipMemcpyAsync(ddt, dt, sizeof(double) * S->P, hipMemcpyHostToDevice, up), "copy dt") &&
       S->ok(hipMemcpyAsync(ddx, dx, 3 * sizeof(double) * S->P, hipMemcpyHostToDevice, up), "copy dx");
  for (int j = 0; j < nsub && ok; ++j) {
    const int k = j % K;
    mhd_bunch* h = S->sub[j];
    const size_t off = (size_t)S->base[j] * es, nb = (size_t)h->state_elems * es;
    char* in = S->slot_in(k);
    char* outb = S->slot_out(k);
    // copy in: the slot's input is free once the update of sub-bunch j - K has read it
    if (j >= K) ok = S->ok(hipStreamWaitEvent(up, ev_comp[k], 0), "wait slot input");
    ok = ok && S->ok(hipMemcpyAsync(in, (const char*)Uin + off, nb, hipMemcpyHostToDevice, up), "copy in") &&
         S->ok(hipEventRecord(ev_in[k], up), "record input");
    // compute: its output is free once sub-bunch j - K has been copied out
    ok = ok && S->ok(hipStreamWaitEvent(comp, ev_in[k], 0), "wait input");
    if (j >= K) ok = ok && S->ok(hipStreamWaitEvent(comp, ev_out[k], 0), "wait slot output");
    // the output carries the input's guards (the update writes owned values only)
    ok = ok && S->ok(hipMemcpyAsync(outb, in, nb, hipMemcpyDeviceToDevice, comp), "copy guards");
    if (ok) {
      const mhd_status st = mhd_bunch_update(h, in, outb, ddt + S->p0[j], ddx + 3 * S->p0[j], comp);
      if (st != MHD_OK) {
        snprintf(S->last_error, sizeof(S->last_error), "update of sub-bunch %d: %s", j, h->last_error);
        return st;
      }
    }
    ok = ok && S->ok(hipEventRecord(ev_comp[k], comp), "record compute");
    // copy out
    ok = ok && S->ok(hipStreamWaitEvent(down, ev_comp[k], 0), "wait compute") &&
         S->ok(hipMemcpyAsync((char*)Uout + off, outb, nb, hipMemcpyDeviceToHost, down), "copy out") &&
         S->ok(hipEventRecord(ev_out[k], down), "record output");
  }
  // the caller's stream continues after every copy out
  for (int k = 0; k < std::min(K, nsub) && ok; ++k)
    ok = S->ok(hipStreamWaitEvent(s, ev_out[k], 0), "join");
  return ok ? MHD_OK : MHD_EDEVICE;
}

mhd_status mhd_stream_check(mhd_stream* S, hipStream_t s) {
  if (!S) return MHD_EINVAL;
  if (!S->bound) return MHD_ESTATE;
  mhd_status worst = MHD_OK;
  for (mhd_bunch* h : S->sub) {
    const mhd_status st = mhd_bunch_check(h, s);
    if (st != MHD_OK && worst == MHD_OK) worst = st;
  }
  return worst;
}

const char* mhd_stream_last_error(const mhd_stream* S) { return S ? S->last_error : "null handle"; }

mhd_status mhd_bunch_lts_graph_capture(mhd_bunch* h, int32_t nsteps, void* U_cur, void* U_new,
                                       void* U_prev, double* t, double* t_prev, double* dt,
                                       const double* dt_fixed, const double* dx,
                                       const int32_t* nbr, double t_end, double dt_quantum,
                                       hipStream_t s) {
  (void)s;
  if (!h || nsteps < 1) return MHD_EINVAL;
  if (!h->bound) return MHD_ESTATE;
  h->drop_graph();
  hipStream_t cs = nullptr;
  if (!h->hip_ok(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream"))
    return MHD_EDEVICE;
  const bool prof = h->prof;
  h->prof = false;
  mhd_status st = MHD_OK;
  if (!h->hip_ok(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture")) {
    st = MHD_EDEVICE;
  } else {
    for (int k = 0; k < nsteps && st == MHD_OK; ++k)
      st = mhd_bunch_lts_step(h, U_cur, U_new, U_prev, t, t_prev, dt, dt_fixed, dx, nbr, t_end,
                              dt_quantum, cs);
    hipGraph_t g = nullptr;
    const bool ended = h->hip_ok(hipStreamEndCapture(cs, &g), "end capture");
    if (st == MHD_OK && !ended) st = MHD_EDEVICE;
    if (st == MHD_OK) {
      h->graph = g;
      if (!h->hip_ok(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0), "instantiate graph")) {
        h->gexec = nullptr;
        st = MHD_EDEVICE;
      }
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  h->prof = prof;
  (void)hipStreamDestroy(cs);
  if (st != MHD_OK) h->drop_graph();
  return st;
}

mhd_status mhd_bunch_graph_launch(mhd_bunch* h, hipStream_t s) {
  if (!h) return MHD_EINVAL;
  if (!h->gexec) return MHD_ESTATE;
  return h->hip_ok(hipGraphLaunch(h->gexec, s), "graph launch") ? MHD_OK : MHD_EDEVICE;
}

}  // extern "C"
