// Host build of the device stage code: the edge-line pass (solver form 3) against the
// per-tile owned-edge pass (solver form 2) on random predictor values, for ragged 3D patches,
// both EMF solvers and both precisions.  Every edge slot must be written by both passes,
// with the same bits (the two passes apply the same corner and UCT arithmetic to the same
// values; compiled with expression-level contraction, as the device code is).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>
using std::fabs;
using std::sqrt;
#define __host__
#define __device__
#define __forceinline__ inline __attribute__((always_inline))
#include "mhd_stages.hpp"
using namespace mhd;

struct SerialGroup {  // a work-group of one thread
  int tid() { return 0; }
  int nthr() { return 1; }
  void sync() {}
};

template <typename T, int EMF, int TX, int TY, int TZ>
int check(int nx, int ny, int nz, int g, unsigned seed) {
  PatchDev P = {};
  P.n[0] = nx; P.n[1] = ny; P.n[2] = nz;
  for (int d = 0; d < 3; ++d) P.N[d] = P.n[d] + 2 * g;
  P.act = 7;
  P.Nc = (int64_t)P.N[0] * P.N[1] * P.N[2];
  P.off[0] = 1; P.off[1] = P.N[0]; P.off[2] = (int64_t)P.N[0] * P.N[1];
  P.woff[0] = 1; P.woff[1] = nx + 2; P.woff[2] = (int64_t)(nx + 2) * (ny + 2);
  P.Nwc = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
  P.sbase = 0;
  P.wbase = 11 * P.Nc;
  std::vector<T> S(11 * P.Nc + NW * P.Nwc, T(0));
  std::mt19937 rng(seed);
  std::uniform_real_distribution<double> pos(0.2, 1.5), sym(-0.5, 0.5);
  for (int v = 0; v < NW; ++v)
    for (int64_t c = 0; c < P.Nwc; ++c) S[P.wbase + v * P.Nwc + c] = (T)(v == 0 || v == 4 ? pos(rng) : sym(rng));
  Consts<T> cs = {};
  cs.gamma = (T)(5.0 / 3.0); cs.gm1 = cs.gamma - T(1); cs.rho_floor = (T)1e-10; cs.p_floor = (T)1e-10;
  cs.tiny = (T)1e-30; cs.limiter = 1; cs.emf = EMF;
  for (int64_t i = 8 * P.Nc; i < 11 * P.Nc; ++i) S[i] = (T)NAN;
  std::vector<T> A = S, B = S;
  SerialGroup ex;
  const double dx[3] = {1.0, 1.0, 1.0};
  for (int z = 0; z < nz; z += TZ)
    for (int y = 0; y < ny; y += TY)
      for (int x = 0; x < nx; x += TX) {
        const TileDev tl = {0, x, y, z};
        solve_tile<T, TX, TY, TZ, 3, EMF>(ex, (T*)nullptr, P, g, tl, A.data(), A.data(), A.data(), 1.0, dx, cs);
      }
  for (int it = 0; it < edge_line_count(P); ++it) edge_line_item<EMF>(P, g, it, B.data(), cs);
  int bad = 0, written = 0;
  for (int64_t i = 8 * P.Nc; i < 11 * P.Nc; ++i) {
    const bool na = std::isnan((double)A[i]), nb = std::isnan((double)B[i]);
    written += !na;
    if (na != nb || (!na && std::memcmp(&A[i], &B[i], sizeof(T)) != 0)) ++bad;
  }
  const int expect = nx * (ny + 1) * (nz + 1) + (nx + 1) * ny * (nz + 1) + (nx + 1) * (ny + 1) * nz;
  std::printf("%s EMF=%d n=(%d,%d,%d) g=%d tile=(%d,%d,%d): %d edges (expected %d), %d differ\n",
              sizeof(T) == 8 ? "f64" : "f32", EMF, nx, ny, nz, g, TX, TY, TZ, written, expect, bad);
  return bad + (written != expect);
}

int main() {
  int bad = 0;
  bad += check<double, 0, 4, 2, 2>(8, 6, 4, 3, 1);
  bad += check<double, 1, 4, 2, 2>(8, 6, 4, 3, 2);
  bad += check<float, 0, 4, 2, 2>(7, 5, 3, 2, 3);
  bad += check<float, 1, 8, 4, 2>(9, 4, 6, 3, 4);
  bad += check<double, 0, 8, 4, 2>(13, 3, 5, 2, 5);
  bad += check<double, 1, 4, 2, 2>(1, 1, 1, 3, 6);
  std::printf(bad ? "FAIL\n" : "OK\n");
  return bad != 0;
}
