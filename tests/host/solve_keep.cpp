// Host build of the device stage code: the solver tile of a local time step (KEEP: in place,
// the cell's state before the update written to a previous-slice buffer) against the
// ordinary out-of-place tile, for solver forms 0, 1 and 2 (form 2 after the form-3 edge pass),
// ragged 3D patches, both EMF solvers and both precisions.  The in-place state must equal the
// out-of-place result bit for bit on every owned cell and face, the previous slice must hold
// the input's owned values exactly, and no guard value of either buffer may change.
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

template <typename T>
bool same(T a, T b) { return std::memcmp(&a, &b, sizeof(T)) == 0; }

template <typename T, int FORM, int EMF, int TX, int TY, int TZ>
int check(int nx, int ny, int nz, int g, unsigned seed) {
  PatchDev P = {};
  P.n[0] = nx; P.n[1] = ny; P.n[2] = nz;
  for (int d = 0; d < 3; ++d) P.N[d] = P.n[d] + 2 * g;
  P.act = 7;
  P.Nc = (int64_t)P.N[0] * P.N[1] * P.N[2];
  P.off[0] = 1; P.off[1] = P.N[0]; P.off[2] = (int64_t)P.N[0] * P.N[1];
  P.woff[0] = 1; P.woff[1] = nx + 2; P.woff[2] = (int64_t)(nx + 2) * (ny + 2);
  P.Nwc = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
  P.ubase = 0;
  P.sbase = 0;
  P.wbase = 11 * P.Nc;
  std::vector<T> S(11 * P.Nc + NW * P.Nwc, T(0)), U(8 * P.Nc);
  std::mt19937 rng(seed);
  std::uniform_real_distribution<double> pos(0.2, 1.5), sym(-0.5, 0.5);
  for (int v = 0; v < NW; ++v)
    for (int64_t c = 0; c < P.Nwc; ++c) S[P.wbase + v * P.Nwc + c] = (T)(v == 0 || v == 4 ? pos(rng) : sym(rng));
  for (auto& u : U) u = (T)pos(rng);
  Consts<T> cs = {};
  cs.gamma = (T)(5.0 / 3.0); cs.gm1 = cs.gamma - T(1); cs.rho_floor = (T)1e-10; cs.p_floor = (T)1e-10;
  cs.tiny = (T)1e-30; cs.limiter = 1; cs.emf = EMF;
  SerialGroup ex;
  const double dx[3] = {0.5, 0.7, 0.9};
  const double dt = 0.05;
  std::vector<T> lds(TileShape<TX, TY, TZ>::template Lds<FORM>::value > 0
                         ? TileShape<TX, TY, TZ>::template Lds<FORM>::value : 1);
  if (FORM == 2)  // the edge EMFs the faces tile reads: the form-3 pass writes them
    for (int z = 0; z < nz; z += TZ)
      for (int y = 0; y < ny; y += TY)
        for (int x = 0; x < nx; x += TX) {
          const TileDev tl = {0, x, y, z};
          solve_tile<T, TX, TY, TZ, 3, EMF>(ex, (T*)nullptr, P, g, tl, S.data(), S.data(), S.data(), 1.0, dx, cs);
        }
  std::vector<T> out(U.size(), (T)NAN), inplace = U, prev(U.size(), (T)NAN);
  for (int z = 0; z < nz; z += TZ)
    for (int y = 0; y < ny; y += TY)
      for (int x = 0; x < nx; x += TX) {
        const TileDev tl = {0, x, y, z};
        solve_tile<T, TX, TY, TZ, FORM, EMF>(ex, lds.data(), P, g, tl, U.data(), out.data(), S.data(), dt, dx, cs);
        solve_tile<T, TX, TY, TZ, FORM, EMF, true>(ex, lds.data(), P, g, tl, inplace.data(), inplace.data(),
                                                   S.data(), dt, dx, cs, nullptr, 0, prev.data());
      }
  int bad = 0, owned = 0, changed = 0;
  for (int m = 0; m < 8; ++m)
    for (int k = 0; k < P.N[2]; ++k)
      for (int j = 0; j < P.N[1]; ++j)
        for (int i = 0; i < P.N[0]; ++i) {
          const int64_t e = m * P.Nc + cell_of(P, i, j, k);
          const bool own = i >= g && i < g + nx && j >= g && j < g + ny && k >= g && k < g + nz;
          if (own) {
            ++owned;
            changed += !same(inplace[e], U[e]);
            bad += !same(inplace[e], out[e]) || !same(prev[e], U[e]);
          } else {
            bad += !same(inplace[e], U[e]) || !std::isnan((double)prev[e]);
          }
        }
  std::printf("%s form %d EMF=%d n=(%d,%d,%d) g=%d tile=(%d,%d,%d): %d owned values, %d changed by "
              "the update, %d differ\n", sizeof(T) == 8 ? "f64" : "f32", FORM, EMF, nx, ny, nz, g, TX,
              TY, TZ, owned, changed, bad);
  return bad + (changed < owned / 2);
}

int main() {
  int bad = 0;
  bad += check<double, 0, 0, 4, 2, 2>(8, 6, 4, 3, 1);
  bad += check<double, 1, 1, 4, 2, 2>(7, 5, 3, 3, 2);
  bad += check<double, 2, 0, 8, 4, 2>(13, 3, 5, 2, 3);
  bad += check<double, 2, 1, 4, 2, 2>(5, 6, 7, 3, 4);
  bad += check<float, 0, 1, 8, 4, 2>(9, 4, 6, 3, 5);
  bad += check<float, 2, 0, 4, 2, 2>(7, 5, 3, 2, 6);
  std::printf(bad ? "FAIL\n" : "OK\n");
  return bad != 0;
}
