// Host build of the device stage code: the adjoint gathers skip forward items that cannot read
// the seeded input.  Checked here on random states: every skipped (item, seed) pair has an
// exactly zero dual-number derivative, for faces and edges (both EMF solvers) against the
// predictor slots, and for the predictor, time-n EMF and primitive items against seeds in the
// primitives, edge EMFs and state -- so skipping them changes no sum.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>
using std::fabs;
using std::sqrt;
#define __host__
#define __device__
#define __forceinline__ inline __attribute__((always_inline))
#include "mhd_stages.hpp"
using namespace mhd;
typedef double T;
typedef Dual<T> D;

static int fails = 0, checked = 0, nonzero = 0;
static void expect_zero(bool skipped, T deriv, const char* what, int a, int b, int c) {
  ++checked;
  if (deriv != 0.0) ++nonzero;
  if (skipped && deriv != 0.0) {
    if (fails < 10) std::printf("  %s (%d, %d, %d): skipped but derivative %.3e\n", what, a, b, c, deriv);
    ++fails;
  }
}

int main() {
  const int n = 6, g = 3;
  PatchDev P = {};
  for (int d = 0; d < 3; ++d) { P.n[d] = n; P.N[d] = n + 2 * g; }
  P.act = 7;
  P.Nc = (int64_t)P.N[0] * P.N[1] * P.N[2];
  P.off[0] = 1; P.off[1] = P.N[0]; P.off[2] = (int64_t)P.N[0] * P.N[1];
  P.woff[0] = 1; P.woff[1] = n + 2; P.woff[2] = (int64_t)(n + 2) * (n + 2);
  P.Nwc = (int64_t)(n + 2) * (n + 2) * (n + 2);
  P.ubase = 0; P.sbase = 0; P.wbase = 11 * P.Nc;
  std::mt19937 rng(11);
  std::uniform_real_distribution<double> pos(0.5, 1.5), sym(-0.3, 0.3);
  std::vector<T> U(8 * P.Nc), S(11 * P.Nc + NW * P.Nwc);
  for (int m = 0; m < 8; ++m)
    for (int64_t c = 0; c < P.Nc; ++c) U[m * P.Nc + c] = (m == 0 || m == 4) ? pos(rng) + 2.0 : sym(rng);
  for (int m = 0; m < 11; ++m)
    for (int64_t c = 0; c < P.Nc; ++c) S[m * P.Nc + c] = (m == 0 || m == 4) ? pos(rng) : sym(rng);
  for (int v = 0; v < NW; ++v)
    for (int64_t c = 0; c < P.Nwc; ++c) S[P.wbase + v * P.Nwc + c] = (v == 0 || v == 4) ? pos(rng) : sym(rng);
  Consts<T> c0 = {};
  c0.gamma = 5.0 / 3.0; c0.gm1 = 2.0 / 3.0; c0.rho_floor = 1e-10; c0.p_floor = 1e-10;
  c0.tiny = 1e-30; c0.limiter = 1;
  const double dxp[3] = {0.1, 0.12, 0.15};
  const int x[3] = {g + 2, g + 3, g + 2};  // an interior cell
  const T* W = S.data() + P.wbase;

  // faces and edges against predictor slots
  for (int emf = 0; emf < 2; ++emf) {
    c0.emf = emf;
    const Consts<D> cd = lift<D>(c0);
    for (int v = 0; v < NW; ++v) {
      const int64_t seed = (int64_t)v * P.Nwc + wcell_of(P, g, x[0], x[1], x[2]);
      const LdSeed<T> acc{W, seed, P.Nwc};
      for (int d = 0; d < 3 && emf == 0; ++d)
        for (int s = 0; s < 2; ++s) {  // the faces on either side of x
          int f[3] = {x[0], x[1], x[2]};
          f[d] += s;
          D F[5];
          face_point(P, g, d, f[0], f[1], f[2], acc, cd, F);
          T sum = 0;
          for (int t = 0; t < 5; ++t) sum += fabs(F[t].d);
          expect_zero(!face_reads_slot(d, v), sum, "face d, s, slot", d, s, v);
        }
      for (int e = 0; e < 3; ++e) {
        const int a = (e + 1) % 3, b = (e + 2) % 3;
        for (int sb = 0; sb < 2; ++sb)
          for (int sa = 0; sa < 2; ++sa) {  // the four edges with x as a corner cell
            int y[3] = {x[0], x[1], x[2]};
            y[a] += sa;
            y[b] += sb;
            const D em = emf == 1 ? edge_point<1>(P, g, e, y[0], y[1], y[2], acc, cd)
                                  : edge_point<0>(P, g, e, y[0], y[1], y[2], acc, cd);
            expect_zero(!edge_reads_slot(e, v), fabs(em.d), "edge e, corner, slot", e, 2 * sb + sa, v);
          }
      }
    }
  }
  // predictor, time-n EMF and primitive items against seeds at x, over the 27 cells around x
  c0.emf = 0;
  const Consts<D> cd = lift<D>(c0);
  const int64_t cx = cell_of(P, x[0], x[1], x[2]);
  for (int kind = 0; kind < 3; ++kind)        // seed in: 0 primitives, 1 time-n EMFs, 2 state
    for (int m = 0; m < (kind == 1 ? 3 : 8); ++m) {
      const int64_t sq = kind == 0 ? P.sbase + m * P.Nc + cx : -1;
      const int64_t se = kind == 1 ? P.sbase + (8 + m) * P.Nc + cx : -1;
      const int64_t su = kind == 2 ? P.ubase + m * P.Nc + cx : -1;
      const LdSeed<T> q{S.data(), sq, 0}, e{S.data(), se, 0}, u{U.data(), su, 0};
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int o[3] = {dx, dy, dz};
            const int y[3] = {x[0] + dx, x[1] + dy, x[2] + dz};
            const int nz = (dx != 0) + (dy != 0) + (dz != 0);
            const bool neg = dx > 0 || dy > 0 || dz > 0;
            // predictor at y (what pred_gather visits: cross stencil, lower half for EMF seeds)
            D w[NW];
            pred_point(P, y[0], y[1], y[2], u, q, e, 1e-3, dxp, cd, w);
            T sw = 0;
            for (int v = 0; v < NW; ++v) sw += fabs(w[v].d);
            const bool pred_skip = nz > 1 || (kind == 1 && neg) || (kind == 2 && m < 5);
            expect_zero(pred_skip, sw, "predictor kind, m, offset", kind, m, dx + 3 * dy + 9 * dz);
            // time-n EMFs at y (en_gather visits {0, 1}^3 but (1, 1, 1))
            if (kind != 1) {
              D E[3];
              en_point(P, cell_of(P, y[0], y[1], y[2]), q, u, E);
              const T se3 = fabs(E[0].d) + fabs(E[1].d) + fabs(E[2].d);
              const bool en_skip = dx < 0 || dy < 0 || dz < 0 || nz == 3;
              expect_zero(en_skip, se3, "edge EMF kind, m, offset", kind, m, dx + 3 * dy + 9 * dz);
            }
            // primitives at y (adj_u visits y = x and x - e_d)
            if (kind == 2) {
              D qq[8];
              prim_point(P, cell_of(P, y[0], y[1], y[2]), u, cd, qq);
              T sp = 0;
              for (int t = 0; t < 8; ++t) sp += fabs(qq[t].d);
              const bool prim_skip = dx > 0 || dy > 0 || dz > 0 || nz > 1;
              expect_zero(prim_skip, sp, "primitive m, offset", m, o[0], o[1] + 3 * o[2]);
            }
          }
    }
  std::printf("%d (item, seed) pairs checked, %d with a nonzero derivative, %d skipped but nonzero\n",
              checked, nonzero, fails);
  std::printf(fails ? "FAIL\n" : "OK\n");
  return fails != 0;
}
