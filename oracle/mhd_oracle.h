/*
 * mhd_oracle.h -- C interface of the FP64 CPU oracle for the ideal-MHD patch update.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product library
 * (include/mhd_bunch.h) never links or calls it, and the two share no source.
 *
 * Data layout (one patch): 8 fields, field-major, each a padded box Nx*Ny*Nz with x
 * fastest.  N_d = n_d + 2g for an active direction (n_d > 1), N_d = 1 for a collapsed
 * one.  Field order rho, rho*u, rho*v, rho*w, E, Bx, By, Bz (state vector of the
 * paper's conservative system, eq:MHD_vector).  Bx[i] is the face-centred value on the
 * lower x face (i - 1/2) of cell i, likewise By, Bz (staggering of Fig. 2).
 *
 * Return codes: 0 ok, -1 invalid argument.  Nothing here allocates device memory.
 */
#ifndef MHD_ORACLE_H
#define MHD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double gamma;      /* adiabatic index */
  double cfl;        /* Courant number C of the time-step rule */
  double rho_floor;  /* density floor applied to every reconstructed state */
  double p_floor;    /* pressure floor applied to every reconstructed state */
  double eps_deg;    /* relative threshold of the HLLD degeneracy switch */
  int32_t limiter;   /* 0 = monotonised central (MC), 1 = minmod */
  int32_t emf_solver; /* edge EMF: 0 = UCT-HLL, 1 = UCT-HLLD (four-state compositions) */
} mhd_oracle_params;

/* Threads the multi-patch entry points use (OpenMP over patches). */
int mhd_oracle_threads(void);
/* Sets the OpenMP thread count of the multi-patch entry points (n >= 1). */
void mhd_oracle_set_threads(int n);

/* One update of one patch: U_out interior <- U_in advanced by dt.  Guards of U_out are a
 * copy of U_in's.  nfloor (may be NULL) is int64_t[3] and accumulates floor activations
 * in cell primitives, face states and edge-corner states.  g >= 3. */
int mhd_oracle_step(const int32_t n[3], int32_t g, const double* U_in, double* U_out,
                    double dt, const double dx[3], const mhd_oracle_params* prm,
                    int64_t* nfloor);

/* Same as mhd_oracle_step for many patches (OpenMP over patches).  dims[P][3],
 * patch p starts at element offset 8*sum_{q<p} Nc(q); dt[P], dx[P][3]. */
int mhd_oracle_step_many(int32_t npatch, const int32_t* dims, int32_t g, const double* U_in,
                         double* U_out, const double* dt, const double* dx,
                         const mhd_oracle_params* prm, int64_t* nfloor);

/* Time step of one patch: C * min over interior cells of 1 / sum_d (|u_d| + c_f,d)/dx_d. */
double mhd_oracle_cfl(const int32_t n[3], int32_t g, const double* U, const double dx[3],
                      const mhd_oracle_params* prm);
int mhd_oracle_cfl_many(int32_t npatch, const int32_t* dims, int32_t g, const double* U,
                        const double* dx, const mhd_oracle_params* prm, double* dt_out);

/* Guard fill from a 27-entry neighbour table per patch (entry (ox+1)+3(oy+1)+9(oz+1),
 * -1 = domain boundary with zero-gradient outflow).  Neighbours share interior dims. */
int mhd_oracle_fill_guards(int32_t npatch, const int32_t* dims, int32_t g, double* U,
                           const int32_t* nbr);

/* Forward-mode derivative of one patch update at fixed dt (dual numbers):
 * dU_out = (d U_out / d U_in) . dU_in. */
int mhd_oracle_step_jvp(const int32_t n[3], int32_t g, const double* U_in, const double* dU_in,
                        double* U_out, double* dU_out, double dt, const double dx[3],
                        const mhd_oracle_params* prm);
int mhd_oracle_step_jvp_many(int32_t npatch, const int32_t* dims, int32_t g,
                             const double* U_in, const double* dU_in, double* U_out,
                             double* dU_out, const double* dt, const double* dx,
                             const mhd_oracle_params* prm);

/* Same result as mhd_oracle_step (bitwise), plus a branch signature: a 64-bit hash of
 * the outcome of every comparison the update makes (limiter cases, min/max/|.| choices,
 * HLLD regions and degeneracy switch, floors), in program order.  Two inputs with equal
 * signatures took the same branch of the piecewise-smooth update (up to hash collisions).
 * sig is uint64_t[1], resp. uint64_t[P] for the multi-patch form. */
int mhd_oracle_step_sig(const int32_t n[3], int32_t g, const double* U_in, double* U_out,
                        double dt, const double dx[3], const mhd_oracle_params* prm,
                        uint64_t* sig);
int mhd_oracle_step_sig_many(int32_t npatch, const int32_t* dims, int32_t g,
                             const double* U_in, double* U_out, const double* dt,
                             const double* dx, const mhd_oracle_params* prm, uint64_t* sig);

/* The update and the guard fill in x87 extended precision (long double, 64-bit
 * significand), with the branch signature as above (sig may be NULL).  The scheme,
 * parameters, dt and dx are the FP64 ones; only the rounding of the state arithmetic is
 * finer.  For finite differences whose step must be smaller than FP64 round-off allows. */
int mhd_oracle_step_ext_many(int32_t npatch, const int32_t* dims, int32_t g,
                             const long double* U_in, long double* U_out, const double* dt,
                             const double* dx, const mhd_oracle_params* prm, uint64_t* sig);
int mhd_oracle_fill_guards_ext(int32_t npatch, const int32_t* dims, int32_t g, long double* U,
                               const int32_t* nbr);

/* Guard fill at each patch's own time t[p] from two time slices of the owners: the owner q's
 * value linearly interpolated between (t_prev[q], U_prev) and (t[q], U); its current value
 * when t[q] == t_prev[q].  Patches with mask[p] == 0 are skipped (mask NULL: all). */
int mhd_oracle_fill_guards_at(int32_t npatch, const int32_t* dims, int32_t g, double* U,
                              const double* U_prev, const double* t, const double* t_prev,
                              const int32_t* nbr, const int32_t* mask);

/* Arithmetic performed by one patch update, counted by class:
 * counts[0] add/sub, [1] mul, [2] div, [3] sqrt, [4] compare/min/max/abs. */
int mhd_oracle_count_ops(const int32_t n[3], int32_t g, const double* U_in, double dt,
                         const double dx[3], const mhd_oracle_params* prm, int64_t counts[5]);

/* Algorithmic arithmetic per interior cell-update, without halo recomputation: each
 * pass of the update over a box (cells, faces of one direction, edges of one direction)
 * contributes its operations per item, since an interior cell owns one item of every
 * pass.  out[5] by class as in mhd_oracle_count_ops. */
int mhd_oracle_ops_per_cell(const int32_t n[3], int32_t g, const double* U_in, double dt,
                            const double dx[3], const mhd_oracle_params* prm, double out[5]);

/* ---- single-building-block entry points (for pinning the pieces one by one) ---- */

/* HLLD flux through one face.  L, R: (rho, u_n, u_t1, u_t2, p, B_n, B_t1, B_t2); the
 * normal field is taken from L.  F: (rho, m_n, m_t1, m_t2, E).  region (may be NULL):
 * 0 F_L, 1 F*_L, 2 F**_L, 3 F**_R, 4 F*_R, 5 F_R. */
void mhd_oracle_hlld(const double L[8], const double R[8], const mhd_oracle_params* prm,
                     double F[5], int32_t* region);

/* The same flux with the wave fan it was built from: speeds[6] = (S_L, S*_L, S_M, S*_R,
 * S_R, total pressure of the intermediate states) and states[4] = U*_L, U**_L, U**_R, U*_R,
 * each (rho, m_n, m_t1, m_t2, E, B_n, B_t1, B_t2) in the face frame.  For checks of the
 * jump conditions across every wave. */
void mhd_oracle_hlld_fan(const double L[8], const double R[8], const mhd_oracle_params* prm,
                         double F[5], int32_t* region, double speeds[6], double states[4][8]);

/* Fast magnetosonic speed along a direction with normal field bn. */
double mhd_oracle_cfast(double rho, double p, double bn, double bt1, double bt2, double gamma);

/* Slope limiter applied to backward/forward differences. */
double mhd_oracle_limiter(double dl, double dr, int32_t limiter);

/* Edge EMF (z component) from the four corner states around a z edge, each given as
 * (rho, u, v, w, p, Bx, By, Bz) in the order SW, SE, NW, NE; solver per prm->emf_solver. */
double mhd_oracle_uct(const double W[4][8], const mhd_oracle_params* prm);

/* Primitive-variable time derivative used by the half-step predictor.
 * q: (rho,u,v,w,p,Bx,By,Bz); D[d][m]: spatial derivative of q_m along d; act[d] != 0 for
 * active directions.  Output dqdt[8]. */
void mhd_oracle_dqdt(const double q[8], const double D[3][8], const int32_t act[3],
                     double gamma, double dqdt[8]);

#ifdef __cplusplus
}
#endif
#endif
