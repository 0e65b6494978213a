/*
 * mhd_bunch.h -- C ABI of the MI355X (gfx950) ideal-MHD bunch update.
 *
 * A "bunch" is a set of guard-zoned patches updated together (the paper's §2.3
 * "HLLD Mockup" and §2.4 "DISPATCH Integration": patches ready for update are gathered
 * into a work array and updated collectively to amortise launch overhead).  One call
 * of mhd_bunch_update advances the 8 conserved fields (rho, rho u, E, face-centred B)
 * of every patch by its own time step: unsplit MUSCL-Hancock prediction in primitive
 * variables (§2.1 "The MUSCL Scheme"), HLLD face fluxes (§2.1 "HLLD Solver", Fig. 1),
 * edge EMFs from four predicted corner states and constrained transport
 * (§2.1 "Constrained transport and 2D-extension", eq:EMF_to_B, Fig. 2-3).
 *
 * Conventions
 *  - Memory: every device buffer (state, workspace, dt/dx arrays, neighbour table) is
 *    allocated and owned by the caller; the library never frees caller memory.  Its own
 *    allocations are the host-side handle and, after mhd_bunch_graph_capture, a HIP graph.
 *  - Streams: all work is enqueued on the caller's stream; calls return without
 *    synchronising, except mhd_bunch_check.
 *  - Errors: status codes only.  Argument errors are detected before any launch.
 *    Non-physical input states (rho <= 0, p <= 0 or non-finite) set a device status
 *    word that mhd_bunch_check reports.
 *  - State layout: patch p occupies elements [base_p, base_p + 8*Nc_p) of the state
 *    buffer, base_p = sum_{q<p} 8*Nc_q.  Inside a patch: 8 fields, field-major, each a
 *    padded box Nx*Ny*Nz with x fastest, N_d = n_d + 2g for an active direction
 *    (n_d > 1) and N_d = 1 for a collapsed one.  Field order rho, rho u, rho v, rho w,
 *    E, Bx, By, Bz (state vector of eq:MHD_vector).  B_d[i] is the value on the lower
 *    d-face of cell i (Fig. 2); a patch owns cells and lower faces [g, g+n).
 *  - Element type: double (precision 8) or float (precision 4).  dt and dx are always
 *    double device arrays: dt[P], dx[P][3] (per-patch time step and per-direction cell
 *    size, §2.2: each patch carries its own time step; §2.3: spacing per direction).
 */
#ifndef MHD_BUNCH_H
#define MHD_BUNCH_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mhd_bunch mhd_bunch; /* opaque; not thread-safe */

typedef enum {
  MHD_OK = 0,
  MHD_EINVAL = -1,        /* invalid argument (nothing was launched) */
  MHD_ENOMEM = -2,        /* host allocation failed */
  MHD_EDEVICE = -3,       /* a HIP call failed */
  MHD_ESTATE = -4,        /* call out of order (e.g. update before bind) */
  MHD_ENONPHYS = -5,      /* a non-physical state was met on the device */
  MHD_EUNSUPPORTED = -6   /* valid but not supported by this build */
} mhd_status;

typedef struct {
  int32_t n_patches;      /* number of patches, >= 1 */
  const int32_t* dims;    /* host array [n_patches][3]: interior cells, 1 = collapsed */
  int32_t guard;          /* guard width g >= 3 (the stencil reaches 2 cells down, 3 faces
                             up); the paper's patches use 3 (24^3 active, 30^3 total) */
  int32_t precision;      /* 4 = float, 8 = double */
  double gamma;           /* adiabatic index */
  double cfl;             /* Courant number of mhd_bunch_cfl */
  int32_t limiter;        /* 0 = monotonised central, 1 = minmod */
  double rho_floor;       /* floors applied to every reconstructed state */
  double p_floor;
  double eps_deg;         /* relative threshold of the HLLD degeneracy switch */
  int64_t max_scratch_bytes; /* cap of the per-call scratch (patches are processed in
                                chunks that fit); 0 = no cap */
  int32_t emf_solver;     /* edge EMF from the four predicted corner states (§2.1 "Constrained
                             transport and 2D-extension of the HLLD solver", Fig. 3):
                             0 = UCT-HLL (two composed one-dimensional HLL fluxes, outer
                             speeds bounded over the four states);
                             1 = UCT-HLLD (the four one-dimensional HLLD problems of the rows
                             and columns; reduces to the HLLD flux of the transverse field
                             for data varying along one direction) */
} mhd_bunch_desc;

/* Validates the description and builds the host-side patch and launch tables.  No
 * device memory is touched.  *out receives a handle to free with mhd_bunch_destroy.
 * MHD_EUNSUPPORTED for patches of different dimensionality, and for a patch whose scratch
 * of one update (11 (n+2g)^D + 38 (n+2)^D values, D active directions) exceeds 4 GiB: the
 * kernels address it by 32-bit offsets (g = 3: up to 219^3 cells in double and 276^3 in
 * float in 3D, 3307^2 in double in 2D). */
mhd_status mhd_bunch_create(mhd_bunch** out, const mhd_bunch_desc* desc);
void mhd_bunch_destroy(mhd_bunch* h);

/* Element count and byte size of one state buffer (all patches, guards included). */
int64_t mhd_bunch_state_elems(const mhd_bunch* h);
int64_t mhd_bunch_state_bytes(const mhd_bunch* h);
/* Element offset of patch p inside a state buffer, or -1 if p is out of range. */
int64_t mhd_bunch_patch_offset(const mhd_bunch* h, int32_t p);

/* Bytes of device workspace the caller must provide to mhd_bunch_bind (patch and launch
 * tables, CFL reduction slots, status word, and the scratch of one chunk of patches). */
int64_t mhd_bunch_workspace_bytes(const mhd_bunch* h);

/* Attaches a caller-owned device workspace (>= workspace_bytes, 256-byte aligned) and
 * uploads the tables on `stream`.  Must precede every call below. */
mhd_status mhd_bunch_bind(mhd_bunch* h, void* workspace_dev, hipStream_t stream);

/* Copies one patch (8 fields of the padded box, layout above, same element type) from
 * src into the state buffer U_dev, or out of it into dst.  src/dst may be host or
 * device memory (flag).  Asynchronous on `stream`; host memory must stay valid until
 * the stream reaches the copy. */
mhd_status mhd_bunch_load(mhd_bunch* h, void* U_dev, int32_t patch, const void* src,
                          int32_t src_is_device, hipStream_t stream);
mhd_status mhd_bunch_store(const mhd_bunch* h, const void* U_dev, int32_t patch, void* dst,
                           int32_t dst_is_device, hipStream_t stream);

/* Fills the guard zones of every patch in place from a device neighbour table
 * nbr_dev[P][27] (entry (ox+1) + 3(oy+1) + 9(oz+1) = id of the patch at that offset,
 * -1 = domain boundary: zero-gradient copy of the nearest owned value).  Patches that
 * are neighbours must have equal interior dims. */
mhd_status mhd_bunch_fill_guards(mhd_bunch* h, void* U_dev, const int32_t* nbr_dev,
                                 hipStream_t stream);

/* Time step per patch: dt[p] = cfl * min over its interior cells of
 * 1 / sum_{active d} (|u_d| + c_f,d) / dx_d, with c_f,d the fast magnetosonic speed
 * along d.  global != 0 writes the minimum over all patches into every dt[p]. */
mhd_status mhd_bunch_cfl(mhd_bunch* h, const void* U_dev, const double* dx_dev,
                         double* dt_dev, int32_t global, hipStream_t stream);

/* One step of local time stepping (§2.2 "DISPATCH": every patch carries time slices and
 * advances with its own time step; §3.1 "DISPATCH Validation": guard zones are interpolated
 * between asynchronous patch times).  Device arrays: two state buffers (U_cur at times
 * t[p], U_prev at t_prev[p]; U_new is not accessed and may be NULL: the update runs in place),
 * t[P], t_prev[P], dt[P] (written), dt_fixed[P] or NULL,
 * dx[P][3], nbr[P][27] as for mhd_bunch_fill_guards.  On the stream, in order:
 *  1. ready[p] = t[p] < t_end and no neighbour q (any of the 26 entries) has t[q] < t[p];
 *  2. the guards of every ready patch p in U_cur are filled at its time t[p]: the owner q's
 *     value (1 - th) U_prev + th U_cur with th = (t[p] - t_prev[q]) / (t[q] - t_prev[q]),
 *     or its U_cur value when t[q] == t_prev[q] (weight and blend in double, then rounded);
 *  3. dt[p] = ready ? min(d, t_end - t[p]) : 0 with d = dt_fixed ? dt_fixed[p] : the patch's
 *     own CFL step, rounded down to dt_quantum x 2^k (k any integer) when dt_quantum > 0 (time
 *     levels: patches then advance in lock-step groups, fewer steps per run; take a power
 *     of two, so that the times of a level are exact sums);
 *  4. the ready patches are updated in place: U_prev's owned cells and faces <- U_cur's,
 *     U_cur's owned cells and faces <- their update (patches at rest are neither computed
 *     nor written; U_prev's guard cells are never written: the guard fill reads owned
 *     values only);
 *  5. for every ready patch: t_prev[p] = t[p], t[p] += dt[p] (exactly t_end when the step
 *     was clipped to it).
 * With free steps (dt_quantum == 0) and a bunch processed in one chunk (no scratch cap) the
 * launches of steps 2-4 run over device-compacted tables of the ready patches' entries
 * (persistent grids), so a step costs in proportion to the patches that advance; with time
 * levels (most patches advance together) they run over the full tables.
 * A ready patch whose step (given or its own CFL step) is not finite and > 0 gets dt[p] = 0,
 * stays where it is and raises a status bit that mhd_bunch_check reports as MHD_EINVAL.
 * On return U_cur holds every patch at its time t[p] (no buffers to swap).  Start with
 * t = t_prev (one slice per patch) and U_prev any buffer of the right size.  The run is over
 * when every t[p] == t_end.  The state
 * buffers (U_new if given) must not overlap, t, t_prev, dt and dt_fixed must be distinct, dt_fixed must
 * hold finite steps > 0 and dt_quantum must be finite and >= 0 (MHD_EINVAL).  Only kernels are enqueued (no host synchronisation, no
 * memset or copy calls). */
mhd_status mhd_bunch_lts_step(mhd_bunch* h, void* U_cur, void* U_new, void* U_prev, double* t_dev,
                              double* t_prev_dev, double* dt_dev, const double* dt_fixed_dev,
                              const double* dx_dev, const int32_t* nbr_dev, double t_end,
                              double dt_quantum, hipStream_t stream);

/* One update of every patch: U_out owned cells and faces <- U_in advanced by dt[p].
 * U_in guards must be filled; U_out guards are not written.  U_in and U_out must not
 * overlap.  A patch with dt[p] == 0 (at rest in a local-time-stepping run) is copied
 * without computing anything (its guards are not read and its state is not checked). */
mhd_status mhd_bunch_update(mhd_bunch* h, const void* U_in, void* U_out, const double* dt_dev,
                            const double* dx_dev, hipStream_t stream);

/* The update followed by the next step's time step, reduced in the update's own tiles
 * (§2.2: each patch carries its own time step; the time-step rule of mhd_bunch_cfl): the same
 * U_out as mhd_bunch_update, and dt_next[p] = the minimum over all patches of the time step
 * that mhd_bunch_cfl(global != 0) computes on U_out after mhd_bunch_fill_guards(U_out, nbr).
 * For the cell-centred field of a patch's last cells the update uses the upper faces as that
 * exchange will leave them: at a face shared with a neighbour, the value the neighbour's update
 * writes there, which the tile computes from the same edge EMFs (so dt must be the same for
 * neighbouring patches, as in a globally stepped run); at a domain boundary (nbr entry -1), the
 * last owned face.  Patches with dt[p] == 0 contribute nothing.  dt_next must not alias dt.
 * Saves the separate time-step pass over the state. */
mhd_status mhd_bunch_update_cfl(mhd_bunch* h, const void* U_in, void* U_out, const double* dt_dev,
                                const double* dx_dev, const int32_t* nbr_dev, double* dt_next_dev,
                                hipStream_t stream);

/* ---- allocation-free update ----
 * For callers that cannot allocate device memory around the update (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same result, argument
 * meaning and errors as mhd_bunch_update (same kernels), but the predictor scratch of the
 * update is a static device array of MHD_STATIC_SCRATCH_BYTES inside the library instead of
 * the bound workspace's scratch; the call allocates and frees nothing.  Each device the
 * library runs on holds one such array until the process ends; its address is resolved by
 * mhd_bunch_bind on the device current there, and the call must be made with that device
 * current (else MHD_EINVAL).  Patches are processed in the handle's chunks: the bunch must
 * have been created with max_scratch_bytes in (0, MHD_STATIC_SCRATCH_BYTES] or have a whole
 * scratch that fits, else MHD_EINVAL (mhd_bunch_last_error gives the sizes).  Every call on a
 * device shares that device's array: calls that overlap in time on one device (other
 * streams, other handles, other threads) race and give wrong results; calls in one stream
 * order are safe.  Nothing in the array needs clearing between calls (every value read in a
 * call is written earlier in that call). */
#define MHD_STATIC_SCRATCH_BYTES (128ll << 20)
mhd_status mhd_bunch_update_static(mhd_bunch* h, const void* U_in, void* U_out,
                                   const double* dt_dev, const double* dx_dev, hipStream_t stream);

/* ---- adjoint of one update (reverse mode at fixed dt) ----
 * The step map is U^{n+1}(owned) = update(fill_guards(U^n)).  mhd_bunch_adjoint returns
 * lam_in = (d U^{n+1} / d U^n)^T lam_out: lam_out holds dL/dU^{n+1} on owned cells and faces
 * (its guard entries are ignored); lam_in receives dL/dU^n on owned entries and zero in the
 * guards, the guard copies' adjoints having been added to their owners.  U_in must be U^n
 * with guards filled (the update's input).  Every adjoint element is a deterministic gather
 * over the forward items that read the corresponding input, differentiated in dual numbers.
 *
 * nbr_host: the host copy of the neighbour table used by mhd_bunch_fill_guards ([P][27]),
 * or NULL when guards are frozen inputs (then guard entries of lam_in are their own
 * adjoints and nothing is folded).  mhd_bunch_adjoint_workspace_bytes builds the
 * owner -> guard-copies map on the host and returns the device bytes that
 * mhd_bunch_adjoint_bind needs (caller-owned, 256-byte aligned). */
int64_t mhd_bunch_adjoint_workspace_bytes(mhd_bunch* h, const int32_t* nbr_host);
mhd_status mhd_bunch_adjoint_bind(mhd_bunch* h, const int32_t* nbr_host, void* adjoint_workspace_dev,
                                  hipStream_t stream);
mhd_status mhd_bunch_adjoint(mhd_bunch* h, const void* U_in, const void* lam_out, void* lam_in,
                             const double* dt_dev, const double* dx_dev, hipStream_t stream);

/* ---- launch configuration and autotuning ----
 * The solver kernel works on 3D tiles of a patch's interior (every face flux and edge EMF
 * of the tile into shared memory, then the update).  A bunch has 3*S launch
 * configurations: S tile shapes for its dimensionality, each in three launch modes:
 *   0 plain grid (one work-group per tile or block of 256 items);
 *   1 the same with the XCD remap (work-groups, handed round-robin to the 8 XCDs, take
 *     contiguous ranges of the tile and block tables, so neighbouring tiles share an L2);
 *   2 persistent grids sized to the device (work-groups loop over the tables), remapped.
 * Configuration 0 is the default.  mhd_bunch_tile_get fills
 * cfg = {tile x, tile y, tile z, mode}.  Every configuration gives the same bits. */
int32_t mhd_bunch_tile_count(const mhd_bunch* h);
int32_t mhd_bunch_tile_current(const mhd_bunch* h);
mhd_status mhd_bunch_tile_get(const mhd_bunch* h, int32_t index, int32_t cfg[4]);
mhd_status mhd_bunch_tile_set(mhd_bunch* h, int32_t index);

/* Predictor stages (the half-step prediction of §2.1 "The MUSCL Scheme"): mode 0 = three
 * kernels (primitives, edge EMFs at time n, predictor) through the workspace scratch;
 * mode k >= 1 = one tiled kernel that keeps the primitives and face fields of a tile (plus
 * one cell around it) in shared memory, with the k-th tile shape of the bunch's
 * dimensionality.  mhd_bunch_predictor_count returns the number of modes (staged + fused
 * shapes); mhd_bunch_predictor_shape fills tile3 with the tile of a mode ({0, 0, 0} for 0).
 * Same values in every mode.  Default 0; mhd_bunch_set_predictor returns MHD_EINVAL for a
 * mode outside [0, count). */
mhd_status mhd_bunch_set_predictor(mhd_bunch* h, int32_t mode);
int32_t mhd_bunch_predictor(const mhd_bunch* h);
int32_t mhd_bunch_predictor_count(const mhd_bunch* h);
mhd_status mhd_bunch_predictor_shape(const mhd_bunch* h, int32_t mode, int32_t tile3[3]);

/* Solver form: 0 = face fluxes and edge EMFs of the tile held in shared memory together,
 * then the whole update; 1 = two phases (face fluxes, hydro update; then edge EMFs, field
 * update) that share the shared memory, for more work-groups per compute unit; 2 = a
 * separate pass computes every edge EMF once into the workspace scratch and the tile does
 * the face fluxes and the update (no halo edges recomputed); 3 = form 2 with that pass taken
 * as lines of edges (one thread steps along a line and loads each corner plane once instead
 * of twice); form 3 is form 2 itself unless all three directions are active.  Same values
 * in every form.  Default 0; MHD_EINVAL for a form outside [0, 3]. */
mhd_status mhd_bunch_set_solver_split(mhd_bunch* h, int32_t split);
int32_t mhd_bunch_solver_split(const mhd_bunch* h);

/* Times every configuration, each with every solver form, on the caller's data (one
 * warm-up and `reps` timed updates of U_in -> U_out each, HIP events on `stream`) and keeps
 * the fastest pair; then, with it, times every predictor mode and keeps the fastest.
 * Synchronises `stream`; overwrites U_out.  best (may be NULL) receives the chosen
 * configuration index, ms (may be NULL, else float[mhd_bunch_tile_count]) the mean update
 * time of each configuration (the fastest of its solver forms).  On an error the
 * configuration, solver form and predictor mode stay as they were before the call. */
mhd_status mhd_bunch_autotune(mhd_bunch* h, const void* U_in, void* U_out, const double* dt_dev,
                              const double* dx_dev, int32_t reps, hipStream_t stream,
                              int32_t* best, float* ms);

/* ---- batched multi-step runs in one HIP graph ----
 * Captures nsteps steps into a HIP graph owned by the handle (replacing any earlier one):
 * step k advances U_a -> U_b for even k and U_b -> U_a for odd k, with
 *   nbr_dev != NULL: the guards of the step's input filled first (as mhd_bunch_fill_guards);
 *                    NULL: guards are frozen inputs;
 *   dt_mode 0: dt_dev used as given; 1: dt_dev[p] = the patch's own CFL step of the step's
 *              input (each patch steps independently at its own dt: valid with frozen
 *              guards only, so nbr_dev must be NULL, else MHD_EINVAL -- a guard exchange
 *              between patches at different times needs mhd_bunch_lts_step); 2: global
 *              minimum.
 * Every launch of every step uses the launch configuration current at capture time.
 * Buffers are bound by address: they must stay allocated while the graph is launched.
 * Capture uses a private stream; nothing runs until mhd_bunch_graph_launch enqueues the
 * whole run on `stream`. */
mhd_status mhd_bunch_graph_capture(mhd_bunch* h, int32_t nsteps, void* U_a, void* U_b,
                                   double* dt_dev, const double* dx_dev, const int32_t* nbr_dev,
                                   int32_t dt_mode, hipStream_t stream);
mhd_status mhd_bunch_graph_launch(mhd_bunch* h, hipStream_t stream);

/* Captures `nsteps` local time steps (mhd_bunch_lts_step with these arguments, validated the
 * same way) into the handle's HIP graph, replacing any earlier one; mhd_bunch_graph_launch
 * runs them.  A bunch processed in one chunk (no max_scratch_bytes cap, or one that holds the
 * whole bunch) and free steps (dt_quantum == 0) compacts its launch tables to the ready patches
 * on the device in every step (as mhd_bunch_lts_step does), so each captured step does work in
 * proportion to the patches that advance.  Steps after every
 * patch reached t_end do nothing.  Buffers are bound by address. */
mhd_status mhd_bunch_lts_graph_capture(mhd_bunch* h, int32_t nsteps, void* U_cur, void* U_new,
                                       void* U_prev, double* t_dev, double* t_prev_dev,
                                       double* dt_dev, const double* dt_fixed_dev,
                                       const double* dx_dev, const int32_t* nbr_dev, double t_end,
                                       double dt_quantum, hipStream_t stream);

/* ---- bunches whose state stays in host memory (§2.4 "DISPATCH Integration": patches are
 * bunched on the host and sent to the GPU, three bunches active at once -- one being
 * filled, one computed, one emptied; §3.2: a third of the time went to transfers; §4:
 * asynchronous transfers hide them) ----
 * mhd_stream_create cuts a bunch description into consecutive sub-bunches of at most
 * `patches_per_bunch` patches (one internal bunch handle each) and plans `slots` (1..8)
 * device slots, each holding one sub-bunch's input and output state.  The caller provides
 * one device allocation of mhd_stream_device_bytes (tables of every sub-bunch, one shared
 * predictor scratch, dt/dx, the slots; 256-byte aligned) to mhd_stream_bind, which uploads
 * the tables on `stream` and creates three non-blocking streams of default priority.
 * mhd_stream_update advances a host-resident state U_in (guards filled, layout of the whole
 * description) into the host buffer U_out with host arrays dt[P], dx[P][3]: per sub-bunch,
 * copy in (first stream), update (second stream; the output slot starts as a copy of the
 * input, so U_out's guard entries are U_in's), copy out (third stream), ordered by events,
 * so that with slots >= 2 the copies of neighbouring sub-bunches overlap the update.  All
 * work is ordered after earlier work on `stream`, and later work on `stream` waits for every
 * copy out; the call itself returns without synchronising.  The host buffers must stay valid
 * and unchanged until then and should be page-locked (hipHostMalloc) for the copies to run
 * asynchronously.  U_in and U_out must not overlap.  mhd_stream_configure applies one launch
 * configuration (mhd_bunch_tile_set index, predictor mode, solver form) to every sub-bunch;
 * mhd_stream_check synchronises `stream` and reports the sub-bunches' device status as
 * mhd_bunch_check does.  Results are those of mhd_bunch_update on the same state. */
typedef struct mhd_stream mhd_stream;
mhd_status mhd_stream_create(mhd_stream** out, const mhd_bunch_desc* desc, int32_t patches_per_bunch,
                             int32_t slots);
void mhd_stream_destroy(mhd_stream* s);
int64_t mhd_stream_device_bytes(const mhd_stream* s);
int32_t mhd_stream_bunch_count(const mhd_stream* s);
mhd_status mhd_stream_bind(mhd_stream* s, void* device_buffer, hipStream_t stream);
mhd_status mhd_stream_configure(mhd_stream* s, int32_t tile, int32_t predictor, int32_t split);
mhd_status mhd_stream_update(mhd_stream* s, const void* U_in_host, void* U_out_host,
                             const double* dt_host, const double* dx_host, hipStream_t stream);
mhd_status mhd_stream_check(mhd_stream* s, hipStream_t stream);
const char* mhd_stream_last_error(const mhd_stream* s);

/* Synchronises `stream`, then returns MHD_ENONPHYS if any kernel since the last check
 * met a non-physical state, MHD_EINVAL if a guard fill met an inconsistent neighbour table or
 * a local time step met a step that is not finite and > 0 (and clears the flags), else
 * MHD_OK. */
mhd_status mhd_bunch_check(mhd_bunch* h, hipStream_t stream);

/* Kernel timing with HIP events recorded on the caller's stream around every launch.
 * mhd_bunch_profile(h, 1) clears the record and starts recording; mhd_bunch_profile(h, 0)
 * stops.  mhd_bunch_profile_read synchronises
 * on the recorded events and returns the summed duration (ms) and launch count of one
 * kernel kind since recording started. */
enum {
  MHD_KERNEL_PRIM = 0,        /* primitives */
  MHD_KERNEL_EDGE_EMF_N = 1,  /* edge EMFs at time n */
  MHD_KERNEL_PREDICT = 2,     /* slopes, half-step state and face field */
  MHD_KERNEL_SOLVE = 3,       /* HLLD fluxes, edge EMFs (forms 0, 1), update */
  MHD_KERNEL_CFL = 4,         /* time step (three small kernels, timed together) */
  MHD_KERNEL_GUARDS = 5,      /* guard fill */
  MHD_KERNEL_EDGE = 6,        /* half-step edge EMFs (solver forms 2, 3) */
  MHD_KERNEL_COUNT = 7
};
mhd_status mhd_bunch_profile(mhd_bunch* h, int32_t enable);
mhd_status mhd_bunch_profile_read(mhd_bunch* h, int32_t kernel, double* total_ms, int64_t* launches);

const char* mhd_status_string(mhd_status s);

/* Text of the HIP failure behind the last MHD_EDEVICE returned for this handle ("" if
 * none).  The string is owned by the handle. */
const char* mhd_bunch_last_error(const mhd_bunch* h);

#ifdef __cplusplus
}
#endif
#endif
