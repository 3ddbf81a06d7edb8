/*
 * lbboil: MI355X (gfx950) library for the hybrid thermal pseudopotential
 * lattice Boltzmann boiling model of Li, Kang, Francois, He and Luo,
 * "Lattice Boltzmann modeling of boiling heat transfer: the boiling curve and
 * the effects of wettability" (arXiv:1501.03857).
 *
 * One time step (Sec. 2) advances
 *   - the D2Q9 distributions f by the MRT collision with the improved forcing
 *     term (Eqs. (2), (4), (5), (8)) and streaming (Eq. (3)), driven by the
 *     Peng-Robinson pseudopotential force (Eq. (7), Eq. (21)), the fluid-solid
 *     force (Eq. (22)) and buoyancy (Eq. (9)), with Zou-He no-slip walls and
 *     periodic x (Sec. 3.1);
 *   - the temperature T by one classical RK4 step (Eqs. (19)-(20)) of the
 *     finite-difference temperature equation (Eq. (18)) with rho and v frozen
 *     at the old time level, Dirichlet walls T_b (bottom) and T_s (top);
 * and samples the bottom-wall heat flux q(t) = <-lambda dT/dy>_x (Sec. 3.2).
 *
 * Conventions of every call:
 *   - Return value: LBB_OK (0) or a negative LBB_E* code; nothing else crosses
 *     the boundary.  lbb_last_error() returns a message for the last failure
 *     of the calling thread (valid until that thread's next call).
 *   - Handles are opaque, owned by the library, released with lbb_destroy.
 *     A handle must not be used by two threads at once.
 *   - All array arguments are caller-owned HOST buffers in row-major order
 *     [ny][nx] (x fastest), FP64, unless stated otherwise.  The library never
 *     keeps a pointer past the call.  Distribution arrays are [9][ny][nx] with
 *     velocities ordered rest, E, N, W, S, NE, NW, SW, SE.
 *   - Calls are synchronous with respect to the host unless the name ends in
 *     _async.
 *   - Lattice units throughout (c = dx = dt = 1, c_s^2 = 1/3).
 */
#ifndef LBBOIL_H
#define LBBOIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBB_OK 0
#define LBB_EINVAL (-1)       /* invalid argument or parameter                 */
#define LBB_ENOMEM (-2)       /* device or host allocation failed              */
#define LBB_EDEVICE (-3)      /* HIP runtime error or no usable gfx950 device  */
#define LBB_ENONFINITE (-4)   /* non-finite value, rho <= 0, T <= 0 or a
                                 negative pseudopotential radicand detected     */
#define LBB_EUNSUPPORTED (-5) /* request not supported by the library          */
#define LBB_ESTATE (-6)       /* domain poisoned by an earlier LBB_ENONFINITE  */

enum { LBB_FP64 = 0, LBB_FP32 = 1 };
/* Test modes: COUPLED is the model; ISOTHERMAL freezes T; THERMAL_ONLY
 * freezes f and advances only T with v = sum_a e_a f_a / rho. */
enum { LBB_COUPLED = 0, LBB_ISOTHERMAL = 1, LBB_THERMAL_ONLY = 2 };

/* Model parameters (Sec. 2 and Sec. 3.1).  lbb_default_params fills the
 * paper's values (with a = 2/49; the paper's own runs use a = 3/49). */
typedef struct lbb_params {
    int32_t nx, ny;          /* lattice nodes; rows 0 and ny-1 are the walls   */
    int32_t precision;       /* LBB_FP64, or LBB_FP32: f, T, rho, v stored in
                                FP32; LB, EOS and reductions in FP64, the RK4
                                stages in FP32 on T - T_s                      */
    int32_t periodic_y;      /* 1: no walls, periodic in y (test mode)         */
    int32_t thermal_mode;    /* LBB_COUPLED / LBB_ISOTHERMAL / LBB_THERMAL_ONLY */
    int32_t liquid_rows;     /* built-in initial state: rows j < liquid_rows
                                are liquid (used when rho0 == NULL)            */
    /* Peng-Robinson EOS, Eq. (21) */
    double a, b, R, omega;
    double Ts_over_Tc;       /* saturation temperature T_s / T_c               */
    /* pseudopotential force, Eq. (7), and improved forcing, Eq. (8) */
    double G, sigma;         /* G < 0                                          */
    /* MRT relaxation rates of Eq. (4); the shear rate follows from nu        */
    double s_rho, s_e, s_zeta, s_j, s_q;
    double nu_L, nu_V;       /* kinematic viscosities of liquid and vapour     */
    double rho_L, rho_V;     /* densities between which tau_nu is interpolated
                                linearly; both 0: Maxwell coexistence at T_s   */
    /* temperature equation, Eq. (18): lambda = rho c_v chi */
    double cv, cv_chi;
    double g;                /* gravity magnitude, Eq. (9), along -y           */
    double Gw_bottom, Gw_top;/* fluid-solid strengths, Eq. (22)                */
    double noise_amp;        /* built-in initial state: uniform noise in
                                [-noise_amp, noise_amp) on rho                 */
    uint64_t seed;           /* built-in initial state: SplitMix64 seed        */
    int32_t ghost_layer;     /* 1: the fluid-fluid force of Eq. (7) also acts
                                on the wall rows (Sec. 3.2), with a ghost fluid
                                layer beyond each wall mirroring the first
                                fluid row, psi(i,-1) = psi(i,1): F_m there is
                                tangential; buoyancy still skips the wall rows.
                                0 (default): no fluid-fluid force on them.
                                No effect with periodic_y (no walls).
                                lbb_adjoint refuses 1 (LBB_EUNSUPPORTED)       */
    int32_t reserved;        /* must be 0                                      */
} lbb_params;

typedef struct lbb_domain lbb_domain;

/* Fill *p with the paper's parameters (Sec. 3.1): a = 2/49, b = 2/21, R = 1,
 * omega = 0.344, T_s = 0.86 T_c, G = -1, sigma = 1.2, s = (1, 0.8, 0.8, 1, 1.1),
 * nu_L = 0.1, nu_V = 0.5/3, c_v = 6, c_v chi = 0.028, g = 3e-5, G_w = 0,
 * 128x64 FP64, liquid_rows = 0.6 ny, noise 1e-3, seed 1, rho_L = rho_V = 0. */
void lbb_default_params(lbb_params *p);

/* T_c and kappa(omega) of the Peng-Robinson EOS, Eq. (21):
 * T_c = (a/b)(0.0778/0.45724)/R. */
int lbb_eos_constants(double a, double b, double R, double omega, double *Tc, double *kappa);

/* Maxwell equal-area coexistence densities of Eq. (21) at temperature T < T_c
 * (the coexistence the paper starts from, Sec. 3.1).  EINVAL if T >= T_c. */
int lbb_coexistence(double a, double b, double R, double omega, double T,
                    double *rho_V, double *rho_L);

/* Peng-Robinson pressure p_EOS(rho, T) of Eq. (21) (host arithmetic), the
 * bulk pressure of the pseudopotential fluid (Sec. 2): the quantity the
 * paper records at the centre of the top wall (Sec. 3.2, Fig. 3).
 * EINVAL unless rho > 0, T > 0, b rho < 1 and p is non-NULL. */
int lbb_eos_pressure(double a, double b, double R, double omega, double rho, double T, double *p);

/* Create a domain on the current HIP device (Sec. 3.1 set-up).
 *   T_bottom [nx] : bottom-wall temperature T_b(x); NULL means T_s.
 *   rho0 [ny*nx]  : initial density; NULL builds the layered state
 *                   (liquid below vapour at rho_L/rho_V plus SplitMix64 noise
 *                   of the (j*nx+i+1)-th output of the generator seeded with
 *                   seed, top 53 bits mapped to [0,1), amplitude noise_amp).
 * f starts at equilibrium at rest, T = T_s with the Dirichlet wall rows.
 * EINVAL: nx < 3, ny < 4 (ny < 3 when periodic_y), a field plane of 2^32
 * bytes or more (nx*ny*sizeof(real) >= 2^32: 2^30 nodes in FP32, 2^29 in
 * FP64), G >= 0, non-finite or non-positive inputs, b*rho >= 1,
 * rho_L == rho_V.  ENOMEM/EDEVICE on HIP
 * failures.  Device memory: about (20 + 5) * nx * ny * sizeof(real) bytes. */
int lbb_init_domain(const lbb_params *p, const double *T_bottom, const double *rho0,
                    lbb_domain **out);

/* Replace the state: f = f_eq(rho, u) (equilibrium with velocity u) and T
 * (wall rows of T are then reset to T_b and T_s unless periodic_y).  ux, uy,
 * T may be NULL (zero velocity; T_s).  Resets the step counter and the
 * heat-flux average. */
int lbb_set_fields(lbb_domain *d, const double *rho, const double *ux, const double *uy,
                   const double *T);

/* Advance n >= 0 time steps and append one heat-flux sample per step (state
 * after the step).  On LBB_ENONFINITE the message names the first failing
 * step and the domain is poisoned (LBB_ESTATE) until lbb_load_state or
 * lbb_set_fields. */
int lbb_step(lbb_domain *d, int64_t n);

/* Enqueue n steps on the library stream without waiting and without the
 * error check (for timing).  lbb_sync waits and performs the check. */
int lbb_step_async(lbb_domain *d, int64_t n);
int lbb_sync(lbb_domain *d);
/* The HIP stream (hipStream_t) the library launches on, so a caller can
 * record events around lbb_step_async. */
void *lbb_stream(lbb_domain *d);

/* Advance n >= 1 steps with single launches (no graph), each launch
 * carrying HIP events that its dispatch records at kernel start and end;
 * returns the mean kernel duration in milliseconds of the LB launch
 * (collision, forces, streaming) and of the thermal launch (RK4 temperature
 * step), and the mean wall time per step of the whole sequence.  For
 * measurement only; the state advances exactly as with lbb_step. */
int lbb_time_kernels(lbb_domain *d, int64_t n, double *ms_lb, double *ms_thermal, double *ms_step);

/* Fields of lbb_read_fields' mask. */
#define LBB_FIELD_RHO 1u
#define LBB_FIELD_UX 2u
#define LBB_FIELD_UY 4u
#define LBB_FIELD_T 8u
#define LBB_FIELD_F 16u
#define LBB_FIELD_ALL 31u

/* Read the current state, widened to FP64: rho = sum_a f_a; v from Eq. (6)
 * with the total force of the current state; T; and f (post-streaming, wall
 * rule applied).  Host buffers, nx*ny each, f 9*nx*ny, layout [a][y][x].  A
 * field is written when its LBB_FIELD_* bit is set in `mask` and its pointer
 * is not NULL; the others are left alone.  The domain's state is not
 * changed. */
int lbb_read_fields(const lbb_domain *d, uint32_t mask, double *rho, double *ux, double *uy, double *T,
                    double *f);
/* The same fields into caller-owned device buffers (FP64, nx*ny each, f
 * 9*nx*ny, layout [a][y][x]; NULL skipped), without a host wait.  The read
 * is ordered after the library's earlier work on the domain, after the
 * caller's earlier work on `stream` (a hipStream_t; NULL is the null stream)
 * and before the caller's later work there.  EDEVICE if the launch or the
 * stream ordering fails. */
int lbb_read_fields_dev(lbb_domain *d, double *rho, double *ux, double *uy, double *T, double *f, void *stream);

/* Bottom-wall heat flux (Sec. 3.2): q_now = q(t) of the current state, q_mean
 * = mean of the samples since creation or lbb_reset_average, n_samples their
 * count; q_local [nx] (optional) = q_w(x) of the current state.
 * q_w = -c_v chi rho (-3 T_0 + 4 T_1 - T_2)/2 at each bottom-wall node. */
int lbb_wall_heat_flux(const lbb_domain *d, double *q_now, double *q_mean, double *q_local,
                       int64_t *n_samples);
int lbb_reset_average(lbb_domain *d);

/* Change the bottom-wall temperature T_b(x) [nx] (the paper raises the
 * superheat mid-run, Sec. 3.2) or the bottom-wall strength G_w (Eq. (22)). */
int lbb_set_heater(lbb_domain *d, const double *T_bottom);
int lbb_set_wettability(lbb_domain *d, double Gw_bottom);

/* Checkpoint: *len in/out.  With buf == NULL, *len receives the size needed.
 * The blob holds f, T, T_b, G_w, the step counter and the heat-flux
 * accumulators, with a parameter hash and a checksum; load rejects a blob of
 * another domain shape/parameters or a corrupted one (EINVAL). */
int lbb_save_state(lbb_domain *d, void *buf, size_t *len);
int lbb_load_state(lbb_domain *d, const void *buf, size_t len);

/* ---- Batched lattices (boiling-curve sweeps) ---------------------------
 * n independent lattices of any sizes and parameters (superheat, wettability,
 * seed) advanced together: each step is one LB launch and one thermal launch
 * covering every lattice, replayed from captured HIP graphs.  Each lattice
 * evolves bitwise as it would alone.  All members share precision and
 * thermal_mode.
 *   ps [n]        : parameters of each lattice (validated as lbb_init_domain).
 *   T_bottoms [n] : per-lattice bottom-wall temperature arrays [nx_i], or NULL
 *                   (the array itself or an entry: T_s).
 *   rho0s [n]     : per-lattice initial densities [ny_i*nx_i], or NULL
 *                   (built-in layered state).
 * EINVAL on an empty batch, mixed precision or modes, or any invalid member. */
typedef struct lbb_batch lbb_batch;
int lbb_batch_init(const lbb_params *ps, int n, const double *const *T_bottoms, const double *const *rho0s,
                   lbb_batch **out);
int lbb_batch_step(lbb_batch *b, int64_t n);
int lbb_batch_step_async(lbb_batch *b, int64_t n);
int lbb_batch_sync(lbb_batch *b);
void *lbb_batch_stream(lbb_batch *b);
/* Per-lattice heat flux [n] each (any pointer may be NULL), as
 * lbb_wall_heat_flux. */
int lbb_batch_heat_flux(lbb_batch *b, double *q_now, double *q_mean, int64_t *n_samples);
/* Borrowed handle of member i for the single-lattice calls (read_fields,
 * heat flux, save/load, set_heater ...); owned by the batch, NULL if out of
 * range.  Stepping a member alone puts it out of phase with the batch, which
 * then refuses to step (EINVAL). */
lbb_domain *lbb_batch_domain(lbb_batch *b, int i);
int lbb_batch_size(lbb_batch *b);
int lbb_batch_destroy(lbb_batch *b);

/* ---- Adjoint -----------------------------------------------------------
 * J = (1/N) sum_{n=1..N} q^n, the bottom-wall heat flux (Sec. 3.2) averaged
 * over the next N steps from the current state, and its gradient with
 * respect to the bottom-wall temperatures of the heater nodes,
 * dJ_dTb[k] = dJ/dT_b(heater_idx[k]) for k < n_heater (heater_idx NULL: all
 * nx nodes in order, n_heater must be nx), and the bottom wall strength G_w
 * (Eq. (22)), by a hand-written discrete adjoint of the whole coupled step
 * (FP64 arithmetic; the population adjoints, the per-node work arrays and
 * the temperature adjoint's LDS planes are stored in the domain's precision,
 * the adjoint of T and the sums in FP64).  J is required; dJ_dTb and dJ_dGw
 * may be NULL.  EINVAL for a heater index outside [0, nx).  States are checkpointed
 * every K steps and each segment but the last is recomputed before its
 * reverse sweep.  K <= 0 lets the library choose: every state kept (K = N,
 * no recompute) when N + 2 states take at most a quarter of the free device
 * memory, else K = ceil(sqrt(N)).  The domain's state, step count and
 * heat-flux average are restored afterwards.  Device memory, allocated on
 * the first call and kept by the domain (reported by lbb_info): about
 * (N/K + K + 2) * 10 * nx*ny * sizeof(real) + 38 * nx*ny * sizeof(real) +
 * 4 * nx*ny * 8 bytes.
 * EUNSUPPORTED for periodic_y or a test mode; EINVAL for N < 1; ENOMEM when
 * the workspace cannot be allocated. */
int lbb_adjoint(lbb_domain *d, int64_t N, int64_t K, const int32_t *heater_idx, int32_t n_heater, double *J,
                double *dJ_dTb, double *dJ_dGw);

/* The adjoint of every batch member at once (the same N and K for all),
 * each lattice's forward, recompute and reverse steps sharing the batch's
 * launches.  Outputs: J[n], dJ_dTb[sum of the members' nx] (member after
 * member), dJ_dGw[n]; J required, the others may be NULL.  Results equal
 * lbb_adjoint on each member alone.  Members are restored and left in phase;
 * EINVAL if the members are out of phase, the member's error code (with its
 * index in the message) if one cannot be differentiated. */
int lbb_batch_adjoint(lbb_batch *b, int64_t N, int64_t K, double *J, double *dJ_dTb, double *dJ_dGw);

/* Device bytes held by the batch: its members and its adjoint workspace. */
int lbb_batch_info(lbb_batch *b, int64_t *device_bytes);

/* ---- Tile shapes and autotuning ---------------------------------------
 * The LB launch works on tiles 62 nodes wide and the thermal launch on tiles
 * 56 wide (plus their halos, one wave64 wide); their heights and waves per
 * block come from small tables of shapes.  lbb_tile_shapes reports them:
 * n_lb and n_thermal entries of (width, height, waves) in lb[3 n_lb] and
 * thermal[3 n_thermal] (any pointer may be NULL).  Shape 0 of each is the
 * default of a new domain or batch.  Results do not depend on the shapes
 * beyond the summation order of the domain-mean density (ulp level). */
int lbb_tile_shapes(int32_t *n_lb, int32_t *n_thermal, int32_t *lb, int32_t *thermal);
int lbb_get_tiles(lbb_domain *d, int32_t *shape_lb, int32_t *shape_thermal);
/* Select the shapes (indices into the tables); EINVAL for an unknown index.
 * A batch member takes its batch's shapes when the batch next steps. */
int lbb_set_tiles(lbb_domain *d, int32_t shape_lb, int32_t shape_thermal);
/* Time every LB shape, then every thermal shape with the best LB shape, for
 * `steps` steps each on the domain's own state (per-kernel durations from
 * events recorded by the dispatches), keep the fastest of each, and restore
 * the state, step count and heat-flux average.  Outputs (may be NULL): the
 * chosen shapes and the mean durations in ms per shape (ms_lb[n_lb],
 * ms_thermal[n_thermal]).  EINVAL for steps < 1; ESTATE on a poisoned
 * domain; ENONFINITE if a trial step produces an invalid state (the state is
 * restored all the same). */
int lbb_autotune(lbb_domain *d, int32_t steps, int32_t *shape_lb, int32_t *shape_thermal, double *ms_lb,
                 double *ms_thermal);
int lbb_batch_set_tiles(lbb_batch *b, int32_t shape_lb, int32_t shape_thermal);
/* As lbb_autotune, for the batch's shared launches (one shape pair for all
 * members). */
int lbb_batch_autotune(lbb_batch *b, int32_t steps, int32_t *shape_lb, int32_t *shape_thermal, double *ms_lb,
                       double *ms_thermal);

/* Device-memory budget of the process: the library refuses (ENOMEM, before
 * touching the device) any domain, batch member or adjoint workspace that
 * would take the bytes it holds over `bytes`; 0 (the default) means no
 * budget.  EINVAL for bytes < 0.  lbb_device_bytes_held reports the bytes
 * held against it (all live domains and adjoint workspaces). */
int lbb_set_device_budget(int64_t bytes);
int64_t lbb_device_bytes_held(void);

/* ---- Stepping without allocation ---------------------------------------
 * For callers that cannot allocate device memory: code running under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same n time steps as lbb_step (the same kernels and default tile
 * shapes) on a lattice whose state the caller holds in its own device
 * buffers.  The domain-mean density of the first step is summed from the
 * given state as lbb_init_domain and lbb_set_fields sum it, so the result is
 * bitwise that of lbb_step on a domain just created with the same state; from
 * a domain that has stepped it differs by that sum's rounding order.  The library allocates nothing: the
 * per-block partial sums, the launch table and the scalars (domain-mean
 * density, heat-flux accumulators, error flag) live in one static device
 * array of LBB_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends
 * and shared by every call on that GPU, so calls that overlap on one GPU
 * (two host threads, or two streams in flight) race and must not be made.
 * Each call re-initialises what it uses; nothing carries over between calls.
 *   p           : parameters, validated as lbb_init_domain (rho_L = rho_V = 0:
 *                 Maxwell coexistence at T_s); the lattice's scratch need is
 *                 8 (ceil(nx/62) ny + ceil(nx/56)) + 4 (blocks + 2) + 1 KiB
 *                 bytes and must not exceed LBB_NOALLOC_SCRATCH_BYTES (EINVAL
 *                 with the need in the message): up to about 1e6 rows of
 *                 nx = 62, or 8192 x 6500.
 *   f[2]        : two device buffers of 9*nx*ny values of the storage type
 *                 (double for LBB_FP64, float for LBB_FP32), layout
 *                 [a][y][x], velocities rest, E, N, W, S, NE, NW, SW, SE:
 *                 post-streaming populations; on wall rows the three
 *                 populations arriving from outside are ignored (completed
 *                 by the Zou-He rule on read).  The layout lbb_save_state
 *                 writes after its header.
 *   T[2]        : two device buffers of nx*ny values of the storage type
 *                 holding T - T_ref (T_ref = 0 in FP64, T_s in FP32); both
 *                 must hold the Dirichlet wall rows (T_b on row 0, T_s on
 *                 row ny-1), which the steps never write.
 *   rho, vx, vy : device buffers of nx*ny values of the storage type
 *                 (overwritten: rho and the velocity the temperature equation
 *                 sees, of the last step's old state).
 *   phase [2]   : host, in/out: which buffer of f (phase[0]) and of T
 *                 (phase[1]) holds the state, 0 or 1; updated on return (f
 *                 alternates every step unless THERMAL_ONLY, T unless
 *                 ISOTHERMAL).
 *   n           : steps, >= 0.
 *   result      : device pointer to an lbb_noalloc_result, written after the
 *                 last step: q(t) of the final state, the mean of the n
 *                 samples (NaN for n = 0), the sample count, and the first
 *                 failing step and error bits (err_step = -1 when none;
 *                 bits 1: rho, 2: pseudopotential radicand, 4: T).
 *   stream      : hipStream_t the work is enqueued on (NULL: null stream).
 * Asynchronous: returns once the work is enqueued; the caller synchronises
 * the stream and reads *result.  EINVAL on invalid parameters, NULL buffers,
 * n < 0, a phase other than 0/1 or a lattice beyond the scratch; EDEVICE on
 * a HIP error (no usable gfx950 device, launch failure). */
#define LBB_NOALLOC_SCRATCH_BYTES (8u << 20)
typedef struct lbb_noalloc_result {
    double q_now, q_mean;
    int64_t n_samples;
    int64_t err_step;
    uint32_t err_code, reserved;
} lbb_noalloc_result;
int lbb_step_noalloc(const lbb_params *p, void *const f[2], void *const T[2], void *rho, void *vx, void *vy,
                     int32_t phase[2], int64_t n, lbb_noalloc_result *result, void *stream);

/* ---- Three-dimensional lattices (D3Q19) ---------------------------------
 * The same time step on a nx x ny x nz lattice: the extension to three
 * dimensions the paper names as its future work (Sec. 4).  The D3Q19 MRT
 * collision in the standard orthogonal moment basis with the improved
 * forcing (Eqs. (2), (4), (5), (8); the sigma term adds to each diagonal
 * component of the second moment the increment of the two-dimensional
 * term), the interaction force Eq. (7) with weights 1/6 (axes) and 1/12
 * (edges), the fluid-solid force Eq. (22), buoyancy Eq. (9), zero-velocity
 * Zou-He walls at y = 0 and y = ny-1 with transverse-momentum correction
 * (periodic x and z), and the RK4 temperature step Eqs. (18)-(20) with the
 * isotropic D3Q19 stencils; the bottom-wall heat flux averages over x and z.
 * Arrays are row-major [nz][ny][nx] (x fastest), FP64 host buffers:
 *   T_bottom [nz*nx], rho0 [nz*ny*nx] (NULL: layered state with noise as
 *   lbb_init_domain, counter (z*ny + y)*nx + x), u [3][nz][ny][nx],
 *   f [19][nz][ny][nx] with velocities rest, +x, -x, +y, -y, +z, -z,
 *   (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1),
 *   (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1); q_local [nz][nx].
 * Parameters as lbb_init_domain; the relaxation rates of the D3Q19 basis are
 * s_rho, s_e, s_zeta (epsilon and the pi moments), s_j, s_q (q and the m
 * moments) and s_nu.  EINVAL for nz < 3 or a lattice of 2^32 / 19 nodes or
 * more; EUNSUPPORTED for ghost_layer = 1.  Steps, errors, poisoning,
 * samples and averages behave as in two dimensions. */
typedef struct lbb3_domain lbb3_domain;
int lbb3_init_domain(const lbb_params *p, int32_t nz, const double *T_bottom, const double *rho0,
                     lbb3_domain **out);
/* Replace the state: f = f_eq(rho, u), T (u, T may be NULL: rest; T_s),
 * Dirichlet rows reset; counters and average reset. */
int lbb3_set_fields(lbb3_domain *d, const double *rho, const double *u, const double *T);
int lbb3_step(lbb3_domain *d, int64_t n);
int lbb3_step_async(lbb3_domain *d, int64_t n);
int lbb3_sync(lbb3_domain *d);
void *lbb3_stream(lbb3_domain *d);
/* rho, u (Eq. (6) with the force of the current state), T, f (completed),
 * widened to FP64; any pointer may be NULL. */
int lbb3_read_fields(lbb3_domain *d, double *rho, double *u, double *T, double *f);
int lbb3_wall_heat_flux(lbb3_domain *d, double *q_now, double *q_mean, double *q_local, int64_t *n_samples);
int lbb3_reset_average(lbb3_domain *d);
int lbb3_set_heater(lbb3_domain *d, const double *T_bottom);
int lbb3_info(lbb3_domain *d, int64_t *t, int64_t *device_bytes);
int lbb3_destroy(lbb3_domain *d);

/* Current step count, grid shape and device bytes held by the domain. */
int lbb_info(lbb_domain *d, int64_t *t, int32_t *nx, int32_t *ny, int64_t *device_bytes);

int lbb_destroy(lbb_domain *d);

const char *lbb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBBOIL_H */
