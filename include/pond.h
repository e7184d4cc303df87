/*
 * pond.h -- C ABI of the MI355X (gfx950) library for the time step of the
 * two-population Particles-on-Demand kinetic model of compressible multiphase
 * flow: Reyhanian, Dorschner & Karlin, "Thermokinetic model of compressible
 * multiphase flows", arXiv:2002.09217.
 *
 * One handle owns one lattice (D1Q3, D2Q9 or D3Q27) and its device state.  A time step
 *   1. streams f (mass, momentum) and g (energy) semi-Lagrangianly at the shifted
 *      velocities v_i = sqrt(p/(rho T_L)) c_i + u                     (eqs. 1, 3-4)
 *      re-expressing every donor in the receiving node's gauge        (App. C)
 *      with cubic Lagrange reconstruction                             (App. D)
 *      inside a fixed-count predictor-corrector on (rho, u, E) through the van
 *      der Waals equation of state                                    (main text; App. A)
 *      or, in isothermal runs, the van der Waals, Dieterici or double-well
 *      pressure at a fixed temperature                                (Supplement)
 *   2. evaluates the Korteweg stress and force F = -div K              (eq. 18; App. F)
 *      and the heat-flux correction M0                                (eq. 9)
 *   3. relaxes f and g to their equilibria with the force source S_i, the
 *      force-extended g equilibrium and the sources g~ + phi          (eqs. 16-22)
 * on the device: for D1Q3 and D2Q9 one fused kernel per step by default (the step keeps
 * the streamed state and recomputes each tile's collision on chip), or two kernels
 * (streaming; force, closure and collision) with two_kernel = 1 and for D3Q27.
 *
 * Conventions for every call below
 *   - All functions return a pond_status (0 = POND_OK, negative = error).
 *   - Host arrays are caller-owned, plain C doubles, copied synchronously.
 *   - Node order: index = x + n[0] * (y + n[1] * z).  A vector field is `dim`
 *     consecutive planes of N = n[0]*n[1]*n[2] values (x component first).
 *   - Device memory is owned by the library (allocated in pond_create, released in
 *     pond_destroy).  Work is enqueued on cfg.stream (a hipStream_t, e.g. PyTorch's
 *     current stream) or on a library-owned stream when cfg.stream is NULL.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - After an error in pond_step the state is that of the last completed step,
 *     the handle refuses further steps (POND_E_STATE) until pond_init_fields is
 *     called again, and pond_last_error() describes the failure.
 */
#ifndef POND_H
#define POND_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pond_handle pond_handle; /* opaque, library-owned */
typedef struct pond_batch pond_batch;   /* opaque, library-owned */

typedef enum {
    POND_OK = 0,
    POND_E_INVALID = -1,   /* bad argument or configuration                          */
    POND_E_NOMEM = -2,     /* device or host allocation failed                        */
    POND_E_DEVICE = -3,    /* HIP runtime error                                       */
    POND_E_PRESSURE = -4,  /* p <= 0, rho <= 0 or 1 - b rho <= 0 at some node         */
    POND_E_NONFINITE = -5, /* NaN or Inf in the state                                 */
    POND_E_HALO = -6,      /* a departure stencil leaves the +-2 node window:
                              |u| + sqrt(theta) times dt reached 1                    */
    POND_E_STATE = -7,     /* handle not initialised, or in the error state           */
    POND_E_SCRATCH = -8    /* pond_step_noalloc: the lattice needs more scratch than
                              POND_NOALLOC_SCRATCH_BYTES                              */
} pond_status;

enum { POND_BC_PERIODIC = 0, POND_BC_OUTFLOW = 1, POND_BC_INFLOW = 2 };
enum { POND_FP64 = 0, POND_FP32_STORE = 1, POND_FP32_STORE_FP64_MATH = 2 };
/* equation of state (main text; Supplement: coexistence curve and speed of sound) */
enum { POND_EOS_VDW = 0, POND_EOS_DIETERICI = 1, POND_EOS_DOUBLE_WELL = 2 };

typedef struct {
    int dim;                  /* 1 (D1Q3), 2 (D2Q9) or 3 (D3Q27, periodic faces only),
                                 App. B                                                 */
    int n[3];                 /* nodes per axis; unused axes = 1                        */
    int bc[3][2];             /* per axis, [low face, high face]: POND_BC_*             */
    double inflow[3][2][5];   /* state of an inflow face: rho, u_x, u_y, u_z, T (the
                                 actual velocity); its ghost nodes hold the equilibrium
                                 of that state with F = 0                              */
    double a, b, R;           /* van der Waals p = rho R T/(1 - b rho) - a rho^2, or
                                 Dieterici p = rho R T/(1 - b rho) exp(-a rho/(R T))  */
    double delta;             /* C_v = R/delta, 0 < delta <= 2/3 (main text)            */
    int eos;                  /* POND_EOS_VDW (e = C_v T - a rho) and POND_EOS_DIETERICI
                                 (e = C_v T + the integral of T (dp/dT)_v - p over v
                                 from the ideal-gas limit; T from e by Newton's method;
                                 Supplement, thermodynamics) run with the energy
                                 equation or isothermally; POND_EOS_DOUBLE_WELL needs
                                 isothermal.  Double well: p = p0 + rho dE0/drho - E0
                                 with E0 = beta (rho - rho_l)^2 (rho - rho_v)^2.  The
                                 Dieterici energy is evaluated for T > a/(150 R b).     */
    int isothermal;           /* nonzero: T = T0 wherever the step needs a temperature
                                 (passes, closure, initial and inflow states, read-back;
                                 the T given to pond_init_fields is not used).  The
                                 energy population is then passive and carries
                                 e(rho, T0) of the law (C_v T for the double well).    */
    double T0;                /* isothermal temperature, > 0                            */
    double eos_c[4];          /* POND_EOS_DOUBLE_WELL: beta > 0, rho_l > rho_v > 0, p0 > 0 */
    double omega;             /* BGK relaxation, 0 < omega < 2; mu = (1/omega - 1/2) p dt */
    double kappa;             /* Korteweg coefficient of eq. 18; 0 switches the force off */
    double k_scale;           /* conductivity k = k_scale mu C_p^ig, C_p^ig = R(1+delta)/delta;
                                 k_scale < 0 switches the heat-flux correction off     */
    double dt;                /* time step in lattice units (dx = 1, App. D)            */
    int n_pass;               /* streaming passes of the predictor-corrector, >= 1      */
    int precision;            /* POND_FP64; POND_FP32_STORE: populations stored and
                                 streamed (interpolated) in FP32, with moments, EoS,
                                 gauge, forcing and collision in FP64;
                                 POND_FP32_STORE_FP64_MATH: stored in FP32, every
                                 operation in FP64.  Both FP32 forms store each set as
                                 its FP64 sum and FP32 deviations from W_q times it.  */
    int tile;                 /* tile shape of the streaming kernel: -1 = measure the
                                 compiled shapes on the first pond_init_fields and keep
                                 the fastest; k >= 0 = shape k (see pond_tile_info).
                                 Results depend on the shape at round-off level only. */
    int two_kernel;           /* 1D and 2D lattices.  0 (default): each step is one kernel
                                 that recomputes the collision of the previous step on its
                                 tile and a 2-node halo and streams; the state kept between
                                 steps is the streamed moments (18 planes in 2D, 6 in 1D;
                                 in the FP32 storage precisions rho, u and 2 rho E in FP64,
                                 the other moments in FP32), so the collided populations
                                 never reach device memory.  1: two kernels per step, with
                                 the collided populations and side fields stored (the FP32
                                 precisions store the populations in FP32).  D3Q27
                                 lattices always store populations.  Both give the same
                                 results up to round-off (FP32 precisions: within their
                                 FP32 rounding).                                         */
    void *stream;             /* hipStream_t or NULL                                    */
} pond_config;

/* Validate cfg and allocate the device state.  *out receives the handle (NULL on
 * error).  Errors: POND_E_INVALID (dim, sizes: N <= 2^30 nodes, 2^29 in 3D;
 * 0 < delta <= 2/3, 0 < omega < 2, n_pass >= 1, dt > 0, tile in range, two_kernel
 * not 0 or 1, inflow state
 * with p <= 0, a non-periodic face in 3D; eos out of range, the double well
 * without isothermal, T0 <= 0 when isothermal, double-well constants other than
 * beta > 0, rho_l > rho_v > 0, p0 > 0), POND_E_NOMEM, POND_E_DEVICE. */
int pond_create(const pond_config *cfg, pond_handle **out);

/* Set the state from the macroscopic fields rho (N), actual velocity u (dim planes
 * of N) and temperature T (N), host arrays.  The force F0 = -div K(rho) follows from
 * rho; the gauge velocity is u - F0 dt/(2 rho); the stored populations are the
 * collision of the equilibrium populations f = rho W, g = g^eq (eqs. 7, 16-22).
 * Before returning, the call records the HIP graphs that pond_step replays (fused
 * step: runs of 45 and of 3 steps from each of the three ring slots; two kernels: runs
 * of 16 and of 2 steps from either state buffer), so that stepping itself captures and
 * instantiates nothing.
 * Errors: POND_E_INVALID (NULL pointer), POND_E_PRESSURE / POND_E_NONFINITE when a
 * node is outside the EoS domain or a field holds NaN or Inf (state then undefined,
 * handle not initialised). */
int pond_init_fields(pond_handle *h, const double *rho, const double *u, const double *T);

/* Advance nsteps >= 0 time steps, then synchronise the stream.  Returns the first
 * error met; the state is then that of the last completed step. */
int pond_step(pond_handle *h, int nsteps);

/* Macroscopic fields of the current state into host arrays (any may be NULL):
 * rho = sum_i f_i; u = u_gauge + F dt/(2 rho) (the actual velocity u-hat, eq. 17 and
 * App. F); p = rho theta T_L; T from the EoS (T0 when isothermal); E = e + |u|^2/2
 * (dim planes for u). */
int pond_moments(pond_handle *h, double *rho, double *u, double *T, double *p, double *E);

/* Conservation monitors of the current state (eq. 2 and App. F), FP64 sums in a
 * fixed order: out[0] = sum rho, out[1..dim] = sum rho u-hat, out[dim+1] = sum rho E,
 * out[dim+2] = sum (rho E + kappa |grad rho|^2/2), out[dim+3] = min p,
 * out[dim+4] = max over nodes and directions of |v_i| dt.  out holds dim + 5 values. */
int pond_monitors(pond_handle *h, double *out);

/* Number of completed steps since the last pond_init_fields. */
int pond_steps_done(const pond_handle *h, long long *out);

/* Human-readable description of the last error of the handle (never NULL). */
const char *pond_last_error(const pond_handle *h);

/* Tile shape in use by the streaming kernel: out[0] = shape index, out[1], out[2] =
 * receivers per workgroup along x and y; out[3] = number of compiled shapes for the
 * handle's dimension. */
int pond_tile_info(const pond_handle *h, int *out);

/* Release everything owned by h.  NULL is accepted. */
int pond_destroy(pond_handle *h);

/* Checkpoint / resume.  A checkpoint holds the current state of the last completed step
 * (fused step: the streamed-state moment planes; two kernels and D3Q27: the stored
 * populations and side fields; in the handle's precision), the step count, the step form,
 * the streaming tile shape in use and the configuration it belongs to.  Loading it into a
 * handle of the same configuration and stepping on gives bitwise the results the saving
 * handle gets (the handle adopts the checkpoint's tile shape for that).
 *
 * pond_checkpoint_size: bytes of a checkpoint of h (depends only on the configuration).
 * pond_save: write the checkpoint of h's current state into the caller-owned host buffer
 *   buf of at least that many bytes.  Errors: POND_E_INVALID (NULL, buffer too small),
 *   POND_E_STATE (not initialised).
 * pond_load: make the state of buf current in h, as if h had just completed the saved
 *   number of steps; clears the error state and records the step graphs as
 *   pond_init_fields does.  Errors: POND_E_INVALID (NULL, buffer too
 *   small, not a checkpoint, or saved from another lattice shape, precision, step form or
 *   set of parameters), POND_E_STATE (h is a member of a batch). */
int pond_checkpoint_size(const pond_handle *h, unsigned long long *bytes);
int pond_save(pond_handle *h, void *buf, unsigned long long bytes);
int pond_load(pond_handle *h, const void *buf, unsigned long long bytes);

/* Measurement: launch kernel `which` (0 = streaming with the predictor-corrector,
 * 1 = Korteweg force, closure and collision) `reps` times back to back on the
 * handle's stream on the current state and return the mean duration per launch in
 * microseconds, from HIP events recorded on that stream.  The launches read the
 * current state and overwrite only scratch planes and the next-state buffer, so the
 * state is unchanged.  Errors: POND_E_STATE (not initialised), POND_E_INVALID. */
int pond_time_kernel(pond_handle *h, int which, int reps, double *avg_us);

/* Measurement: advance nsteps >= 1 time steps exactly as pond_step does, but with
 * the kernels launched one by one, each with a pair of HIP events that the runtime
 * records at that kernel's start and end on the handle's stream; kernel_us[0] and
 * kernel_us[1] receive the mean duration of the streaming kernel and of the
 * force/collision kernel inside the step pipeline.
 * Errors and state as for pond_step. */
int pond_step_timed(pond_handle *h, int nsteps, double *kernel_us);

/* Device bytes that pond_create allocates for cfg (all state, scratch and monitor
 * buffers; HIP's own allocation granularity not included).  For admission control of
 * many resident lattices.  Errors: POND_E_INVALID as for pond_create. */
int pond_footprint(const pond_config *cfg, unsigned long long *bytes);

/* ---------------------------------------------------------------------------
 * Batches: many independent lattices advanced together.  Every step of a batch is
 * one launch of each step kernel per group of members that share dim, precision and
 * streaming tile shape, over the tiles of all of them; each member keeps its own
 * device state, parameters, error flags and step counter, so its results are
 * bitwise those of pond_step on the same handle alone.  The main-text time step of
 * each lattice is unchanged (eqs. 1-22); batching is scheduling only.
 * --------------------------------------------------------------------------- */

/* Create an empty batch whose steps run on `stream` (a hipStream_t; NULL = a
 * library-owned stream).  Errors: POND_E_INVALID (out NULL), POND_E_NOMEM,
 * POND_E_DEVICE. */
int pond_batch_create(void *stream, pond_batch **out);

/* Add an initialised handle that is in no batch.  While it is a member, pond_step,
 * pond_step_timed, pond_time_kernel and pond_init_fields refuse the handle
 * (POND_E_STATE); pond_moments, pond_monitors, pond_steps_done, pond_last_error and
 * pond_tile_info work as usual, and pond_destroy removes it first.  The handle's
 * stream is synchronised before it joins.  Errors: POND_E_INVALID (NULL, already
 * a member of a batch, a D3Q27 lattice, or its group would exceed 2^21 workgroups
 * per launch),
 * POND_E_STATE (not initialised or in the error state), POND_E_NOMEM. */
int pond_batch_add(pond_batch *b, pond_handle *h);

/* Remove a member (its state and step count are kept).  Errors: POND_E_INVALID when
 * h is not a member of b. */
int pond_batch_remove(pond_batch *b, pond_handle *h);

/* Advance every member nsteps >= 0 time steps, then synchronise.  A member that fails
 * is left as pond_step leaves a failed handle (state of its last completed step,
 * error state, pond_last_error set) and leaves the batch; the others complete all
 * nsteps.  Returns POND_OK when every member completed, else the status of the
 * first failed member in order of addition (POND_E_PRESSURE, POND_E_NONFINITE,
 * POND_E_HALO), or POND_E_DEVICE. */
int pond_batch_step(pond_batch *b, int nsteps);

/* Number of members. */
int pond_batch_size(const pond_batch *b, int *out);

/* Remove all members and release the batch.  NULL is accepted. */
int pond_batch_destroy(pond_batch *b);

/* ---------------------------------------------------------------------------
 * Stepping without device allocation.  For callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the caller owns the two state buffers, and every other buffer a step
 * needs lives in a static device array of POND_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends.
 * --------------------------------------------------------------------------- */
#define POND_NOALLOC_SCRATCH_BYTES (64ull * 1024ull * 1024ull)

/* Advance a 1D or 2D lattice nsteps >= 0 time steps with the two-kernel step of pond_step
 * (cfg->two_kernel must be 1: the state is stored populations), on the current device
 * and cfg->stream, then synchronise that stream.  Allocates no device memory and records
 * no graph.
 *   state0, state1  device buffers of one state each (caller-owned, read and written):
 *                   the population planes, then the five FP64 side planes u_x, u_y,
 *                   theta, F_x, F_y of N values each.  Populations: FP64, the 2Q planes
 *                   f_0..f_{Q-1}, g_0..g_{Q-1}; FP32 forms, the 2Q FP32 deviation planes
 *                   f_q - W_q sum f, g_q - W_q sum g, then the two FP64 sum planes.  A
 *                   checkpoint of the same configuration (pond_save) holds one such
 *                   buffer after its header, whose size is pond_checkpoint_size minus
 *                   the bytes of a state buffer.  8-byte alignment is required.  1D
 *                   lattices neither read nor write the planes u_y and F_y.
 *   *cur            in: 0 or 1, the buffer holding the current state; out: the buffer
 *                   holding the last completed state.
 *   *done           out (may be NULL): the number of completed steps.
 * cfg->tile selects the streaming tile shape (-1: shape 0, nothing is measured); the
 * results are bitwise those of pond_step on a handle of the same configuration and
 * tile shape.  The scratch holds 4096 bytes plus the streamed-state moment planes,
 * 18 (2D) or 6 (1D) FP64 values per node, so 2D lattices of up to 466 005 nodes fit.
 * All calls on one GPU share its scratch array: calls that overlap in time on the
 * same GPU (other threads, or other streams before this call's synchronisation) race
 * and give undefined results.  Each call sets up its scratch contents itself.
 * Errors: POND_E_INVALID (cfg as for pond_create, dim 3, two_kernel 0, NULL buffers, *cur
 * not 0 or 1, nsteps < 0), POND_E_SCRATCH (the lattice needs more than the scratch array; nothing
 * is launched), POND_E_DEVICE, and the step errors of pond_step (POND_E_PRESSURE,
 * POND_E_NONFINITE, POND_E_HALO), after which *cur is the last completed state. */
int pond_step_noalloc(const pond_config *cfg, void *state0, void *state1, int *cur, int nsteps, int *done);

#ifdef __cplusplus
}
#endif

#endif /* POND_H */
