/*
 * dmrt.h -- C ABI of libdmrt: the double-MRT thermal lattice Boltzmann time
 * step of Z. Li, M. Yang and Y. Zhang, "Double MRT Thermal Lattice Boltzmann
 * Method for Simulating Natural Convection of Low Prandtl Number Fluids"
 * (arXiv:1601.04633), on AMD MI355X (gfx950).
 *
 * Problem (Section 2, Eqs. 1-8 and 14-17): a square cavity of side H filled
 * with a Boussinesq fluid, left wall hot, right wall cold, top and bottom
 * adiabatic, no slip everywhere; governed by Ra, Pr and the lattice Mach
 * number Ma (Eq. 9).  Outputs: U, V, theta, P (Eq. 9) and the wall Nusselt
 * number (Eqs. 18-19).
 *
 * Method (Section 3): per node and step, a D2Q9 MRT collision with the
 * Boussinesq force (Eqs. 22-34), a D2Q5 MRT collision for the temperature
 * (Eqs. 35-43), streaming, and halfway bounce-back walls (no-slip for the
 * flow; Eq. 44 adiabatic and Eq. 45 isothermal for the temperature).
 *
 * Conventions shared by every call
 *  - Lattice units: dx = dt = c = 1, c_s^2 = 1/3, rho0 = 1.  The grid has
 *    n x n nodes; the walls lie half a link outside the outer nodes, so
 *    H = n and node (x, y) sits at X = (x + 1/2)/n, Y = (y + 1/2)/n.
 *  - Host field arrays are double, n*n, y-major with x fastest
 *    (index y*n + x).  They are caller-owned.
 *  - theta is stored shifted so that the default walls are +0.5 / -0.5;
 *    the paper's theta (0 at the cold wall, 1 at the hot wall) is
 *    theta + 1/2 for those defaults.
 *  - Return value: DMRT_OK (0) or a negative error code.  No call throws.
 *    After an error the handle stays valid unless stated otherwise.
 *  - Threading: one host thread at a time per handle.  dmrt_step and the
 *    set-up calls only enqueue work on the handle's stream; calls that
 *    return host data synchronise that stream.
 *  - Device memory: the library owns everything it allocates.  External
 *    distribution buffers passed to dmrt_create stay owned by the caller,
 *    who must keep them alive until dmrt_destroy.
 *
 * Readings of the paper that this library implements (the paper's text is
 * garbled or silent at these places):
 *  - Eq. 34: the energy moment equilibrium is -2 drho + 3 rho0 |u|^2.
 *  - Eq. 37: the last row of N is (0, 1, -1, 1, -1).
 *  - Eq. 26: F_i = 3 G.(e_i - u) f_i^eq(rho0, u)  (divisor rho0 c_s^2).
 *  - Eq. 27: G = (force_x, gbeta (theta - theta_ref)).
 *  - Eqs. 40/43: by default a is fixed and sigma_k solved from Eq. 43, with
 *    sigma_e = sigma_nu from Eq. 39 (DMRT_Q5_FIXED_A); DMRT_Q5_PAPER takes
 *    Eq. 40 literally and requires the resulting a < 1.
 *  - Eq. 45: the anti-bounce-back constant is (4 + a)/10 theta_w.
 *  - Eq. 18: second-order one-sided wall gradient
 *    Nu(y) = H (8 theta_w - 9 theta(0, y) + theta(1, y)) / (3 dT).
 */
#ifndef DMRT_H
#define DMRT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes */
#define DMRT_OK           0
#define DMRT_EINVAL      -1  /* NULL pointer, bad size or mode, non-finite input */
#define DMRT_EUNSTABLE   -2  /* parameters outside the scheme's stable range     */
#define DMRT_ENOMEM      -3  /* host or device allocation failed                 */
#define DMRT_EHIP        -4  /* a HIP runtime call failed (see dmrt_last_error)   */
#define DMRT_ENONFINITE  -5  /* the state holds NaN or Inf (watchdog)            */
#define DMRT_ENODEV      -6  /* no usable gfx950 device                          */

/* Storage and arithmetic precision of the distributions */
#define DMRT_FP32 0
#define DMRT_FP64 1

/* D2Q5 parameterisation (Eqs. 38-43) */
#define DMRT_Q5_FIXED_A 0   /* a given; sigma_k from Eq. 43; sigma_e = sigma_nu from Eq. 39 */
#define DMRT_Q5_PAPER   1   /* Eq. 40 literally; a = 20 sqrt(3) alpha - 4, must be < 1     */

/* Collision operator.  MRT is the paper's scheme (Eqs. 28 and 36).  LBGK is
 * the double single-relaxation-time scheme the paper's introduction
 * contrasts it with: every non-conserved moment of f relaxes at s_nu
 * (s_q = s_nu) and every non-conserved moment of g at sigma_k
 * (sigma_e = sigma_nu = sigma_k), which is the BGK collision
 * f* = f - s_nu (f - f^eq) + F, g* = g - sigma_k (g - g^eq) written in
 * moment space; same kernels, same cost. */
#define DMRT_COLL_MRT  0
#define DMRT_COLL_LBGK 1

/* Wall configuration.  CAVITY is the paper's problem; the others are test
 * boxes that share the same kernel: PERIODIC (no walls), CHANNEL_X
 * (periodic in x, no-slip adiabatic walls at y = 0 and y = n) and
 * ADIABATIC_BOX (no-slip adiabatic walls on all four sides). */
#define DMRT_BC_CAVITY        0
#define DMRT_BC_PERIODIC      1
#define DMRT_BC_CHANNEL_X     2
#define DMRT_BC_ADIABATIC_BOX 3

typedef struct {
    int    n;               /* nodes per side, >= 4; 14 planes of the state must  *
                             * stay under 4 GiB: n <= 8747 (FP32), 6177 (FP64)     */
    double Ra, Pr, Ma;      /* Eq. 9; all > 0                                      */
    double theta_hot;       /* hot-wall temperature (default +0.5)                 */
    double theta_cold;      /* cold-wall temperature (default -0.5)                */
    int    precision;       /* DMRT_FP32 or DMRT_FP64                              */
    int    q5_mode;         /* DMRT_Q5_FIXED_A or DMRT_Q5_PAPER                    */
    double a;               /* D2Q5 parameter a of Eq. 42 in FIXED_A mode (-2/3)   */
    int    bc_mode;         /* DMRT_BC_*                                           */
    double gbeta_override;  /* NaN: g beta = Ma^2 / (3 H dT) from Eq. 9; else used */
    double force_x;         /* constant horizontal body force (test modes only;    *
                             * DMRT_BC_CAVITY requires 0, else EINVAL), 0          */
    double theta_ref;       /* reference temperature of Eq. 27 (default 0)         */
    int    collision;       /* DMRT_COLL_MRT (default) or DMRT_COLL_LBGK           */
} dmrt_params;

/* Derived lattice parameters (Eqs. 9, 11-13, 32, 38-43). */
typedef struct {
    double nu, alpha, gbeta;            /* viscosity, diffusivity, g beta            */
    double s_nu, s_q;                   /* Eq. 32 (s_e = s_eps = s_nu)               */
    double sigma_k, sigma_e, sigma_nu;  /* Eq. 38                                    */
    double a;                           /* Eq. 42                                    */
    double w0, wm;                      /* D2Q5 equilibrium weights (1-a)/5, (4+a)/20 */
    double H;                           /* = n                                       */
} dmrt_derived;

typedef struct dmrt_cavity dmrt_cavity;   /* opaque, library-owned */

/* Fill *p with the defaults: n = 64, Ra = 1e3, Pr = 0.01, Ma = 0.1, walls
 * +-0.5, FP64, FIXED_A with a = -2/3, CAVITY, gbeta derived, no force_x,
 * theta_ref = 0, MRT collision.  Returns DMRT_EINVAL if p is NULL. */
int dmrt_params_default(dmrt_params *p);

/* Parameter map of Eq. 9 / Eqs. 11-13 (H = n, c_s^2 = 1/3):
 *   nu = Ma H sqrt(Pr / (3 Ra)), alpha = nu / Pr, g beta = Ma^2 / (3 H dT);
 * Eq. 32 for s_nu, s_q; Eqs. 39-43 for sigma_k, sigma_e, sigma_nu and a.
 * Host only, touches no device.  DMRT_EINVAL for NULL or non-finite input,
 * n < 4 or n above the size limit of dmrt_params.n, or a horizontal force
 * in the cavity; DMRT_EUNSTABLE for Ma, Ra or Pr <= 0, a outside (-4, 1), or any
 * relaxation rate outside (0, 2). */
int dmrt_derive(const dmrt_params *p, dmrt_derived *out);

/* Bytes that external distribution buffers must provide for these
 * parameters: f_bytes for both ping-pong copies of the 9 D2Q9 planes,
 * g_bytes for both copies of the 5 D2Q5 planes.  Layout of each buffer:
 * [copy 0..1][population][y 0..n-1][x 0..pitch-1], pitch = n rounded up to
 * a multiple of 64 elements, element = float (FP32) or double (FP64).
 * The stored f is the deviation from w_i rho0 (Eq. 33: sum f = drho). */
int dmrt_buffer_bytes(const dmrt_params *p, size_t *f_bytes, size_t *g_bytes);

/* Create a cavity on the current HIP device.  ext_f / ext_g: NULL to let
 * the library allocate, or device pointers of at least dmrt_buffer_bytes
 * bytes, 256-byte aligned (both NULL or both non-NULL).  hip_stream: the
 * hipStream_t to enqueue on, or NULL for a library-created stream.  The
 * state starts at rest with theta = 0 (call dmrt_set_theta to change it).
 * Errors: EINVAL, EUNSTABLE (as dmrt_derive), ENOMEM, EHIP, ENODEV. */
int dmrt_create(const dmrt_params *p, void *ext_f, void *ext_g, void *hip_stream,
                dmrt_cavity **out);

/* Re-initialise at rest: pre-collision f = 0 (drho = 0, u = 0) and g at the
 * D2Q5 equilibrium of theta0 (n*n host doubles), then one collision; the
 * step counter is reset to 0.  Enqueued; theta0 may be reused on return. */
int dmrt_set_theta(dmrt_cavity *h, const double *theta0);

/* Re-initialise at the equilibria of the given fields (Eqs. 34, 42): drho,
 * U, V, theta are n*n host doubles, any of them NULL for zero. */
int dmrt_set_equilibrium(dmrt_cavity *h, const double *drho, const double *U,
                         const double *V, const double *theta);

/* Hot-wall temperature per row, theta_w(y) for y = 0..n-1 (n host doubles),
 * used by Eq. 45 on the left wall and by the hot-wall Nusselt number.
 * Takes effect from the next step. */
int dmrt_set_hot_wall(dmrt_cavity *h, const double *theta_w);

/* Advance nsteps >= 0 time steps (Eqs. 25 and 36 with the walls).  Enqueued
 * only; long runs replay a captured graph of the step kernel.  Each call
 * with nsteps > 0 runs a watchdog check of the populations of the two
 * isothermal-wall columns of the state it starts from (a non-finite value
 * anywhere reaches one of them within n steps), in extra workgroups of its
 * first launch, or as a launch of its own when the call starts with a graph
 * replay.  When a check has found a non-finite value, dmrt_step returns
 * DMRT_ENONFINITE and enqueues nothing; the report is asynchronous (it comes
 * from a later call once the check has run, or from dmrt_sync).
 * dmrt_set_theta, dmrt_set_equilibrium and dmrt_load_state clear it. */
int dmrt_step(dmrt_cavity *h, long nsteps);

/* Wait for all work enqueued on the handle's stream, after a watchdog check
 * of the current state when steps were taken since the last one.  Returns
 * DMRT_ENONFINITE when a check has found a non-finite state (then up to
 * date). */
int dmrt_sync(dmrt_cavity *h);

/* Steps taken since the last (re)initialisation. */
int dmrt_get_step(dmrt_cavity *h, long *step);

/* Fields at the current step (Eq. 9, Eq. 33, Eq. 41): U = u, V = v
 * (U = u / (sqrt(3) c_s)), theta, P = drho / 3.  Any output may be NULL.
 * Synchronises.  u is the velocity of Eq. 33 (first moment of the
 * pre-collision populations over rho0). */
int dmrt_get_fields(dmrt_cavity *h, double *U, double *V, double *theta, double *P);

/* Wall Nusselt number (Eqs. 18-19, second-order wall gradient, midpoint
 * rule over the n rows).  wall 0: hot wall x = 0; wall 1: cold wall x = H,
 * where Nu = -dtheta/dX as well (heat flowing out).  nu_local: n doubles or
 * NULL.  Synchronises. */
int dmrt_nusselt(dmrt_cavity *h, int wall, double *nu_avg, double *nu_local);

/* Record the hot-wall Nu_avg on the device every `stride` steps (counted
 * from the last initialisation), into a ring of `cap` doubles; stride 0
 * switches recording off.  Resets the ring.  With K steps per launch the
 * launches take the samples due on their steps and one small kernel per
 * dmrt_step chunk (and per 32 samples) appends them; device memory: 64 n
 * doubles of sample slots besides the ring. */
int dmrt_nu_series(dmrt_cavity *h, int stride, long cap);

/* Copy the recorded samples, oldest first, into out (room for cap doubles);
 * *count receives how many were copied (at most cap; older ones are
 * overwritten).  Synchronises. */
int dmrt_nu_series_read(dmrt_cavity *h, double *out, long *count);

/* Relative change of theta and of (U, V) since the previous call (or since
 * initialisation): ||x_now - x_prev||_2 / ||x_now||_2, accumulated in FP64
 * on the device, then the reference is updated.  Returns DMRT_ENONFINITE
 * if any distribution is NaN or Inf.  Synchronises. */
int dmrt_residual(dmrt_cavity *h, double *res_theta, double *res_u);

/* dmrt_residual for callers that cannot allocate device memory (serving
 * loops, harnesses that forbid hipMalloc): the same quantities and the same
 * kernels, with no hipMalloc or hipFree in the call.
 *  ref: caller-owned device memory of 3 n^2 doubles (8-byte aligned) with
 *    the previous theta, U and V (Eq. 33 velocity), y-major; read, then
 *    overwritten with the current fields.  Zero it before the first call
 *    (which then returns 1 and 1).  The caller keeps its size right: the
 *    library cannot check it.
 *  The FP64 partial sums live in a library-owned device array of fixed size
 *  (at most 1024 workgroup partials: 41,000 bytes on each device the call
 *  runs on, held until the process ends).  The reduction uses at most 1024
 *  workgroups whatever n, so every cavity fits; EINVAL if it would not.
 *  Every call on one device shares that array and leaves its last contents
 *  there: calls that overlap on one device (several host threads or
 *  streams) race and must be serialised by the caller.
 * Returns DMRT_ENONFINITE as dmrt_residual.  EINVAL for NULL h or ref or a
 * misaligned ref.  Synchronises the handle's stream. */
int dmrt_residual_noalloc(dmrt_cavity *h, double *ref, double *res_theta, double *res_u);

/* Host checkpoint of the complete state (distributions at the current step,
 * step counter, hot-wall profile).  dmrt_state_bytes gives the size;
 * dmrt_load_state requires a blob saved with the same n and precision and
 * resumes bitwise identically.  Both synchronise. */
int dmrt_state_bytes(dmrt_cavity *h, size_t *bytes);
int dmrt_save_state(dmrt_cavity *h, void *host, size_t bytes);
int dmrt_load_state(dmrt_cavity *h, const void *host, size_t bytes);

/* Launch shape of the step kernel: block_x in {64, 128, 256, 512},
 * block_y >= 1 with block_x * block_y <= 1024, xcd_remap 0/1 (assign
 * contiguous tiles to each of the 8 accelerator dies), graph_steps >= 0
 * (steps per captured graph; 0 = never capture).  Defaults at creation:
 * 256 x 1, die-aware order, graphs of 60 steps (a multiple of every
 * steps-per-launch K offered).  Results do not depend on the launch shape. */
int dmrt_set_launch(dmrt_cavity *h, int block_x, int block_y, int xcd_remap,
                    int graph_steps);

/* Steps per launch K of dmrt_step: 1 (one fused kernel per step) or 2..4
 * (K steps per launch through LDS: each workgroup computes the intermediate
 * steps on its 64 x tile_rows footprint, shrinking by one node per step, and
 * keeps them in LDS; every population is read and written once per launch,
 * so HBM traffic per node update drops from 28 to about 28/K words plus
 * halo).  tile_rows in {4, 6, 10, 16} for K <= 2, {6, 10, 12, 14, 16} for
 * K = 3, {10, 12, 14, 16} for K = 4.  K >= 2 is available for
 * DMRT_BC_CAVITY only (EINVAL otherwise).  Results are identical to
 * single steps; Nusselt samples are still taken after every stride-th step
 * (a sample due on any step of a launch is taken by that launch, with the
 * same value as after a single step, and appended to the ring, in order, by
 * the end of the dmrt_step call's enqueued work).
 * Default at creation: K = 1.  On MI355X K = 4 with 16 rows is the fastest
 * tile shape from about 512^2 up, 12 rows below that; from 1024^2 up the
 * marching form (dmrt_set_temporal_march) is faster. */
int dmrt_set_temporal(dmrt_cavity *h, int steps_per_launch, int tile_rows);

/* K = steps_per_launch steps per launch of dmrt_step with workgroups that
 * march up the rows (the same time steps, Eqs. 25-45, as dmrt_set_temporal,
 * with less recomputed halo).  Each workgroup holds K groups of group_rows
 * wavefronts, group j computing step t + j on rows that trail group j - 1
 * by group_rows + 1, with the newest group_rows + 2 rows of each
 * intermediate step in an LDS ring; it owns 64 - 2(K - 1) columns and
 * chunk_rows rows, so the halo recomputed at the K - 1 rows of each chunk
 * end replaces the one of each 16-row tile.  The first group gathers the
 * row of its next iteration from global memory one iteration ahead.
 * (K, group_rows) in {(2, 8), (3, 2), (3, 4), (4, 1), (4, 2), (4, 3),
 * (4, 4), (6, 2)} (the LDS rings, (K - 1) x 14 x (group_rows + 2) x 64
 * elements, fit 160 KB in both precisions); chunk_rows >= 1 (clamped to n),
 * or 0 to pick the largest chunk that keeps one launch's workgroups
 * resident on the device at once.  DMRT_BC_CAVITY only (EINVAL otherwise).
 * Results are identical to single steps.  The adjoint's forward run uses
 * the same launches, except in the objective window, where it takes the
 * tile form's Nusselt-accumulating launches when K <= 4 and single steps
 * otherwise.
 * dmrt_set_temporal switches the marching off.  EHIP if the device query for
 * chunk_rows = 0 fails.  On MI355X with chunk_rows = 0: K = 4 with 3 rows
 * (FP32) or 4 rows (FP64) is the fastest at 1024^2, K = 6 with 2 rows at
 * 2048^2 (where the state no longer fits the last-level cache and fewer
 * launches per step pay); below about 512^2 the tile kernel of
 * dmrt_set_temporal is faster. */
int dmrt_set_temporal_march(dmrt_cavity *h, int steps_per_launch, int group_rows, int chunk_rows);

/* The marching mode of dmrt_set_temporal_march: group_rows (0 when off) and
 * the rows per workgroup in use (0 when off).  Either pointer may be NULL. */
int dmrt_get_temporal_march(const dmrt_cavity *h, int *group_rows, int *chunk_rows);

/* Device pointers of the two ping-pong copies and the index (0/1) of the
 * copy holding the current state; for callers that manage memory. */
int dmrt_buffers(dmrt_cavity *h, void **f, void **g, int *current);

/* Release the handle and the device memory the library allocated.  Waits
 * for pending work.  NULL is accepted. */
int dmrt_destroy(dmrt_cavity *h);

/* ------------------------------------------------------------------------
 * Gradient of the time-averaged hot-wall Nusselt number (reverse mode).
 * Objective: J = mean of Nu_avg (Eqs. 18-19, hot wall) over the last
 * avg_last of nsteps steps, started from the rest state with the
 * temperature field theta0 of the last dmrt_set_theta (set_equilibrium with
 * only theta also qualifies).  Gradients with respect to the hot-wall
 * profile theta_w(y) (Eq. 45 and Eq. 18) and theta0.  Only DMRT_BC_CAVITY.
 * The forward stores a checkpoint every ckpt_every steps; the backward
 * recomputes each segment from its checkpoint, keeping of every step only
 * the point the collision Jacobian depends on (the u, v and theta of the
 * pre-collision state), and runs the hand-written adjoint step kernel (the
 * discrete adjoint of the step: the transposed collision Jacobian at each
 * node, then the transposed streaming and wall map).  Device memory:
 * ceil(nsteps/ckpt_every) + 4 states of 14 n^2 elements and 2 ckpt_every
 * points of 3 n^2 elements (plus n^2 + 2 n doubles), held until
 * dmrt_adjoint_release or dmrt_destroy.
 * ------------------------------------------------------------------------ */

/* Forward run: re-initialises from theta0, advances nsteps (the handle ends
 * at step nsteps) and returns J (FP64).  EINVAL if no rest-state theta0 was
 * set, if 1 <= avg_last <= nsteps or ckpt_every >= 1 fails, or for a
 * non-cavity handle.  Synchronises. */
int dmrt_adjoint_forward(dmrt_cavity *h, long nsteps, long avg_last, long ckpt_every, double *J);

/* Backward run after dmrt_adjoint_forward: dJ_dthetaw (n doubles) and
 * dJ_dtheta0 (n*n doubles, y-major), either may be NULL.  The parameter
 * gradient is accumulated in FP64 on the device.  Synchronises.  EINVAL when
 * no forward run is stored, or when it no longer matches the handle:
 * dmrt_set_hot_wall, dmrt_set_theta, dmrt_set_equilibrium or
 * dmrt_load_state since the last dmrt_adjoint_forward (the backward would
 * linearise about another wall or initial field), or a launch-mode call
 * that released the adjoint buffers (dmrt_set_launch, dmrt_set_temporal,
 * dmrt_set_temporal_march, dmrt_adjoint_set_temporal,
 * dmrt_adjoint_release).  Stepping the handle does not affect it. */
int dmrt_adjoint_backward(dmrt_cavity *h, double *dJ_dthetaw, double *dJ_dtheta0);

/* Generation of the forward run that the next dmrt_adjoint_backward would
 * differentiate: 1 for the handle's first successful dmrt_adjoint_forward,
 * increasing by one with each later one; 0 when no forward run is stored
 * or it was invalidated (see dmrt_adjoint_backward).  Lets a caller that
 * keeps several objectives of one handle check that the stored run is its
 * own.  Host only. */
int dmrt_adjoint_generation(const dmrt_cavity *h, long *gen);

/* dmrt_adjoint_forward followed by dmrt_adjoint_backward. */
int dmrt_adjoint_nu(dmrt_cavity *h, long nsteps, long avg_last, long ckpt_every, double *J,
                    double *dJ_dthetaw, double *dJ_dtheta0);

/* Adjoint steps (and recompute steps) per backward launch: 1, or 2..4
 * through LDS with footprints of 64 x tile_rows threads (the same pairs as
 * dmrt_set_temporal).  The gradients do not depend on it (bitwise).
 * Releases the adjoint buffers.  EINVAL for an unsupported pair or a
 * non-cavity handle.  Synchronises. */
int dmrt_adjoint_set_temporal(dmrt_cavity *h, int steps_per_launch, int tile_rows);

/* Free the checkpoint, segment and adjoint buffers. */
int dmrt_adjoint_release(dmrt_cavity *h);

/* ------------------------------------------------------------------------
 * Batched sweep: many independent cavities (the paper's Ra x Pr study,
 * Section 4 and Table 1, run as one workload).  Every member is a cavity
 * (DMRT_BC_CAVITY) with its own n, Ra, Pr, Ma and walls; all members share
 * one precision.  One launch per step advances every member; each member
 * evolves bitwise as the same cavity would under dmrt_step.
 * ------------------------------------------------------------------------ */
typedef struct dmrt_batch dmrt_batch;   /* opaque, library-owned */

/* p: array of `count` parameter sets (1 <= count <= 65535).  Members start
 * at rest with theta = 0.  Errors: as dmrt_create for any member, EINVAL
 * for mixed precision or a non-cavity member. */
int dmrt_batch_create(const dmrt_params *p, int count, void *hip_stream, dmrt_batch **out);

/* Re-initialise member `index` at rest with temperature theta0 (n*n host
 * doubles of that member); the batch step counter is unchanged and a
 * member marked dead is revived. */
int dmrt_batch_set_theta(dmrt_batch *b, int index, const double *theta0);

/* Hot-wall temperature profile of member `index` (n host doubles). */
int dmrt_batch_set_hot_wall(dmrt_batch *b, int index, const double *theta_w);

/* Schedule of the batched launch (results do not depend on it):
 *  block_x in {64,128,256,512}, block_y >= 1, block_x*block_y <= 1024:
 *    workgroup tile of block_x x block_y nodes of one member;
 *  order: 0 members in the given order, 1 largest first, 2 tiles of the
 *    members of a group interleaved round-robin;
 *  grid_blocks: workgroups per launch, 0 = one per tile, else a persistent
 *    grid-stride launch of that many workgroups;
 *  group_bytes: 0 = one group; else members are packed in order into
 *    groups of at most this much state (both copies), and
 *  group_steps >= 1: each group advances this many steps before the next
 *    group runs (also the number of steps per captured graph; even values
 *    enable graph replay). */
int dmrt_batch_set_schedule(dmrt_batch *b, int block_x, int block_y, int order, int grid_blocks,
                            size_t group_bytes, int group_steps);

/* Steps per launch K of dmrt_batch_step for every member: 1, or 2..4
 * through LDS as dmrt_set_temporal (same tile_rows rules); each group
 * advances its group_steps K at a time (the remainder one at a time).
 * Results do not depend on it. */
int dmrt_batch_set_temporal(dmrt_batch *b, int steps_per_launch, int tile_rows);

/* K = steps_per_launch steps per launch with the row-marching sweep of
 * dmrt_set_temporal_march (same Eqs. 25-45, same (K, group_rows) pairs and
 * LDS rings): every workgroup takes one member's column band and chunk of
 * rows, so each member evolves bitwise as it would alone.  chunk_rows >= 1
 * rows per workgroup for every member of a group, or 0 for, per group, the
 * shortest chunk that leaves all of the group's workgroups resident on the
 * device at once.  The table deals each die a contiguous range of
 * workgroups.  Remainders of a group's steps go one per launch.
 * dmrt_batch_set_temporal switches the marching off.  EINVAL for a pair
 * not built or whose rings exceed 160 KB in the batch's precision; EHIP if
 * the device query for chunk_rows = 0 fails. */
int dmrt_batch_set_temporal_march(dmrt_batch *b, int steps_per_launch, int group_rows, int chunk_rows);

/* Advance every live member nsteps >= 0 steps.  Enqueued only. */
int dmrt_batch_step(dmrt_batch *b, long nsteps);
int dmrt_batch_sync(dmrt_batch *b);
int dmrt_batch_get_step(dmrt_batch *b, long *step);

/* Hot-wall Nu_avg (Eqs. 18-19) of every member into nu_avg[count], reduced
 * on the device in FP64; NaN for dead members.  Synchronises. */
int dmrt_batch_nusselt(dmrt_batch *b, double *nu_avg);

/* Per-member status into status[count]: DMRT_OK, or DMRT_ENONFINITE when
 * the member's state holds NaN/Inf.  Such members are marked dead and
 * skipped by later steps; the others continue.  Synchronises. */
int dmrt_batch_status(dmrt_batch *b, int *status);

/* Fields of member `index` as dmrt_get_fields.  Synchronises. */
int dmrt_batch_get_fields(dmrt_batch *b, int index, double *U, double *V, double *theta,
                          double *P);

/* Raw post-collision distributions of member `index` at the current step:
 * host_f gets 9*n*n, host_g 5*n*n elements of the batch precision,
 * [population][y][x]; either may be NULL.  Synchronises. */
int dmrt_batch_member_state(dmrt_batch *b, int index, void *host_f, void *host_g);

/* Overwrite member `index`'s current distributions from host arrays laid
 * out as dmrt_batch_member_state returns them (a per-member checkpoint
 * restore); revives a dead member.  Synchronises. */
int dmrt_batch_load_member_state(dmrt_batch *b, int index, const void *host_f,
                                 const void *host_g);

int dmrt_batch_destroy(dmrt_batch *b);

/* Static description of an error code. */
const char *dmrt_strerror(int code);

/* Text of the last HIP error seen by this thread (empty if none). */
const char *dmrt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DMRT_H */
