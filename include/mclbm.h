/*
 * mclbm: moment-chain lattice Boltzmann method for hyperelastic solids on
 * AMD Instinct MI355X (gfx950).  C ABI of the device library.
 *
 * The method (arXiv 2502.00920): a D2Q9 lattice (Tab. 1) carries the moment
 * chain r, j, Pi of a solid in the reference configuration (Sect. 3.1); the
 * part of the first Piola-Kirchhoff stress P(H) that the bare chain does not
 * carry enters through the forcing term psi with the source
 * S = rho0 b + Div(P(H) + Pi(H)) (Eq. source, Eq. forcing); BGK collision and
 * streaming (Algorithm 1) run with modified bounce-back walls that prescribe a
 * momentum j* (Eq. bbcon) and modified anti-bounce-back walls that prescribe a
 * traction T* (Eq. abbcon, Sect. 3.3); the displacement follows from j by the
 * trapezoidal rule (Sect. 3.2).  Materials: St. Venant-Kirchhoff and neo-Hooke
 * (Sect. 4), plane strain; a linear-elastic material for tests.
 *
 * Units: the lattice velocity c = sqrt(3) c_s with c_s = sqrt(mu/rho0)
 * (Sect. 3.2) and c = dX/dt (Sect. 2), so dt is derived from dx, mu and rho0;
 * tau is dimensionless (relaxation time in units of dt).
 *
 * Memory: the caller owns all device memory.  mclbm_plan reports the arena
 * size; the caller allocates it (e.g. torch.empty(bytes, dtype=uint8,
 * device="cuda")) and hands it to mclbm_create together with a HIP stream.
 * The library never allocates or frees device memory.  All work is enqueued on
 * that stream; mclbm_read and mclbm_diag synchronise it.
 *
 * Fields exchanged with the caller are FP64, component-major, x fastest:
 * [comp][ny][nx].  Node (i, k) sits at X = ((i + 1/2) dx, (k + 1/2) dx); the
 * walls lie half way beyond the outermost nodes.
 *
 * Errors: every int function returns MCLBM_OK (0) or a negative status;
 * mclbm_last_error() gives a message for the calling thread.  A handle is not
 * thread safe; distinct handles may be used from distinct threads.
 */
#ifndef MCLBM_H
#define MCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum mclbm_status {
    MCLBM_OK = 0,
    MCLBM_EINVAL = -1,    /* invalid argument or parameter                      */
    MCLBM_ETOOSMALL = -2, /* arena smaller than mclbm_plan reported             */
    MCLBM_EHIP = -3,      /* a HIP runtime call failed (message has the detail) */
    MCLBM_EUNSTABLE = -4, /* non-finite values, or growth past growth_limit     */
    MCLBM_ESTATE = -5     /* call out of order (e.g. step before init)          */
};

enum mclbm_material { MCLBM_SVK = 0, MCLBM_NEOHOOKE = 1, MCLBM_LINEAR = 2 };

/* Storage of the populations and the arithmetic of the step.  The displacement
 * u is stored and integrated in FP64 in every mode, and its differences (the
 * displacement gradient) are taken in FP64.
 *   F64   populations FP64, arithmetic FP64 (the plain method)
 *   F32   populations stored in FP32; stresses, source and pulls in FP32; the
 *         moments, the equilibrium and the BGK relaxation in FP64 (the D2Q9
 *         weights are inexact in FP32, and an FP32 equilibrium would scale j
 *         and Pi by about 1 + 1e-8 in every collision); at wall nodes the
 *         stresses and the wall rules, i.e. the boundary-traction balance
 *         Pi N = -T* + (P + Pi(H)) N of Sect. 3.3 and the bounce-back values,
 *         in FP64 (T* and P(H) N nearly cancel on a loaded wall)
 *   F16   populations stored as FP16, arithmetic as F32.  The rest state of the
 *         scheme has f = 0, so the stored values are the deviations from that
 *         equilibrium; they are kept times 2^(12 - floor(log2 rho0)), which
 *         holds |f| from about 1.5e-8 rho0 to 16 rho0 in FP16's normal range
 *   BF16  populations stored as BF16 (unscaled), arithmetic as F32
 * The two 16-bit modes keep 18 bytes per node and buffer instead of 36 (F32)
 * or 72 (F64).  Their error against F64 is reported per workload; no bound is
 * claimed. */
enum mclbm_precision { MCLBM_F64 = 0, MCLBM_F32 = 1, MCLBM_F16 = 2, MCLBM_BF16 = 3 };

enum mclbm_side { MCLBM_LEFT = 0, MCLBM_RIGHT = 1, MCLBM_BOTTOM = 2, MCLBM_TOP = 3 };

/* Wall types (Sect. 3.3).  PERIODIC must be set on both opposite sides. */
enum mclbm_bc { MCLBM_DIRICHLET = 0, MCLBM_NEUMANN = 1, MCLBM_PERIODIC = 2 };

/* Time programs of a wall load, evaluated at the step index n (the step whose
 * post-collision populations the wall reflects):
 *   ZERO        0
 *   CONST       amp
 *   DISP_RAMP   Dirichlet only: a wall displacement amp reached at constant
 *               speed over t1 steps and then held: j* = rho0 amp / (t1 dt)
 *               for n < t1, else 0
 *   LINEAR_RAMP amp * min(n / t1, 1)
 *   SIN2_RAMP   amp * sin^2(pi n / (2 t1)) for n < t1, amp after (tension
 *               load of Sect. 4.1 with the time in steps)
 *   SIN_PULSE   amp * sin(pi n / t1) for n < t1, 0 after (shear momentum of
 *               Sect. 4.2)
 *   GAUSS       amp * exp(-(n - t0)^2 / (2 width^2)) for n <= t1, 0 after
 *   RICKER      amp * 2/sqrt(3 width sqrt(pi)) (1 - (n-t0)^2/width)
 *               * exp(-(n-t0)^2 / (2 width)) for n < t1, 0 after (Eq. of the
 *               Ricker wavelet in Sect. 4.3, s = width, times in steps)
 *   TABLE       amp * table[n] for n < table_len, amp * table[table_len - 1]
 *               after (any load history sampled at the steps; the table is
 *               copied when the side is set)
 * For a Dirichlet wall the value is j* (momentum density), for a Neumann wall
 * T* (traction, force per reference length). */
enum mclbm_load_kind {
    MCLBM_LOAD_ZERO = 0, MCLBM_LOAD_CONST = 1, MCLBM_LOAD_DISP_RAMP = 2,
    MCLBM_LOAD_LINEAR_RAMP = 3, MCLBM_LOAD_SIN2_RAMP = 4, MCLBM_LOAD_SIN_PULSE = 5,
    MCLBM_LOAD_GAUSS = 6, MCLBM_LOAD_RICKER = 7, MCLBM_LOAD_TABLE = 8
};

/* Fields for mclbm_read, at t_n after n steps:
 *   U  2 comps  displacement u_n
 *   J  2        momentum j = sum_q c_q f_q + dt/2 S (the j of the collision
 *               at t_n, Algorithm 1)
 *   R  1        r = sum_q f_q
 *   PI 3        Pi = sum_q c_q c_q f_q, (xx, xy, yy)
 *   H  4        H = grad u by finite differences, (xx, xy, yx, yy),
 *               H_ab = d u_a / d X_b
 *   P  4        first Piola-Kirchhoff stress P(H), (xx, xy, yx, yy)
 *   S  2        source S = rho0 b + Div(P(H) + Pi(H)) */
enum mclbm_field {
    MCLBM_FIELD_U = 0, MCLBM_FIELD_J = 1, MCLBM_FIELD_R = 2, MCLBM_FIELD_PI = 3,
    MCLBM_FIELD_H = 4, MCLBM_FIELD_P = 5, MCLBM_FIELD_S = 6
};

typedef struct {
    int32_t nx, ny;       /* lattice nodes, each >= 3                          */
    int32_t material;     /* enum mclbm_material                                */
    int32_t precision;    /* enum mclbm_precision                               */
    double dx;            /* lattice spacing dX > 0                             */
    double rho0;          /* reference density > 0                              */
    double mu;            /* shear modulus > 0                                  */
    double nu;            /* Poisson ratio in (-1, 0.5); lambda = 2 mu nu/(1-2nu)*/
    double tau;           /* relaxation time in units of dt, > 0.5              */
    double body[2];       /* body force b per unit mass                         */
    double tau_plus;      /* 0: BGK collision (the paper's).  > 0.5: two
                           * relaxation times, an option for stability (the
                           * paper's conclusion, Sect. 6, names collision
                           * operators beyond BGK): the non-equilibrium part
                           * n = f - f_eq splits into its odd part
                           * (n_q - n_qbar)/2, relaxed at 1/tau as in BGK, and
                           * its even part (n_q + n_qbar)/2, relaxed at
                           * 1/tau_plus.  tau_plus = tau is BGK.                */
    double growth_limit;  /* 0: off.  > 0: a displacement |u| above it at any
                           * node counts as growth, the sign of a run that has
                           * left the regime the scheme is stable in (Sect. 3.2
                           * bounds nu for stability; beyond it runs diverge):
                           * mclbm_diag sets growth and returns EUNSTABLE, and
                           * mclbm_step_checked stops, like for a non-finite
                           * value.  In units of length, like dx.               */
    int32_t extrap;       /* Neumann walls (Sect. 3.3): the stresses in the
                           * quasi-boundary traction -T* + (P + Pi(H)) N and the
                           * entry of Pi_bd the traction does not set are carried
                           * from the wall node X to the half-way wall.
                           * 0: zeroth order, the node's value (default).
                           * 1: linear, (3 v(X) - v(X - N dX)) / 2; with the
                           * one-sided source differences of Sect. 3.2 this
                           * closes the discrete momentum balance exactly.     */
    int32_t corner;       /* the shear entry of Pi_bd for a link that crosses
                           * two Neumann walls (the paper gives no corner rule):
                           * 0 the mean of the two walls' entries (default),
                           * 1 the x wall's, 2 the y wall's.                     */
    int32_t boundary_order; /* one-sided differences (u -> H, T -> S) at the
                           * outermost nodes: 1 first order, with the inward
                           * neighbour (Sect. 3.2; default); 2 second order,
                           * (-3 v0 + 4 v1 - v2) / (2 dX), the stencils for which
                           * the CFL discussion of Sect. 3.2 admits nu <= 5/11.
                           * 2 runs the multi-pass step (see time_levels).      */
    int32_t time_levels;  /* 0: the stresses and the source of step n are taken
                           * from u_n before the collision, so the collision,
                           * the moment j(t_{n+1}) and the walls all use level n
                           * (Sect. 3.1 states S at the current level; default).
                           * 1: the order printed in Algorithm 1: the collision
                           * and the walls of step n use S and T of level n - 1
                           * (from u_{n-1}), j(t_{n+1}) uses S_n.  Options 1 and
                           * boundary_order 2 run a multi-pass step (stresses,
                           * source, then the step, three launches, FP64
                           * arithmetic) with S and T held in the arena; the
                           * default runs one fused launch.                     */
    int32_t diag_every;   /* 0: off.  k > 0: mclbm_step runs the diagnostics on
                           * the device after every step whose count is a
                           * multiple of k, without synchronising, and records
                           * the first such step at which u or j was not finite
                           * (mclbm_diag_out.first_bad_step).                   */
    int32_t reserved_;    /* must be 0                                          */
} mclbm_params;

typedef struct {
    int32_t bc;           /* enum mclbm_bc                                      */
    int32_t kind;         /* enum mclbm_load_kind                               */
    double amp[2];        /* load vector                                        */
    double t0, t1, width; /* time-program parameters, in steps                  */
    const double* table;  /* TABLE: the scalar program per step (host memory,
                           * copied by mclbm_set_side / mclbm_server_submit)   */
    int64_t table_len;    /* TABLE: entries, 1..2^26; other kinds ignore both   */
} mclbm_side_spec;

typedef struct {
    int64_t step;         /* n                                                  */
    double momentum[2];   /* sum_X sum_q c_q f_q(t_n)                           */
    double ekin;          /* sum_X |j|^2 / (2 rho0), j as MCLBM_FIELD_J          */
    double max_u;         /* max_X |u_n|                                        */
    int32_t nonfinite;    /* 1 when any u or j is NaN or infinite               */
    int32_t growth;       /* 1 when growth_limit > 0 and max_u exceeds it       */
    int32_t cfl_excess;   /* 1 when the dilatational wave speed exceeds the
                           * lattice speed, c_d > c, i.e. nu > 1/4: beyond the
                           * CFL bound of first-order boundary stencils
                           * (Sect. 3.2); with boundary_order 2, when nu > 5/11.
                           * A warning about the parameters, not an error: such
                           * runs often diverge near walls.                     */
    int32_t pad_;
    int64_t first_bad_step; /* diag_every > 0: the first step checked during
                           * mclbm_step at which u or j was not finite, -1 when
                           * none (or diag_every = 0)                          */
} mclbm_diag_out;

typedef struct mclbm_sim mclbm_sim; /* opaque host-side handle */

/* Arena size for these parameters, the alignment the arena needs (256 bytes)
 * and the derived time step dt (any output pointer may be NULL).  Host only;
 * validates the parameters.  Returns EINVAL for nx or ny < 3, dx, rho0 or
 * mu <= 0, tau <= 0.5, nu outside (-1, 0.5), unknown enums or option values,
 * reserved_ != 0, a lattice of 2^28 nodes or more once nx is rounded up to
 * a multiple of 64 (the device addresses a displacement buffer, 16 bytes per
 * node, through one 32-bit range; about 16320^2 is the largest square), or a
 * rounded-up nx of 2^32 / 72 or more (one lattice row's populations, at most
 * 72 bytes per node, through another). */
int mclbm_plan(const mclbm_params* p, size_t* arena_bytes, size_t* align, double* dt_out);

/* Create a simulation on the current HIP device inside the caller's arena
 * (device pointer, at least mclbm_plan bytes, 256-byte aligned) and stream
 * (a hipStream_t; NULL means the null stream).  Sides start as traction-free
 * Neumann walls.  The arena and stream must outlive the handle; the handle
 * owns no device memory.  Returns EINVAL, ETOOSMALL (arena too small or
 * misaligned). */
int mclbm_create(const mclbm_params* p, void* arena, size_t arena_bytes, void* stream,
                 mclbm_sim** out);

/* Wall program of one side (Sect. 3.3); allowed before every mclbm_init and
 * between steps (the new program applies from the next step).  Periodic sides
 * must be set in opposite pairs before mclbm_init.  Returns EINVAL for unknown
 * enums, DISP_RAMP on a non-Dirichlet side, t1 <= 0 for programs that divide
 * by it, or PERIODIC paired with a non-periodic side at init. */
int mclbm_set_side(mclbm_sim* s, int side, const mclbm_side_spec* spec);

/* Initial state (Algorithm 1, Initialise): u = u0 and populations at the
 * equilibrium f_eq(r0 = -rho0 tr H(u0), j0, Pi(H(u0))).  u0 and j0 are
 * [2][ny][nx] FP64 arrays on the host (on_device = 0) or the device
 * (on_device = 1); NULL means zero.  Resets the step counter to 0. */
int mclbm_init(mclbm_sim* s, const double* u0, const double* j0, int on_device);

/* Advance nsteps >= 0 time steps, enqueued asynchronously on the stream.
 * Capturable into a HIP graph on the simulation's stream (no allocation, no
 * memset; diag_every = 0): the captured launches keep the arguments of the
 * steps captured (buffers by step parity, the wall values of those steps), so
 * a replay repeats those steps; it continues the run correctly for constant
 * wall programs and an even number of captured steps.  The handle's step
 * count advances at capture, not at replay. */
int mclbm_step(mclbm_sim* s, int64_t nsteps);

/* Advance nsteps (1..100000) time steps as mclbm_step does, with HIP events
 * recorded on the stream before each step's launches, after its main kernel
 * and after the last step, and return the mean duration of one step (ms_step)
 * and of its main kernel (ms_main: march_kernel, which carries the wall
 * blocks; the whole step for the multi-pass step), in
 * milliseconds; either pointer may be NULL, not both.  Synchronises the
 * stream.  For measurement; the results equal those of mclbm_step bitwise. */
int mclbm_step_timed(mclbm_sim* s, int64_t nsteps, double* ms_step, double* ms_main);

/* Advance nsteps as mclbm_step does, in runs of `every` (>= 1) steps, and after
 * each run scan the displacement for values that are not finite or, with a
 * growth_limit, for |u| above it (the failure modes the paper names: the CFL
 * limit and large-strain instability, Sect. 3.2 and Sect. 4).  Stops at the
 * first run that leaves one and returns
 * MCLBM_EUNSTABLE; *steps_run (may be NULL) receives the steps taken by this
 * call either way.  Synchronises the stream after every run.  Uses the
 * arena's diagnostics result area, so it must not overlap a mclbm_diag on
 * another stream.  Results equal those of mclbm_step bitwise. */
int mclbm_step_checked(mclbm_sim* s, int64_t nsteps, int64_t every, int64_t* steps_run);

/* Plain device copy of nbytes (a multiple of 4, buffers 4-byte aligned) from
 * src to dst, enqueued on stream (a hipStream_t; NULL = null stream).  Not
 * part of the method: the reference kernel of known traffic against which the
 * hardware byte counters of the step kernels are calibrated, and the copy
 * bandwidth they are compared with. */
int mclbm_copy(void* dst, const void* src, size_t nbytes, void* stream);

/* Number of steps taken since mclbm_init. */
int64_t mclbm_stepno(const mclbm_sim* s);

/* Components of a field (see enum mclbm_field), 0 for an unknown field. */
int mclbm_field_components(int field);

/* Write one field at t_n into dst, FP64 [comp][ny][nx], on the host
 * (on_device = 0) or the device (on_device = 1).  Synchronises the stream. */
int mclbm_read(mclbm_sim* s, int field, double* dst, int on_device);

/* Global diagnostics at t_n (deterministic reductions on the device).
 * Returns EUNSTABLE (with *out filled) when u or j hold non-finite values or
 * max_u exceeds the growth_limit. */
int mclbm_diag(mclbm_sim* s, mclbm_diag_out* out);

/* For callers that cannot allocate device memory or use a workspace (code under
 * graph capture, serving loops, harnesses that forbid allocation): mclbm_diag
 * with its block partials and result in a fixed array of the library's own
 * device memory instead of the arena's diagnostics areas.  The array holds
 * 1025 x 8 doubles (65 600 bytes) per device, for the life of the process; the
 * reduction uses at most 1024 blocks, each taking several 64 x 4 node tiles,
 * so every lattice fits it.  Call it with the simulation's device current.
 * Nothing is allocated: the array's address is looked up once per device.
 * Calls on one device share the array: calls that overlap (on several streams
 * or threads) race and must be serialised by the caller.  The results equal
 * mclbm_diag's up to the summation order (more nodes per block).  Same
 * statuses as mclbm_diag; EHIP if the device's array cannot be reached. */
int mclbm_diag_noalloc(mclbm_sim* s, mclbm_diag_out* out);

/* Checkpoints: a 64-byte header (magic, format version, nx, ny, storage
 * precision, material, byte counts, step counter) followed by the state
 * (populations, displacement, and with time_levels = 1 the source and stresses
 * of the previous level), copied to or from host (on_device = 0) or device
 * (on_device = 1) memory of at least mclbm_state_bytes bytes.  A simulation
 * loaded from a checkpoint continues bitwise as the one saved.  mclbm_load
 * returns EINVAL, leaving the simulation as it was, when src_bytes is short or
 * the header does not match this simulation's lattice, storage and options. */
size_t mclbm_state_bytes(const mclbm_sim* s);
int mclbm_save(mclbm_sim* s, void* dst, size_t dst_bytes, int on_device);
int mclbm_load(mclbm_sim* s, const void* src, size_t src_bytes, int on_device);

/* Release the host handle (the arena stays with the caller). */
int mclbm_destroy(mclbm_sim* s);

/* Message of the last error on the calling thread ("" when none). */
const char* mclbm_last_error(void);

/* ---- Serving: continuous batching of many simulations on one GPU -------------
 *
 * A server advances every admitted simulation in rounds of steps_per_round
 * steps.  The batch is split into four groups (two per material, balanced by
 * lattice nodes); each round uploads one table (per step and group: the
 * simulations' buffers, wall values at their own step index and work items)
 * and replays, on four streams of the server's own joined to the caller's,
 * one graph per group of batched step launches (captured at the first round,
 * and again when a round's work items outgrow its grid): one wave per work
 * item of all simulations of the group,
 * so requests of different lattice sizes, loads and step counts share every
 * launch, and the groups' launches run side by side.  A simulation's result does not depend on its company:
 * it is bitwise the same alone and in any mix.  Against mclbm_step it agrees
 * to rounding (the batch cuts lattices into longer row chunks).  Between rounds the
 * server collects finished simulations (copying their displacement to the
 * caller's buffer) and admits waiting requests in arrival order while a slot
 * is free and their arena (mclbm_plan bytes) fits in the caller's pool.
 * After every round a scan of each active simulation's displacement flags the
 * ones that are no longer finite or have passed their growth_limit; they
 * finish at the next turn as
 * MCLBM_EUNSTABLE instead of running out their steps (the instabilities of
 * Sect. 3.2 and Sect. 4: CFL excess, large strain).
 *
 * Ownership: the caller owns the device pool (256-byte aligned) and the
 * stream.  The server keeps the first mclbm_server_plan bytes of the pool for
 * its tables and allocates arenas from the rest; it allocates a pinned host
 * staging buffer of the same size, four streams (default priority) and some
 * events, and no device memory.  Single-threaded use. */

typedef struct {
    int32_t precision;       /* enum mclbm_precision; every request must match    */
    int32_t steps_per_round; /* 1..1024                                           */
    int32_t max_active;      /* simulations in flight, 1..1024                    */
} mclbm_server_config;

enum mclbm_request_state { MCLBM_REQ_WAITING = 0, MCLBM_REQ_ACTIVE = 1, MCLBM_REQ_DONE = 2 };

typedef struct mclbm_server mclbm_server;

/* Device bytes the server keeps at the start of its pool.  EINVAL for a bad
 * configuration. */
int mclbm_server_plan(const mclbm_server_config* cfg, size_t* reserved_bytes);

/* Create a server on the current device over the caller's pool.  EINVAL,
 * ETOOSMALL (pool below the reserved bytes), EHIP. */
int mclbm_server_create(const mclbm_server_config* cfg, void* pool, size_t pool_bytes, void* stream,
                        mclbm_server** out);

/* Queue a request: a lattice (mclbm_params, same precision as the server; SVK
 * or neo-Hooke), its four sides (mclbm_side_spec, left, right, bottom, top),
 * an initial displacement u0 [2][ny][nx] FP64 on the host (copied; NULL =
 * zero) and nsteps >= 1.  At completion u_n is written to u_out [2][ny][nx]
 * FP64 (host memory that must stay valid until then).  Host only.  EINVAL
 * for bad arguments, ETOOSMALL if the arena can never fit the pool. */
int mclbm_server_submit(mclbm_server* sv, const mclbm_params* p, const mclbm_side_spec sides[4],
                        const double* u0, int64_t nsteps, double* u_out, int64_t* id_out);

/* One scheduling turn: wait for the round in flight, collect the requests it
 * finished (their ids in done_ids, at most cap of them, count in *ndone),
 * admit waiting requests, enqueue the next round and return without waiting
 * for it.  A failed request is reported as done with its status. */
int mclbm_server_progress(mclbm_server* sv, int64_t* done_ids, int32_t cap, int32_t* ndone);

/* State (enum mclbm_request_state) and status of a request: MCLBM_OK, or
 * MCLBM_EUNSTABLE when the failure scan flagged it, or the error
 * that stopped it. */
int mclbm_server_result(mclbm_server* sv, int64_t id, int32_t* state, int32_t* status);

/* Steps a request has run: nsteps when it finished normally, fewer when it was
 * stopped as unstable or failed.  EINVAL for an unknown id. */
int mclbm_server_steps(mclbm_server* sv, int64_t id, int64_t* steps);

/* Requests waiting, in flight and done so far (any pointer may be NULL). */
int mclbm_server_counts(mclbm_server* sv, int64_t* waiting, int64_t* active, int64_t* done);

/* Wait for the round in flight and release everything (the pool stays with
 * the caller). */
int mclbm_server_destroy(mclbm_server* sv);

#ifdef __cplusplus
}
#endif

#endif /* MCLBM_H */
