/*
 * lbmswim: the coupled lattice-Boltzmann / rigid-body step for three-bead
 * swimmers of Pickl et al., arXiv:1108.0786, on one AMD Instinct MI355X (gfx950).
 *
 * One call of lbm_step advances every box by the coupled step of Alg. 2
 * (Sec. 2.3):
 *   1. the bodies are mapped onto the lattice as moving-boundary cells, cells
 *      that leave a body are refilled with equilibrium populations, cells that
 *      enter one are dropped (Sec. 2.3, flag changes);
 *   2. every fluid cell is collided with LBGK (Sec. 2.1, Eqs. lbgk, collide) and
 *      streamed (Eq. streaming), with halfway bounce-back at the channel walls
 *      (Eq. lbm:bounce_back) and moving bounce-back at body cells (Sec. 2.3);
 *   3. the momentum-exchange force and torque on every body are summed
 *      (Eq. hydroF);
 *   4. the driving forces of Eqs. FB1-FB3 are added;
 *   5. the rigid bodies take one time step (Alg. 1) with the spring-damper
 *      forces of Eqs. osci_i/j (total force of Eq. totalFSwimmer).
 *
 * Conventions
 *   - Lattice: D3Q19, directions numbered 0 (rest), 1..6 = +x,-x,+y,-y,+z,-z,
 *     7..18 = (+x+y),(-x-y),(+x-y),(-x+y),(+x+z),(-x-z),(+x-z),(-x+z),
 *     (+y+z),(-y-z),(+y-z),(-y+z); weights 1/3, 1/18, 1/36.
 *   - Cells (i,j,k), i fastest, linear index i + nx*(j + ny*k), centre
 *     (i+1/2, j+1/2, k+1/2).  Non-periodic axes have halfway bounce-back walls
 *     at coordinates 0 and n.
 *   - Populations are stored as deviations dF = f - w_alpha from the rest
 *     weights, structure of arrays: element [alpha][k][j][i] at
 *     alpha*stride + cell, N = nx*ny*nz <= stride.  Storage LBM_F64 and LBM_F32 hold dF;
 *     LBM_F16S and LBM_BF16S hold dF * 2^shift_log2 in IEEE half / bfloat16.
 *     LBM_F64 collides in double, the others in float; forces, torques and the
 *     rigid-body state are always double.
 *   - Flags, one byte per cell: low 7 bits 0 = fluid, 1+b = inside body b;
 *     bit 7 is set on fluid cells that have at least one D3Q19 neighbour inside
 *     a body (the cells that own boundary links).
 *   - A body is inside-tested at cell centres exactly in this float64
 *     sequence (no fused multiply-add): X = anchor + disp; R = floor(X);
 *     f = X - R; d = cell index - R (integer, wrapped into [-L/2, L - L/2) on
 *     periodic axes); r = (d + 0.5) - f; sphere: (rx*rx + ry*ry) + rz*rz <= rad*rad;
 *     capsule (axis a = body-frame x rotated by quat): t = clamp((rx*ax + ry*ay)
 *     + rz*az, -h, h), s = r - t*a, (sx*sx + sy*sy) + sz*sz <= rad*rad.
 *   - Boundary links are (fluid cell, direction alpha pointing into the body,
 *     body index), sorted by (cell, alpha).
 *
 * Memory ownership: population, flag and trajectory buffers are device
 * memory owned by the caller and never freed by the library.  The context
 * and its scratch (link lists, body tables, per-cell link offsets) belong to
 * the library and are released by lbm_destroy.  Host structures passed in are
 * copied before the call returns.
 *
 * Ordering: calls are enqueued on the stream given in lbm_params and return
 * without waiting, except the ones documented as synchronising.  A context
 * must not be used from two threads at once.
 *
 * Errors: every function returns LBM_OK or a negative code; nothing aborts.
 * After LBM_E_HIP the context is poisoned and only lbm_last_error and
 * lbm_destroy may be called.  lbm_last_error describes the last failure.
 */
#ifndef LBMSWIM_H
#define LBMSWIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

enum {
    LBM_OK = 0,
    LBM_E_ARG = -1,       /* invalid argument or configuration */
    LBM_E_HIP = -2,       /* HIP runtime error; context poisoned */
    LBM_E_OVERLAP = -3,   /* bodies overlap each other or a wall */
    LBM_E_UNSTABLE = -4,  /* a body force or state became non-finite */
    LBM_E_STATE = -5,     /* call not valid in the current state */
    LBM_E_CAPACITY = -6,  /* link list exceeded its capacity */
    LBM_E_SYNC = -7       /* the coupling kernel's workgroups timed out at a barrier */
};

enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3 };
/* LBM_SLAB is for tests only: the half-space r . axis > 0 beyond the plane
 * through the body position normal to the body's x axis (a moving wall for
 * Couette flow, Sec. 2.3).  It must be kinematic (kinematic = 1), may reach
 * the walls, and must not overlap other bodies; radius, half_len, mass and
 * inertia are not used. */
enum { LBM_SPHERE = 0, LBM_CAPSULE = 1, LBM_SLAB = 2 };

/* doubles per body per step in the trajectory record:
 * disp[3], vel[3], omega[3], F_hydro[3], T_hydro[3], step */
#define LBM_TRAJ_DOUBLES 16

/* One box.  tau > 0.5 is the LBGK relaxation time in units of the time step
 * (Eq. lbgk).  pop[0] holds the initial deviations (the caller fills it;
 * zero is the fluid at rest); pop[1] is the second buffer of the two-buffer
 * sweep.  traj (optional, may be NULL) receives LBM_TRAJ_DOUBLES * nb
 * doubles per step at record (step % traj_cap). */
typedef struct {
    int32_t nx, ny, nz;
    uint32_t periodic_mask;   /* bit 0 = x, bit 1 = y, bit 2 = z */
    double tau;
    int32_t storage;          /* LBM_F64, LBM_F32, LBM_F16S, LBM_BF16S */
    int32_t shift_log2;       /* scale exponent of LBM_F16S / LBM_BF16S */
    void *pop[2];             /* device, 19*N elements of the storage type each */
    uint8_t *flags;           /* device, N bytes; cleared by lbm_init */
    double *traj;             /* device, optional */
    int64_t traj_cap;         /* records in traj */
    void *stream;             /* hipStream_t; all work of the context goes here */
    int64_t stride;           /* elements from one direction's array to the next,
                                 >= N (0 means N); each pop buffer holds 19*stride
                                 elements.  Padding N breaks the power-of-two
                                 spacing of the 19 streams in HBM. */
    int32_t force_average;    /* 0: the rigid-body step of step n uses the
                                 momentum-exchange force and torque of step n
                                 (Alg. 2); 1: it uses the mean of those of steps
                                 n and n-1 (zero before the first step after
                                 lbm_set_bodies).  The paper does not say; the
                                 mean removes the period-2 mode that the explicit
                                 coupling amplifies for tau < 1.  lbm_adjoint
                                 differentiates either form. */
    int32_t reserved;         /* must be 0 */
    double body_force[3];     /* TEST ONLY, not part of the method: a uniform
                                 force per unit volume on the fluid (lattice
                                 units), entered by Guo's scheme (velocity
                                 u = (j + g/2)/rho in the equilibrium, source
                                 (1 - 1/(2 tau)) w [3 (e - u) + 9 (e.u) e].g),
                                 for Poiseuille flow and the drag of a sphere
                                 array.  Zero for every workload of the paper.
                                 A box with a force cannot sample a flow
                                 average or run lbm_adjoint (LBM_E_STATE). */
} lbm_params;

/* A rigid body (Sec. 2.2).  Positions are anchor + disp; disp accumulates
 * the motion so that small displacements keep full precision.  quat =
 * (w, x, y, z) rotates the body frame, whose x axis is a capsule's axis.
 * inertia holds the principal moments in the body frame.  kinematic = 1:
 * the body keeps its prescribed vel and omega (infinitely heavy);
 * kinematic = 2: its rotation is locked (omega prescribed, torque still
 * computed) while it translates freely; 0: free. */
typedef struct {
    int32_t shape;            /* LBM_SPHERE, LBM_CAPSULE, or LBM_SLAB (tests) */
    int32_t kinematic;        /* 0 free, 1 prescribed motion, 2 rotation locked */
    double radius, half_len;  /* half_len: half the cylinder length of a capsule */
    double mass, inertia[3];
    double anchor[3], disp[3], quat[4], vel[3], omega[3];
} lbm_body;

/* Damped spring between bodies i and j (Eqs. spring_i, damp_i, osci_i/j):
 * with d = x_i - x_j, body i feels -k (|d| - rest_len) d/|d| - gamma (u_i - u_j)
 * and body j the opposite; rest_len is the centre-to-centre rest length. */
typedef struct {
    int32_t i, j;
    double k, gamma, rest_len;
} lbm_spring;

/* Driving protocol of Eqs. FB1-FB3 along x at step t, omega = 2 pi / period:
 * left body -a sin(omega t), right body a sin(omega t - phase_lag), middle
 * body minus their sum.  gate_lagged holds the right force at zero while
 * omega t < phase_lag; off_left / off_right (-1 = never) switch the left /
 * right force off from that step on. */
typedef struct {
    int32_t left, middle, right, gate_lagged;
    double amplitude, period, phase_lag;
    int64_t off_left, off_right;
} lbm_drive;

/* Create a context for one box.  Validates the parameters (LBM_E_ARG),
 * allocates the library's scratch and clears params->flags. */
int lbm_init(const lbm_params *params, lbm_ctx **out);

/* Create a context for nbox independent boxes that are stepped together by
 * single launches (parameter sweeps).  All boxes must share one storage type
 * and params[0].stream.  Box b is addressed by the *_box calls. */
int lbm_init_batch(const lbm_params *params, int32_t nbox, lbm_ctx **out);

/* Set the bodies, springs and driving protocols of box 0 (lbm_set_bodies)
 * or of box `box`, and map them onto the lattice (Sec. 2.3).  Bodies must keep
 * at least one cell between their surfaces and from the walls, measured on
 * the exact sphere and capsule shapes (LBM_E_OVERLAP); indices must be in
 * range (LBM_E_ARG).  On a box that already holds bodies, cells that leave a
 * body are refilled as in a step. */
int lbm_set_bodies(lbm_ctx *ctx, const lbm_body *bodies, int32_t nb,
                   const lbm_spring *springs, int32_t ns,
                   const lbm_drive *drives, int32_t nd);
int lbm_set_bodies_box(lbm_ctx *ctx, int32_t box, const lbm_body *bodies, int32_t nb,
                       const lbm_spring *springs, int32_t ns,
                       const lbm_drive *drives, int32_t nd);

/* Stop box `box` once it has taken max_steps steps (-1: no limit).  Boxes
 * that reached their limit are left out of later launches. */
int lbm_set_step_limit(lbm_ctx *ctx, int32_t box, int64_t max_steps);

/* Advance every box that has not reached its limit by nsteps coupled steps
 * (Alg. 2), asynchronously on the context's stream. */
int lbm_step(lbm_ctx *ctx, int64_t nsteps);

/* Build the launch sequence that lbm_step(ctx, nsteps) replays (HIP graphs
 * of LBM_TUNE_GRAPH_STEPS steps and one of the remainder), without launching
 * any of it, so that a timed lbm_step does not include capturing graphs.
 * Graphs are kept until the tuning, the timing mode or the set of active
 * boxes changes; lbm_step builds what is missing itself.  Synchronising only
 * when the active boxes changed since the last call. */
int lbm_prepare(lbm_ctx *ctx, int64_t nsteps);

/* Hydrodynamic force and torque on every body from the last step
 * (Eq. hydroF), nb x 3 doubles each.  on_device = 1: F and T are device
 * pointers and the copy is enqueued; on_device = 0: host pointers and the
 * call synchronises the stream. */
int lbm_body_forces(lbm_ctx *ctx, double *F, double *T, int32_t on_device);
int lbm_body_forces_box(lbm_ctx *ctx, int32_t box, double *F, double *T, int32_t on_device);

/* Copy the current body states into out[0..nb) (host).  Synchronising. */
int lbm_get_bodies(lbm_ctx *ctx, lbm_body *out, int32_t nb);
int lbm_get_bodies_box(lbm_ctx *ctx, int32_t box, lbm_body *out, int32_t nb);

/* Copy box `box`'s boundary links into host arrays of capacity cap; *n gets
 * the number of links (LBM_E_CAPACITY if cap is too small).  Synchronising. */
int lbm_get_links(lbm_ctx *ctx, int32_t box, int32_t *cell, int8_t *dir, int8_t *body,
                  int64_t cap, int64_t *n);

/* Write box `box`'s current pre-collision deviations dF as double into the
 * device array dst (19*N, same layout as the populations), zero at body cells. */
int lbm_export_populations(lbm_ctx *ctx, int32_t box, double *dst);

/* Write the current deviations of n chosen cells of box `box` as double into
 * dst (device, 19*n, dst[alpha*n + m] for cells[m]); cells is a device array
 * of n linear cell indices; an index outside the box yields NaN in its
 * column.  Zero at body cells. */
int lbm_export_cells(lbm_ctx *ctx, int32_t box, const int32_t *cells, int64_t n, double *dst);

/* Overwrite box `box`'s current populations from the device array src
 * (19*N doubles of dF), converting to the storage type. */
int lbm_import_populations(lbm_ctx *ctx, int32_t box, const double *src);

/* Time-averaged flow field (Sec. 6, Fig. flowfields13: flow fields averaged
 * over swimming cycles).  lbm_flow_average_begin(ctx, box, every) with
 * every >= 1 clears box `box`'s sums and from then on adds, at every step n
 * with n % every == 0 (n the box's step counter), the fluid velocity
 * u = sum_alpha e_alpha f_alpha / rho of the pre-collision state of step n
 * at every cell that is fluid in that step, in double, together with a
 * per-cell count of the samples.  every = 0 stops sampling and keeps the
 * sums.  The sums (3N doubles and N ints) are library-owned, allocated on
 * first use and freed by lbm_destroy.  Steps that sample run a variant of
 * the sweep that reads and writes 28 more bytes per fluid cell; the plain
 * sweep is used while no box samples.  Synchronising.  LBM_E_ARG for a bad
 * box or every < 0; lbm_adjoint returns LBM_E_STATE while a box samples.
 *
 * lbm_flow_average_get writes the mean velocity sum / count into the
 * caller-owned device array `mean` (3*N doubles: x, then y, then z, each
 * [nz][ny][nx]; zero where the cell was never fluid in a sample) and, if
 * `count` is not null, the counts into the device array `count` (N int32).
 * Asynchronous on the context's stream.  LBM_E_STATE if no average was
 * begun on the box. */
int lbm_flow_average_begin(lbm_ctx *ctx, int32_t box, int32_t every);
int lbm_flow_average_get(lbm_ctx *ctx, int32_t box, double *mean, int32_t *count);

/* Steps taken by box `box` so far.  Synchronising. */
int lbm_step_count(lbm_ctx *ctx, int32_t box, int64_t *steps);

/* Synchronise and report a device-side failure: LBM_E_UNSTABLE if a body
 * force or state became non-finite, LBM_E_CAPACITY if a link list overflowed,
 * LBM_E_SYNC if the workgroups of a cooperative mapping (LBM_TUNE_COOP_REMAP)
 * waited at a barrier for longer than about a second (they then give up, so
 * that the kernel always ends; the box's state is not valid afterwards).
 * Such a mapping only starts once all of the box's workgroups are running;
 * if they are not within tens of microseconds (other work holds the device),
 * the box's first workgroup maps alone instead, with the same results. */
int lbm_status(lbm_ctx *ctx);

/* Hand-written reverse mode (adjoint) of nsteps coupled steps of box 0 of a
 * single-box context, from its current state.  The objective is the linear
 * function of the final body displacements
 *     J = sum_b dJ_ddisp[3b..3b+2] . disp_b(t + nsteps),
 * (dJ_ddisp: host array, nb x 3), e.g. 1/nb on x for the swimmer centroid.
 * On return *J holds its value and grad[0..2] (host) its derivatives with
 * respect to the driving amplitude and the phase lag (shared by all drives of
 * the box, Eqs. FB1-FB3) and the spring stiffness k (shared by all springs,
 * Eq. spring_i).  The forward states are kept as checkpoints every
 * checkpoint_every steps and recomputed segment by segment during the reverse
 * pass (scratch: nsteps/checkpoint_every + checkpoint_every + 1 population
 * states, two adjoint fields in double, owned by the context).  The mapping
 * must not change during the run (the flags are held fixed in the reverse
 * pass): LBM_E_STATE if any cell changed its owner at any step of the run,
 * even if it changed back before the end.  Capsule orientation is treated as a constant
 * in the reverse pass.  Afterwards the context is in the same state as after
 * lbm_step(ctx, nsteps).  Synchronising. */
int lbm_adjoint(lbm_ctx *ctx, int64_t nsteps, int32_t checkpoint_every, const double *dJ_ddisp,
                double *J, double *grad);

/* Launch tuning of a context (values outside the listed ones give LBM_E_ARG):
 *   LBM_TUNE_BLOCK        sweep workgroup size: 128, 256 (default) or 512
 *   LBM_TUNE_XCD_ORDER    1: give each XCD a contiguous slab of tiles; 0: hand
 *                         out tiles in order.  Default 1 when the context's
 *                         two population buffers hold more than 2 GiB in all,
 *                         else 0.  Results are identical.
 *   LBM_TUNE_GRAPH_STEPS  0: launch every kernel; n > 0 (default 32): replay
 *                         captured HIP graphs of n steps, and the remainder of
 *                         a run as one graph of its own length
 *   LBM_TUNE_FULL_REMAP   1: map the bodies every step even when no cell can
 *                         have changed side (default 0; results are identical)
 *   LBM_TUNE_NONTEMPORAL  1: streaming (non-temporal) loads of the
 *                         populations in the sweep; stores are always plain.
 *                         Default 1 when the context's two population buffers
 *                         hold at most 768 MiB in all and the storage is not
 *                         LBM_F64, else 0.  Results are identical.
 *   LBM_TUNE_COOP_REMAP   1 (default): when every workgroup of the coupling
 *                         launch can be resident at once (up to the device's
 *                         occupancy for it: a few boxes per launch), all
 *                         workgroups of a box share its mapping, once all of
 *                         them have joined (else the first maps alone); 0:
 *                         one workgroup maps each box; 2 (a test aid): the
 *                         workgroups join as for 1, and the first one always
 *                         maps alone.  Results are identical.
 *   LBM_TUNE_STREAMING    0: the sweep reads one population buffer and
 *                         pushes into the other (Eq. streaming as written;
 *                         default for LBM_F64, LBM_F16S, LBM_BF16S); 1
 *                         (default for LBM_F32): it streams in place in one
 *                         buffer (the
 *                         "AA" access pattern of Bailey et al. 2009: at even
 *                         steps every cell reads and writes only its own
 *                         slots, at odd steps it pulls from and pushes to its
 *                         neighbours).  Switching converts the current
 *                         populations between the layouts; results are
 *                         identical bit for bit.  The adjoint runs the
 *                         two-buffer sweep either way. */
enum { LBM_TUNE_BLOCK = 0, LBM_TUNE_XCD_ORDER = 1, LBM_TUNE_GRAPH_STEPS = 2, LBM_TUNE_FULL_REMAP = 3,
       LBM_TUNE_NONTEMPORAL = 4, LBM_TUNE_COOP_REMAP = 5, LBM_TUNE_STREAMING = 6 };
int lbm_tune(lbm_ctx *ctx, int32_t key, int64_t value);

/* Kernel timing.  With enable = 1, lbm_step launches every kernel itself (no
 * graph replay) and records a pair of HIP events
 * on the context's stream around every sweep launch and every coupling
 * launch (and keeps them until lbm_get_timing); enable = 0 stops recording
 * and drops the recorded events.  lbm_get_timing synchronises, and writes the
 * summed durations in milliseconds and the launch counts since timing was
 * enabled: out_ms[0] sweep, out_ms[1] coupling; out_n likewise. */
int lbm_set_timing(lbm_ctx *ctx, int32_t enable);
int lbm_get_timing(lbm_ctx *ctx, double out_ms[2], int64_t out_n[2]);

/* Integrator-only runs: the swimmer in vacuum of Sec. 4 (its Lagrangian
 * with the spring damping of Eq. damp_i), used there to validate the spring
 * forces against the analytic model and to trace the amplitude resonances
 * of Fig. vacuumVal2.  Advances nsys independent systems by nsteps steps of
 * the rigid-body step that lbm_step uses (driving, Eqs. FB1-FB3; springs,
 * Eqs. osci_i/j; semi-implicit Euler with dt = 1), with the hydrodynamic
 * force and torque zero.  Every system has nb bodies, ns springs and nd
 * drives: system s uses bodies[s*nb .. s*nb+nb-1], springs[s*ns ..] and
 * drives[s*nd ..] (host arrays, copied; same limits as lbm_set_bodies).
 * Steps are numbered from 0 for every system.  traj (optional) is a
 * caller-owned device ring of traj_cap records per system laid out
 * [nsys][traj_cap][nb][16] like the lbm_params trajectory.  out (optional)
 * receives the nsys*nb final body states on the host.  Runs on `stream`
 * (hipStream_t, 0 for the default stream), one workgroup per system, and
 * synchronises; the few device tables it needs are allocated and freed
 * inside the call.  LBM_E_ARG for bad counts or indices, non-positive mass,
 * inertia or period; LBM_E_UNSTABLE if a state became non-finite;
 * LBM_E_HIP on a runtime error (no context, so no message). */
int lbm_vacuum_run(const lbm_body *bodies, int32_t nb, const lbm_spring *springs, int32_t ns,
                   const lbm_drive *drives, int32_t nd, int32_t nsys, int64_t nsteps, double *traj,
                   int64_t traj_cap, lbm_body *out, void *stream);

/* Bytes of the per-GPU array that lbm_vacuum_run_noalloc keeps its device
 * tables in. */
#define LBM_NOALLOC_SCRATCH_BYTES (1 << 20)

/* lbm_vacuum_run for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, run and results, with no hipMalloc or hipFree.  The
 * device tables of the nsys systems (bodies, springs, drives and one
 * descriptor per system: 256 nb + 32 ns + 56 nd + 344 bytes per system, each
 * of the four tables padded to 256 bytes) go into an array of
 * LBM_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it runs
 * on until the process ends (850 systems of three beads, two springs and one
 * drive fit); the caller still owns traj and out.  LBM_E_ARG when the
 * tables do not fit, or for the argument errors of lbm_vacuum_run.  Every
 * call on one GPU uses that GPU's array, so calls that overlap in time on
 * one GPU race; the call writes every table before it runs, and nothing of
 * an earlier call carries over.  Synchronising. */
int lbm_vacuum_run_noalloc(const lbm_body *bodies, int32_t nb, const lbm_spring *springs, int32_t ns,
                           const lbm_drive *drives, int32_t nd, int32_t nsys, int64_t nsteps, double *traj,
                           int64_t traj_cap, lbm_body *out, void *stream);

/* Measurement aid, not part of the method: copy `bytes` bytes (a multiple
 * of 16) from device memory src to device memory dst with a plain streaming
 * kernel on `stream` (hipStream_t): with blocks_per_cu = 0 one 16-byte vector
 * per thread over the whole range, else at most 256 * blocks_per_cu
 * workgroups looping over it; non-temporal loads and stores if `nontemporal`.  Used as the practical
 * HBM ceiling and to calibrate hardware byte counters against a known
 * transfer. */
int lbm_copy_kernel(const void *src, void *dst, int64_t bytes, int32_t blocks_per_cu, int32_t nontemporal,
                    void *stream);

/* Measurement aid, not part of the method: the sweep's memory access
 * pattern without its arithmetic, as the practical ceiling of that pattern
 * at a given box size.  Copies 19 streams of n elements of elem_bytes bytes
 * each (2, 4 or 8), stream a starting at element a * stride, from src to dst
 * (device memory, each at least 19 * stride elements, not overlapping), on
 * `stream` (hipStream_t): one element per thread, its 19 loads issued before
 * its 19 stores, non-temporal loads if `nontemporal`, plain stores.
 * LBM_E_ARG for a null pointer, n <= 0, stride < n, another element size or
 * sizes whose offsets overflow; LBM_E_HIP when the launch fails. */
int lbm_stream_copy(const void *src, void *dst, int64_t n, int64_t stride, int32_t elem_bytes, int32_t nontemporal,
                    void *stream);

/* Write sizeof(lbm_params), sizeof(lbm_body), sizeof(lbm_spring) and
 * sizeof(lbm_drive) into out[0..3] so that a binding can check its struct
 * layout.  Touches no device. */
int lbm_struct_sizes(int64_t out[4]);

const char *lbm_last_error(const lbm_ctx *ctx);
void lbm_destroy(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBMSWIM_H */
