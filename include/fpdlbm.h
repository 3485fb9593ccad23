/*
 * fpdlbm.h -- C ABI of the MI355X (gfx950) library for one time step of the fluid
 * particle dynamics (FPD) method for a flexible bead-spring fiber in confined shear flow,
 * solved by a D2Q9 multiple-relaxation-time lattice Boltzmann (MRT-LBM) scheme
 * (arXiv:2212.14153, Sec. II).
 *
 * What one step computes (Sec. II.C, integration steps (1)-(3)):
 *   (1) from the bead centres R_i^n: the interface profiles phi_i^n (Eq. 2), the bead
 *       forces F_i^n (Eqs. 10-12), the force density f^n (Eq. 4) and the viscosity
 *       eta^n (Eq. 1);
 *   (2) one MRT-LBM collide-and-stream update of the fluid with the local viscosity
 *       eta^n and the force density f^n, walls at y = 0 and y = H moving at -U and +U
 *       (Sec. IV.A, Fig. 1b), x periodic; or, for the driven-particle benchmark of
 *       Sec. III.B, no walls (x and y periodic, FPD_PERIODIC);
 *   (3) the bead velocities V_i^{n+1} (Eq. 5) and the forward-Euler update
 *       R_i^{n+1} = R_i^n + dt V_i^{n+1}.
 *
 * Units and geometry: lattice units, dx = dt = 1, c_s^2 = 1/3, reference density 1.
 * The paper's z axis is y.  Node (i, j), 0 <= i < nx, 0 <= j < ny, sits at the square
 * centre (i + 1/2, j + 1/2) (Sec. II.C); the walls lie at y = 0 and y = ny; bead
 * coordinates are continuous in [0, nx) x (0, ny) (x may leave [0, nx); it is taken
 * modulo nx through the minimum image).
 *
 * Array layouts on the host side of this ABI (all arrays are caller-owned, float64,
 * C order):
 *   populations f[9][ny][nx], direction k = 0..8 with
 *     e_0 = (0,0), e_1..e_4 = (1,0),(0,1),(-1,0),(0,-1),
 *     e_5..e_8 = (1,1),(-1,1),(-1,-1),(1,-1);
 *   per-node fields [ny][nx]; bead arrays [n_beads][2].
 * Device-side layout (not visible through this ABI): two buffers (pull streaming) of
 * f - w_k; value (k, j, i) at j * 9P + k * P + i with P = nx rounded up to 64 (the nine
 * direction rows of a lattice row side by side).
 *
 * Errors: every int-returning call returns FPD_OK (0) or a negative FPD_E* code and
 * never throws; fpd_last_error() gives a message for the calling thread.  Calls on one
 * simulation must come from one thread at a time.  Calls that return data to the host
 * synchronise the simulation's stream; fpd_step only enqueues work.
 */
#ifndef FPDLBM_H
#define FPDLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes ---- */
#define FPD_OK          0
#define FPD_EINVAL     -1   /* invalid argument or parameter set                         */
#define FPD_ENOMEM     -2   /* device allocation failed or the HBM budget is exhausted    */
#define FPD_EUNSTABLE  -3   /* a health check tripped (see FPD_HEALTH_*)                  */
#define FPD_EDEVICE    -4   /* HIP runtime error                                          */
#define FPD_ESTATE     -5   /* call not valid in the current state                        */

/* population storage formats (arithmetic is FP64 for FPD_F64, FP32 otherwise) */
#define FPD_F64        0    /* float64 f - w_k                                            */
#define FPD_F32        1    /* float32 f - w_k                                            */
#define FPD_F16DEV     2    /* binary16 of (f - w_k) * 2^14                               */
#define FPD_BF16DEV    3    /* bfloat16 of (f - w_k)                                      */

/* initial flow (the paper starts from a flat fiber in the shear flow, Sec. IV.C) */
#define FPD_INIT_REST            0   /* rho = 1, u = 0 everywhere                         */
#define FPD_INIT_LINEAR_COUETTE  1   /* equilibrium at u_x = U (2 y / H - 1)              */

/* boundary in y */
#define FPD_WALLS     0   /* moving walls at y = 0 and y = ny (Sec. IV.A)                  */
#define FPD_PERIODIC  1   /* no walls: y periodic too (the box of Sec. III.B)               */

/* flags */
#define FPD_FLAG_CLAMP_PHI     0x1u  /* clamp sum_i phi_i to 1 in Eq. (1)                 */
#define FPD_FLAG_NO_GRAPH      0x2u  /* launch every kernel directly (no graph replay)    */
#define FPD_FLAG_TIME_KERNELS  0x4u  /* time the lattice pass and bead kernel (no graph)    */
#define FPD_FLAG_NO_SPLIT      0x8u  /* one lattice kernel per step (no split steps)      */

/* health bits, sticky until fpd_clear_health */
#define FPD_HEALTH_NAN      0x1u   /* NaN or Inf in a bead position or velocity           */
#define FPD_HEALTH_STRAIN   0x2u   /* a bond is stretched or compressed by more than 50%  */
#define FPD_HEALTH_MACH     0x4u   /* a bead moves faster than 0.3 c_s                    */
#define FPD_HEALTH_WALL     0x8u   /* a bead came within a + xi of a wall (FPD_WALLS)     */
#define FPD_HEALTH_SUPPORT  0x10u  /* the fiber outgrew the reserved support window       */

#define FPD_MAX_BEADS 256

/* Parameters of one simulation, lattice units.  Names follow the paper: r_eta = eta_s /
 * eta_f (Sec. II.A remark (1)), xi and a of Eq. (2), k_s, k_b, l_0 of Eq. (9). */
typedef struct fpd_params {
    int32_t  nx, ny;        /* lattice squares along x (periodic) and y (between walls)    */
    double   u_wall;        /* U: bottom wall moves at -U, top wall at +U (|U| < 0.1)       */
    double   nu_f;          /* fluid kinematic viscosity eta_f / rho (> 0)                  */
    double   eta_ratio;     /* r_eta = eta_s / eta_f (>= 1)                                 */
    double   xi;            /* interface thickness xi (> 0)                                 */
    int32_t  n_beads;       /* N, 0 (no fiber) .. FPD_MAX_BEADS                             */
    double   radius;        /* bead radius a (> 0)                                          */
    double   l0;            /* spring rest length l_0 (> 0)                                 */
    double   k_s, k_b;      /* stretching and bending constants (>= 0)                      */
    double   s_e, s_eps;    /* MRT rates of the energy moments, in (0, 2)                   */
    double   s_q_fixed;     /* > 0: heat-flux rate; <= 0: per-node value with
                               (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16                            */
    double   cutoff;        /* phi is evaluated within a + cutoff * xi of each bead and
                               taken as 0 beyond; <= 0 selects 20 (FPD_F64) or 9 (others)    */
    int32_t  storage;       /* FPD_F64 | FPD_F32 | FPD_F16DEV | FPD_BF16DEV                 */
    int32_t  init_flow;     /* FPD_INIT_REST | FPD_INIT_LINEAR_COUETTE                      */
    uint32_t flags;         /* FPD_FLAG_*                                                   */
    int32_t  boundary;      /* FPD_WALLS | FPD_PERIODIC (then u_wall = 0, FPD_INIT_REST)    */
    double   f_ext[2];      /* external force added to F_i of every bead (the driving force
                               F0 of Sec. III.B), spread by Eq. (4) like F_i               */
    double   g_body[2];     /* uniform body force density on every node; in a periodic box
                               g = -N f_ext / (nx ny) keeps the total momentum constant     */
    int32_t  n_chains;      /* fibers: beads c L .. c L + L - 1 form fiber c, L = n_beads /
                               n_chains (<= 1: one fiber); springs and bending act inside a
                               fiber only, and fibers meet through the fluid (and the
                               excluded volume below); the force window then spans the
                               whole lattice                                                 */
    double   ev_k;          /* excluded volume between fibers, which the paper does not
                               specify (0: none): beads of different fibers closer than d
                               repel with the force of (ev_k / 2)(d - r)^2 (>= 0)          */
    double   ev_range;      /* d; <= 0 selects 2 a (contact of the bead surfaces)          */
} fpd_params;

/* Launch shape of the fused lattice kernel; any field <= 0 keeps the current value. */
typedef struct fpd_launch {
    int32_t block_x;          /* threads per block along x: 64, 128 or 256                 */
    int32_t block_y;          /* thread rows per block: 1, 2, 4 (block_x*block_y <= 256)   */
    int32_t rows_per_thread;  /* lattice rows per thread: 1, 2 or 4                         */
    int32_t xcd_remap;        /* 1: consecutive tiles on one XCD; 2: off                    */
    int32_t graph_chunk;      /* steps per captured graph (even, >= 2)                      */
} fpd_launch;

typedef struct fpd_sim fpd_sim;

/* ------------------------------------------------------------- parameters ---- */

/* Fill p with defaults: no fiber, nu_f = 1/6, r_eta = 50, xi = 1, s_e = 1.64,
 * s_eps = 1.54, magic s_q, FPD_F32, linear Couette start. */
void fpd_params_default(fpd_params *p);

/* Lattice parameters from the physical groups of Eq. (18): K = 2 k_b / (eta_f gamma
 * l_c^2), C = l_c / H, Re_ps = rho gamma l_c^2 / (4 eta_f), with gamma = 2U/H and
 * l_c = N l_0, l_0 = 2a (touching beads, Sec. II.B).  ny = l_c / C, nx = nx_over_ny * ny,
 * k_s / l_0^2 = 0.1 pi a^2 (explicit-coupling stability; the paper's K_s = 3.33e6 is not
 * reachable in lattice units).  Fills *out (other fields from fpd_params_default).
 * Returns FPD_EINVAL when the result violates fpd_create's checks. */
int fpd_params_from_physical(double re_ps, double confinement, double kappa, int32_t n_beads,
                             double radius, double eta_ratio, double xi, double u_wall,
                             int32_t nx_over_ny, fpd_params *out);

/* Bytes of one population buffer for p (the library keeps two). */
size_t fpd_population_bytes(const fpd_params *p);

/* ------------------------------------------------------------- lifecycle ----- */

/* The problem of Sec. IV.A (Fig. 1b): a channel of nx x ny squares between walls moving
 * at -U and +U, fluid of viscosity eta_f, fiber beads of radius a and interface xi
 * (Eqs. 1, 2, 9), on the lattice of Sec. II.C.  Validate p (tau_f > 1/2, |U| < 0.1,
 * N <= FPD_MAX_BEADS, 1 <= nx < 2^31 / 9, 1 <= ny <= 65535, rates in (0,2); FPD_EINVAL
 * otherwise), allocate device state on the current HIP device (FPD_ENOMEM when that
 * fails), initialise the populations per p->init_flow.  hip_stream is a hipStream_t (NULL:
 * the library creates its own).  The caller owns *out and frees it with fpd_destroy.
 * The fiber is absent until fpd_init_fiber. */
int fpd_create(const fpd_params *p, void *hip_stream, fpd_sim **out);

/* As fpd_create (the problem of Sec. IV.A), but the two population buffers of the pull
 * scheme are caller-owned device memory of bytes_each >= fpd_population_bytes(p) bytes
 * each (e.g. torch tensors), 16-byte aligned (FPD_EINVAL otherwise); the library writes
 * the initial state into f_a and never frees them; they must outlive the simulation. */
int fpd_create_with_buffers(const fpd_params *p, void *hip_stream, void *f_a, void *f_b,
                            size_t bytes_each, fpd_sim **out);

/* Place the fiber: R is host [n_beads][2].  Computes A_i = int phi_i, the forces F_i and
 * the support window on the device.  Beads closer than a + xi to a wall are rejected
 * (FPD_EINVAL). */
int fpd_init_fiber(fpd_sim *s, const double *R);

/* Straight fiber centred at (cx, cy) at angle theta (radians):
 * R_i = c + (i - (N + 1)/2) l_0 (cos theta, sin theta), i = 1..N. */
int fpd_init_fiber_line(fpd_sim *s, double cx, double cy, double theta);

/* Enqueue n_steps >= 0 time steps on the simulation's stream (asynchronous): each is the
 * three integration steps of Sec. II.C, (1) phi, F, f and eta from R^n (Eqs. 1, 2, 4,
 * 10-12), (2) the MRT collide-and-stream update with moving-wall bounce-back, (3) V^{n+1}
 * by Eq. (5) and R^{n+1} = R^n + V^{n+1}.  FPD_EINVAL for n_steps < 0, FPD_ESTATE before
 * fpd_init_fiber when the simulation has beads; an unstable run is reported by health
 * bits (fpd_sync), not here.
 * Split steps: with a fiber whose reserved window spans at most about a quarter of the
 * lattice's tiles (no fixed profile, not FPD_FLAG_NO_SPLIT),
 * step (2) runs as two kernels, the tiles away from the fiber on a second stream of the
 * library's own (non-blocking, default priority) while the bead kernel of the step before
 * finishes, and the tiles near it after that bead kernel; the results are the same bits.
 * The simulation's stream waits for the second stream before fpd_step returns, so work
 * enqueued on it afterwards follows every step.  The first step after fpd_init_fiber or
 * fpd_load runs whole.  FPD_HEALTH_SUPPORT is raised if a bead outran the split's margin
 * of three nodes (far beyond FPD_HEALTH_MACH). */
int fpd_step(fpd_sim *s, int64_t n_steps);

/* Capture now, without running any step, the graph that fpd_step(s, n_steps) replays
 * (steps are replayed in captured chunks of graph_chunk steps when n_steps >= graph_chunk
 * and neither FPD_FLAG_NO_GRAPH nor FPD_FLAG_TIME_KERNELS is set; otherwise there is
 * nothing to capture and the call does nothing), so that the capture cost stays out of a
 * timed fpd_step; with split steps right after fpd_init_fiber or fpd_load, the graph of
 * the steps after the whole first one.  Synchronous with respect to the host; enqueues no
 * work. */
int fpd_capture(fpd_sim *s, int64_t n_steps);

/* Wait for the stream; FPD_EUNSTABLE if a health bit is set. */
int fpd_sync(fpd_sim *s);

/* Health bits (FPD_HEALTH_*) and the largest relative bond strain seen; synchronises. */
int fpd_health(fpd_sim *s, uint32_t *flags, double *max_strain);
int fpd_clear_health(fpd_sim *s);

/* Number of steps taken since creation (or the loaded checkpoint). */
int fpd_step_count(fpd_sim *s, int64_t *steps);

void fpd_destroy(fpd_sim *s);

/* Message of the last error on the calling thread ("" if none). */
const char *fpd_last_error(void);

/* -------------------------------------------------------------- read-back ---- */

/* Host arrays [ny][nx], NULL to skip: density rho, velocity u = (j + f^n/2) / rho with the
 * force density of the current bead state (Guo's macroscopic velocity), viscosity eta^n of
 * Eq. (1).  Pressure is rho / 3. */
int fpd_read_fields(fpd_sim *s, double *rho, double *ux, double *uy, double *eta);

/* Host f[9][ny][nx] (caller-owned, filled here): the pre-collision (post-stream)
 * populations f_k of the MRT-LBM scheme (Sec. II.C) at the current step, decoded to
 * float64 whatever the storage.  Synchronises; FPD_EDEVICE on a HIP error. */
int fpd_read_populations(fpd_sim *s, double *f);

/* Replace the current pre-collision populations with host f[9][ny][nx] (encoded into the
 * storage format). */
int fpd_write_populations(fpd_sim *s, const double *f);

/* Host [n_beads][2] each, NULL to skip: R^n, V^n (velocity of the last step), F^n. */
int fpd_read_beads(fpd_sim *s, double *R, double *V, double *F);

/* A fixed interface profile phi_s(y), host [ny] (>= 0), added to sum_i phi_i in Eq. (1)
 * at every node of row y: the solid slabs of the sandwich benchmark (Sec. III.A,
 * Eq. 14).  NULL removes it.  The library keeps a device copy; checkpoints do not hold
 * it (set it again after fpd_load).  Synchronises. */
int fpd_set_static_phi(fpd_sim *s, const double *phi);

/* Fiber-ends recorder for the tumbling analysis of Sec. IV (orientation theta(t),
 * angular velocity, period, end-to-end length): from now on, every `every` steps the
 * state R^n of each fiber is summarised on the device (at the start of the step, by the
 * lattice kernel) as its end-to-end vector R_last - R_first and its centroid, into a ring
 * of `capacity` records (older records are overwritten).  Restarts any recording.
 * FPD_ESTATE without a fiber. */
int fpd_record_start(fpd_sim *s, int32_t every, int64_t capacity);
int fpd_record_stop(fpd_sim *s);

/* The records held, oldest first: *n_records receives their number (out may be NULL to
 * ask); out[n][1 + 4 * fibers] receives [step n, then (ex, ey, cx, cy) per fiber].
 * FPD_EINVAL if cap_records is smaller than the number held. */
int fpd_record_read(fpd_sim *s, double *out, int64_t cap_records, int64_t *n_records);

/* Diagnostics of the driven-particle benchmark (Sec. III.B) for bead `bead` on the
 * current state (pre-collision populations at step n, positions R^n, force density f^n
 * of that state), computed on the device with fixed-order FP64 sums; synchronises.
 * out[8] (host): A = sum_x phi_b; V0 = sum_x phi_b v / A with v = (j + f^n/2)/rho
 * (Eq. 5 on this state); eps_v = sum_x phi_b |v - V0|^2 / A (Eq. 15); the viscous
 * force -sum_x sigma . grad phi_b with sigma = eta (grad v + grad v^T), eta of Eq. (1),
 * and the pressure force sum_x ((rho - 1)/3) grad phi_b (the reference pressure 1/3
 * contributes nothing) (Eq. 17 in diffuse-interface form:
 * n dA -> -grad phi dr).  Gradients use the isotropic D2Q9 stencil
 * grad q (x) = 3 sum_k w_k e_k q(x + e_k).  Sums run over the bead's support box grown by
 * one node.  FPD_EINVAL if there is no such bead or, with walls, if that box reaches the
 * first or last row (the stencil would leave the channel). */
int fpd_particle_stats(fpd_sim *s, int32_t bead, double *out);

/* ---------------------------------------------------------------- tuning ----- */

/* Launch shape of the fused lattice kernel (results are bitwise the same for every shape;
 * the shape only changes speed).  Defaults: 128 x 1 for FPD_F64, 256 x 1 for FPD_F32,
 * 256 x 1 with two rows per thread for the two-byte formats, and 64 x 1 for FPD_F32 and
 * the two-byte formats at 2^20 nodes or fewer; graph_chunk 64.  FPD_EINVAL for a value
 * outside those fpd_launch allows (nothing changes then); synchronises. */
int fpd_set_launch(fpd_sim *s, const fpd_launch *cfg);

/* Replace the FPD_FLAG_NO_GRAPH / FPD_FLAG_TIME_KERNELS / FPD_FLAG_NO_SPLIT bits
 * (FPD_FLAG_CLAMP_PHI is fixed at creation and ignored here); synchronises. */
int fpd_set_flags(fpd_sim *s, uint32_t flags);
int fpd_get_launch(fpd_sim *s, fpd_launch *cfg);

/* Whether fpd_step splits its steps as things stand (see fpd_step): *on = 1 or 0.  The
 * first step after fpd_init_fiber or fpd_load runs whole either way. */
int fpd_split_active(fpd_sim *s, int32_t *on);

/* Kernel timing with FPD_FLAG_TIME_KERNELS: summed duration (ms) and count of the lattice
 * passes and of the bead kernels since the last reset.  Each duration is that of the
 * dispatches themselves: their events are stamped by the launch (hipExtLaunchKernel), not
 * recorded as separate queue entries around it.  A whole step's lattice pass is its fused
 * lattice kernel; a split step's (fpd_step) runs from the earlier start to the later end of
 * its fluid and fiber kernels, which run beside each other.  The first split step after
 * fpd_init_fiber or fpd_load runs whole and untimed. */
int fpd_kernel_times(fpd_sim *s, double *ms_lattice, int64_t *n_lattice, double *ms_bead,
                     int64_t *n_bead);
int fpd_reset_kernel_times(fpd_sim *s);

/* Device-to-device copy of `bytes` (multiple of 16) on hip_stream, repeated `iters` times
 * after one warm-up; *gbps receives (read + write bytes) / mean time.  A bandwidth yardstick
 * for the lattice kernel. */
int fpd_copy_probe(void *hip_stream, size_t bytes, int32_t iters, double *gbps);

/* ------------------------------------------------------------- checkpoint ---- */

/* Save / restore the whole state of the time integration of Sec. II.C: populations (in
 * storage format), bead state (R, V, F of Sec. II.B and the derived A_i, window and health),
 * step count and parameters, to / from the file at path.  fpd_load requires a simulation
 * created with the same parameters (FPD_EINVAL otherwise, the simulation unchanged); a
 * file that cannot be opened or is truncated gives FPD_EINVAL, a failed write FPD_EDEVICE.
 * Both synchronise. */
int fpd_save(fpd_sim *s, const char *path);
int fpd_load(fpd_sim *s, const char *path);

/* ---------------------------------------------------- no device allocation ---- */
/* For callers that cannot allocate device memory: code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc.  fpd_run_static runs one simulation of p for
 * n_steps steps with the results of fpd_create_with_buffers + fpd_init_fiber + fpd_step
 * (bitwise the same populations and bead positions) but calls no allocator: the bead state
 * and the force-density window live in a device array of FPD_STATIC_SCRATCH_BYTES that the
 * library holds on every device it runs on until the process ends.
 *   f_a, f_b   caller-owned device buffers of bytes_each >= fpd_population_bytes(p) bytes,
 *              16-byte aligned, holding populations in the library's storage format.  The
 *              state is read from f_a; after the call it sits in f_a if n_steps is even,
 *              in f_b if it is odd (the other buffer is overwritten).
 *   init_populations  non-zero: first write the initial state of p->init_flow into f_a
 *              (what fpd_create_with_buffers writes there).
 *   R_in       device [n_beads][2]: the bead positions to start from (read on the stream
 *              before any step; NULL when n_beads = 0).
 *   R_out      device [n_beads][2]: receives the positions after n_steps (may be R_in).
 *   health     device uint32 or NULL: receives the FPD_HEALTH_* bits of this call; bead
 *              positions fpd_init_fiber would refuse show here (e.g. FPD_HEALTH_WALL).
 *   hip_stream hipStream_t, NULL for the null stream.  The call only enqueues work.
 * FPD_EINVAL, with nothing enqueued, if p is invalid, a buffer is missing, too small or
 * misaligned, or the bead state and force window need more than FPD_STATIC_SCRATCH_BYTES
 * (fpd_static_scratch_need gives the size: one fiber whose window side
 * 1.5 (N - 1) l_0 + 2 (a + cutoff xi) + 4 is up to about 720 nodes in FP64 and 1020
 * otherwise; several fibers up to about 0.5M (FP64) or 1M lattice nodes).
 * Every call on a device uses that device's one array, which keeps the last call's
 * contents (each call clears what it needs): calls that overlap on one device, from other
 * streams or threads, race and give wrong results. */
#define FPD_STATIC_SCRATCH_BYTES 8388608

/* Bytes of the static scratch array that fpd_run_static needs for p (0 without beads). */
size_t fpd_static_scratch_need(const fpd_params *p);

int fpd_run_static(const fpd_params *p, void *hip_stream, void *f_a, void *f_b,
                   size_t bytes_each, int32_t init_populations, const double *R_in,
                   double *R_out, uint32_t *health, int64_t n_steps);

/* ------------------------------------------------------------------ batch ---- */
/* A batch holds independent simulations of different lattice sizes (one storage format)
 * and advances all active ones together: each step is one forces kernel (a block per
 * simulation), one lattice kernel over every (simulation, tile) pair and one bead kernel
 * over every (simulation, bead) pair, replayed from a captured graph.  The parameter-sweep workload of the paper
 * (Sec. IV: stiffness, Re_ps 1-10, confinement) is the intended use.  Per-simulation
 * arithmetic is the single-simulation path's, so a result is bitwise the same alone and
 * in any mix. */

typedef struct fpd_batch fpd_batch;

#define FPD_SIM_ACTIVE  0   /* still running                                             */
#define FPD_SIM_DONE    1   /* reached its step target; results readable until release   */
#define FPD_SIM_FAILED  2   /* evicted by a health check (FPD_HEALTH_* bits set)          */

/* Device bytes one simulation of p occupies in a batch (populations, fiber window, bead
 * state). */
size_t fpd_sim_footprint(const fpd_params *p);

/* A batch for the parameter sweeps of Sec. IV (Figs. 7-10): hbm_budget_bytes caps the sum
 * of footprints of held simulations; max_slots caps their number (<= 4096); storage is one
 * of FPD_F64..FPD_BF16DEV for every member (FPD_EINVAL otherwise).  hip_stream as for
 * fpd_create.  The caller owns *out and frees it with fpd_batch_destroy. */
int fpd_batch_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t storage,
                     void *hip_stream, fpd_batch **out);

/* Launch shape of the batch's lattice kernel (graph_chunk: steps per replayed graph). */
int fpd_batch_set_launch(fpd_batch *b, const fpd_launch *cfg);

/* Admit one simulation of the problem of Sec. IV.A (as fpd_create + fpd_init_fiber):
 * p->storage must be the batch's; R is host [n_beads][2] (NULL when n_beads = 0); it will
 * run n_steps >= 0 steps.  FPD_ENOMEM when no slot is free or the footprint would exceed
 * the budget (nothing is allocated then); FPD_EINVAL for invalid parameters or beads.
 * *sim_id > 0. */
int fpd_batch_add(fpd_batch *b, const fpd_params *p, const double *R, int64_t n_steps,
                  int64_t *sim_id);

/* Advance every active simulation by min(max_steps, smallest remaining count) steps of
 * Sec. II.C (*advanced receives it; 0 when none is active), then check health: a
 * simulation with a health bit set becomes FPD_SIM_FAILED, the others continue.
 * Synchronises; FPD_EDEVICE on a HIP error. */
int fpd_batch_run(fpd_batch *b, int64_t max_steps, int64_t *advanced);

/* fpd_batch_run in two halves, so that batches on different streams advance at the same
 * time from one host thread (while one batch's latency-bound bead and force kernels run,
 * another's lattice kernel fills the device).  fpd_batch_launch enqueues on the batch's
 * stream the steps fpd_batch_run would take and the health read-back, and returns without
 * waiting (*advanced receives the step count, 0 when none is active); fpd_batch_wait waits
 * for them and then updates step counts and statuses as fpd_batch_run does (FPD_OK at once
 * when nothing is pending).  While a launch is pending every other call on the batch
 * except fpd_batch_poll, fpd_batch_stats and fpd_batch_destroy fails with FPD_EINVAL, and
 * fpd_batch_poll reports statuses as of the last wait.  FPD_EDEVICE on a HIP error. */
int fpd_batch_launch(fpd_batch *b, int64_t max_steps, int64_t *advanced);
int fpd_batch_wait(fpd_batch *b);

/* Simulations that became DONE or FAILED since the last poll: ids[i], status[i]
 * (up to cap; *n receives the count). */
int fpd_batch_poll(fpd_batch *b, int64_t *ids, int32_t *status, int32_t cap, int32_t *n);

/* Read-back of a held simulation (same conventions as the single-simulation calls). */
int fpd_batch_read_beads(fpd_batch *b, int64_t sim_id, double *R, double *V, double *F);
int fpd_batch_read_populations(fpd_batch *b, int64_t sim_id, double *f);
int fpd_batch_read_fields(fpd_batch *b, int64_t sim_id, double *rho, double *ux, double *uy,
                          double *eta);
int fpd_batch_particle_stats(fpd_batch *b, int64_t sim_id, int32_t bead, double *out);
/* fpd_set_static_phi, fpd_record_start, fpd_record_read for a simulation of the batch. */
int fpd_batch_set_static_phi(fpd_batch *b, int64_t sim_id, const double *phi);
int fpd_batch_record_start(fpd_batch *b, int64_t sim_id, int32_t every, int64_t capacity);
int fpd_batch_record_read(fpd_batch *b, int64_t sim_id, double *out, int64_t cap_records,
                          int64_t *n_records);
int fpd_batch_sim_info(fpd_batch *b, int64_t sim_id, int64_t *steps, int32_t *status,
                       uint32_t *health);

/* Free a held simulation (any status). */
int fpd_batch_release(fpd_batch *b, int64_t sim_id);

/* Active and held simulation counts and device bytes in use. */
int fpd_batch_stats(fpd_batch *b, int32_t *active, int32_t *held, size_t *bytes_in_use);

void fpd_batch_destroy(fpd_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* FPDLBM_H */
