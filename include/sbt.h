/*
 * sbt.h -- C ABI of the MI355X (gfx950) lattice-Boltzmann / immersed-boundary
 * hot path of SBoTFlow (arXiv 2402.04606).
 *
 * The calls follow the paper's statement of the problem (Sec. 2.5): the
 * solver receives geometry and refinement, motion and flow parameters,
 * builds a block mesh, initialises the populations, runs the recursive
 * LBM/IBM time step of Algorithm 1 and hands back macroscopic fields, the
 * per-marker forces and the total body force of Eq. (16).
 *
 * Conventions
 *  - Every function returns sbt_status: 0 on success, < 0 on failure; the
 *    message of the last failure of the calling thread is sbt_last_error().
 *    No C++ exception crosses this boundary.
 *  - Host pointers are borrowed for the duration of the call only.
 *  - Device memory: the caller allocates one buffer of the size sbt_plan()
 *    reports and passes it, with a HIP stream, to sbt_create(); the library
 *    carves all device state out of it and never frees it.  The caller keeps
 *    ownership of buffer and stream and must keep both alive until
 *    sbt_destroy().  The library owns its host metadata and HIP graphs.
 *  - All device work is enqueued on that stream, in order.  sbt_step() does
 *    not block; the read functions synchronise the stream.
 *  - Coordinates are cell-centred: the centre of cell i is at i + 1/2, in the
 *    lattice units of the level concerned.  Marker data are in finest-level
 *    units of their case.  Velocities are lattice velocities (the same number
 *    on every level under the acoustic scaling used here).
 *  - Dense field arrays of level l are row-major [ny0*2^l][nx0*2^l].
 *  - One context is not thread-safe: do not call it from two threads at once.
 *  - Several cases may share one context (a batch).  They are advanced
 *    together: with V = max n_levels, level l of a case with m levels runs as
 *    virtual level l + V - m, and one sbt_step is one virtual-level-0 step, i.e.
 *    2^(V-m) coarse steps of that case.
 */
#ifndef SBT_H
#define SBT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbt_ctx sbt_ctx;
typedef int32_t sbt_status;

enum {
    SBT_OK = 0,
    SBT_ERR_ARG = -1,            /* bad argument or descriptor                    */
    SBT_ERR_TOPOLOGY = -2,       /* refinement violates nesting / 2:1 / edges     */
    SBT_ERR_DEVICE = -3,         /* a HIP call failed                             */
    SBT_ERR_NOMEM = -4,          /* device buffer smaller than sbt_plan() asked   */
    SBT_ERR_STATE = -5,          /* call not allowed in the current state         */
    SBT_ERR_NONFINITE = -6,      /* a density became NaN or Inf                   */
    SBT_ERR_MARKER_OUTSIDE = -7, /* a marker stencil left the finest owned cells  */
    SBT_ERR_BUFSIZE = -8         /* host buffer of the wrong size                 */
};

/* Population storage.  F64 stores f_i and computes in FP64.  F32, F16S and
 * BF16S store the deviation f_i - w_i rho0 and compute in FP32; F16S/BF16S
 * round to nearest even.  Marker kinematics, the MDF force accumulation and
 * all reductions are FP64 in every mode. */
enum { SBT_F64 = 0, SBT_F32 = 1, SBT_F16S = 2, SBT_BF16S = 3 };

/* Domain edge kinds (Sec. 2.1 names them; the formulas are textbook):
 * PERIODIC; WALL = half-way bounce-back with moving-wall term (velocity
 * bc_u, wall density rho0); INFLOW_EQ = equilibrium at (rho0, bc_u);
 * OUTFLOW = zero-gradient copy from the interior neighbour; SYMMETRY =
 * specular (free-slip) reflection.  A corner population (source beyond two
 * non-periodic edges) takes the W/E edge's rule unless only the S/N edge is a
 * wall or inflow; cells that rule refers to are clamped into the domain. */
enum { SBT_BC_PERIODIC = 0, SBT_BC_WALL = 1, SBT_BC_INFLOW_EQ = 2, SBT_BC_OUTFLOW = 3,
       SBT_BC_SYMMETRY = 4 };
enum { SBT_EDGE_W = 0, SBT_EDGE_E = 1, SBT_EDGE_S = 2, SBT_EDGE_N = 3 };

/* Coarse-fine interface operator (Sec. 2.4, steps (2) and (6)).
 * HOMOGENEOUS: halo cells take the coarse post-collision populations as
 * they are; coarse cells take the mean of their four children (Rohde's
 * mass-conservative scheme cited by the paper).  RESCALE additionally scales
 * the non-equilibrium part by (tau_f - 1)/(2 (tau_c - 1)) coarse->fine and by
 * 2 tau_c / tau_f fine->coarse; it requires |tau - 1| > 1e-6 on coarse levels. */
enum { SBT_CF_HOMOGENEOUS = 0, SBT_CF_RESCALE = 1 };

/* Collision (Sec. 2.1).  BGK: Eqs. (2)-(3) with Guo forcing.  MRT: the
 * multiple-relaxation-time option the paper names for low viscosity, on the
 * orthogonal D2Q9 moment basis (rho, e, eps, jx, qx, jy, qy, pxx, pxy).  The
 * moments relax toward those of the Eq. (7) equilibrium at rates
 * (-, s_e, s_eps, -, s_q, -, s_q, 1/tau_l, 1/tau_l); Guo's forcing enters in
 * moment space as (I - S/2) M Fbar, Fbar being Eq. (3)'s term without its
 * 1 - 1/(2 tau) factor.  Equal rates 1/tau reproduce BGK.  Same viscosity
 * nu = (tau - 1/2)/3; the interface rescaling uses tau as for BGK. */
enum { SBT_COLL_BGK = 0, SBT_COLL_MRT = 1 };

/* Body kinematics (marker positions r_j(t) of Sec. 2.2):
 * FIXED: r_j = (p[0] + xb_j, p[1] + yb_j), desired velocity 0.
 * FLAP : the flapping law of Sec. 3.6 with free amplitudes:
 *        ts = t p[8] / p[9] (t = finest substep), theta = 2 pi ts / p[6],
 *        alpha = p[2] - p[3] sin(theta + p[7]),
 *        centre = (p[0], p[1]) + (p[4]/2) cos(theta) (cos p[5], sin p[5]),
 *        r_j = centre + (xb cos a + yb sin a, -xb sin a + yb cos a).
 *        p = {x0, y0, alpha0, A_pitch, A0, beta, T, phi, U_ref, chord}.
 * HOST : positions and desired velocities given by sbt_set_markers.
 * RAMP : the pitch-up ramp of Sec. 3.5, a pure pitch about the pivot
 *        (p[0], p[1]) (the body-frame origin; the paper pivots about the
 *        leading edge): ts as for FLAP, t2 = t1 + A / (2K),
 *        G(ts) = log[cosh(a_s (ts - t1)) / cosh(a_s (ts - t2))] - a_s (t1 - t2),
 *        alpha = A G / (2 a_s (t2 - t1)) (the supremum of G, so alpha -> A),
 *        r_j = (p[0], p[1]) + (xb cos a + yb sin a, -xb sin a + yb cos a).
 *        p = {x0, y0, A, a_s, K, t1, -, -, U_ref, chord}; a_s, K > 0.
 * TRI  : the smoothed asymmetric triangular pitching law of Sec. 3.6 about
 *        (p[0], p[1]), period T in ts units (T = pi / k for reduced
 *        frequency k = pi f c / U), ta = p[5] T: ramps of rate
 *        2 alpha0 / (xi T - ta) and -2 alpha0 / ((1 - xi) T - ta) joined by
 *        quartic blends of duration ta before and after each extreme
 *        +alpha0 at ts = xi T / 2 and -alpha0 at ts = T (1 - xi / 2); the
 *        quartics use ta in every denominator (the only choice that keeps
 *        alpha and its rate continuous).  alpha(0) = 0, rising.
 *        p = {x0, y0, alpha0, xi, T, ta/T, -, -, U_ref, chord};
 *        0 < xi < 1, 0 < ta/T <= min(xi, 1 - xi) / 2.
 * Every moving kind: desired velocity u_d = r_j(t + 1) - r_j(t). */
enum { SBT_BODY_FIXED = 0, SBT_BODY_FLAP = 1, SBT_BODY_HOST = 2, SBT_BODY_RAMP = 3, SBT_BODY_TRI = 4 };

typedef struct {
    int32_t level;                 /* >= 1                                        */
    int32_t bx0, by0, bx1, by1;    /* half-open box in level-`level` block units  */
} sbt_box;

/* Solid cells with interpolated bounce-back: the paper's solid-cell
 * alternative to the IBM (Sec. 2.1; compared with it in Sec. 3.2), in the
 * linear form of Bouzidi, Firdaouss and Lallemand for a resting wall.  A
 * fluid cell x pulls population i from a solid neighbour x - c_i instead
 * from the population o = opposite(i) it sent toward the wall, which sits at
 * fraction q of the link x -> x + c_o:
 *   q <  1/2:  f_i(x) = 2q f*_o(x) + (1 - 2q) f*_o(x - c_o),
 *   q >= 1/2:  f_i(x) = f*_o(x) / (2q) + (2q - 1)/(2q) f*_i(x)
 * (q = 1/2 is half-way bounce-back; where q < 1/2 and x - c_o is solid too,
 * the link takes q = 1/2).  Solid cells are not collided and read out as NaN.
 * mask: dense level cells [ny][nx], nonzero = solid.  q: dense [ny][nx][9],
 * q[x][i] the wall fraction of the link from fluid cell x toward a solid
 * x + c_i (0 < q <= 1, read only there); NULL = 1/2 everywhere.  Every cell
 * within two cells of a solid cell must be an owned cell of that level not
 * covered by a finer level (no halo, no interface, inside the domain or
 * across a periodic edge).  Host arrays, read during sbt_plan/sbt_create. */
typedef struct {
    int32_t level;
    const uint8_t *mask;
    const double *q;
} sbt_solid;

typedef struct {
    int32_t nx0, ny0;              /* level-0 cells, multiples of block_n          */
    int32_t block_n;               /* cells per block edge; must be 16             */
    int32_t n_levels;              /* m, 1..6                                      */
    const sbt_box *refine;         /* region of level l = union of its boxes;      */
    int32_t n_refine;              /*   validated for nesting, 2:1 and edges       */
    double tau0, rho0;             /* tau_l = 1/2 + 2^l (tau0 - 1/2)               */
    int32_t bc[4];                 /* edge kinds, order W, E, S, N                 */
    double bc_u[4][2];             /* wall / inflow velocity per edge              */
    double fext[2];                /* uniform body-force density (level-0 units);
                                      level l uses fext / 2^l                      */
    int32_t storage;               /* SBT_F64 ... (same for every case of a ctx)   */
    int32_t cf_mode;               /* SBT_CF_*                                     */
    int32_t mdf_iters;             /* N_F of the multi-direct-forcing loop         */
    int32_t max_markers;           /* capacity for sbt_set_body; 0 = no body       */
    int32_t history_cap;           /* finest substeps of force history kept        */
    int32_t collision;             /* SBT_COLL_* (same for every case of a ctx)    */
    double mrt_rates[3];           /* SBT_COLL_MRT: s_e, s_eps, s_q in (0, 2)      */
    const sbt_solid *solids;       /* solid regions (at most one per level)        */
    int32_t n_solids;
} sbt_case_desc;

typedef struct {
    int32_t n;                     /* markers, <= max_markers                      */
    const double *xb, *yb, *ds;    /* body-frame coordinates and arc length
                                      (SBT_BODY_HOST: absolute marker positions in
                                      finest-level cells, desired velocity 0 until
                                      sbt_set_markers)                              */
    int32_t kind;                  /* SBT_BODY_*                                   */
    double p[16];                  /* kinematic parameters                         */
} sbt_body;

/* Validate the cases and report the device bytes sbt_create() needs.  Host
 * only; makes no HIP call.  Errors: SBT_ERR_ARG, SBT_ERR_TOPOLOGY. */
sbt_status sbt_plan(const sbt_case_desc *cases, int32_t n_cases, size_t *device_bytes);

/* Build the block forest (Sec. 2.3: square 16x16-cell blocks, levels
 * 0..m-1, blocks Morton-ordered per level), upload tables into device_buf
 * (at least the planned bytes, 256-byte aligned) and set every case to rest
 * at rho0.  hip_stream is a hipStream_t (NULL = legacy default stream). */
sbt_status sbt_create(const sbt_case_desc *cases, int32_t n_cases, void *device_buf, size_t bytes,
                      void *hip_stream, sbt_ctx **out);
sbt_status sbt_destroy(sbt_ctx *ctx);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, hosts that forbid hipMalloc): sbt_create
 * with the context's device memory in the library's file-scope static
 * device array of SBT_STATIC_BYTES per GPU (each GPU the library runs on
 * holds its own copy until the process ends) instead of a caller buffer.
 * The current device's array is used; the cases must plan to at most
 * SBT_STATIC_BYTES (else SBT_ERR_NOMEM, nothing created).  One such context
 * may live per device at a time: a call while another one is alive on the
 * same device returns SBT_ERR_STATE; sbt_destroy frees the array for the
 * next.  Calls that overlap on one device from several threads race for
 * the array and must be serialised by the caller.  Everything else is
 * sbt_create's: same kernels, same results, the same calls on the context
 * afterwards.  Makes no device allocation (no hipMalloc or hipFree). */
#define SBT_STATIC_BYTES ((size_t)128 << 20)
sbt_status sbt_create_static(const sbt_case_desc *cases, int32_t n_cases, void *hip_stream, sbt_ctx **out);

/* Blocks of a case's level that own at least one cell, Morton order; origins
 * in level cells.  ox/oy may be NULL (then only the count is returned). */
sbt_status sbt_level_blocks(sbt_ctx *ctx, int32_t c, int32_t level, int32_t *n_blocks,
                            int32_t *ox, int32_t *oy);
/* out = {owned cells, owned-cell blocks, halo blocks, substeps per sbt_step}. */
sbt_status sbt_level_info(sbt_ctx *ctx, int32_t c, int32_t level, int64_t out[4]);

/* f = f^eq(rho, u) (Eq. (7)) on the owned cells of a level, from dense FP64
 * arrays; other cells' values are ignored.  Puts the context back to its
 * initial (pre-collision) state: force history and substep count restart. */
sbt_status sbt_init_fields(sbt_ctx *ctx, int32_t c, int32_t level, const double *rho,
                           const double *ux, const double *uy);
/* f = f^eq(rho, (ux, uy)) on every owned cell of every level of a case (a
 * uniform initial state); same state semantics as sbt_init_fields. */
sbt_status sbt_init_uniform(sbt_ctx *ctx, int32_t c, double rho, double ux, double uy);
/* Attach a body to a case (copied in).  Only before the first sbt_step after
 * create/init.  n <= max_markers. */
sbt_status sbt_set_body(sbt_ctx *ctx, int32_t c, const sbt_body *body);
/* Markers placed by the caller (Sec. 2.2 takes the Lagrangian positions and
 * their desired velocities as given): for a case whose body is
 * SBT_BODY_HOST, every forcing loop that the following sbt_step calls run
 * uses positions x, y (finest-level cells) and desired velocities udx, udy
 * (finest-level lattice units), n = the body's marker count, until the next
 * call; ds (may be NULL: keep the current values) replaces the markers'
 * arc-length weights ds_j of Eqs. (15)-(16) as well.  A step collides one
 * finest substep ahead of what the readouts show: after the readouts show
 * finest substep s, the next forcing loop is that of substep s + 1 (the
 * first sbt_step runs substeps 0 and 1).  Host arrays, copied in; waits for
 * the context's stream.  Errors: SBT_ERR_ARG (not a HOST body, n differs
 * from the body's marker count, null positions or velocities, ds not
 * positive and finite). */
sbt_status sbt_set_markers(sbt_ctx *ctx, int32_t c, int32_t n, const double *x, const double *y,
                           const double *udx, const double *udy, const double *ds);

/* Advance every case by n virtual-level-0 steps (Algorithm 1, each level
 * sub-cycled 2^l times).  Asynchronous, stream-ordered. */
sbt_status sbt_step(sbt_ctx *ctx, int32_t n);
/* Wait for the stream; report SBT_ERR_NONFINITE / SBT_ERR_MARKER_OUTSIDE if
 * the device raised them (the flags are then cleared). */
sbt_status sbt_synchronize(sbt_ctx *ctx);

/* rho and u = (sum_i c_i f_i + F_ext/2)/rho (Eq. (8) without the IBM force,
 * which is defined only inside a substep) on owned cells of the level; NaN on
 * other cells.  Dense FP64 arrays.  Synchronises. */
sbt_status sbt_read_fields(sbt_ctx *ctx, int32_t c, int32_t level, double *rho, double *ux,
                           double *uy);
/* As sbt_read_fields, in block order: out[n_blocks][3][256] holds rho, ux,
 * uy of the blocks sbt_level_blocks lists (NaN on cells covered by the finer
 * level).  Synchronises. */
sbt_status sbt_read_fields_blocks(sbt_ctx *ctx, int32_t c, int32_t level, double *out);
/* Total MDF force F_j of every marker at the last completed finest substep
 * (sum over the N_F iterations of Eq. (11)). */
sbt_status sbt_read_marker_forces(sbt_ctx *ctx, int32_t c, double *fx, double *fy);
/* Body force F_s = -sum_j F_j ds_j (Eq. (16)) per completed finest substep,
 * oldest first; at most min(cap, history_cap) most recent entries. */
sbt_status sbt_read_force_history(sbt_ctx *ctx, int32_t c, int32_t cap, double *fx, double *fy,
                                  int32_t *n_out);
/* out = {mass, momentum x, momentum y}: sums over owned cells of rho,
 * sum_i c_i f_i, weighted by the cell volume 4^-l.  Computed on the device in
 * FP64 with a fixed reduction order. */
sbt_status sbt_diagnostics(sbt_ctx *ctx, int32_t c, double out[3]);

/* Force-coefficient statistics of Sec. 3.3, Eq. (21), over the most recent
 * min(n_last, recorded, history_cap) finest substeps of the force history:
 * C_D = F_s,x / (rho0 U^2 L / 2), C_L = F_s,y / (rho0 U^2 L / 2), with U the
 * reference velocity (lattice units) and L the reference length (finest
 * cells).  out = {mean C_D, mean C_L, rms of C_D about its mean (C_D'), rms
 * of C_L about its mean (C_L'), St, upward crossings of C_L through its mean,
 * samples}.  St = f L / U, where f is the lift frequency taken from the
 * history: (crossings - 1) periods between the first and the last upward
 * crossing, crossing times interpolated linearly between substeps (finest
 * substeps as the time unit); St = 0 with fewer than two crossings.
 * Computed on the device in FP64 (fixed reduction order).  Errors:
 * SBT_ERR_ARG (n_last <= 0, U or L not positive, null out), SBT_ERR_STATE
 * (no body, or fewer than two recorded substeps).  Synchronises. */
sbt_status sbt_force_stats(sbt_ctx *ctx, int32_t c, int32_t n_last, double U, double L, double out[7]);

/* Convergence criterion of Sec. 3.2: E = sum_x |u(x, t) - u(x, t0)| /
 * sum_x |u(x, t)| over the leaf cells x of the case (owned cells not covered
 * by a finer level, every level), each weighted by its area 4^-l (a uniform
 * grid gives the paper's plain sums); |.| is the Euclidean norm of the
 * velocity (Eq. (8) without the IBM force, as sbt_read_fields).  The velocity
 * at t0 lives in a caller-owned DEVICE buffer `snapshot` (8-byte aligned, at
 * least sbt_snapshot_bytes; layout [level][owned block][ux, uy][256] FP64,
 * levels in order, blocks in sbt_level_blocks order; covered cells hold 0).
 * mode SBT_SNAP_STORE: the snapshot takes the current velocity (out unused,
 * may be NULL); SBT_SNAP_COMPARE: out = {sum |u - u0|, sum |u|, E};
 * both: compare, then store (a rolling check every fixed number of steps,
 * 1000 in the paper).  Device reductions in FP64, fixed order.  Errors:
 * SBT_ERR_ARG (bad mode, null or misaligned snapshot), SBT_ERR_BUFSIZE.
 * Synchronises. */
enum { SBT_SNAP_STORE = 1, SBT_SNAP_COMPARE = 2 };
sbt_status sbt_snapshot_bytes(sbt_ctx *ctx, int32_t c, size_t *bytes);
sbt_status sbt_convergence(sbt_ctx *ctx, int32_t c, void *snapshot, size_t bytes, int32_t mode,
                           double out[3]);

/* Checkpoint: raw state (populations of both lattices of every level, halo
 * cells, substep counters, marker forces, force history).  sbt_state_bytes
 * gives the size; write_state requires the same descriptors. */
sbt_status sbt_state_bytes(sbt_ctx *ctx, size_t *bytes);
sbt_status sbt_read_state(sbt_ctx *ctx, void *host, size_t bytes);
sbt_status sbt_write_state(sbt_ctx *ctx, const void *host, size_t bytes);

/* Tuning and measurement.
 * SBT_OPT_GRAPH (default 1): replay steps as captured HIP graphs (of 4, 2 and 1
 *   steps; all are captured at the first step that uses one).
 * SBT_OPT_TILE: interior 16x16 blocks per workgroup of the stream+collide
 *   launch, 1..16 for every level (a workgroup loads block j+1 while it
 *   computes block j); 0 (default) = automatic per launch size.
 * SBT_OPT_XCD_REMAP (default 1): map consecutive Morton blocks to one XCD.
 * SBT_OPT_PERSISTENT (default 0): run each step as one persistent launch
 *   (plan builder, forcing loops and level substeps as phases separated by
 *   grid barriers, every level block through the generic per-cell path)
 *   instead of the chain of launches.  FP64 results are the same bit for
 *   bit; the deviation forms may differ in the last bits (the per-cell path
 *   rounds some FP32 sums differently).  A barrier that times out makes
 *   sbt_synchronize report SBT_ERR_DEVICE.  The
 *   launch sizes its grid to fill every CU, so kernels of other streams
 *   running at the same time can keep a workgroup from starting and make a
 *   barrier time out.
 * SBT_OPT_BARRIER_SPINS: polls a grid-barrier wait of the persistent step
 *   makes before it gives up; 0 (default) = 2^21 (about a second).  A small
 *   value forces the time-out path (for tests of it). */
enum { SBT_OPT_GRAPH = 0, SBT_OPT_TILE = 1, SBT_OPT_XCD_REMAP = 2, SBT_OPT_PERSISTENT = 3, SBT_OPT_BARRIER_SPINS = 4 };
sbt_status sbt_set_option(sbt_ctx *ctx, int32_t option, int32_t value);
/* Pick the blocks per workgroup of each level by timing `steps` steps per
 * trial (1, 2, 3, 4, 6, 8; finest level first, one level at a time) and keep the
 * fastest; if cache_path is non-NULL the choice is read from / written to
 * that JSON file keyed by the storage and the block counts.  The simulation
 * state is restored afterwards. */
sbt_status sbt_autotune(sbt_ctx *ctx, int32_t steps, const char *cache_path);
/* Run n steps eagerly with HIP events around every launch, on the context's
 * stream.  out[0] = total ms of level (collide+stream) kernels, out[1] = their
 * launch count, out[2] = total ms of MDF kernels, out[3] = their count,
 * out[4] = algorithmic bytes moved by the level kernels (2 Q s per cell
 * update), out[5] = cell updates, out[6] = ms of the per-substep tile kernel
 * (all owned blocks and halo bands), out[7] = its launch count, out[8] = its
 * algorithmic bytes. */
sbt_status sbt_profile(sbt_ctx *ctx, int32_t n, double out[9]);
/* Cell updates performed per sbt_step, summed over cases and levels. */
sbt_status sbt_updates_per_step(sbt_ctx *ctx, int64_t *updates);

const char *sbt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SBT_H */
