/*
 * oracle.h -- plain FP64 CPU oracle for the lattice-Boltzmann / multi-direct-
 * forcing immersed-boundary time step of SBoTFlow (arXiv 2402.04606).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check
 * and the CPU-baseline leg of the benchmark may load this library.  It shares
 * no code, header, table or helper with the GPU library; the two meet only
 * through the seeded workload generators in `workloads/`.
 *
 * Data layout: every refinement level l is held as a dense array covering the
 * whole domain at that level's resolution (nx0*2^l x ny0*2^l cells), row-major,
 * 9 populations per cell, direction order of Eq. (1).  Cells that are neither
 * owned nor halo cells of the level hold NaN, so any read of an undefined
 * population shows up in the results.
 *
 * All functions return 0 on success or a negative code (ORC_ERR_*).
 */
#ifndef SBT_ORACLE_H
#define SBT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_TOPOLOGY = -2, ORC_ERR_MARKER = -7 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_WALL = 1, ORC_BC_INFLOW = 2, ORC_BC_OUTFLOW = 3,
       ORC_BC_SYMMETRY = 4 };
enum { ORC_CF_HOMOGENEOUS = 0, ORC_CF_RESCALE = 1 };
enum { ORC_BODY_NONE = -1, ORC_BODY_FIXED = 0, ORC_BODY_FLAP = 1, ORC_BODY_HOST = 2,
       ORC_BODY_RAMP = 3, ORC_BODY_TRI = 4 };
enum { ORC_W = 0, ORC_E = 1, ORC_S = 2, ORC_N = 3 };
enum { ORC_COLL_BGK = 0, ORC_COLL_MRT = 1 };

typedef struct {
    int32_t nx0, ny0;        /* level-0 cells                                   */
    int32_t block_n;         /* cells per block edge (boxes are in block units) */
    int32_t n_levels;        /* m >= 1                                           */
    int32_t n_boxes;         /* refinement boxes, 5 ints each:                   */
    const int32_t *boxes;    /*   level, bx0, by0, bx1, by1 (half-open, level-l
                                   block units); region_l = union of its boxes   */
    double tau0, rho0;       /* level-0 relaxation time, reference density      */
    int32_t bc[4];           /* edge kinds, order W, E, S, N                     */
    double bc_u[8];          /* (ux, uy) per edge: wall / inflow velocity        */
    double fext[2];          /* uniform body-force density, level-0 units        */
    int32_t cf_mode;         /* ORC_CF_*                                         */
    int32_t mdf_iters;       /* N_F                                              */
    int32_t body_kind;       /* ORC_BODY_*                                       */
    int32_t n_markers;
    const double *xb, *yb;   /* body-frame marker coordinates, finest cells
                                (ORC_BODY_HOST: absolute positions)              */
    const double *ds;        /* marker arc lengths, finest cells                 */
    double bp[16];           /* kinematic parameters (see orc_body_positions)    */
    int32_t collision;       /* ORC_COLL_*                                       */
    double mrt[3];           /* MRT rates s_e, s_eps, s_q (shear rate 1/tau_l)   */
} orc_case;

typedef struct orc_sim orc_sim;

int  orc_create(const orc_case *c, orc_sim **out);
void orc_destroy(orc_sim *s);
int  orc_level_size(const orc_sim *s, int level, int32_t *nx, int32_t *ny);
/* Kind map of a level: 0 none, 1 own, 2 ghost (halo), 3 hidden (covered by l+1). */
int  orc_level_kinds(const orc_sim *s, int level, uint8_t *kind);
/* f = f^eq(rho, u) with F = 0 on the owned cells of `level` (dense arrays). */
int  orc_init_fields(orc_sim *s, int level, const double *rho, const double *ux,
                     const double *uy);
/* Pre-collision populations of the owned cells of `level`, dense [ny][nx][9]. */
int  orc_init_populations(orc_sim *s, int level, const double *f);
/* RESCALE factors {s_cf (coarse -> fine, post-collision), s_fc (fine ->
 * coarse, pre-collision)} for relaxation times tau_c (coarse), tau_f (fine). */
void orc_interface_factors(double tau_c, double tau_f, double out[2]);
/* Advance n coarse (level-0) time steps. */
int  orc_step(orc_sim *s, int32_t n);
/* rho and u = (sum_i c_i f_i + F_ext/2)/rho on owned cells, NaN elsewhere. */
int  orc_read_fields(const orc_sim *s, int level, double *rho, double *ux, double *uy);
/* Raw populations of a level, dense [ny][nx][9]. */
int  orc_read_populations(const orc_sim *s, int level, double *f);
int  orc_marker_forces(const orc_sim *s, double *fx, double *fy);
/* ORC_BODY_HOST: marker positions X, Y (finest cells) and desired velocities
 * used by every finest substep from the next orc_step on (Sec. 2.2 takes
 * both as given); ds (NULL: unchanged) replaces the markers' arc-length
 * weights. */
int  orc_set_markers(orc_sim *s, int32_t n, const double *X, const double *Y, const double *udx,
                     const double *udy, const double *ds);
int  orc_force_history(const orc_sim *s, int32_t cap, double *fx, double *fy, int32_t *n_out);
/* out = {mass, momentum x, momentum y}, each summed over owned cells with
 * volume weight 4^-l; momentum is the bare first moment sum_i c_i f_i. */
int  orc_diagnostics(const orc_sim *s, double out[3]);
int64_t orc_substeps(const orc_sim *s);
/* Solid cells of a level with interpolated bounce-back on their links (the
 * solid-cell alternative to the IBM, Sec. 2.1 / Sec. 3.2): mask dense level
 * cells (1 = solid), q dense [cell][9] wall fraction of link i from a fluid
 * cell toward a solid x + c_i (NULL: 1/2).  Before the first step. */
int  orc_set_solid(orc_sim *s, int level, const uint8_t *mask, const double *q);

/* ---- building blocks, exposed so the test-suite can pin them ------------ */
void   orc_velocity_set(int32_t cx[9], int32_t cy[9], double w[9]);
void   orc_feq(double rho, double ux, double uy, double out[9]);
void   orc_guo(double tau, double ux, double uy, double Fx, double Fy, double out[9]);
void   orc_collide_cell(double tau, const double f[9], double Fx, double Fy, double out[9]);
/* MRT collision (moment basis M, its inverse; rates = {s_e, s_eps, s_q}). */
void   orc_mrt_matrices(double M[81], double Minv[81]);
void   orc_collide_cell_mrt(double tau, const double rates[3], const double f[9], double Fx,
                            double Fy, double out[9]);
double orc_phi(double r);
/* Marker positions of the body at finest substep k (time t_k = k). */
int    orc_body_positions(const orc_case *c, double k, double *X, double *Y);
/* Pitch angle of the ramp (Sec. 3.5) and triangular (Sec. 3.6) laws at t*. */
double orc_ramp_alpha(const double *p, double tstar);
double orc_tri_alpha(const double *p, double tstar);
/* The multi-direct-forcing loop on a dense periodic nx x ny grid of cell
 * moments: rho (fixed), u (corrected in place), F (accumulated in place);
 * markers X, Y, desired velocity ud, arc length ds; returns the per-marker
 * total force ftot over all iterations. */
int    orc_mdf(int32_t nx, int32_t ny, const double *rho, double *ux, double *uy,
               double *Fx, double *Fy, int32_t n, const double *X, const double *Y,
               const double *udx, const double *udy, const double *ds, int32_t iters,
               double *ftx, double *fty);
/* Velocity interpolation Eq. (12) at arbitrary points on a dense periodic grid. */
int    orc_interpolate(int32_t nx, int32_t ny, const double *ux, const double *uy,
                       int32_t n, const double *X, const double *Y, double *U, double *V);
/* Force spreading Eq. (15) on a dense periodic grid (adds into Fx, Fy). */
int    orc_spread(int32_t nx, int32_t ny, int32_t n, const double *X, const double *Y,
                  const double *Fjx, const double *Fjy, const double *ds,
                  double *Fx, double *Fy);
/* Eq. (21) statistics of a force history (coefficients C = scale F):
 * out = {mean C_D, mean C_L, C_D', C_L', St, upward crossings, n}. */
int    orc_force_stats(const double *fx, const double *fy, int32_t n, double scale,
                       double l_over_u, double out[7]);
int    orc_num_threads(void);

/* ---- three dimensions: D3Q19 or D3Q27 (q), one periodic level ------------ */
typedef struct orc3_sim orc3_sim;
void orc3_velocity_set(int32_t q, int32_t *cx, int32_t *cy, int32_t *cz, double *w);
void orc3_feq(int32_t q, double rho, double ux, double uy, double uz, double *out);
int  orc3_create(int32_t nx, int32_t ny, int32_t nz, int32_t q, double tau, const double F[3], orc3_sim **out);
void orc3_destroy(orc3_sim *s);
/* f = f^eq(rho, u), dense arrays, cell (z ny + y) nx + x. */
int  orc3_init_fields(orc3_sim *s, const double *rho, const double *ux, const double *uy, const double *uz);
int  orc3_step(orc3_sim *s, int32_t steps);
/* Half-way bounce-back walls below z = 0 and above z = nz - 1 (velocities
 * ub, ut; NULL = at rest; wall density rho0) instead of the periodic z faces. */
int  orc3_set_walls(orc3_sim *s, double rho0, const double ub[3], const double ut[3]);
/* Solid cells with interpolated bounce-back (mask [cell], q [cell][q] wall
 * fraction of the link from a fluid cell toward a solid x + c_i, NULL = 1/2).
 * After orc3_set_walls when both are used. */
int  orc3_set_solid(orc3_sim *s, const uint8_t *mask, const double *q);
/* A fixed immersed body (Sec. 2.2 in 3D): n markers X, Y, Z (cells), surface
 * elements dA, N_F iterations of the forcing loop before every collision. */
int  orc3_set_body(orc3_sim *s, int32_t n, const double *X, const double *Y, const double *Z,
                   const double *dA, int32_t iters);
/* Motion: kind 0 fixed (markers absolute), kind 1 pitch about the y axis and
 * plunge along z, p = {x0, y0, z0, alpha0, A_pitch, A0, T, phi, U_ref, chord}
 * (markers in the body frame); desired velocity r(t + 1) - r(t). */
int  orc3_set_motion(orc3_sim *s, int32_t kind, const double p[10]);
/* F_s = -sum_j F_j dA_j of the last step. */
int  orc3_body_force(const orc3_sim *s, double out[3]);
/* Marker positions of the body at step t (after orc3_set_body/_motion). */
int  orc3_marker_positions(const orc3_sim *s, double t, double *X, double *Y, double *Z);
int  orc3_read_fields(const orc3_sim *s, double *rho, double *ux, double *uy, double *uz);

/* ---- three dimensions on a block forest (periodic, D3Q19 or D3Q27) ------ */
typedef struct {
    int32_t nx0, ny0, nz0;   /* level-0 cells                                     */
    int32_t block_n;         /* cells per block edge (boxes are in block units)   */
    int32_t n_levels, q;     /* m >= 1; 19 or 27                                  */
    int32_t n_boxes;         /* refinement boxes, 7 ints each: level, bx0, by0,   */
    const int32_t *boxes;    /*   bz0, bx1, by1, bz1 (half-open, level-l blocks)  */
    double tau0, rho0;       /* level-0 relaxation time, reference density       */
    double fext[3];          /* uniform body-force density, level-0 units         */
    int32_t cf_mode;         /* ORC_CF_*                                          */
} orc3f_case;
typedef struct orc3f_sim orc3f_sim;
int  orc3f_create(const orc3f_case *c, orc3f_sim **out);
void orc3f_destroy(orc3f_sim *s);
int  orc3f_level_size(const orc3f_sim *s, int level, int32_t out[3]);
/* Kind map of a level: 0 none, 1 own, 2 halo, 3 hidden (dense [z][y][x]). */
int  orc3f_level_kinds(const orc3f_sim *s, int level, uint8_t *kind);
int  orc3f_init_fields(orc3f_sim *s, int level, const double *rho, const double *ux, const double *uy,
                       const double *uz);
int  orc3f_step(orc3f_sim *s, int32_t n);
int  orc3f_read_fields(const orc3f_sim *s, int level, double *rho, double *ux, double *uy, double *uz);
int  orc3f_diagnostics(const orc3f_sim *s, double out[4]);

#ifdef __cplusplus
}
#endif
#endif
