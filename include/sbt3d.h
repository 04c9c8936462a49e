/*
 * sbt3d.h -- the three-dimensional (D3Q19) form of the lattice-Boltzmann
 * collide+stream of SBoTFlow (arXiv 2402.04606, Sec. 2.1 written for the
 * 3D lattices the method extends to), on one periodic level.
 *
 * One step is Eqs. (2)-(3), (6)-(8) in 3D: BGK collision with Guo's forcing
 * term and the half-force velocity, then streaming f(x + c_i, i) = f*(x, i)
 * across periodic faces (or, across z, half-way bounce-back walls with the
 * moving-wall term f_i = f*_o - 6 w_i rho0 (c_o . u_wall), o = opposite(i),
 * as the 2D walls).  Solid cells (solid_mask) take the interpolated
 * bounce-back of the 2D solid cells (linear Bouzidi form, resting wall): a
 * fluid cell pulls direction i from a solid x - c_i as
 *   q <  1/2: 2q f*_o(x) + (1 - 2q) f*_o(x - c_o),
 *   q >= 1/2: f*_o(x) / (2q) + (2q - 1)/(2q) f*_i(x),  o = opposite(i),
 * q = 1/2 where a short link has no fluid cell behind it; solid cells are
 * not collided and read out as NaN.  They add a 4-byte code per cell to
 * each step's reads.  An immersed body (n_markers > 0; Sec. 2.2 in 3D, fixed
 * or in the pitch/plunge motion of motion_p, desired velocity
 * r(t + 1) - r(t)) runs the multi-direct forcing loop before every
 * collision with Peskin's kernel (Eq. (14)) in each axis: N_F passes of
 * U_j, rho_j interpolation over the 4x4x4 taps, g_j = 2 rho_j (u_d - U_j),
 * spreading g_j w dA_j in marker order and u += dF / (2 rho); the cells
 * collide with F_ext + F.  It needs a fully periodic box without solid
 * cells.  Each step's stencils must stay inside the box (no wrap) and
 * inside a box of at most ibm_box_cells cells; a step where they do not
 * runs without the body force and sbt3_synchronize reports
 * SBT_ERR_MARKER_OUTSIDE.  D3Q19: rest (w = 1/3), 6 axis (1/18) and 12 edge
 * (1/36) velocities; D3Q27 adds the 8 corners (rest 8/27, axis 2/27, edge
 * 1/54, corner 1/216); c_s^2 = 1/3 for both.  Direction order: rest,
 * +x -x +y -y +z -z, the edges (+-1, +-1, 0), (+-1, 0, +-1), (0, +-1, +-1),
 * then the corners.
 *
 * Storage forms as for the 2D library (sbt.h): SBT_F64 (f itself, FP64
 * arithmetic) and SBT_F32 / SBT_F16S / SBT_BF16S (the deviation
 * f - w rho0, FP32 arithmetic).  Layout in the caller's device buffer:
 * two lattices [Q][nz][ny][nx] (x fastest) and a staging area for the
 * field transfers.  The kernels pull: after a step a lattice holds
 * post-collision populations and the readout gathers the streamed state
 * from the lattice the last step read.  All functions return sbt_status; sbt_last_error()
 * describes the last failure.  A context must not be used from two threads
 * at once.
 */
#ifndef SBT3D_H
#define SBT3D_H
#include <stddef.h>
#include <stdint.h>

#include "sbt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbt3_ctx sbt3_ctx;

typedef struct {
    int32_t nx, ny, nz;            /* cells per axis, each >= 1 (periodic)          */
    double tau, rho0;              /* relaxation time (> 1/2), reference density     */
    double fext[3];                /* uniform body-force density                     */
    int32_t storage;               /* SBT_F64 ... SBT_BF16S                          */
    int32_t lattice;               /* 19 (D3Q19) or 27 (D3Q27)                       */
    int32_t walls_z;               /* 0: periodic in z; 1: half-way bounce-back
                                      walls below z = 0 and above z = nz - 1         */
    double wall_u[2][3];           /* bottom and top wall velocities (walls_z = 1)   */
    const uint8_t *solid_mask;     /* solid cells [nz][ny][nx] (nonzero = solid), or
                                      NULL; read during sbt3_plan / sbt3_create      */
    const double *solid_q;         /* [nz][ny][nx][Q] wall fraction of the link from a
                                      fluid cell x toward a solid x + c_i (0 < q <= 1,
                                      read there only); NULL = 1/2 everywhere         */
    int32_t n_markers;             /* fixed immersed body (0 = none): markers        */
    const double *marker_xyz;      /* [3][n_markers] positions (cells; centres at
                                      i + 1/2); read during plan / create           */
    const double *marker_dA;       /* [n_markers] surface element of each marker     */
    int32_t mdf_iters;             /* N_F of the forcing loop                        */
    int64_t ibm_box_cells;         /* capacity (>= 64) of the box of stencil cells
                                      the body's forcing works in; 0: the library
                                      sizes it from the markers' reach over the
                                      motion plus the stencil, capped at the box     */
    int32_t body_motion;           /* 0: fixed (marker_xyz absolute); 1: pitch about
                                      the y axis and plunge along z (marker_xyz in
                                      the body frame)                                */
    double motion_p[10];           /* motion 1: x0, y0, z0, alpha0, A_pitch, A0, T,
                                      phi, U_ref, chord: t* = t U_ref / chord,
                                      theta = 2 pi t* / T, alpha = alpha0 - A_pitch
                                      sin(theta + phi), centre (x0, y0, z0 + (A0/2)
                                      cos theta), X = xc + xb cos a + zb sin a,
                                      Y = yc + yb, Z = zc - xb sin a + zb cos a      */
} sbt3_desc;

/* Device bytes sbt3_create needs.  Host only.  Errors: SBT_ERR_ARG. */
sbt_status sbt3_plan(const sbt3_desc *desc, size_t *device_bytes);
/* Lay the lattices out in device_buf (caller-owned, >= planned bytes,
 * 256-byte aligned) and bind hip_stream (a hipStream_t; NULL = legacy
 * default stream).  The state is undefined until sbt3_init_slab has covered
 * every plane. */
sbt_status sbt3_create(const sbt3_desc *desc, void *device_buf, size_t bytes, void *hip_stream,
                       sbt3_ctx **out);
sbt_status sbt3_destroy(sbt3_ctx *ctx);
/* f = f^eq(rho, u) (Eq. (7) in 3D) on planes z0 .. z0 + nz - 1, from host
 * FP64 arrays [nz][ny][nx].  Puts the context back to an initial
 * (pre-collision) state: after a step, every plane must be initialised
 * again before the next one.  Synchronises.  Errors: SBT_ERR_ARG (planes
 * out of range, null arrays). */
sbt_status sbt3_init_slab(sbt3_ctx *ctx, int32_t z0, int32_t nz, const double *rho, const double *ux,
                          const double *uy, const double *uz);
/* Advance n steps.  Asynchronous, stream-ordered. */
sbt_status sbt3_step(sbt3_ctx *ctx, int32_t n);
/* Wait for the stream; SBT_ERR_NONFINITE if a density became NaN or Inf,
 * SBT_ERR_MARKER_OUTSIDE if a body's stencils left the box or outgrew
 * ibm_box_cells. */
sbt_status sbt3_synchronize(sbt3_ctx *ctx);
/* Body force F_s = -sum_j F_j dA_j of the last completed step (sum over
 * the N_F passes of each marker's force).  Synchronises.  SBT_ERR_STATE
 * without a body or before the first step; SBT_ERR_MARKER_OUTSIDE when a
 * step since the last sbt3_synchronize ran without the body force (its
 * stencils left the box or outgrew ibm_box_cells), leaving the flag set. */
sbt_status sbt3_body_force(sbt3_ctx *ctx, double out[3]);
/* rho and u = (sum_i c_i f_i + F/2) / rho on planes z0 .. z0 + nz - 1 into
 * host FP64 arrays [nz][ny][nx].  Synchronises. */
sbt_status sbt3_read_slab(sbt3_ctx *ctx, int32_t z0, int32_t nz, double *rho, double *ux, double *uy,
                          double *uz);

#ifdef __cplusplus
}
#endif
#endif
