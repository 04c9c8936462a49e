/*
 * sbt3f.h -- the three-dimensional block forest of SBoTFlow (arXiv
 * 2402.04606): the topology-confined refinement of Sec. 2.3 and the
 * coarse-fine interface of Sec. 2.4 written for the 3D lattices (D3Q19 or
 * D3Q27) the method extends to, fully periodic.
 *
 * Level l has (nx0, ny0, nz0) * 2^l cells in blocks of 8^3; level 0 covers
 * the domain and level l >= 1 the union of its boxes (in level-l blocks).  A
 * level-l cell whose children (2x + a, 2y + b, 2z + c), a, b, c in {0, 1},
 * lie on level l + 1 is hidden; the others of the region are owned.  The
 * halo of level l >= 1 is every cell outside its region within Chebyshev
 * distance 2 of an owned cell; its parent must be owned on level l - 1
 * (else SBT_ERR_TOPOLOGY).  tau_l = 1/2 + 2^l (tau0 - 1/2), F_l = F_0 / 2^l
 * (Eq. (9) in 3D).
 *
 * One coarse step runs 2^l substeps on level l in the order of Algorithm 1.
 * A substep of level l streams (Eq. (10)) and collides (BGK with Guo's term
 * and the half-force velocity, Eqs. (2)-(8) in 3D) its owned cells.  Across
 * the interface (Sec. 2.4):
 *   - before the first of a fine level's two substeps its halo cells take
 *     the post-collision populations of their coarse parents (explosion;
 *     cf_mode RESCALE: non-equilibrium part times (tau_f - 1)/(2 (tau_c - 1)));
 *   - the halo cells stream in that first substep and are the sources of
 *     their own second one;
 *   - after the coarse stream, an owned coarse cell's populations whose
 *     source is hidden are the mean over its 8 children of their post-stream
 *     values (coalescence; RESCALE: non-equilibrium part about the moments
 *     of the assembled set times 2 tau_c / tau_f).
 *
 * Storage forms as for the 2D library (sbt.h): SBT_F64 (f itself, FP64
 * arithmetic) and SBT_F32 / SBT_F16S / SBT_BF16S (the deviation f - w rho0,
 * FP32 arithmetic).  Layout in the caller's device buffer: per level a pool
 * of the blocks that hold owned or halo cells, two lattices [block][Q][512]
 * (cell = (z * 8 + y) * 8 + x within a block), block tables and per-cell
 * codes, and a staging area for field transfers.  All functions return
 * sbt_status; sbt_last_error() describes the last failure.  A context must
 * not be used from two threads at once.
 */
#ifndef SBT3F_H
#define SBT3F_H
#include <stddef.h>
#include <stdint.h>

#include "sbt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbt3f_ctx sbt3f_ctx;

typedef struct {
    int32_t nx0, ny0, nz0;         /* level-0 cells per axis, multiples of 8         */
    int32_t n_levels;              /* 1 .. 6                                         */
    int32_t n_boxes;               /* refinement boxes, 7 ints each: level (>= 1),   */
    const int32_t *boxes;          /*   bx0, by0, bz0, bx1, by1, bz1 (half-open range
                                      of level-l blocks of 8^3 cells, inside the
                                      level's grid); read during plan / create       */
    double tau0, rho0;             /* level-0 relaxation time (> 1/2), density       */
    double fext[3];                /* uniform body-force density, level-0 units      */
    int32_t storage;               /* SBT_F64 ... SBT_BF16S                          */
    int32_t lattice;               /* 19 (D3Q19) or 27 (D3Q27)                       */
    int32_t cf_mode;               /* SBT_CF_HOMOGENEOUS or SBT_CF_RESCALE (this one
                                      needs tau_l != 1 below the finest level)       */
} sbt3f_desc;

/* Device bytes sbt3f_create needs; validates the forest.  Host only.
 * Errors: SBT_ERR_ARG, SBT_ERR_TOPOLOGY. */
sbt_status sbt3f_plan(const sbt3f_desc *desc, size_t *device_bytes);
/* Build the forest in device_buf (caller-owned, >= planned bytes, 256-byte
 * aligned) and bind hip_stream (a hipStream_t; NULL = legacy default
 * stream).  Every owned cell starts at rest at rho0 (pre-collision). */
sbt_status sbt3f_create(const sbt3f_desc *desc, void *device_buf, size_t bytes, void *hip_stream,
                        sbt3f_ctx **out);
sbt_status sbt3f_destroy(sbt3f_ctx *ctx);
/* The forest desc describes, for one level: info[6] = cells per axis (nx,
 * ny, nz) and its counts of owned, halo and hidden cells; and, when kind is
 * not NULL, the kinds of the level's cells inside box {x0, y0, z0, nx, ny,
 * nz} (level cells, inside the grid) into kind[nz][ny][nx]: 0 none, 1
 * owned, 2 halo, 3 hidden.  Host only, makes no HIP call.  Errors:
 * SBT_ERR_ARG, SBT_ERR_TOPOLOGY. */
sbt_status sbt3f_level_kinds(const sbt3f_desc *desc, int32_t level, const int32_t box[6], uint8_t *kind,
                             int64_t info[6]);
/* f = f^eq(rho, u) (Eq. (7) in 3D) on the owned cells of a level inside the
 * box {x0, y0, z0, nx, ny, nz} (level cells, inside the grid), from host FP64
 * arrays [nz][ny][nx]; densities must be positive and finite.  Puts the
 * context back to an initial (pre-collision) state: the first call after a
 * step resets every level to rest at rho0 before taking its box.
 * Synchronises.  Errors: SBT_ERR_ARG (box outside the grid, null arrays,
 * bad densities). */
sbt_status sbt3f_init_box(sbt3f_ctx *ctx, int32_t level, const int32_t box[6], const double *rho,
                          const double *ux, const double *uy, const double *uz);
/* Advance n coarse steps.  Asynchronous, stream-ordered. */
sbt_status sbt3f_step(sbt3f_ctx *ctx, int32_t n);
/* Wait for the stream; SBT_ERR_NONFINITE if a density became NaN or Inf. */
sbt_status sbt3f_synchronize(sbt3f_ctx *ctx);
/* rho and u = (sum_i c_i f_i + F_l / 2) / rho of the streamed (pre-collision)
 * state on a level's cells inside the box, into host FP64 arrays
 * [nz][ny][nx]; NaN where the level owns no cell.  Synchronises. */
sbt_status sbt3f_read_box(sbt3f_ctx *ctx, int32_t level, const int32_t box[6], double *rho, double *ux,
                          double *uy, double *uz);
/* out[4] = mass and first moment (sum_i c_i f_i, no force term) of the
 * streamed state, summed over owned cells with volume weight 8^-l, in a
 * fixed order.  Synchronises. */
sbt_status sbt3f_diagnostics(sbt3f_ctx *ctx, double out[4]);

#ifdef __cplusplus
}
#endif
#endif
