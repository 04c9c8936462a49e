/*
 * oracle.c -- plain FP64 CPU oracle for the SBoTFlow time step (arXiv 2402.04606).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the package smoke check
 * and the benchmark's CPU-baseline leg, never by the GPU library.  It is kept
 * deliberately literal: dense per-level arrays, one loop per step of the
 * method's steps (Sec. 2.1-2.5), no blocking, no fusion.  OpenMP only splits the
 * per-cell loops (each cell is written by exactly one thread), so results do
 * not depend on the thread count; every reduction runs sequentially in index
 * order.
 *
 * What each function follows in the paper:
 *   velocity set ............ Sec. 2.1, Eq. (1)
 *   collision + Guo forcing . Sec. 2.1, Eqs. (2)-(8)
 *   streaming ............... Sec. 2.1, Eq. (10)
 *   domain boundaries ....... Sec. 2.1 (kinds named only; formulas are the
 *                             textbook readings listed in the design notes)
 *   IBM, MDF loop ........... Sec. 2.2, Eqs. (11)-(16)
 *   coarse/fine interface ... Sec. 2.4 (steps (1)-(6))
 *   level schedule .......... Sec. 2.4-2.5 (Algorithm 1's order, walked as a
 *                             clock over the finest substeps)
 *
 * Readings where the paper is silent (same list as the design notes):
 *   - tau per level: tau_l - 1/2 = 2^l (tau_0 - 1/2) (same viscosity, dt ~ dx).
 *   - body force per level: F_l = F_0 / 2^l.
 *   - MDF: N_F iterations; rho_j interpolated with the delta kernel; the first
 *     interpolation uses the uncorrected velocity, later ones the corrected one.
 *   - halo ("ghost") cells are never collided; they are streamed in both fine
 *     substeps; coarse-to-fine fills them only before the first substep; the
 *     halo cells' post-stream values are the sources of the
 *     second stream.
 *   - fine-to-coarse replaces f(X,i) exactly when X - c_i is covered by the
 *     finer level, with the mean of the 4 children of X.
 *   - RESCALE interface mode multiplies the non-equilibrium part by
 *     (tau_f - 1)/(2 (tau_c - 1)) coarse->fine (post-collision) and
 *     2 tau_c / tau_f fine->coarse (pre-collision).
 *   - domain edges: half-way bounce-back with the moving-wall term (wall
 *     density rho0), equilibrium inflow at rho0, zero-gradient outflow,
 *     specular symmetry, periodic; corner diagonals follow the rule stated
 *     at edge_rules().
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXL 8
#define Q 9

/* Eq. (1): D2Q9 directions, and the weights of Eq. (7). */
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

enum { K_NONE = 0, K_OWN = 1, K_GHOST = 2, K_HIDDEN = 3 };

typedef struct {
    int nx, ny;
    double tau, fx, fy;
    uint8_t *kind;
    double *f, *fs;           /* pre-collision / post-collision populations */
    double *rho, *ux, *uy;    /* moments used by the last collision          */
    double *Fx, *Fy;          /* IBM force density (finest level only)       */
    uint8_t *solid;           /* solid (bounce-back) cells, or NULL          */
    double *sq;               /* [cell][9] wall fraction of link i from a fluid
                                 cell toward a solid neighbour x + c_i       */
    /* the cells each step visits, in ascending index: the dense arrays are
       the data, these lists only spare the scans over cells that take no
       part (a refined level covers a small part of its dense grid)       */
    int64_t *own, *ghost, *act;   /* owned; halo; owned or halo            */
    int64_t n_own, n_ghost, n_act;
    int64_t *fcell, n_fcell;      /* finest level: cells the last forcing wrote */
} olev;

struct orc_sim {
    orc_case c;
    int32_t *boxes;
    double *xb, *yb, *ds;
    int m, per_x, per_y;
    olev L[MAXL];
    int64_t k;                /* finest-level substeps done */
    double *hist;             /* 2 doubles per finest substep */
    int64_t nhist, cap;
    double *ftx, *fty;        /* per-marker total force of the last substep */
    double *hud;              /* ORC_BODY_HOST: desired velocity, 2 x n       */
    int err;
};

/* ------------------------------------------------------------------------ */
/* Building blocks                                                           */
/* ------------------------------------------------------------------------ */

void orc_velocity_set(int32_t cx[9], int32_t cy[9], double w[9]) {
    for (int i = 0; i < Q; ++i) { cx[i] = CX[i]; cy[i] = CY[i]; w[i] = WT[i]; }
}

/* Eq. (7), c_s^2 = 1/3. */
void orc_feq(double rho, double ux, double uy, double out[9]) {
    double usq = ux * ux + uy * uy;
    for (int i = 0; i < Q; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        out[i] = WT[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    }
}

/* Eq. (3), Guo et al. forcing term. */
void orc_guo(double tau, double ux, double uy, double Fx, double Fy, double out[9]) {
    double uF = ux * Fx + uy * Fy;
    double pre = 1.0 - 0.5 / tau;
    for (int i = 0; i < Q; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        double cF = CX[i] * Fx + CY[i] * Fy;
        out[i] = WT[i] * pre * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF);
    }
}

/* Eqs. (6), (8): moments with the half-force velocity, then BGK + forcing.
 * Returns the moments through the last three slots of `mom` when non-NULL. */
static void collide_cell(double tau, const double *f, double Fx, double Fy, double *out,
                         double *mom) {
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < Q; ++i) { rho += f[i]; jx += CX[i] * f[i]; jy += CY[i] * f[i]; }
    double ux = (jx + 0.5 * Fx) / rho;
    double uy = (jy + 0.5 * Fy) / rho;
    double feq[Q], fi[Q];
    orc_feq(rho, ux, uy, feq);
    orc_guo(tau, ux, uy, Fx, Fy, fi);
    for (int i = 0; i < Q; ++i) out[i] = f[i] - (f[i] - feq[i]) / tau + fi[i];
    if (mom) { mom[0] = rho; mom[1] = ux; mom[2] = uy; }
}

void orc_collide_cell(double tau, const double f[9], double Fx, double Fy, double out[9]) {
    collide_cell(tau, f, Fx, Fy, out, NULL);
}

/* The multiple-relaxation-time collision the paper names as an option for
 * low viscosity (Sec. 2.1, after Du et al.), on the usual orthogonal D2Q9
 * moment basis m = M f: density, energy e, energy square eps, momentum jx,
 * energy flux qx, jy, qy, and the stresses pxx, pxy.  Row k of M is the
 * polynomial of c_i named below; the rows are orthogonal, so
 * M^-1 = M^T diag(1 / |row_k|^2). */
void orc_mrt_matrices(double M[81], double Minv[81]) {
    for (int i = 0; i < Q; ++i) {
        double cx = CX[i], cy = CY[i], c2 = cx * cx + cy * cy;
        M[0 * Q + i] = 1.0;
        M[1 * Q + i] = -4.0 + 3.0 * c2;
        M[2 * Q + i] = 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
        M[3 * Q + i] = cx;
        M[4 * Q + i] = (3.0 * c2 - 5.0) * cx;
        M[5 * Q + i] = cy;
        M[6 * Q + i] = (3.0 * c2 - 5.0) * cy;
        M[7 * Q + i] = cx * cx - cy * cy;
        M[8 * Q + i] = cx * cy;
    }
    for (int k = 0; k < Q; ++k) {
        double n2 = 0.0;
        for (int i = 0; i < Q; ++i) n2 += M[k * Q + i] * M[k * Q + i];
        for (int i = 0; i < Q; ++i) Minv[i * Q + k] = M[k * Q + i] / n2;
    }
}

/* MRT step: every moment relaxes toward the moments of the Eq. (7)
 * equilibrium, m_eq = M f^eq(rho, u), at its own rate, and Guo's forcing
 * enters in moment space as (I - S/2) M Fbar, Fbar_i = w_i (3 c.F +
 * 9 (c.u)(c.F) - 3 u.F) (Eq. (3) without its 1 - 1/(2 tau) factor):
 *   m* = m - S (m - m_eq) + (I - S/2) M Fbar,  f* = M^-1 m*,
 *   S = diag(1, s_e, s_eps, 1, s_q, 1, s_q, 1/tau, 1/tau).
 * u is the half-force velocity of Eq. (8).  With every rate 1/tau this is
 * Eqs. (2)-(3) exactly.  rates = {s_e, s_eps, s_q}. */
static void collide_mrt(double tau, const double rates[3], const double *f, double Fx, double Fy,
                        double *out, double *mom) {
    double M[81], Minv[81];
    orc_mrt_matrices(M, Minv);
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < Q; ++i) { rho += f[i]; jx += CX[i] * f[i]; jy += CY[i] * f[i]; }
    double ux = (jx + 0.5 * Fx) / rho;
    double uy = (jy + 0.5 * Fy) / rho;
    double feq[Q], fbar[Q];
    orc_feq(rho, ux, uy, feq);
    double uF = ux * Fx + uy * Fy;
    for (int i = 0; i < Q; ++i) {
        double cu = CX[i] * ux + CY[i] * uy, cF = CX[i] * Fx + CY[i] * Fy;
        fbar[i] = WT[i] * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF);
    }
    double S[Q] = {1.0, rates[0], rates[1], 1.0, rates[2], 1.0, rates[2], 1.0 / tau, 1.0 / tau};
    double ms[Q];
    for (int k = 0; k < Q; ++k) {
        double m = 0.0, me = 0.0, g = 0.0;
        for (int i = 0; i < Q; ++i) {
            m += M[k * Q + i] * f[i];
            me += M[k * Q + i] * feq[i];
            g += M[k * Q + i] * fbar[i];
        }
        ms[k] = m - S[k] * (m - me) + (1.0 - 0.5 * S[k]) * g;
    }
    for (int i = 0; i < Q; ++i) {
        double v = 0.0;
        for (int k = 0; k < Q; ++k) v += Minv[i * Q + k] * ms[k];
        out[i] = v;
    }
    if (mom) { mom[0] = rho; mom[1] = ux; mom[2] = uy; }
}

void orc_collide_cell_mrt(double tau, const double rates[3], const double f[9], double Fx, double Fy,
                          double out[9]) {
    collide_mrt(tau, rates, f, Fx, Fy, out, NULL);
}

/* Eq. (14): Peskin's 4-point kernel (dx = 1). */
double orc_phi(double r) {
    double a = fabs(r);
    if (a <= 1.0) return 0.125 * (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a));
    if (a <= 2.0) return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
    return 0.0;
}

/* Pitch-up ramp of Sec. 3.5 (Eldredge's smoothing function G):
 *   G(t*) = log[cosh(a_s (t* - t1*)) / cosh(a_s (t* - t2*))] - a_s (t1* - t2*),
 *   t2* = t1* + A / (2K),   alpha = A G / max G.
 * G rises monotonically from 0 to its supremum 2 a_s (t2* - t1*), the value
 * the paper calls approximately max G; that supremum is used, so alpha ends
 * at A.  log cosh is evaluated as |x| - log 2 + log1p(exp(-2|x|)), the same
 * function without the overflow of cosh for |x| > 710.
 * p = {x0, y0, A, a_s, K, t1*, -, -, U_ref, c}. */
static double logcosh(double x) {
    double a = fabs(x);
    return a - M_LN2 + log1p(exp(-2.0 * a));
}

double orc_ramp_alpha(const double *p, double tstar) {
    double A = p[2], as = p[3], K = p[4], t1 = p[5];
    double t2 = t1 + A / (2.0 * K);
    double G = logcosh(as * (tstar - t1)) - logcosh(as * (tstar - t2)) - as * (t1 - t2);
    return A * G / (2.0 * as * (t2 - t1));
}

/* Smoothed asymmetric triangular pitching of Sec. 3.6 (E5): straight ramps
 * of rate adot1 = 2 alpha0 / (xi T - ta) and adot2 = -2 alpha0 / ((1 - xi) T - ta)
 * joined at the extremes alpha0 (t2 = xi T / 2) and -alpha0 (t5 = T (1 - xi/2))
 * by quartics of duration ta on each side.  The printed law has t2 in place
 * of ta in some quartic denominators; only ta makes alpha and its rate
 * continuous at every breakpoint, so ta is used throughout.  Time runs in
 * t* = t U_ref / c, periodic in T.
 * p = {x0, y0, alpha0, xi, T, ta/T, -, -, U_ref, c}. */
double orc_tri_alpha(const double *p, double tstar) {
    double a0 = p[2], xi = p[3], T = p[4], ta = p[5] * p[4];
    double r1 = 2.0 * a0 / (xi * T - ta);
    double r2 = -2.0 * a0 / ((1.0 - xi) * T - ta);
    double t2 = 0.5 * xi * T, t1 = t2 - ta, t3 = t2 + ta;
    double t5 = T * (1.0 - 0.5 * xi), t4 = t5 - ta, t6 = t5 + ta;
    double t = fmod(tstar, T);
    if (t < 0.0) t += T;
    double ta2 = ta * ta, ta3 = ta2 * ta;
    if (t < t1) return r1 * t;
    if (t < t2) { double s = t - t2; return r1 / (2.0 * ta3) * s * s * s * s + r1 / ta2 * s * s * s + a0; }
    if (t < t3) { double s = t - t2; return -r2 / (2.0 * ta3) * s * s * s * s + r2 / ta2 * s * s * s + a0; }
    if (t < t4) return r2 * (t - t4) - r2 * ta / 2.0 - a0;
    if (t < t5) { double s = t - t5; return r2 / (2.0 * ta3) * s * s * s * s + r2 / ta2 * s * s * s - a0; }
    if (t < t6) { double s = t - t5; return -r1 / (2.0 * ta3) * s * s * s * s + r1 / ta2 * s * s * s - a0; }
    return r1 * (t - T);
}

/* Kinematics.  FIXED: X = (x0 + xb, y0 + yb).  FLAP (Sec. 3.6 law, with the
 * pitch amplitude and stroke angle as parameters):
 *   t* = t U_ref / c,  theta = 2 pi t* / T
 *   alpha = alpha0 - A_pitch sin(theta + phi)
 *   (xc, yc) = (x0, y0) + (A0/2) cos(theta) (cos beta, sin beta)
 * bp = {x0, y0, alpha0, A_pitch, A0, beta, T, phi, U_ref, c}.
 * RAMP and TRI: pure pitch alpha(t*) (orc_ramp_alpha, orc_tri_alpha) about
 * the pivot (xc, yc) = (x0, y0), t* = t U_ref / c.
 * Every moving body: X = xc + xb cos(alpha) + yb sin(alpha),
 *                    Y = yc - xb sin(alpha) + yb cos(alpha). */
int orc_body_positions(const orc_case *c, double k, double *X, double *Y) {
    const double *p = c->bp;
    if (c->body_kind == ORC_BODY_FIXED) {
        for (int j = 0; j < c->n_markers; ++j) { X[j] = p[0] + c->xb[j]; Y[j] = p[1] + c->yb[j]; }
        return ORC_OK;
    }
    if (c->body_kind == ORC_BODY_HOST) {      /* caller-placed markers */
        for (int j = 0; j < c->n_markers; ++j) { X[j] = c->xb[j]; Y[j] = c->yb[j]; }
        return ORC_OK;
    }
    double tstar = k * p[8] / p[9];
    double alpha, xc = p[0], yc = p[1];
    if (c->body_kind == ORC_BODY_FLAP) {
        double theta = 2.0 * M_PI * tstar / p[6];
        alpha = p[2] - p[3] * sin(theta + p[7]);
        double h = 0.5 * p[4] * cos(theta);
        xc = p[0] + h * cos(p[5]);
        yc = p[1] + h * sin(p[5]);
    } else if (c->body_kind == ORC_BODY_RAMP) {
        alpha = orc_ramp_alpha(p, tstar);
    } else if (c->body_kind == ORC_BODY_TRI) {
        alpha = orc_tri_alpha(p, tstar);
    } else {
        return ORC_ERR_ARG;
    }
    double ca = cos(alpha), sa = sin(alpha);
    for (int j = 0; j < c->n_markers; ++j) {
        X[j] = xc + c->xb[j] * ca + c->yb[j] * sa;
        Y[j] = yc - c->xb[j] * sa + c->yb[j] * ca;
    }
    return ORC_OK;
}

static inline int wrapi(int a, int n) { a %= n; return a < 0 ? a + n : a; }

/* First of the 4 cells (centres at i + 1/2) within distance 2 of X. */
static inline int tap0(double X) { return (int)floor(X - 1.5); }

/* Eq. (12) on a dense periodic grid: sum over taps, y outer, x inner. */
int orc_interpolate(int32_t nx, int32_t ny, const double *ux, const double *uy, int32_t n,
                    const double *X, const double *Y, double *U, double *V) {
    for (int j = 0; j < n; ++j) {
        int i0 = tap0(X[j]), j0 = tap0(Y[j]);
        double su = 0.0, sv = 0.0;
        for (int b = 0; b < 4; ++b) {
            double py = orc_phi(j0 + b + 0.5 - Y[j]);
            int yy = wrapi(j0 + b, ny);
            for (int a = 0; a < 4; ++a) {
                double w = orc_phi(i0 + a + 0.5 - X[j]) * py;
                int xx = wrapi(i0 + a, nx);
                su += ux[(size_t)yy * nx + xx] * w;
                sv += uy[(size_t)yy * nx + xx] * w;
            }
        }
        U[j] = su; V[j] = sv;
    }
    return ORC_OK;
}

/* Eq. (15) on a dense periodic grid, markers in index order. */
int orc_spread(int32_t nx, int32_t ny, int32_t n, const double *X, const double *Y,
               const double *Fjx, const double *Fjy, const double *ds, double *Fx, double *Fy) {
    for (int j = 0; j < n; ++j) {
        int i0 = tap0(X[j]), j0 = tap0(Y[j]);
        for (int b = 0; b < 4; ++b) {
            double py = orc_phi(j0 + b + 0.5 - Y[j]);
            int yy = wrapi(j0 + b, ny);
            for (int a = 0; a < 4; ++a) {
                double w = orc_phi(i0 + a + 0.5 - X[j]) * py;
                int xx = wrapi(i0 + a, nx);
                Fx[(size_t)yy * nx + xx] += Fjx[j] * w * ds[j];
                Fy[(size_t)yy * nx + xx] += Fjy[j] * w * ds[j];
            }
        }
    }
    return ORC_OK;
}

/* The multi-direct-forcing loop (Sec. 2.2, Eqs. (11)-(15), iterated N_F
 * times): interpolate velocity and density at the markers, boundary force
 * Eq. (11) with dt = 1, spread, correct the cell velocity by dF/(2 rho)
 * (consistent with the half-force velocity of Eq. (8)) and accumulate. */
/* Cells within the 4x4 stencil of any marker (periodic wrap), ascending;
 * returns their count, the list in *out (caller frees). */
static int64_t stencil_cells(int32_t nx, int32_t ny, int32_t n, const double *X, const double *Y,
                             int64_t **out) {
    const size_t ncell = (size_t)nx * ny;
    uint8_t *mark = calloc(ncell, 1);
    int64_t cnt = 0;
    for (int j = 0; j < n; ++j) {
        int i0 = tap0(X[j]), j0 = tap0(Y[j]);
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a) {
                size_t c = (size_t)wrapi(j0 + b, ny) * nx + wrapi(i0 + a, nx);
                if (!mark[c]) { mark[c] = 1; ++cnt; }
            }
    }
    int64_t *list = malloc(sizeof(int64_t) * (cnt + 1));
    int64_t k = 0;
    if (cnt > 0)
        for (int j = 0; j < n; ++j) {
            int i0 = tap0(X[j]), j0 = tap0(Y[j]);
            for (int b = 0; b < 4; ++b)
                for (int a = 0; a < 4; ++a) {
                    size_t c = (size_t)wrapi(j0 + b, ny) * nx + wrapi(i0 + a, nx);
                    if (mark[c] == 1) { mark[c] = 2; list[k++] = (int64_t)c; }
                }
        }
    free(mark);
    /* ascending (insertion sort of a short list) */
    for (int64_t i = 1; i < k; ++i) {
        int64_t v = list[i], t = i;
        while (t > 0 && list[t - 1] > v) { list[t] = list[t - 1]; --t; }
        list[t] = v;
    }
    *out = list;
    return k;
}

int orc_mdf(int32_t nx, int32_t ny, const double *rho, double *ux, double *uy, double *Fx,
            double *Fy, int32_t n, const double *X, const double *Y, const double *udx,
            const double *udy, const double *ds, int32_t iters, double *ftx, double *fty) {
    size_t ncell = (size_t)nx * ny;
    double *U = malloc(sizeof(double) * n * 4);
    double *dFx = calloc(ncell, sizeof(double)), *dFy = calloc(ncell, sizeof(double));
    if (!U || !dFx || !dFy) { free(U); free(dFx); free(dFy); return ORC_ERR_ARG; }
    double *V = U + n, *R = U + 2 * n, *Rv = U + 3 * n;
    double *zero = calloc(ncell, sizeof(double));
    /* spreading and the corrections touch only the stencil cells; the other
       cells keep dF = 0 and are skipped as in a scan of the whole grid */
    int64_t *cells = NULL;
    const int64_t ns = stencil_cells(nx, ny, n, X, Y, &cells);
    for (int j = 0; j < n; ++j) { ftx[j] = 0.0; fty[j] = 0.0; }
    for (int it = 0; it < iters; ++it) {
        orc_interpolate(nx, ny, ux, uy, n, X, Y, U, V);
        orc_interpolate(nx, ny, rho, zero, n, X, Y, R, Rv);
        double *gx = malloc(sizeof(double) * n * 2), *gy = gx + n;
        for (int j = 0; j < n; ++j) {
            gx[j] = 2.0 * R[j] * (udx[j] - U[j]);
            gy[j] = 2.0 * R[j] * (udy[j] - V[j]);
            ftx[j] += gx[j];
            fty[j] += gy[j];
        }
        for (int64_t k = 0; k < ns; ++k) dFx[cells[k]] = dFy[cells[k]] = 0.0;
        orc_spread(nx, ny, n, X, Y, gx, gy, ds, dFx, dFy);
        for (int64_t k = 0; k < ns; ++k) {
            const size_t c = (size_t)cells[k];
            if (dFx[c] == 0.0 && dFy[c] == 0.0) continue;
            Fx[c] += dFx[c];
            Fy[c] += dFy[c];
            ux[c] += dFx[c] / (2.0 * rho[c]);
            uy[c] += dFy[c] / (2.0 * rho[c]);
        }
        free(gx);
    }
    free(U); free(dFx); free(dFy); free(zero); free(cells);
    return ORC_OK;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Topology                                                                  */
/* ------------------------------------------------------------------------ */

static int in_region(const orc_sim *s, int l, int x, int y) {
    if (l == 0) return 1;
    int B = s->c.block_n;
    for (int b = 0; b < s->c.n_boxes; ++b) {
        const int32_t *q = s->boxes + 5 * b;
        if (q[0] != l) continue;
        if (x >= q[1] * B && x < q[3] * B && y >= q[2] * B && y < q[4] * B) return 1;
    }
    return 0;
}

static inline size_t cid(const olev *L, int x, int y) { return (size_t)y * L->nx + x; }

/* Wrap (x, y) on level L if the axis is periodic.  Returns 0 if outside. */
static int wrap_level(const orc_sim *s, const olev *L, int *x, int *y) {
    if (*x < 0 || *x >= L->nx) { if (!s->per_x) return 0; *x = wrapi(*x, L->nx); }
    if (*y < 0 || *y >= L->ny) { if (!s->per_y) return 0; *y = wrapi(*y, L->ny); }
    return 1;
}

static int build_topology(orc_sim *s) {
    int m = s->m;
    for (int l = 0; l < m; ++l) {
        olev *L = &s->L[l];
        for (int y = 0; y < L->ny; ++y)
            for (int x = 0; x < L->nx; ++x) {
                uint8_t kd = K_NONE;
                if (in_region(s, l, x, y)) {
                    kd = K_OWN;
                    if (l + 1 < m && in_region(s, l + 1, 2 * x, 2 * y)) kd = K_HIDDEN;
                }
                L->kind[cid(L, x, y)] = kd;
            }
        /* nesting: every cell of region_l has its parent in region_{l-1} */
        if (l > 0)
            for (int y = 0; y < L->ny; ++y)
                for (int x = 0; x < L->nx; ++x)
                    if (L->kind[cid(L, x, y)] != K_NONE && !in_region(s, l - 1, x / 2, y / 2))
                        return ORC_ERR_TOPOLOGY;
    }
    /* ghost (halo) cells: outside region_l, Chebyshev distance <= 2 from an
     * owned cell of level l, parent owned on level l-1 (Sec. 2.4: two halo
     * layers over faces, edges and vertices). */
    for (int l = 1; l < m; ++l) {
        olev *L = &s->L[l], *P = &s->L[l - 1];
        uint8_t *mark = calloc((size_t)L->nx * L->ny, 1);
        for (int y = 0; y < L->ny; ++y)
            for (int x = 0; x < L->nx; ++x) {
                if (L->kind[cid(L, x, y)] != K_OWN) continue;
                for (int dy = -2; dy <= 2; ++dy)
                    for (int dx = -2; dx <= 2; ++dx) {
                        int xx = x + dx, yy = y + dy;
                        if (!wrap_level(s, L, &xx, &yy)) { free(mark); return ORC_ERR_TOPOLOGY; }
                        if (L->kind[cid(L, xx, yy)] == K_NONE) mark[cid(L, xx, yy)] = 1;
                    }
            }
        for (int y = 0; y < L->ny; ++y)
            for (int x = 0; x < L->nx; ++x) {
                if (!mark[cid(L, x, y)]) continue;
                if (P->kind[cid(P, x / 2, y / 2)] != K_OWN) { free(mark); return ORC_ERR_TOPOLOGY; }
                L->kind[cid(L, x, y)] = K_GHOST;
            }
        free(mark);
    }
    /* refined levels may not reach a non-periodic domain edge */
    for (int l = 1; l < m; ++l) {
        olev *L = &s->L[l];
        for (int y = 0; y < L->ny; ++y)
            for (int x = 0; x < L->nx; ++x) {
                if (L->kind[cid(L, x, y)] == K_NONE) continue;
                if ((!s->per_x && (x == 0 || x == L->nx - 1)) ||
                    (!s->per_y && (y == 0 || y == L->ny - 1)))
                    return ORC_ERR_TOPOLOGY;
            }
    }
    /* cell lists of each level, ascending */
    for (int l = 0; l < m; ++l) {
        olev *L = &s->L[l];
        const size_t n = (size_t)L->nx * L->ny;
        int64_t no = 0, ng = 0;
        for (size_t q = 0; q < n; ++q) {
            no += L->kind[q] == K_OWN;
            ng += L->kind[q] == K_GHOST;
        }
        L->own = malloc(sizeof(int64_t) * (no + 1));
        L->ghost = malloc(sizeof(int64_t) * (ng + 1));
        L->act = malloc(sizeof(int64_t) * (no + ng + 1));
        L->fcell = NULL;
        L->n_own = L->n_ghost = L->n_act = L->n_fcell = 0;
        for (size_t q = 0; q < n; ++q) {
            if (L->kind[q] == K_OWN) L->own[L->n_own++] = (int64_t)q;
            if (L->kind[q] == K_GHOST) L->ghost[L->n_ghost++] = (int64_t)q;
            if (L->kind[q] == K_OWN || L->kind[q] == K_GHOST) L->act[L->n_act++] = (int64_t)q;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Life cycle                                                                */
/* ------------------------------------------------------------------------ */

void orc_destroy(orc_sim *s) {
    if (!s) return;
    for (int l = 0; l < MAXL; ++l) {
        olev *L = &s->L[l];
        free(L->kind); free(L->f); free(L->fs); free(L->rho); free(L->ux); free(L->uy);
        free(L->Fx); free(L->Fy); free(L->solid); free(L->sq);
        free(L->own); free(L->ghost); free(L->act); free(L->fcell);
    }
    free(s->boxes); free(s->xb); free(s->yb); free(s->ds); free(s->hist); free(s->hud);
    free(s->ftx); free(s->fty);
    free(s);
}

int orc_create(const orc_case *c, orc_sim **out) {
    *out = NULL;
    if (c->n_levels < 1 || c->n_levels > MAXL || c->nx0 <= 0 || c->ny0 <= 0 || c->block_n <= 0 ||
        c->tau0 <= 0.5)
        return ORC_ERR_ARG;
    if (c->collision != ORC_COLL_BGK && c->collision != ORC_COLL_MRT) return ORC_ERR_ARG;
    if (c->collision == ORC_COLL_MRT)
        for (int k = 0; k < 3; ++k)
            if (!(c->mrt[k] > 0.0 && c->mrt[k] < 2.0)) return ORC_ERR_ARG;
    for (int e = 0; e < 4; ++e)
        if (c->bc[e] < 0 || c->bc[e] > ORC_BC_SYMMETRY) return ORC_ERR_ARG;
    if ((c->bc[ORC_W] == ORC_BC_PERIODIC) != (c->bc[ORC_E] == ORC_BC_PERIODIC) ||
        (c->bc[ORC_S] == ORC_BC_PERIODIC) != (c->bc[ORC_N] == ORC_BC_PERIODIC))
        return ORC_ERR_ARG;
    orc_sim *s = calloc(1, sizeof(orc_sim));
    s->c = *c;
    s->m = c->n_levels;
    s->per_x = c->bc[ORC_W] == ORC_BC_PERIODIC;
    s->per_y = c->bc[ORC_S] == ORC_BC_PERIODIC;
    s->boxes = malloc(sizeof(int32_t) * 5 * (c->n_boxes > 0 ? c->n_boxes : 1));
    if (c->n_boxes > 0) memcpy(s->boxes, c->boxes, sizeof(int32_t) * 5 * c->n_boxes);
    s->c.boxes = s->boxes;
    int nm = c->body_kind == ORC_BODY_NONE ? 0 : c->n_markers;
    s->c.n_markers = nm;
    s->xb = malloc(sizeof(double) * (nm + 1));
    s->yb = malloc(sizeof(double) * (nm + 1));
    s->ds = malloc(sizeof(double) * (nm + 1));
    s->ftx = calloc(nm + 1, sizeof(double));
    s->fty = calloc(nm + 1, sizeof(double));
    s->hud = calloc(2 * nm + 1, sizeof(double));
    if (nm) {
        memcpy(s->xb, c->xb, sizeof(double) * nm);
        memcpy(s->yb, c->yb, sizeof(double) * nm);
        memcpy(s->ds, c->ds, sizeof(double) * nm);
    }
    s->c.xb = s->xb; s->c.yb = s->yb; s->c.ds = s->ds;
    for (int l = 0; l < s->m; ++l) {
        olev *L = &s->L[l];
        L->nx = c->nx0 << l;
        L->ny = c->ny0 << l;
        L->tau = 0.5 + (double)(1 << l) * (c->tau0 - 0.5);
        L->fx = c->fext[0] / (double)(1 << l);
        L->fy = c->fext[1] / (double)(1 << l);
        size_t n = (size_t)L->nx * L->ny;
        L->kind = calloc(n, 1);
        L->f = malloc(sizeof(double) * n * Q);
        L->fs = malloc(sizeof(double) * n * Q);
        L->rho = malloc(sizeof(double) * n);
        L->ux = malloc(sizeof(double) * n);
        L->uy = malloc(sizeof(double) * n);
        if (!L->kind || !L->f || !L->fs || !L->rho || !L->ux || !L->uy) {
            orc_destroy(s);
            return ORC_ERR_ARG;
        }
        for (size_t q = 0; q < n * Q; ++q) { L->f[q] = NAN; L->fs[q] = NAN; }
        for (size_t q = 0; q < n; ++q) { L->rho[q] = NAN; L->ux[q] = NAN; L->uy[q] = NAN; }
    }
    olev *Lf = &s->L[s->m - 1];
    size_t nf = (size_t)Lf->nx * Lf->ny;
    Lf->Fx = calloc(nf, sizeof(double));
    Lf->Fy = calloc(nf, sizeof(double));
    int rc = build_topology(s);
    if (rc) { orc_destroy(s); return rc; }
    if (c->cf_mode == ORC_CF_RESCALE)
        for (int l = 0; l + 1 < s->m; ++l)
            if (fabs(s->L[l].tau - 1.0) < 1e-6) { orc_destroy(s); return ORC_ERR_ARG; }
    /* default state: rest at rho0 */
    for (int l = 0; l < s->m; ++l) {
        olev *L = &s->L[l];
        double feq[Q];
        orc_feq(c->rho0, 0.0, 0.0, feq);
        for (size_t q = 0; q < (size_t)L->nx * L->ny; ++q)
            if (L->kind[q] == K_OWN) memcpy(L->f + q * Q, feq, sizeof feq);
    }
    s->cap = 1024;
    s->hist = malloc(sizeof(double) * 2 * s->cap);
    *out = s;
    return ORC_OK;
}

int orc_level_size(const orc_sim *s, int level, int32_t *nx, int32_t *ny) {
    if (level < 0 || level >= s->m) return ORC_ERR_ARG;
    *nx = s->L[level].nx; *ny = s->L[level].ny;
    return ORC_OK;
}

int orc_level_kinds(const orc_sim *s, int level, uint8_t *kind) {
    if (level < 0 || level >= s->m) return ORC_ERR_ARG;
    memcpy(kind, s->L[level].kind, (size_t)s->L[level].nx * s->L[level].ny);
    return ORC_OK;
}

int orc_init_fields(orc_sim *s, int level, const double *rho, const double *ux, const double *uy) {
    if (level < 0 || level >= s->m) return ORC_ERR_ARG;
    olev *L = &s->L[level];
    for (size_t q = 0; q < (size_t)L->nx * L->ny; ++q)
        if (L->kind[q] == K_OWN) orc_feq(rho[q], ux[q], uy[q], L->f + q * Q);
    return ORC_OK;
}

/* Pre-collision populations of the owned cells of a level, dense [ny][nx][9]
 * (a state with a non-equilibrium part; the other cells keep theirs). */
int orc_init_populations(orc_sim *s, int level, const double *f) {
    if (level < 0 || level >= s->m) return ORC_ERR_ARG;
    olev *L = &s->L[level];
    for (size_t q = 0; q < (size_t)L->nx * L->ny; ++q)
        if (L->kind[q] == K_OWN) memcpy(L->f + q * Q, f + q * Q, sizeof(double) * Q);
    return ORC_OK;
}

/* Scale factors of the non-equilibrium part under the RESCALE interface
 * mode, for a coarse level of relaxation time tau_c over a fine level of
 * tau_f (Sec. 2.4 names no factor; this is the reading that converts a
 * first-order Chapman-Enskog non-equilibrium part, -tau dt c.grad f^eq,
 * between two grids of spacing ratio 2 under acoustic scaling):
 *   out[0] = s_cf = (tau_f - 1) / (2 (tau_c - 1)), coarse -> fine, applied
 *            to post-collision populations (their part is (tau - 1)/tau of
 *            the pre-collision one);
 *   out[1] = s_fc = 2 tau_c / tau_f, fine -> coarse, applied to pre-
 *            collision populations. */
void orc_interface_factors(double tau_c, double tau_f, double out[2]) {
    out[0] = (tau_f - 1.0) / (2.0 * (tau_c - 1.0));
    out[1] = 2.0 * tau_c / tau_f;
}

/* ------------------------------------------------------------------------ */
/* The steps of one time step (Sec. 2.1-2.4)                               */
/* ------------------------------------------------------------------------ */

/* Immersed-boundary forcing on the finest level: kinematics, moments of the
 * stencil cells, the multi-direct-forcing loop and the body force (Sec. 2.2). */
static void ibm_forcing(orc_sim *s, int l) {
    if (l != s->m - 1 || s->c.body_kind == ORC_BODY_NONE || s->c.n_markers == 0) return;
    olev *L = &s->L[l];
    int n = s->c.n_markers;
    size_t ncell = (size_t)L->nx * L->ny;
    double *X = malloc(sizeof(double) * n * 6);
    double *Y = X + n, *X1 = X + 2 * n, *Y1 = X + 3 * n, *udx = X + 4 * n, *udy = X + 5 * n;
    orc_body_positions(&s->c, (double)s->k, X, Y);
    if (s->c.body_kind == ORC_BODY_HOST) {    /* desired velocity given with the markers */
        for (int j = 0; j < n; ++j) { udx[j] = s->hud[j]; udy[j] = s->hud[n + j]; }
    } else {
        orc_body_positions(&s->c, (double)(s->k + 1), X1, Y1);
        for (int j = 0; j < n; ++j) { udx[j] = X1[j] - X[j]; udy[j] = Y1[j] - Y[j]; }
    }

    /* Moments of the stencil cells: rho and the uncorrected velocity. */
    double *rho = calloc(ncell, sizeof(double));
    double *ux = calloc(ncell, sizeof(double)), *uy = calloc(ncell, sizeof(double));
    /* F = 0 outside this substep's stencils: clear the cells the last forcing
       wrote, and remember the ones this forcing writes */
    for (int64_t k = 0; k < L->n_fcell; ++k) L->Fx[L->fcell[k]] = L->Fy[L->fcell[k]] = 0.0;
    free(L->fcell);
    L->n_fcell = stencil_cells(L->nx, L->ny, n, X, Y, &L->fcell);
    for (int j = 0; j < n; ++j) {
        int i0 = tap0(X[j]), j0 = tap0(Y[j]);
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a) {
                int x = i0 + a, y = j0 + b;
                /* the stencil and its streaming sources must be owned cells */
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int xx = x + dx, yy = y + dy;
                        if (!wrap_level(s, L, &xx, &yy) || L->kind[cid(L, xx, yy)] != K_OWN)
                            s->err = ORC_ERR_MARKER;
                    }
                if (!wrap_level(s, L, &x, &y)) continue;
                size_t q = cid(L, x, y);
                const double *f = L->f + q * Q;
                double r = 0.0, jx = 0.0, jy = 0.0;
                for (int i = 0; i < Q; ++i) { r += f[i]; jx += CX[i] * f[i]; jy += CY[i] * f[i]; }
                rho[q] = r;
                ux[q] = (jx + 0.5 * L->fx) / r;
                uy[q] = (jy + 0.5 * L->fy) / r;
            }
    }
    if (!s->err)
        orc_mdf(L->nx, L->ny, rho, ux, uy, L->Fx, L->Fy, n, X, Y, udx, udy, s->ds,
                s->c.mdf_iters, s->ftx, s->fty);
    /* Eq. (16): total force on the body */
    double fsx = 0.0, fsy = 0.0;
    for (int j = 0; j < n; ++j) { fsx -= s->ftx[j] * s->ds[j]; fsy -= s->fty[j] * s->ds[j]; }
    if (s->nhist == s->cap) {
        s->cap *= 2;
        s->hist = realloc(s->hist, sizeof(double) * 2 * s->cap);
    }
    s->hist[2 * s->nhist] = fsx;
    s->hist[2 * s->nhist + 1] = fsy;
    s->nhist++;
    free(X); free(rho); free(ux); free(uy);
}

/* Collision of a level's owned cells, Eqs. (2)-(8); F = body force plus the
 * IBM force on the finest level. */
static void collide_level(orc_sim *s, int l) {
    olev *L = &s->L[l];
    int finest = (l == s->m - 1);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < L->n_own; ++k) {
        const size_t q = (size_t)L->own[k];
        if (L->solid && L->solid[q]) continue;
        double Fx = L->fx, Fy = L->fy;
        if (finest) { Fx += L->Fx[q]; Fy += L->Fy[q]; }
        double mom[3];
        if (s->c.collision == ORC_COLL_MRT)
            collide_mrt(L->tau, s->c.mrt, L->f + q * Q, Fx, Fy, L->fs + q * Q, mom);
        else
            collide_cell(L->tau, L->f + q * Q, Fx, Fy, L->fs + q * Q, mom);
        L->rho[q] = mom[0]; L->ux[q] = mom[1]; L->uy[q] = mom[2];
    }
}

/* Explosion (step (2) of Sec. 2.4): each halo cell of the
 * fine level takes the post-collision populations of its coarse parent. */
static void explode(orc_sim *s, int lc, int lf) {
    olev *C = &s->L[lc], *F = &s->L[lf];
    double fac[2];
    orc_interface_factors(C->tau, F->tau, fac);
    const double scf = fac[0];
    int rescale = s->c.cf_mode == ORC_CF_RESCALE;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < F->n_ghost; ++k) {
        const size_t q = (size_t)F->ghost[k];
        const int x = (int)(q % (size_t)F->nx), y = (int)(q / (size_t)F->nx);
        size_t p = cid(C, x / 2, y / 2);
        const double *src = C->fs + p * Q;
        double *dst = F->fs + q * Q;
        if (!rescale) {
            for (int i = 0; i < Q; ++i) dst[i] = src[i];
        } else {
            double feq[Q];
            orc_feq(C->rho[p], C->ux[p], C->uy[p], feq);
            for (int i = 0; i < Q; ++i) dst[i] = feq[i] + scf * (src[i] - feq[i]);
        }
    }
}

/* Streaming, Eq. (10), over owned and halo cells; same-level exchange is
 * implicit in the dense arrays (with the periodic wrap).  Unknown incoming
 * populations are left NaN for the boundary and fine-to-coarse steps. */
static int opposite(int i);

/* Interpolated bounce-back of Bouzidi, Firdaouss and Lallemand (linear form,
 * resting wall), the solid-cell alternative to the IBM named in Sec. 2.1 and
 * used in Sec. 3.2.  The population of direction i that fluid cell x would
 * pull from a solid neighbour x - c_i instead comes from the population
 * o = opposite(i) that x sent toward the wall, which sits at fraction q of
 * the link x -> x + c_o:
 *   q <  1/2:  f_i(x) = 2q f*_o(x) + (1 - 2q) f*_o(x - c_o)
 *   q >= 1/2:  f_i(x) = f*_o(x) / (2q) + (2q - 1)/(2q) f*_i(x).
 * (q = 1/2 is half-way bounce-back.) */
static double bouzidi(const orc_sim *s, const olev *L, int x, int y, int i) {
    int o = opposite(i);
    size_t c = cid(L, x, y);
    double q = L->sq[c * Q + o];
    if (q < 0.5) {
        int ux = x - CX[o], uy = y - CY[o];
        wrap_level(s, L, &ux, &uy);
        return 2.0 * q * L->fs[c * Q + o] + (1.0 - 2.0 * q) * L->fs[cid(L, ux, uy) * Q + o];
    }
    return L->fs[c * Q + o] / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * L->fs[c * Q + i];
}

static void stream_level(orc_sim *s, int l) {
    olev *L = &s->L[l];
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < L->n_act; ++k) {
        const size_t q = (size_t)L->act[k];
        const int x = (int)(q % (size_t)L->nx), y = (int)(q / (size_t)L->nx);
        if (L->solid && L->solid[q]) continue;
        for (int i = 0; i < Q; ++i) {
            int sx = x - CX[i], sy = y - CY[i];
            double v = NAN;
            if (wrap_level(s, L, &sx, &sy)) {
                size_t p = cid(L, sx, sy);
                if (L->solid && L->solid[p]) {
                    v = bouzidi(s, L, x, y, i);
                } else if (L->kind[p] == K_OWN || L->kind[p] == K_GHOST) {
                    v = L->fs[p * Q + i];
                }
            }
            L->f[q * Q + i] = v;
        }
    }
}

/* Halo sources of the second fine stream (step (5) of Sec. 2.4): the halo cells' sources
 * are their own post-stream values of the first substep. */
static void halo_second_sources(orc_sim *s, int l) {
    olev *L = &s->L[l];
    for (int64_t k = 0; k < L->n_ghost; ++k) {
        const size_t q = (size_t)L->ghost[k];
        memcpy(L->fs + q * Q, L->f + q * Q, sizeof(double) * Q);
    }
}

static int opposite(int i) {
    for (int k = 0; k < Q; ++k)
        if (CX[k] == -CX[i] && CY[k] == -CY[i]) return k;
    return -1;
}

static int mirror(int i, int normal_x) {
    for (int k = 0; k < Q; ++k) {
        if (normal_x && CX[k] == -CX[i] && CY[k] == CY[i]) return k;
        if (!normal_x && CX[k] == CX[i] && CY[k] == -CY[i]) return k;
    }
    return -1;
}

/* Clamp a cell reference into the level (used only for corner populations). */
static void clamp_level(const olev *L, int *x, int *y) {
    if (*x < 0) *x = 0;
    if (*x >= L->nx) *x = L->nx - 1;
    if (*y < 0) *y = 0;
    if (*y >= L->ny) *y = L->ny - 1;
}

static int local_kind(int k) { return k == ORC_BC_WALL || k == ORC_BC_INFLOW; }

/* Domain edges: fills the unknown populations of edge cells.  A
 * population whose source lies beyond one non-periodic edge takes that
 * edge's rule; one beyond two edges (a corner diagonal) takes the W/E edge's
 * rule unless only the S/N edge is a wall or inflow, with any cell that rule
 * refers to clamped into the domain. */
static void edge_rules(orc_sim *s, int l) {
    olev *L = &s->L[l];
    if (s->per_x && s->per_y) return;
    const int nrm[4][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}};
    double rho0 = s->c.rho0;
    for (int64_t k = 0; k < L->n_own; ++k) {
        const size_t q = (size_t)L->own[k];
        const int x = (int)(q % (size_t)L->nx), y = (int)(q / (size_t)L->nx);
        for (int i = 1; i < Q; ++i) {
            int sx = x - CX[i], sy = y - CY[i];
            int outx = (sx < 0 || sx >= L->nx) && !s->per_x;
            int outy = (sy < 0 || sy >= L->ny) && !s->per_y;
            if (!outx && !outy) continue;
            int ex = sx < 0 ? ORC_W : ORC_E, ey = sy < 0 ? ORC_S : ORC_N;
            int e = outx ? ex : ey;
            if (outx && outy && !local_kind(s->c.bc[ex]) && local_kind(s->c.bc[ey])) e = ey;
            double *fx = L->f + q * Q;
            const double *fsx = L->fs + q * Q;
            double uwx = s->c.bc_u[2 * e], uwy = s->c.bc_u[2 * e + 1];
            switch (s->c.bc[e]) {
            case ORC_BC_WALL:
                fx[i] = fsx[opposite(i)] + 6.0 * WT[i] * rho0 * (CX[i] * uwx + CY[i] * uwy);
                break;
            case ORC_BC_INFLOW: {
                double feq[Q];
                orc_feq(rho0, uwx, uwy, feq);
                fx[i] = feq[i];
            } break;
            case ORC_BC_OUTFLOW: {
                int px = x - nrm[e][0] - CX[i], py = y - nrm[e][1] - CY[i];
                wrap_level(s, L, &px, &py);
                clamp_level(L, &px, &py);
                fx[i] = L->fs[cid(L, px, py) * Q + i];
            } break;
            case ORC_BC_SYMMETRY: {
                int nx_ = (e == ORC_W || e == ORC_E);
                int px = x - (nx_ ? 0 : CX[i]), py = y - (nx_ ? CY[i] : 0);
                wrap_level(s, L, &px, &py);
                clamp_level(L, &px, &py);
                fx[i] = L->fs[cid(L, px, py) * Q + mirror(i, nx_)];
            } break;
            default: break;
            }
        }
    }
}

/* Coalescence (step (6) of Sec. 2.4). */
static void coalesce(orc_sim *s, int lf, int lc) {
    olev *F = &s->L[lf], *C = &s->L[lc];
    double fac[2];
    orc_interface_factors(C->tau, F->tau, fac);
    const double sfc = fac[1];
    int rescale = s->c.cf_mode == ORC_CF_RESCALE;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < C->n_own; ++k) {
        const size_t q = (size_t)C->own[k];
        const int x = (int)(q % (size_t)C->nx), y = (int)(q / (size_t)C->nx);
        int hid[Q];
        int any = 0;
        for (int i = 0; i < Q; ++i) {
            int sx = x - CX[i], sy = y - CY[i];
            hid[i] = wrap_level(s, C, &sx, &sy) && C->kind[cid(C, sx, sy)] == K_HIDDEN;
            any |= hid[i];
        }
        if (!any) continue;
        double avg[Q];
        for (int i = 0; i < Q; ++i) {
            if (!hid[i]) continue;
            double sum = F->f[cid(F, 2 * x, 2 * y) * Q + i];
            sum += F->f[cid(F, 2 * x + 1, 2 * y) * Q + i];
            sum += F->f[cid(F, 2 * x, 2 * y + 1) * Q + i];
            sum += F->f[cid(F, 2 * x + 1, 2 * y + 1) * Q + i];
            avg[i] = 0.25 * sum;
        }
        double *dst = C->f + q * Q;
        if (!rescale) {
            for (int i = 0; i < Q; ++i) if (hid[i]) dst[i] = avg[i];
        } else {
            double g[Q], r = 0.0, jx = 0.0, jy = 0.0;
            for (int i = 0; i < Q; ++i) g[i] = hid[i] ? avg[i] : dst[i];
            for (int i = 0; i < Q; ++i) { r += g[i]; jx += CX[i] * g[i]; jy += CY[i] * g[i]; }
            double feq[Q];
            orc_feq(r, jx / r, jy / r, feq);
            for (int i = 0; i < Q; ++i)
                if (hid[i]) dst[i] = feq[i] + sfc * (avg[i] - feq[i]);
        }
    }
}

/* One coarse (level-0) time step of the whole forest, Sec. 2.4 and 2.5.
 *
 * Acoustic scaling gives level l a time step of 2^-l coarse units, so the
 * finest level m-1 takes 2^(m-1) substeps per coarse step and substep j of
 * level l covers the finest substeps [j 2^(m-1-l), (j+1) 2^(m-1-l)).  Each
 * level substep collides at the start of its interval and streams at its
 * end.  Walking a clock over the finest substeps therefore gives the order:
 * at the start of finest substep t every level whose interval starts there
 * collides, coarse to fine; at its end every level whose interval ends there
 * streams, fine to coarse.  The interface steps (1)-(6) of Sec. 2.4 fall in
 * place:
 *   (1) the coarse level collides before its two fine substeps;
 *   (2) before the first of them the fine halo takes the coarse
 *       post-collision populations (explosion);
 *   (3) the fine level streams its owned and halo cells;
 *   (4) the fine level collides again (halo cells never collide);
 *   (5) it streams a second time, the halo cells supplying the values they
 *       received in (3);
 *   (6) when the coarse interval ends, the coarse level streams and takes
 *       the fine populations it cannot stream itself (coalescence).
 * The immersed-boundary forcing (Sec. 2.2) precedes every finest collision. */
static void level_collide(orc_sim *s, int l) {
    const int finest = l == s->m - 1;
    if (finest && s->c.body_kind != ORC_BODY_NONE) {
        ibm_forcing(s, l);
        s->k++;
    }
    collide_level(s, l);
}

/* End of substep j of level l: halo preparation (explosion before the first
 * of the two substeps inside a coarse substep, the halo's own first-stream
 * values before the second), streaming, domain edges, coalescence from the
 * finer level. */
static void level_stream(orc_sim *s, int l, int64_t j) {
    if (l > 0) {
        if ((j & 1) == 0) explode(s, l - 1, l);
        else halo_second_sources(s, l);
    }
    stream_level(s, l);
    edge_rules(s, l);
    if (l + 1 < s->m) coalesce(s, l + 1, l);
}

static void coarse_step(orc_sim *s) {
    const int m = s->m;
    const int64_t nsub = (int64_t)1 << (m - 1);      /* finest substeps per coarse step */
    for (int64_t t = 0; t < nsub && !s->err; ++t) {
        for (int l = 0; l < m; ++l) {
            const int64_t span = nsub >> l;              /* finest substeps per level-l substep */
            if (t % span == 0) level_collide(s, l);
        }
        for (int l = m - 1; l >= 0; --l) {
            const int64_t span = nsub >> l;
            if ((t + 1) % span == 0) level_stream(s, l, t / span);
        }
    }
}

int orc_step(orc_sim *s, int32_t n) {
    for (int32_t t = 0; t < n && !s->err; ++t) {
        if (s->c.body_kind == ORC_BODY_NONE) s->k += (int64_t)1 << (s->m - 1);
        coarse_step(s);
    }
    return s->err;
}

int64_t orc_substeps(const orc_sim *s) { return s->k; }

/* ------------------------------------------------------------------------ */
/* Outputs                                                                   */
/* ------------------------------------------------------------------------ */

int orc_read_fields(const orc_sim *s, int level, double *rho, double *ux, double *uy) {
    if (level < 0 || level >= s->m) return ORC_ERR_ARG;
    const olev *L = &s->L[level];
    for (size_t q = 0; q < (size_t)L->nx * L->ny; ++q) {
        if (L->kind[q] != K_OWN || (L->solid && L->solid[q])) { rho[q] = ux[q] = uy[q] = NAN; continue; }
        const double *f = L->f + q * Q;
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int i = 0; i < Q; ++i) { r += f[i]; jx += CX[i] * f[i]; jy += CY[i] * f[i]; }
        rho[q] = r;
        ux[q] = (jx + 0.5 * L->fx) / r;
        uy[q] = (jy + 0.5 * L->fy) / r;
    }
    return ORC_OK;
}

int orc_read_populations(const orc_sim *s, int level, double *f) {
    if (level < 0 || level >= s->m) return ORC_ERR_ARG;
    const olev *L = &s->L[level];
    memcpy(f, L->f, sizeof(double) * Q * L->nx * L->ny);
    return ORC_OK;
}

int orc_marker_forces(const orc_sim *s, double *fx, double *fy) {
    for (int j = 0; j < s->c.n_markers; ++j) { fx[j] = s->ftx[j]; fy[j] = s->fty[j]; }
    return ORC_OK;
}

int orc_set_markers(orc_sim *s, int32_t n, const double *X, const double *Y, const double *udx,
                    const double *udy, const double *ds) {
    if (s->c.body_kind != ORC_BODY_HOST || n != s->c.n_markers) return ORC_ERR_ARG;
    for (int j = 0; j < n; ++j) {
        s->xb[j] = X[j];
        s->yb[j] = Y[j];
        s->hud[j] = udx[j];
        s->hud[n + j] = udy[j];
        if (ds) s->ds[j] = ds[j];
    }
    return ORC_OK;
}

int orc_force_history(const orc_sim *s, int32_t cap, double *fx, double *fy, int32_t *n_out) {
    int64_t n = s->nhist < cap ? s->nhist : cap;
    int64_t first = s->nhist - n;
    for (int64_t t = 0; t < n; ++t) {
        fx[t] = s->hist[2 * (first + t)];
        fy[t] = s->hist[2 * (first + t) + 1];
    }
    *n_out = (int32_t)n;
    return ORC_OK;
}

int orc_diagnostics(const orc_sim *s, double out[3]) {
    double M = 0.0, Px = 0.0, Py = 0.0;
    for (int l = 0; l < s->m; ++l) {
        const olev *L = &s->L[l];
        double vol = 1.0 / (double)(1 << (2 * l));
        double m = 0.0, px = 0.0, py = 0.0;
        for (size_t q = 0; q < (size_t)L->nx * L->ny; ++q) {
            if (L->kind[q] != K_OWN || (L->solid && L->solid[q])) continue;
            const double *f = L->f + q * Q;
            for (int i = 0; i < Q; ++i) { m += f[i]; px += CX[i] * f[i]; py += CY[i] * f[i]; }
        }
        M += vol * m; Px += vol * px; Py += vol * py;
    }
    out[0] = M; out[1] = Px; out[2] = Py;
    return ORC_OK;
}

/* Sec. 3.3, Eq. (21): statistics of the coefficient histories
 * C_D = scale fx, C_L = scale fy (scale = 1 / (rho0 U^2 L / 2)), n samples
 * one finest substep apart.  out = {mean C_D, mean C_L, rms(C_D - mean),
 * rms(C_L - mean), St, upward crossings, n}.  The lift frequency is read off
 * the history as (crossings - 1) periods between the first and the last
 * upward crossing of C_L through its mean, each crossing time interpolated
 * linearly between the two samples around it; St = f L / U = f l_over_u. */
int orc_force_stats(const double *fx, const double *fy, int32_t n, double scale, double l_over_u,
                    double out[7]) {
    if (n < 2) return ORC_ERR_ARG;
    double sd = 0.0, sl = 0.0;
    for (int32_t i = 0; i < n; ++i) { sd += fx[i] * scale; sl += fy[i] * scale; }
    double md = sd / n, ml = sl / n;
    double vd = 0.0, vl = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        double dd = fx[i] * scale - md, dl = fy[i] * scale - ml;
        vd += dd * dd;
        vl += dl * dl;
    }
    int32_t up = 0;
    double first = 0.0, last = 0.0;
    for (int32_t i = 0; i + 1 < n; ++i) {
        double c0 = fy[i] * scale - ml, c1 = fy[i + 1] * scale - ml;
        if (c0 < 0.0 && c1 >= 0.0) {
            double t = (double)i + c0 / (c0 - c1);
            if (up == 0) first = t;
            last = t;
            ++up;
        }
    }
    out[0] = md;
    out[1] = ml;
    out[2] = sqrt(vd / n);
    out[3] = sqrt(vl / n);
    out[4] = up >= 2 ? (double)(up - 1) / (last - first) * l_over_u : 0.0;
    out[5] = up;
    out[6] = n;
    return ORC_OK;
}

/* Solid cells of a level for the interpolated bounce-back (see bouzidi()).
 * mask: dense level cells, 1 = solid.  q: dense [cell][9], read for fluid
 * cells x whose neighbour x + c_i is solid (0 < q <= 1; NULL: 1/2 on every
 * link).  Every cell within two cells of a solid cell must be an owned cell
 * of this level (no halo, no covered cell, no domain edge).  Where q < 1/2
 * and the upstream cell x - c_i is solid too, the link takes q = 1/2
 * (half-way bounce-back).  Only before the first step. */
int orc_set_solid(orc_sim *s, int level, const uint8_t *mask, const double *q) {
    if (level < 0 || level >= s->m || !mask) return ORC_ERR_ARG;
    olev *L = &s->L[level];
    size_t n = (size_t)L->nx * L->ny;
    uint8_t *sm = calloc(n, 1);
    double *sq = malloc(sizeof(double) * n * Q);
    for (size_t c = 0; c < n * Q; ++c) sq[c] = 0.5;
    for (size_t c = 0; c < n; ++c) sm[c] = mask[c] ? 1 : 0;
    for (int y = 0; y < L->ny; ++y)
        for (int x = 0; x < L->nx; ++x) {
            if (!sm[cid(L, x, y)]) continue;
            for (int dy = -2; dy <= 2; ++dy)
                for (int dx = -2; dx <= 2; ++dx) {
                    int xx = x + dx, yy = y + dy;
                    if (!wrap_level(s, L, &xx, &yy) || L->kind[cid(L, xx, yy)] != K_OWN) {
                        free(sm); free(sq);
                        return ORC_ERR_TOPOLOGY;
                    }
                }
        }
    for (int y = 0; y < L->ny; ++y)
        for (int x = 0; x < L->nx; ++x) {
            size_t c = cid(L, x, y);
            if (sm[c]) continue;
            for (int i = 1; i < Q; ++i) {
                int nx_ = x + CX[i], ny_ = y + CY[i];
                if (!wrap_level(s, L, &nx_, &ny_) || !sm[cid(L, nx_, ny_)]) continue;
                double v = q ? q[c * Q + i] : 0.5;
                if (!(v > 0.0 && v <= 1.0)) { free(sm); free(sq); return ORC_ERR_ARG; }
                int ux = x - CX[i], uy = y - CY[i];
                if (v < 0.5 && (!wrap_level(s, L, &ux, &uy) || sm[cid(L, ux, uy)])) v = 0.5;
                sq[c * Q + i] = v;
            }
        }
    free(L->solid); free(L->sq);
    L->solid = sm;
    L->sq = sq;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Three dimensions: D3Q19 and D3Q27 on one periodic level                  */
/* ------------------------------------------------------------------------ */

/* The 3D velocity sets the paper's method extends to, with c_s^2 = 1/3.
 * D3Q19: rest (w = 1/3), 6 axis (1/18), 12 edge (1/36) velocities.  D3Q27
 * adds the 8 corners: rest 8/27, axis 2/27, edge 1/54, corner 1/216.
 * Order: rest, +x -x +y -y +z -z, the edges (+-1, +-1, 0), (+-1, 0, +-1),
 * (0, +-1, +-1), then (D3Q27) the corners. */
static const int C3X[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                            1, -1, 1, -1, 1, -1, 1, -1};
static const int C3Y[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1,
                            1, 1, -1, -1, 1, 1, -1, -1};
static const int C3Z[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1,
                            1, 1, 1, 1, -1, -1, -1, -1};

static double w3(int q, int i) {
    if (q == 19) return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    return i == 0 ? 8.0 / 27.0 : (i < 7 ? 2.0 / 27.0 : (i < 19 ? 1.0 / 54.0 : 1.0 / 216.0));
}

void orc3_velocity_set(int32_t q, int32_t *cx, int32_t *cy, int32_t *cz, double *w) {
    for (int i = 0; i < q; ++i) { cx[i] = C3X[i]; cy[i] = C3Y[i]; cz[i] = C3Z[i]; w[i] = w3(q, i); }
}

/* Eq. (7) in 3D. */
void orc3_feq(int32_t q, double rho, double ux, double uy, double uz, double *out) {
    double usq = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < q; ++i) {
        double cu = C3X[i] * ux + C3Y[i] * uy + C3Z[i] * uz;
        out[i] = w3(q, i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    }
}

static int opposite3(int i) {
    for (int k = 0; k < 27; ++k)
        if (C3X[k] == -C3X[i] && C3Y[k] == -C3Y[i] && C3Z[k] == -C3Z[i]) return k;
    return -1;
}

struct orc3_sim;
static double bouzidi3(const struct orc3_sim *s, int x, int y, int z, int i);

struct orc3_sim {
    int nx, ny, nz, q;
    int walls;                /* 1: half-way bounce-back walls below z = 0 and above z = nz - 1 */
    double uw[2][3];          /* bottom and top wall velocities                                  */
    double rho_w;             /* wall density of the moving-wall term                            */
    uint8_t *solid;           /* solid cells (interpolated bounce-back), or NULL                 */
    double *sq;               /* [cell][q] wall fraction of link i from a fluid cell toward x + c_i */
    int nm, iters;            /* immersed body: markers, N_F                                     */
    double *bx, *by, *bz, *bdA;   /* markers: absolute (kind 0) or body frame (kind 1)           */
    int kind;                 /* 0 fixed, 1 pitch about y + plunge along z                       */
    double bp[10];            /* kind 1: x0, y0, z0, alpha0, A_pitch, A0, T, phi, U_ref, chord   */
    int64_t k;                /* steps whose forcing loop has run                                */
    double *Fb;               /* [3][cell] IBM force density of the current step                 */
    double fsb[3];            /* body force F_s of the last step                                 */
    double tau, F[3];
    double *f, *fs;           /* [cell][q], cell = (z ny + y) nx + x */
};

int orc3_create(int32_t nx, int32_t ny, int32_t nz, int32_t q, double tau, const double F[3], orc3_sim **out) {
    *out = NULL;
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(tau > 0.5) || (q != 19 && q != 27)) return ORC_ERR_ARG;
    orc3_sim *s = calloc(1, sizeof(orc3_sim));
    s->nx = nx; s->ny = ny; s->nz = nz; s->q = q; s->tau = tau;
    for (int k = 0; k < 3; ++k) s->F[k] = F ? F[k] : 0.0;
    size_t n = (size_t)nx * ny * nz * q;
    s->f = malloc(sizeof(double) * n);
    s->fs = malloc(sizeof(double) * n);
    for (size_t c = 0; c < n; ++c) s->f[c] = s->fs[c] = NAN;
    *out = s;
    return ORC_OK;
}

/* The population of direction i that fluid cell (x, y, z) would pull from a
 * solid neighbour x - c_i: o = opposite(i) at wall fraction q of the link
 * x -> x + c_o,  q < 1/2: 2q f*_o(x) + (1 - 2q) f*_o(x - c_o);
 * q >= 1/2: f*_o(x) / (2q) + (2q - 1)/(2q) f*_i(x). */
static double bouzidi3(const struct orc3_sim *s, int x, int y, int z, int i) {
    const int nx = s->nx, ny = s->ny, nz = s->nz, Q3 = s->q;
    int o = opposite3(i);
    size_t c = ((size_t)z * ny + y) * nx + x;
    double q = s->sq[c * Q3 + o];
    if (q < 0.5) {
        int ux = (x - C3X[o] + nx) % nx, uy = (y - C3Y[o] + ny) % ny, uz = (z - C3Z[o] + nz) % nz;
        return 2.0 * q * s->fs[c * Q3 + o] + (1.0 - 2.0 * q) * s->fs[(((size_t)uz * ny + uy) * nx + ux) * Q3 + o];
    }
    return s->fs[c * Q3 + o] / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * s->fs[c * Q3 + i];
}

void orc3_destroy(orc3_sim *s) {
    if (!s) return;
    free(s->f); free(s->fs); free(s->solid); free(s->sq);
    free(s->bx); free(s->Fb); free(s);
}

int orc3_init_fields(orc3_sim *s, const double *rho, const double *ux, const double *uy, const double *uz) {
    size_t n = (size_t)s->nx * s->ny * s->nz;
    for (size_t c = 0; c < n; ++c) orc3_feq(s->q, rho[c], ux[c], uy[c], uz[c], s->f + c * s->q);
    return ORC_OK;
}

/* One step: BGK + Guo forcing with the half-force velocity (Eqs. (2)-(3),
 * (6)-(8) in 3D), then periodic streaming f(x, i) <- f*(x - c_i, i). */
/* Sec. 2.2 in 3D for a fixed body (desired velocity 0): the multi-direct
 * forcing loop on the current pre-collision state, with the Peskin kernel of
 * Eq. (14) in each axis (taps z outer, y, x inner; weight phi_x (phi_y phi_z)).
 * Per iteration: U_j and rho_j interpolated, g_j = 2 rho_j (0 - U_j),
 * spread in marker order as g_j w dA_j, F += dF and u += dF / (2 rho); then
 * F_s = -sum_j F_j dA_j.  Fills s->Fb and s->fs. */
/* Marker positions at step t: kind 0 as given; kind 1 the Sec. 3.6 law in
 * the x-z plane (pitch alpha about the y axis, plunge along z):
 *   t* = t U_ref / c, theta = 2 pi t* / T, alpha = alpha0 - A_pitch sin(theta + phi),
 *   centre (x0, y0, z0 + (A0/2) cos theta),
 *   X = xc + xb cos a + zb sin a,  Y = yc + yb,  Z = zc - xb sin a + zb cos a. */
static void body3_positions(const orc3_sim *s, double t, double *X, double *Y, double *Z) {
    const double *p = s->bp;
    if (s->kind == 0) {
        for (int j = 0; j < s->nm; ++j) { X[j] = s->bx[j]; Y[j] = s->by[j]; Z[j] = s->bz[j]; }
        return;
    }
    double tstar = t * p[8] / p[9];
    double theta = 2.0 * M_PI * tstar / p[6];
    double alpha = p[3] - p[4] * sin(theta + p[7]);
    double zc = p[2] + 0.5 * p[5] * cos(theta);
    double ca = cos(alpha), sa = sin(alpha);
    for (int j = 0; j < s->nm; ++j) {
        X[j] = p[0] + s->bx[j] * ca + s->bz[j] * sa;
        Y[j] = p[1] + s->by[j];
        Z[j] = zc - s->bx[j] * sa + s->bz[j] * ca;
    }
}

static void mdf3(orc3_sim *s) {
    const int nx = s->nx, ny = s->ny, nz = s->nz, Q3 = s->q, nm = s->nm;
    const size_t n = (size_t)nx * ny * nz;
    double *pos = malloc(sizeof(double) * nm * 9), *PX = pos, *PY = pos + nm, *PZ = pos + 2 * nm;
    double *ud = pos + 3 * nm, *Q1 = pos + 6 * nm;
    body3_positions(s, (double)s->k, PX, PY, PZ);
    body3_positions(s, (double)(s->k + 1), Q1, Q1 + nm, Q1 + 2 * nm);
    for (int j = 0; j < nm; ++j) {
        ud[3 * j] = Q1[j] - PX[j];
        ud[3 * j + 1] = Q1[nm + j] - PY[j];
        ud[3 * j + 2] = Q1[2 * nm + j] - PZ[j];
    }
    double *rho = malloc(sizeof(double) * n * 7), *u = rho + n, *dF = rho + 4 * n;
    for (size_t c = 0; c < n; ++c) {
        const double *f = s->f + c * Q3;
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < Q3; ++i) { r += f[i]; jx += C3X[i] * f[i]; jy += C3Y[i] * f[i]; jz += C3Z[i] * f[i]; }
        rho[c] = r;
        u[c] = (jx + 0.5 * s->F[0]) / r;
        u[n + c] = (jy + 0.5 * s->F[1]) / r;
        u[2 * n + c] = (jz + 0.5 * s->F[2]) / r;
    }
    memset(s->Fb, 0, sizeof(double) * 3 * n);
    double *g = malloc(sizeof(double) * nm * 6), *ft = g + 3 * nm;
    for (int j = 0; j < 3 * nm; ++j) ft[j] = 0.0;
    for (int it = 0; it < s->iters; ++it) {
        for (int j = 0; j < nm; ++j) {
            int i0 = tap0(PX[j]), j0 = tap0(PY[j]), k0 = tap0(PZ[j]);
            double U[3] = {0.0, 0.0, 0.0}, R = 0.0;
            for (int cc = 0; cc < 4; ++cc) {
                double pz = orc_phi(k0 + cc + 0.5 - PZ[j]);
                int zz = (k0 + cc + nz) % nz;
                for (int b = 0; b < 4; ++b) {
                    double pyz = orc_phi(j0 + b + 0.5 - PY[j]) * pz;
                    int yy = (j0 + b + ny) % ny;
                    for (int a = 0; a < 4; ++a) {
                        double w = orc_phi(i0 + a + 0.5 - PX[j]) * pyz;
                        size_t c = ((size_t)zz * ny + yy) * nx + (i0 + a + nx) % nx;
                        U[0] += u[c] * w;
                        U[1] += u[n + c] * w;
                        U[2] += u[2 * n + c] * w;
                        R += rho[c] * w;
                    }
                }
            }
            for (int k = 0; k < 3; ++k) {
                g[3 * j + k] = 2.0 * R * (ud[3 * j + k] - U[k]);
                ft[3 * j + k] += g[3 * j + k];
            }
        }
        memset(dF, 0, sizeof(double) * 3 * n);
        for (int j = 0; j < nm; ++j) {
            int i0 = tap0(PX[j]), j0 = tap0(PY[j]), k0 = tap0(PZ[j]);
            for (int cc = 0; cc < 4; ++cc) {
                double pz = orc_phi(k0 + cc + 0.5 - PZ[j]);
                int zz = (k0 + cc + nz) % nz;
                for (int b = 0; b < 4; ++b) {
                    double pyz = orc_phi(j0 + b + 0.5 - PY[j]) * pz;
                    int yy = (j0 + b + ny) % ny;
                    for (int a = 0; a < 4; ++a) {
                        double w = orc_phi(i0 + a + 0.5 - PX[j]) * pyz;
                        size_t c = ((size_t)zz * ny + yy) * nx + (i0 + a + nx) % nx;
                        for (int k = 0; k < 3; ++k) dF[k * n + c] += g[3 * j + k] * w * s->bdA[j];
                    }
                }
            }
        }
        for (size_t c = 0; c < n; ++c) {
            if (dF[c] == 0.0 && dF[n + c] == 0.0 && dF[2 * n + c] == 0.0) continue;
            for (int k = 0; k < 3; ++k) {
                s->Fb[k * n + c] += dF[k * n + c];
                u[k * n + c] += dF[k * n + c] / (2.0 * rho[c]);
            }
        }
    }
    for (int k = 0; k < 3; ++k) {
        double t = 0.0;
        for (int j = 0; j < nm; ++j) t -= ft[3 * j + k] * s->bdA[j];
        s->fsb[k] = t;
    }
    free(g); free(rho); free(pos);
    s->k++;
}

int orc3_set_body(orc3_sim *s, int32_t n, const double *X, const double *Y, const double *Z, const double *dA,
                  int32_t iters) {
    if (n <= 0 || iters < 0) return ORC_ERR_ARG;
    free(s->bx); free(s->Fb);
    s->bx = malloc(sizeof(double) * 4 * n);
    s->by = s->bx + n; s->bz = s->bx + 2 * n; s->bdA = s->bx + 3 * n;
    memcpy(s->bx, X, sizeof(double) * n); memcpy(s->by, Y, sizeof(double) * n);
    memcpy(s->bz, Z, sizeof(double) * n); memcpy(s->bdA, dA, sizeof(double) * n);
    s->nm = n;
    s->iters = iters;
    s->kind = 0;
    s->k = 0;
    s->Fb = calloc((size_t)3 * s->nx * s->ny * s->nz, sizeof(double));
    return ORC_OK;
}

/* Motion of the body (after orc3_set_body): kind 0 fixed (markers absolute),
 * kind 1 the pitch/plunge law of body3_positions (markers in the body frame). */
int orc3_set_motion(orc3_sim *s, int32_t kind, const double p[10]) {
    if (kind != 0 && kind != 1) return ORC_ERR_ARG;
    s->kind = kind;
    for (int i = 0; i < 10; ++i) s->bp[i] = p ? p[i] : 0.0;
    return ORC_OK;
}

int orc3_marker_positions(const orc3_sim *s, double t, double *X, double *Y, double *Z) {
    if (s->nm <= 0) return ORC_ERR_ARG;
    body3_positions(s, t, X, Y, Z);
    return ORC_OK;
}

int orc3_body_force(const orc3_sim *s, double out[3]) {
    for (int k = 0; k < 3; ++k) out[k] = s->fsb[k];
    return ORC_OK;
}

int orc3_step(orc3_sim *s, int32_t steps) {
    const int nx = s->nx, ny = s->ny, nz = s->nz, Q3 = s->q;
    const size_t n = (size_t)nx * ny * nz;
    const double tau = s->tau;
    for (int32_t t = 0; t < steps; ++t) {
        if (s->nm > 0) mdf3(s);
#pragma omp parallel for schedule(static)
        for (size_t c = 0; c < n; ++c) {
            if (s->solid && s->solid[c]) continue;
            double Fx = s->F[0], Fy = s->F[1], Fz = s->F[2];
            if (s->nm > 0) { Fx += s->Fb[c]; Fy += s->Fb[n + c]; Fz += s->Fb[2 * n + c]; }
            const double *f = s->f + c * Q3;
            double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
            for (int i = 0; i < Q3; ++i) { rho += f[i]; jx += C3X[i] * f[i]; jy += C3Y[i] * f[i]; jz += C3Z[i] * f[i]; }
            double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho, uz = (jz + 0.5 * Fz) / rho;
            double feq[27];
            orc3_feq(Q3, rho, ux, uy, uz, feq);
            double uF = ux * Fx + uy * Fy + uz * Fz, pre = 1.0 - 0.5 / tau;
            for (int i = 0; i < Q3; ++i) {
                double cu = C3X[i] * ux + C3Y[i] * uy + C3Z[i] * uz;
                double cF = C3X[i] * Fx + C3Y[i] * Fy + C3Z[i] * Fz;
                double fi = w3(Q3, i) * pre * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF);
                s->fs[c * Q3 + i] = f[i] - (f[i] - feq[i]) / tau + fi;
            }
        }
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    for (int i = 0; i < Q3; ++i) {
                        size_t c = ((size_t)z * ny + y) * nx + x;
                        if (s->solid && s->solid[c]) continue;
                        int zs = z - C3Z[i];
                        if (s->solid && !(s->walls && (zs < 0 || zs >= nz))) {
                            int sx0 = (x - C3X[i] + nx) % nx, sy0 = (y - C3Y[i] + ny) % ny, sz0 = (zs + nz) % nz;
                            if (s->solid[((size_t)sz0 * ny + sy0) * nx + sx0]) {
                                s->f[c * Q3 + i] = bouzidi3(s, x, y, z, i);
                                continue;
                            }
                        }
                        if (s->walls && (zs < 0 || zs >= nz)) {
                            int o = opposite3(i);
                            const double *u = s->uw[zs < 0 ? 0 : 1];
                            double cu = C3X[o] * u[0] + C3Y[o] * u[1] + C3Z[o] * u[2];
                            s->f[c * Q3 + i] = s->fs[c * Q3 + o] - 6.0 * w3(Q3, i) * s->rho_w * cu;
                            continue;
                        }
                        int sx = (x - C3X[i] + nx) % nx, sy = (y - C3Y[i] + ny) % ny, sz = (zs + nz) % nz;
                        s->f[c * Q3 + i] = s->fs[(((size_t)sz * ny + sy) * nx + sx) * Q3 + i];
                    }
    }
    return ORC_OK;
}

/* Walls across z: a population that would stream in from outside the box is
 * the opposite population of the same cell bounced back half-way, with the
 * moving-wall term of the 2D walls (wall density rho0, the reference
 * density): f_i(x) = f*_o(x) - 6 w_i rho0 (c_o . u_wall), o = opposite(i). */
int orc3_set_walls(orc3_sim *s, double rho0, const double ub[3], const double ut[3]) {
    s->walls = 1;
    s->rho_w = rho0;
    for (int k = 0; k < 3; ++k) { s->uw[0][k] = ub ? ub[k] : 0.0; s->uw[1][k] = ut ? ut[k] : 0.0; }
    return ORC_OK;
}

/* Solid cells with the interpolated bounce-back of the 2D solid cells
 * (Bouzidi, Firdaouss and Lallemand, linear form, resting wall) in 3D.
 * mask [cell] nonzero = solid; q [cell][q] the wall fraction of the link from
 * a fluid cell x toward a solid x + c_i (NULL: 1/2), read there only.  A short
 * link (q < 1/2) whose upstream cell x - c_i is solid or beyond a z wall
 * takes q = 1/2.  Solid cells are not collided and read out as NaN. */
int orc3_set_solid(orc3_sim *s, const uint8_t *mask, const double *q) {
    const int nx = s->nx, ny = s->ny, nz = s->nz, Q3 = s->q;
    size_t n = (size_t)nx * ny * nz;
    uint8_t *sm = malloc(n);
    double *sq = malloc(sizeof(double) * n * Q3);
    for (size_t c = 0; c < n; ++c) sm[c] = mask[c] ? 1 : 0;
    for (size_t c = 0; c < n * Q3; ++c) sq[c] = 0.5;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t c = ((size_t)z * ny + y) * nx + x;
                if (sm[c]) continue;
                for (int i = 1; i < Q3; ++i) {
                    int az = z + C3Z[i];
                    if (s->walls && (az < 0 || az >= nz)) continue;
                    int ax = (x + C3X[i] + nx) % nx, ay = (y + C3Y[i] + ny) % ny;
                    az = (az + nz) % nz;
                    if (!sm[((size_t)az * ny + ay) * nx + ax]) continue;
                    double v = q ? q[c * Q3 + i] : 0.5;
                    if (!(v > 0.0 && v <= 1.0)) { free(sm); free(sq); return ORC_ERR_ARG; }
                    int uz = z - C3Z[i];
                    int ux = (x - C3X[i] + nx) % nx, uy = (y - C3Y[i] + ny) % ny;
                    int behind_solid = (s->walls && (uz < 0 || uz >= nz)) ||
                                       sm[((size_t)((uz + nz) % nz) * ny + uy) * nx + ux];
                    if (v < 0.5 && behind_solid) v = 0.5;
                    sq[c * Q3 + i] = v;
                }
            }
    free(s->solid); free(s->sq);
    s->solid = sm;
    s->sq = sq;
    return ORC_OK;
}

/* rho and u = (sum_i c_i f_i + F/2) / rho of every cell (dense arrays). */
int orc3_read_fields(const orc3_sim *s, double *rho, double *ux, double *uy, double *uz) {
    size_t n = (size_t)s->nx * s->ny * s->nz;
    for (size_t c = 0; c < n; ++c) {
        if (s->solid && s->solid[c]) { rho[c] = ux[c] = uy[c] = uz[c] = NAN; continue; }
        const double *f = s->f + c * s->q;
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < s->q; ++i) { r += f[i]; jx += C3X[i] * f[i]; jy += C3Y[i] * f[i]; jz += C3Z[i] * f[i]; }
        rho[c] = r;
        ux[c] = (jx + 0.5 * s->F[0]) / r;
        uy[c] = (jy + 0.5 * s->F[1]) / r;
        uz[c] = (jz + 0.5 * s->F[2]) / r;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Three dimensions on a block forest: the topology-confined refinement of  */
/* Sec. 2.3 and the coarse-fine interface of Sec. 2.4 in 3D (D3Q19 or       */
/* D3Q27), periodic in every direction                                       */
/* ------------------------------------------------------------------------ */

/* The same construction as in 2D, one dimension up: level l is a dense grid
 * of (nx0, ny0, nz0) 2^l cells; region_l is the union of the level's boxes
 * (level 0: everything); own_l = region_l minus the cells covered by
 * region_{l+1} (hidden); the halo of level l >= 1 is every cell outside
 * region_l within Chebyshev distance 2 of own_l, whose parent must be owned
 * on level l-1.  A coarse cell's 8 children are (2x + a, 2y + b, 2z + c),
 * a, b, c in {0, 1}. */
typedef struct {
    int nx, ny, nz;
    double tau, F[3];
    uint8_t *kind;
    double *f, *fs;           /* [cell][q] pre- / post-collision, cell = (z ny + y) nx + x */
    double *rho, *u;          /* moments of the last collision: rho [cell], u [cell][3] */
    int64_t *own, *ghost, *act;
    int64_t n_own, n_ghost, n_act;
} o3lev;

struct orc3f_sim {
    orc3f_case c;
    int32_t *boxes;
    int m, q;
    o3lev L[MAXL];
};

static inline size_t c3(const o3lev *L, int x, int y, int z) { return ((size_t)z * L->ny + y) * L->nx + x; }

static void wrap3(const o3lev *L, int *x, int *y, int *z) {
    *x = wrapi(*x, L->nx);
    *y = wrapi(*y, L->ny);
    *z = wrapi(*z, L->nz);
}

static int in_region3(const orc3f_sim *s, int l, int x, int y, int z) {
    if (l == 0) return 1;
    const int B = s->c.block_n;
    for (int b = 0; b < s->c.n_boxes; ++b) {
        const int32_t *q = s->boxes + 7 * b;
        if (q[0] != l) continue;
        if (x >= q[1] * B && x < q[4] * B && y >= q[2] * B && y < q[5] * B && z >= q[3] * B && z < q[6] * B) return 1;
    }
    return 0;
}

void orc3f_destroy(orc3f_sim *s) {
    if (!s) return;
    for (int l = 0; l < MAXL; ++l) {
        o3lev *L = &s->L[l];
        free(L->kind); free(L->f); free(L->fs); free(L->rho); free(L->u);
        free(L->own); free(L->ghost); free(L->act);
    }
    free(s->boxes);
    free(s);
}

static int topology3(orc3f_sim *s) {
    const int m = s->m;
    for (int l = 0; l < m; ++l) {
        o3lev *L = &s->L[l];
        for (int z = 0; z < L->nz; ++z)
            for (int y = 0; y < L->ny; ++y)
                for (int x = 0; x < L->nx; ++x) {
                    uint8_t kd = K_NONE;
                    if (in_region3(s, l, x, y, z)) {
                        kd = K_OWN;
                        if (l + 1 < m && in_region3(s, l + 1, 2 * x, 2 * y, 2 * z)) kd = K_HIDDEN;
                        if (l > 0 && !in_region3(s, l - 1, x / 2, y / 2, z / 2)) return ORC_ERR_TOPOLOGY;
                    }
                    L->kind[c3(L, x, y, z)] = kd;
                }
    }
    for (int l = 1; l < m; ++l) {
        o3lev *L = &s->L[l], *P = &s->L[l - 1];
        const size_t n = (size_t)L->nx * L->ny * L->nz;
        uint8_t *mark = calloc(n, 1);
        for (int z = 0; z < L->nz; ++z)
            for (int y = 0; y < L->ny; ++y)
                for (int x = 0; x < L->nx; ++x) {
                    if (L->kind[c3(L, x, y, z)] != K_OWN) continue;
                    for (int dz = -2; dz <= 2; ++dz)
                        for (int dy = -2; dy <= 2; ++dy)
                            for (int dx = -2; dx <= 2; ++dx) {
                                int xx = x + dx, yy = y + dy, zz = z + dz;
                                wrap3(L, &xx, &yy, &zz);
                                if (L->kind[c3(L, xx, yy, zz)] == K_NONE) mark[c3(L, xx, yy, zz)] = 1;
                            }
                }
        for (int z = 0; z < L->nz; ++z)
            for (int y = 0; y < L->ny; ++y)
                for (int x = 0; x < L->nx; ++x) {
                    if (!mark[c3(L, x, y, z)]) continue;
                    if (P->kind[c3(P, x / 2, y / 2, z / 2)] != K_OWN) { free(mark); return ORC_ERR_TOPOLOGY; }
                    L->kind[c3(L, x, y, z)] = K_GHOST;
                }
        free(mark);
    }
    for (int l = 0; l < m; ++l) {
        o3lev *L = &s->L[l];
        const size_t n = (size_t)L->nx * L->ny * L->nz;
        int64_t no = 0, ng = 0;
        for (size_t q = 0; q < n; ++q) { no += L->kind[q] == K_OWN; ng += L->kind[q] == K_GHOST; }
        L->own = malloc(sizeof(int64_t) * (no + 1));
        L->ghost = malloc(sizeof(int64_t) * (ng + 1));
        L->act = malloc(sizeof(int64_t) * (no + ng + 1));
        for (size_t q = 0; q < n; ++q) {
            if (L->kind[q] == K_OWN) L->own[L->n_own++] = (int64_t)q;
            if (L->kind[q] == K_GHOST) L->ghost[L->n_ghost++] = (int64_t)q;
            if (L->kind[q] == K_OWN || L->kind[q] == K_GHOST) L->act[L->n_act++] = (int64_t)q;
        }
    }
    return ORC_OK;
}

int orc3f_create(const orc3f_case *c, orc3f_sim **out) {
    *out = NULL;
    if (c->n_levels < 1 || c->n_levels > MAXL || c->nx0 <= 0 || c->ny0 <= 0 || c->nz0 <= 0 || c->block_n <= 0 ||
        c->tau0 <= 0.5 || (c->q != 19 && c->q != 27) || c->n_boxes < 0 || (c->n_boxes > 0 && !c->boxes))
        return ORC_ERR_ARG;
    orc3f_sim *s = calloc(1, sizeof(orc3f_sim));
    s->c = *c;
    s->m = c->n_levels;
    s->q = c->q;
    s->boxes = malloc(sizeof(int32_t) * 7 * (c->n_boxes > 0 ? c->n_boxes : 1));
    if (c->n_boxes > 0) memcpy(s->boxes, c->boxes, sizeof(int32_t) * 7 * c->n_boxes);
    s->c.boxes = s->boxes;
    for (int l = 0; l < s->m; ++l) {
        o3lev *L = &s->L[l];
        L->nx = c->nx0 << l;
        L->ny = c->ny0 << l;
        L->nz = c->nz0 << l;
        L->tau = 0.5 + (double)(1 << l) * (c->tau0 - 0.5);
        for (int k = 0; k < 3; ++k) L->F[k] = c->fext[k] / (double)(1 << l);
        const size_t n = (size_t)L->nx * L->ny * L->nz;
        L->kind = calloc(n, 1);
        L->f = malloc(sizeof(double) * n * s->q);
        L->fs = malloc(sizeof(double) * n * s->q);
        L->rho = malloc(sizeof(double) * n);
        L->u = malloc(sizeof(double) * n * 3);
        if (!L->kind || !L->f || !L->fs || !L->rho || !L->u) { orc3f_destroy(s); return ORC_ERR_ARG; }
        for (size_t q = 0; q < n * s->q; ++q) L->f[q] = L->fs[q] = NAN;
        for (size_t q = 0; q < n; ++q) L->rho[q] = NAN;
        for (size_t q = 0; q < 3 * n; ++q) L->u[q] = NAN;
    }
    int rc = topology3(s);
    if (rc) { orc3f_destroy(s); return rc; }
    if (c->cf_mode == ORC_CF_RESCALE)
        for (int l = 0; l + 1 < s->m; ++l)
            if (fabs(s->L[l].tau - 1.0) < 1e-6) { orc3f_destroy(s); return ORC_ERR_ARG; }
    for (int l = 0; l < s->m; ++l) {      /* rest at rho0 */
        o3lev *L = &s->L[l];
        double feq[27];
        orc3_feq(s->q, c->rho0, 0.0, 0.0, 0.0, feq);
        for (int64_t k = 0; k < L->n_own; ++k) memcpy(L->f + (size_t)L->own[k] * s->q, feq, sizeof(double) * s->q);
    }
    *out = s;
    return ORC_OK;
}

int orc3f_level_size(const orc3f_sim *s, int level, int32_t out[3]) {
    if (level < 0 || level >= s->m) return ORC_ERR_ARG;
    out[0] = s->L[level].nx; out[1] = s->L[level].ny; out[2] = s->L[level].nz;
    return ORC_OK;
}

int orc3f_level_kinds(const orc3f_sim *s, int level, uint8_t *kind) {
    if (level < 0 || level >= s->m) return ORC_ERR_ARG;
    const o3lev *L = &s->L[level];
    memcpy(kind, L->kind, (size_t)L->nx * L->ny * L->nz);
    return ORC_OK;
}

/* f = f^eq(rho, u) on the owned cells of a level (dense [z][y][x] arrays). */
int orc3f_init_fields(orc3f_sim *s, int level, const double *rho, const double *ux, const double *uy,
                      const double *uz) {
    if (level < 0 || level >= s->m) return ORC_ERR_ARG;
    o3lev *L = &s->L[level];
    for (int64_t k = 0; k < L->n_own; ++k) {
        const size_t c = (size_t)L->own[k];
        orc3_feq(s->q, rho[c], ux[c], uy[c], uz[c], L->f + c * s->q);
    }
    return ORC_OK;
}

/* Collision (Eqs. (2)-(8) in 3D, BGK with Guo's term and the half-force
 * velocity) of the owned cells of a level. */
static void collide3f(orc3f_sim *s, int l) {
    o3lev *L = &s->L[l];
    const int Q3 = s->q;
    const double tau = L->tau, pre = 1.0 - 0.5 / tau;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < L->n_own; ++k) {
        const size_t c = (size_t)L->own[k];
        const double *f = L->f + c * Q3;
        const double Fx = L->F[0], Fy = L->F[1], Fz = L->F[2];
        double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < Q3; ++i) { rho += f[i]; jx += C3X[i] * f[i]; jy += C3Y[i] * f[i]; jz += C3Z[i] * f[i]; }
        double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho, uz = (jz + 0.5 * Fz) / rho;
        double feq[27];
        orc3_feq(Q3, rho, ux, uy, uz, feq);
        double uF = ux * Fx + uy * Fy + uz * Fz;
        for (int i = 0; i < Q3; ++i) {
            double cu = C3X[i] * ux + C3Y[i] * uy + C3Z[i] * uz;
            double cF = C3X[i] * Fx + C3Y[i] * Fy + C3Z[i] * Fz;
            double fi = w3(Q3, i) * pre * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF);
            L->fs[c * Q3 + i] = f[i] - (f[i] - feq[i]) / tau + fi;
        }
        L->rho[c] = rho;
        L->u[3 * c] = ux; L->u[3 * c + 1] = uy; L->u[3 * c + 2] = uz;
    }
}

/* Explosion (step (2) of Sec. 2.4): every halo cell of the fine level takes
 * the post-collision populations of its coarse parent (RESCALE: with the
 * non-equilibrium part scaled by s_cf). */
static void explode3f(orc3f_sim *s, int lc, int lf) {
    o3lev *C = &s->L[lc], *F = &s->L[lf];
    const int Q3 = s->q;
    double fac[2];
    orc_interface_factors(C->tau, F->tau, fac);
    const int rescale = s->c.cf_mode == ORC_CF_RESCALE;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < F->n_ghost; ++k) {
        const size_t g = (size_t)F->ghost[k];
        const int x = (int)(g % F->nx), y = (int)((g / F->nx) % F->ny), z = (int)(g / ((size_t)F->nx * F->ny));
        const size_t p = c3(C, x / 2, y / 2, z / 2);
        const double *src = C->fs + p * Q3;
        double *dst = F->fs + g * Q3;
        if (!rescale) {
            for (int i = 0; i < Q3; ++i) dst[i] = src[i];
        } else {
            double feq[27];
            orc3_feq(Q3, C->rho[p], C->u[3 * p], C->u[3 * p + 1], C->u[3 * p + 2], feq);
            for (int i = 0; i < Q3; ++i) dst[i] = feq[i] + fac[0] * (src[i] - feq[i]);
        }
    }
}

/* Streaming, Eq. (10), over owned and halo cells (periodic wrap); a source
 * that is neither owned nor halo leaves NaN. */
static void stream3f(orc3f_sim *s, int l) {
    o3lev *L = &s->L[l];
    const int Q3 = s->q;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < L->n_act; ++k) {
        const size_t c = (size_t)L->act[k];
        const int x = (int)(c % L->nx), y = (int)((c / L->nx) % L->ny), z = (int)(c / ((size_t)L->nx * L->ny));
        for (int i = 0; i < Q3; ++i) {
            int sx = x - C3X[i], sy = y - C3Y[i], sz = z - C3Z[i];
            wrap3(L, &sx, &sy, &sz);
            const size_t p = c3(L, sx, sy, sz);
            L->f[c * Q3 + i] = (L->kind[p] == K_OWN || L->kind[p] == K_GHOST) ? L->fs[p * Q3 + i] : NAN;
        }
    }
}

/* Step (5) of Sec. 2.4: the halo cells' sources of the second fine stream are
 * their own post-stream values of the first. */
static void halo_second3f(orc3f_sim *s, int l) {
    o3lev *L = &s->L[l];
    for (int64_t k = 0; k < L->n_ghost; ++k) {
        const size_t g = (size_t)L->ghost[k];
        memcpy(L->fs + g * s->q, L->f + g * s->q, sizeof(double) * s->q);
    }
}

/* Coalescence (step (6) of Sec. 2.4): an owned coarse cell takes, for each
 * direction whose source is covered by the fine level, the mean of its 8
 * children's post-stream populations (RESCALE: non-equilibrium part scaled by
 * s_fc about the moments of the assembled set). */
static void coalesce3f(orc3f_sim *s, int lf, int lc) {
    o3lev *F = &s->L[lf], *C = &s->L[lc];
    const int Q3 = s->q;
    double fac[2];
    orc_interface_factors(C->tau, F->tau, fac);
    const int rescale = s->c.cf_mode == ORC_CF_RESCALE;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < C->n_own; ++k) {
        const size_t q = (size_t)C->own[k];
        const int x = (int)(q % C->nx), y = (int)((q / C->nx) % C->ny), z = (int)(q / ((size_t)C->nx * C->ny));
        int hid[27], any = 0;
        for (int i = 0; i < Q3; ++i) {
            int sx = x - C3X[i], sy = y - C3Y[i], sz = z - C3Z[i];
            wrap3(C, &sx, &sy, &sz);
            hid[i] = C->kind[c3(C, sx, sy, sz)] == K_HIDDEN;
            any |= hid[i];
        }
        if (!any) continue;
        double avg[27];
        for (int i = 0; i < Q3; ++i) {
            if (!hid[i]) continue;
            double sum = 0.0;
            for (int cz = 0; cz < 2; ++cz)
                for (int cy = 0; cy < 2; ++cy)
                    for (int cx = 0; cx < 2; ++cx)
                        sum += F->f[c3(F, 2 * x + cx, 2 * y + cy, 2 * z + cz) * Q3 + i];
            avg[i] = 0.125 * sum;
        }
        double *dst = C->f + q * Q3;
        if (!rescale) {
            for (int i = 0; i < Q3; ++i) if (hid[i]) dst[i] = avg[i];
        } else {
            double g[27], r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
            for (int i = 0; i < Q3; ++i) g[i] = hid[i] ? avg[i] : dst[i];
            for (int i = 0; i < Q3; ++i) { r += g[i]; jx += C3X[i] * g[i]; jy += C3Y[i] * g[i]; jz += C3Z[i] * g[i]; }
            double feq[27];
            orc3_feq(Q3, r, jx / r, jy / r, jz / r, feq);
            for (int i = 0; i < Q3; ++i)
                if (hid[i]) dst[i] = feq[i] + fac[1] * (avg[i] - feq[i]);
        }
    }
}

/* One coarse step: the same clock over the finest substeps as in 2D (Sec.
 * 2.4-2.5): levels whose substep starts collide, coarse to fine; levels
 * whose substep ends stream, fine to coarse, the fine level's halo prepared
 * by explosion before the first of its two substeps and by its own values
 * before the second, the coarse level coalescing after its stream. */
int orc3f_step(orc3f_sim *s, int32_t n) {
    const int m = s->m;
    const int64_t nsub = (int64_t)1 << (m - 1);
    for (int32_t step = 0; step < n; ++step)
        for (int64_t t = 0; t < nsub; ++t) {
            for (int l = 0; l < m; ++l)
                if (t % (nsub >> l) == 0) collide3f(s, l);
            for (int l = m - 1; l >= 0; --l) {
                const int64_t span = nsub >> l;
                if ((t + 1) % span != 0) continue;
                if (l > 0) {
                    if (((t / span) & 1) == 0) explode3f(s, l - 1, l);
                    else halo_second3f(s, l);
                }
                stream3f(s, l);
                if (l + 1 < m) coalesce3f(s, l + 1, l);
            }
        }
    return ORC_OK;
}

/* rho and u = (sum_i c_i f_i + F/2) / rho on the owned cells of a level, NaN
 * elsewhere (dense [z][y][x]). */
int orc3f_read_fields(const orc3f_sim *s, int level, double *rho, double *ux, double *uy, double *uz) {
    if (level < 0 || level >= s->m) return ORC_ERR_ARG;
    const o3lev *L = &s->L[level];
    const size_t n = (size_t)L->nx * L->ny * L->nz;
    for (size_t c = 0; c < n; ++c) rho[c] = ux[c] = uy[c] = uz[c] = NAN;
    for (int64_t k = 0; k < L->n_own; ++k) {
        const size_t c = (size_t)L->own[k];
        const double *f = L->f + c * s->q;
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < s->q; ++i) { r += f[i]; jx += C3X[i] * f[i]; jy += C3Y[i] * f[i]; jz += C3Z[i] * f[i]; }
        rho[c] = r;
        ux[c] = (jx + 0.5 * L->F[0]) / r;
        uy[c] = (jy + 0.5 * L->F[1]) / r;
        uz[c] = (jz + 0.5 * L->F[2]) / r;
    }
    return ORC_OK;
}

/* out = {mass, momentum x, y, z}: sums over owned cells with volume weight
 * 8^-l; momentum is the bare first moment. */
int orc3f_diagnostics(const orc3f_sim *s, double out[4]) {
    for (int k = 0; k < 4; ++k) out[k] = 0.0;
    for (int l = 0; l < s->m; ++l) {
        const o3lev *L = &s->L[l];
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t k = 0; k < L->n_own; ++k) {
            const double *f = L->f + (size_t)L->own[k] * s->q;
            for (int i = 0; i < s->q; ++i) {
                acc[0] += f[i]; acc[1] += C3X[i] * f[i]; acc[2] += C3Y[i] * f[i]; acc[3] += C3Z[i] * f[i];
            }
        }
        const double wgt = 1.0 / (double)((int64_t)1 << (3 * l));
        for (int k = 0; k < 4; ++k) out[k] += wgt * acc[k];
    }
    return ORC_OK;
}
