// gfx950 kernels of the SBoTFlow LBM-IBM hot path (arXiv 2402.04606).
//
// level_kernel : one refinement level of one substep, fused.  Pull scheme: a
//   lattice holds post-collision populations f*; a launch gathers
//   f(x,i) = f*(x - c_i, i) (streaming, Eq. (10)) including the same-level
//   exchange across block edges, domain-edge rules, halo cells and the
//   fine-to-coarse coalescence, then collides (Eqs. (2)-(8), Guo forcing) and
//   writes f* coalesced; coarse cells next to the finer level also explode
//   their f* into the finer level's halo cells (coarse-to-fine, Sec. 2.4).
//   Halo ("ghost") blocks of the level gather their two halo layers in the
//   first fine substep and are never collided.
// mdf_kernel   : one workgroup per body: kinematics, moments of the stencil
//   cells, the multi-direct-forcing loop (Eqs. (11)-(15)) and the body force
//   (Eq. (16)), all FP64, deterministic (no floating-point atomics).
//
// Layout in HBM: per virtual level a pool of 16x16-cell blocks, SoA
// [block][q][256] in the storage type, two lattices (read / write).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sbt_internal.h"

using namespace sbt;

namespace {

// ---- D2Q9 velocity set (Eq. (1)) and weights (Eq. (7)) -----------------
__device__ constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
__device__ constexpr int MIRX[9] = {0, 3, 2, 1, 4, 6, 5, 8, 7};  // reflect about an x-normal edge
__device__ constexpr int MIRY[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};  // reflect about a y-normal edge

template <typename C>
__device__ __forceinline__ C wgt(int i) {
  return i == 0 ? C(4.0 / 9.0) : (i < 5 ? C(1.0 / 9.0) : C(1.0 / 36.0));
}

// ---- storage types ---------------------------------------------------------
template <int ST> struct Store;
template <> struct Store<0> {  // FP64: f itself, FP64 arithmetic
  using T = double;
  using C = double;
  static constexpr bool kShift = false;
  __device__ static C ld(T v) { return v; }
  __device__ static T st(C v) { return v; }
};
template <> struct Store<1> {  // FP32 deviation
  using T = float;
  using C = float;
  static constexpr bool kShift = true;
  __device__ static C ld(T v) { return v; }
  __device__ static T st(C v) { return v; }
};
template <> struct Store<2> {  // FP16 deviation, round to nearest even
  using T = _Float16;
  using C = float;
  static constexpr bool kShift = true;
  __device__ static C ld(T v) { return (float)v; }
  __device__ static T st(C v) { return (_Float16)v; }
};
template <> struct Store<3> {  // BF16 deviation, round to nearest even
  using T = uint16_t;
  using C = float;
  static constexpr bool kShift = true;
  __device__ static C ld(T v) { return __uint_as_float(((uint32_t)v) << 16); }
  __device__ static T st(C v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (T)((u >> 16) | 0x40);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (T)(u >> 16);
  }
};

// Scalar (wave-uniform) context of one block: the workgroup's block id,
// origin, level, flags and its 8 neighbours and 4 finer children, as named
// scalars (no arrays, so a per-lane choice among them stays a value select
// and never becomes an indexed load from private memory).
struct Blk {
  int self, ox, oy, level, flags, code, cid;
  int nE, nN, nW, nS, nNE, nNW, nSW, nSE;
  int c0, c1, c2, c3;
};

__device__ __forceinline__ Blk load_blk(const BlockMeta *meta, int b) {
  Blk k;
  const BlockMeta &m = meta[b];
  k.self = b;
  k.ox = m.ox;
  k.oy = m.oy;
  k.level = m.level;
  k.flags = m.flags;
  k.code = m.code;
  k.cid = m.case_id;
  k.nE = m.nbr[0]; k.nN = m.nbr[1]; k.nW = m.nbr[2]; k.nS = m.nbr[3];
  k.nNE = m.nbr[4]; k.nNW = m.nbr[5]; k.nSW = m.nbr[6]; k.nSE = m.nbr[7];
  k.c0 = m.child[0]; k.c1 = m.child[1]; k.c2 = m.child[2]; k.c3 = m.child[3];
  return k;
}

// Value select (both operands already loaded; a ?: on two fields would
// select their address instead).
__device__ __forceinline__ int vsel(bool c, int a, int b) { return c ? a : b; }

// Block holding local cell (x, y), x, y in [-1, 16] (-1 if none).
__device__ __forceinline__ int pick_nbr(const Blk &k, int x, int y) {
  int w = vsel(y < 0, k.nSW, vsel(y > 15, k.nNW, k.nW));
  int e = vsel(y < 0, k.nSE, vsel(y > 15, k.nNE, k.nE));
  int c = vsel(y < 0, k.nS, vsel(y > 15, k.nN, k.self));
  return vsel(x < 0, w, vsel(x > 15, e, c));
}

// Same, for a block known only per lane: the neighbour index is read from
// the block table in memory.
__device__ __forceinline__ int pick_nbr_mem(const BlockMeta *meta, int blk, int x, int y) {
  int d;
  if (x < 0) d = y < 0 ? 6 : (y > 15 ? 5 : 2);
  else if (x > 15) d = y < 0 ? 7 : (y > 15 ? 4 : 0);
  else if (y < 0) d = 3;
  else if (y > 15) d = 1;
  else return blk;
  return meta[blk].nbr[d];
}

__device__ __forceinline__ int pick_child(const Blk &k, int x, int y) {
  return vsel(x < 8, vsel(y < 8, k.c0, k.c2), vsel(y < 8, k.c1, k.c3));
}

template <int ST>
__device__ __forceinline__ typename Store<ST>::T ldraw(const void *lat, int blk, int q, int cell) {
  using T = typename Store<ST>::T;
  return static_cast<const T *>(lat)[((size_t)blk * kQ + q) * kCells + cell];
}

template <int ST>
__device__ __forceinline__ typename Store<ST>::C ldv(const void *lat, int blk, int q, int cell) {
  return Store<ST>::ld(ldraw<ST>(lat, blk, q, cell));
}

// Post-collision value of direction q at local cell (x, y) of the block in
// context k (x, y may be one cell outside it).  NaN if no block holds it.
template <int ST>
__device__ __forceinline__ typename Store<ST>::C fetch(const void *lat, const Blk &k, int x, int y, int q) {
  using C = typename Store<ST>::C;
  int nb = pick_nbr(k, x, y);
  if (nb < 0) return C(__builtin_nan(""));
  return ldv<ST>(lat, nb, q, (y & 15) * 16 + (x & 15));
}

template <int ST>
__device__ __forceinline__ typename Store<ST>::C fetch_mem(const void *lat, const BlockMeta *meta, int blk,
                                                         int x, int y, int q) {
  using C = typename Store<ST>::C;
  int nb = pick_nbr_mem(meta, blk, x, y);
  if (nb < 0) return C(__builtin_nan(""));
  return ldv<ST>(lat, nb, q, (y & 15) * 16 + (x & 15));
}

// ---- equilibrium in the storage frame --------------------------------------
// FP64 path: f^eq exactly as Eq. (7) is written.  Deviation paths: f^eq - w rho0.
__device__ __forceinline__ double feq64(int i, double rho, double ux, double uy, double usq) {
#pragma clang fp contract(off)
  double cu = CX[i] * ux + CY[i] * uy;
  return wgt<double>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
}
__device__ __forceinline__ float feqdev(int i, float drho, float rho, float ux, float uy, float usq) {
  float cu = CX[i] * ux + CY[i] * uy;
  return wgt<float>(i) * (drho + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * usq));
}

// Moments in FP64 exactly in the order the paper's sums are written
// (i = 0..8), so FP64 results are reproducible bit for bit.
__device__ __forceinline__ void moments64(const double f[9], double &rho, double &jx, double &jy) {
#pragma clang fp contract(off)
  rho = 0.0;
  jx = 0.0;
  jy = 0.0;
  for (int i = 0; i < 9; ++i) {
    rho += f[i];
    jx += CX[i] * f[i];
    jy += CY[i] * f[i];
  }
}

// ---- collision (Eqs. (3), (6)-(8)) -----------------------------------------
template <int ST>
struct Collide;

template <>
struct Collide<0> {
  __device__ __forceinline__ static void run(const CaseDev &cp, int l, double f[9], double Fx, double Fy, double &rho,
                             double &ux, double &uy) {
#pragma clang fp contract(off)
    double jx, jy;
    moments64(f, rho, jx, jy);
    ux = (jx + 0.5 * Fx) / rho;
    uy = (jy + 0.5 * Fy) / rho;
    double usq = ux * ux + uy * uy;
    double tau = cp.tau[l];
    bool forced = (Fx != 0.0) || (Fy != 0.0);
    double uF = ux * Fx + uy * Fy;
    double pre = cp.pre[l];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      double fe = feq64(i, rho, ux, uy, usq);
      double v = f[i] - (f[i] - fe) / tau;
      if (forced) {
        double cu = CX[i] * ux + CY[i] * uy;
        double cF = CX[i] * Fx + CY[i] * Fy;
        v = v + wgt<double>(i) * pre * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF);
      }
      f[i] = v;
    }
  }
};

template <int ST>
struct Collide {
  // deviation form: f = w rho0 + d;  rho = rho0 + sum d;  sum c f = sum c d
  __device__ __forceinline__ static void run(const CaseDev &cp, int l, float d[9], float Fx, float Fy, float &rho,
                             float &ux, float &uy) {
    float drho = 0.f, jx = 0.f, jy = 0.f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      drho += d[i];
      jx += CX[i] * d[i];
      jy += CY[i] * d[i];
    }
    rho = (float)cp.rho0 + drho;
    float ir = 1.0f / rho;
    ux = (jx + 0.5f * Fx) * ir;
    uy = (jy + 0.5f * Fy) * ir;
    float usq = ux * ux + uy * uy;
    float om = cp.omega_f[l];
    float pre = cp.pre_f[l];
    float uF = ux * Fx + uy * Fy;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      float cu = CX[i] * ux + CY[i] * uy;
      float cF = CX[i] * Fx + CY[i] * Fy;
      float fe = feqdev(i, drho, rho, ux, uy, usq);
      d[i] = d[i] + om * (fe - d[i]) + wgt<float>(i) * pre * (3.f * cF + 9.f * cu * cF - 3.f * uF);
    }
  }
};

// Equilibrium in the storage frame for the interface / boundary operators.
template <int ST>
__device__ __forceinline__ typename Store<ST>::C feq_frame(const CaseDev &cp, int i,
                                                          typename Store<ST>::C rho,
                                                          typename Store<ST>::C ux,
                                                          typename Store<ST>::C uy) {
  using C = typename Store<ST>::C;
  if constexpr (!Store<ST>::kShift) {
    return feq64(i, rho, ux, uy, ux * ux + uy * uy);
  } else {
    C r0 = (C)cp.rho0;
    return feqdev(i, rho - r0, rho, ux, uy, ux * ux + uy * uy);
  }
}

// Moments of a set of populations held in the storage frame.
template <int ST>
__device__ __forceinline__ void frame_moments(const CaseDev &cp, const typename Store<ST>::C f[9],
                                              typename Store<ST>::C &rho, typename Store<ST>::C &jx,
                                              typename Store<ST>::C &jy) {
  if constexpr (!Store<ST>::kShift) {
    moments64(f, rho, jx, jy);
  } else {
    float dr = 0.f, a = 0.f, b = 0.f;
    for (int i = 0; i < 9; ++i) {
      dr += f[i];
      a += CX[i] * f[i];
      b += CY[i] * f[i];
    }
    rho = (float)cp.rho0 + dr;
    jx = a;
    jy = b;
  }
}

// ---- domain-edge rules -----------------------------------------------------
// Unknown population q of cell (x, y) (local coordinates of block `self`,
// level-0 global cell (gx, gy)); its source lies beyond a non-periodic edge.
template <int ST>
__device__ __forceinline__ typename Store<ST>::C edge_value(const CaseDev &cp, const void *src, const Blk &k, int x, int y,
                                            int gx, int gy, int q) {
#pragma clang fp contract(off)
  using C = typename Store<ST>::C;
  const int nx = cp.nx[0], ny = cp.ny[0];
  int sx = gx - CX[q], sy = gy - CY[q];
  bool outx = (sx < 0 || sx >= nx) && !cp.per_x;
  bool outy = (sy < 0 || sy >= ny) && !cp.per_y;
  int ex = sx < 0 ? 0 : 1, ey = sy < 0 ? 2 : 3;
  int e = outx ? ex : ey;
  if (outx && outy) {
    int kx = cp.bc[ex], ky = cp.bc[ey];
    bool lx = kx == 1 || kx == 2, ly = ky == 1 || ky == 2;
    if (!lx && ly) e = ey;
  }
  const double uwx = cp.bcu[e][0], uwy = cp.bcu[e][1];
  switch (cp.bc[e]) {
    case 1: {  // wall: half-way bounce-back with moving-wall term
      C fs = ldv<ST>(src, k.self, OPP[q], y * 16 + x);
      if constexpr (!Store<ST>::kShift) {
        return fs + 6.0 * wgt<double>(q) * cp.rho0 * (CX[q] * uwx + CY[q] * uwy);
      } else {
        return fs + (float)(6.0 * wgt<double>(q) * cp.rho0 * (CX[q] * uwx + CY[q] * uwy));
      }
    }
    case 2: {  // equilibrium inflow at (rho0, u_in)
      if constexpr (!Store<ST>::kShift) {
        return feq64(q, cp.rho0, uwx, uwy, uwx * uwx + uwy * uwy);
      } else {
        double cu = CX[q] * uwx + CY[q] * uwy;
        return (float)(wgt<double>(q) * cp.rho0 *
                       (3.0 * cu + 4.5 * cu * cu - 1.5 * (uwx * uwx + uwy * uwy)));
      }
    }
    case 3:    // zero-gradient outflow: the value that streams into the interior neighbour
    case 4: {  // specular symmetry: mirrored population from the tangential neighbour
      const int nrx = e == 0 ? -1 : (e == 1 ? 1 : 0), nry = e == 2 ? -1 : (e == 3 ? 1 : 0);
      const bool xn = (e == 0 || e == 1);
      int px, py, qq = q;
      if (cp.bc[e] == 3) {
        px = gx - nrx - CX[q];
        py = gy - nry - CY[q];
      } else {
        px = gx - (xn ? 0 : CX[q]);
        py = gy - (xn ? CY[q] : 0);
        qq = xn ? MIRX[q] : MIRY[q];
      }
      // periodic axes wrap through the neighbour table; others clamp (corners)
      if (!cp.per_x) px = px < 0 ? 0 : (px >= nx ? nx - 1 : px);
      if (!cp.per_y) py = py < 0 ? 0 : (py >= ny ? ny - 1 : py);
      return fetch<ST>(src, k, x + (px - gx), y + (py - gy), qq);
    }
    default:
      return C(__builtin_nan(""));
  }
}

// ---- fine-to-coarse coalescence (step (6) of Sec. 2.4), on read ------------
// Mean over the 4 children g of coarse cell (x, y) of the finer level's
// post-stream value f(g, q) = f*(g - c_q, q), read from the finer lattice its
// last substep streamed from.
template <int ST>
__device__ __forceinline__ typename Store<ST>::C coalesce(const LevelArgs &a, const Blk &k, int x, int y, int q) {
#pragma clang fp contract(off)
  using C = typename Store<ST>::C;
  int cb = pick_child(k, x, y);
  if (cb < 0) return C(__builtin_nan(""));
  int fx0 = (2 * x) & 15, fy0 = (2 * y) & 15;
  C v00 = fetch_mem<ST>(a.fprev, a.fmeta, cb, fx0 - CX[q], fy0 - CY[q], q);
  C v10 = fetch_mem<ST>(a.fprev, a.fmeta, cb, fx0 + 1 - CX[q], fy0 - CY[q], q);
  C v01 = fetch_mem<ST>(a.fprev, a.fmeta, cb, fx0 - CX[q], fy0 + 1 - CY[q], q);
  C v11 = fetch_mem<ST>(a.fprev, a.fmeta, cb, fx0 + 1 - CX[q], fy0 + 1 - CY[q], q);
  C sum = v00;
  sum += v10;
  sum += v01;
  sum += v11;
  return C(0.25) * sum;
}

// ---- one cell of a level launch --------------------------------------------
template <int ST>
__device__ __forceinline__ void level_cell(const LevelArgs &a, const Blk &k, int cell, const CaseDev &cp,
                                           bool slow, double *part) {
#pragma clang fp contract(off)
  using S = Store<ST>;
  using T = typename S::T;
  using C = typename S::C;
  const int x = cell & 15, y = cell >> 4;
  const int l = k.level;
  const int b = k.self;
  uint16_t code = (k.flags & BF_CODES) ? a.codes[(size_t)k.code * kCells + cell] : (uint16_t)0;

  if (k.flags & BF_GHOST) {  // halo layers: streamed, never collided
    if (!(code & CC_BAND)) return;
    T g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      int sx = x - CX[i], sy = y - CY[i];
      int nb = pick_nbr(k, sx, sy);
      g[i] = nb < 0 ? S::st(C(__builtin_nan(""))) : ldraw<ST>(a.src, nb, i, (sy & 15) * 16 + (sx & 15));
    }
    T *dst = static_cast<T *>(a.dst);
#pragma unroll
    for (int i = 0; i < 9; ++i) dst[((size_t)b * kQ + i) * kCells + cell] = g[i];
    return;
  }

  const size_t ob = (size_t)(b - a.b0);
  if (code & CC_HIDDEN) {
    if (a.mode & MODE_READOUT) {
#pragma unroll
      for (int q = 0; q < 3; ++q) a.out[(ob * 3 + q) * kCells + cell] = __builtin_nan("");
    }
    return;
  }

  C f[9];
  if (a.mode & MODE_LOCAL) {
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = ldv<ST>(a.src, b, i, cell);
  } else if (!slow) {
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = fetch<ST>(a.src, k, x - CX[i], y - CY[i], i);
  } else {
    const int gx = k.ox + x, gy = k.oy + y;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      int sx = x - CX[i], sy = y - CY[i];
      int nb = pick_nbr(k, sx, sy);
      if (code & (1u << i)) {
        f[i] = coalesce<ST>(a, k, x, y, i);
      } else if (nb < 0) {
        f[i] = edge_value<ST>(cp, a.src, k, x, y, gx, gy, i);
      } else {
        f[i] = ldv<ST>(a.src, nb, i, (sy & 15) * 16 + (sx & 15));
      }
    }
    if ((code & CC_HSRC) && cp.cf_mode == 1) {  // RESCALE the coalesced populations
      C r, jx, jy;
      frame_moments<ST>(cp, f, r, jx, jy);
      C ux = jx / r, uy = jy / r;
      C s;
      if constexpr (!Store<ST>::kShift) s = cp.s_fc[l];
      else s = cp.s_fc_f[l];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        C fe = feq_frame<ST>(cp, i, r, ux, uy);
        C v = fe + s * (f[i] - fe);
        f[i] = (code & (1u << i)) ? v : f[i];
      }
    }
  }

  if (a.mode & MODE_READOUT) {  // moments of the post-stream populations, FP64
    double fd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) fd[i] = (double)f[i];
    double rho, jx, jy;
    moments64(fd, rho, jx, jy);
    if constexpr (Store<ST>::kShift) rho = cp.rho0 + rho;
    double ux = (jx + 0.5 * cp.fx[l]) / rho, uy = (jy + 0.5 * cp.fy[l]) / rho;
    a.out[(ob * 3 + 0) * kCells + cell] = rho;
    a.out[(ob * 3 + 1) * kCells + cell] = ux;
    a.out[(ob * 3 + 2) * kCells + cell] = uy;
    part[0] = rho;
    part[1] = jx;
    part[2] = jy;
    return;
  }

  // Force density: uniform body force (+ IBM force on the finest level).
  C Fx, Fy;
  if constexpr (!Store<ST>::kShift) {
    Fx = cp.fx[l];
    Fy = cp.fy[l];
  } else {
    Fx = cp.fx_f[l];
    Fy = cp.fy_f[l];
  }
  if (k.flags & BF_IBM) {
    const IbmWindow w = *cp.win;
    int wx = k.ox + x - w.x0, wy = k.oy + y - w.y0;
    if (wx >= 0 && wx < w.w && wy >= 0 && wy < w.h) {
      size_t wi = (size_t)wy * w.w + wx;
      Fx = Fx + (C)cp.wF[wi];
      Fy = Fy + (C)cp.wF[(size_t)cp.win_cap + wi];
    }
  }

  C rho, ux, uy;
  Collide<ST>::run(cp, l, f, Fx, Fy, rho, ux, uy);
  if (!(rho == rho) || rho > C(1e30) || rho < C(-1e30)) atomicOr(a.err, ERR_NONFINITE);

  T *dst = static_cast<T *>(a.dst);
#pragma unroll
  for (int i = 0; i < 9; ++i) dst[((size_t)b * kQ + i) * kCells + cell] = S::st(f[i]);

  if (code & CC_IFACE) {  // coarse-to-fine: explode f* into the 4 halo children
    int cb = pick_child(k, x, y);
    if (cb >= 0) {
      C s = 1;
      if constexpr (!Store<ST>::kShift) s = cp.s_cf[l + 1];
      else s = cp.s_cf_f[l + 1];
      const bool resc = cp.cf_mode == 1;
      T *fd = static_cast<T *>(a.fcur);
      int fx0 = (2 * x) & 15, fy0 = (2 * y) & 15;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        C e = f[i];
        if (resc) {
          C fe = feq_frame<ST>(cp, i, rho, ux, uy);
          e = fe + s * (f[i] - fe);
        }
        T v = S::st(e);
        size_t base = ((size_t)cb * kQ + i) * kCells;
        fd[base + fy0 * 16 + fx0] = v;
        fd[base + fy0 * 16 + fx0 + 1] = v;
        fd[base + (fy0 + 1) * 16 + fx0] = v;
        fd[base + (fy0 + 1) * 16 + fx0 + 1] = v;
      }
    }
  }
}

__device__ __forceinline__ int remap_block(int bid, int nblk, int enable) {
  if (!enable) return bid;
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous run of (Morton-ordered) blocks so halo reads hit its own L2.
  int xcd = bid & 7, k = bid >> 3;
  int q = nblk >> 3, r = nblk & 7;
  int start = xcd * q + (xcd < r ? xcd : r);
  return start + k;
}

// Halo-band cell of a halo block: streamed in the first fine substep, never
// collided.
template <int ST>
__device__ __forceinline__ void band_cell(const LevelArgs &a, int packed) {
  using S = Store<ST>;
  using T = typename S::T;
  using C = typename S::C;
  const int b = packed >> 8, cell = packed & 255;
  const int x = cell & 15, y = cell >> 4;
  const Blk k = load_blk(a.meta, b);
  T g[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int sx = x - CX[i], sy = y - CY[i];
    int nb = pick_nbr(k, sx, sy);
    g[i] = nb < 0 ? S::st(C(__builtin_nan(""))) : ldraw<ST>(a.src, nb, i, (sy & 15) * 16 + (sx & 15));
  }
  T *dst = static_cast<T *>(a.dst);
#pragma unroll
  for (int i = 0; i < 9; ++i) dst[((size_t)b * kQ + i) * kCells + cell] = g[i];
}

template <int ST, int CPT>
__global__ __launch_bounds__(256 / CPT) void level_kernel(LevelArgs a) {
  constexpr int NT = 256 / CPT;
  const int w = remap_block(blockIdx.x, gridDim.x, a.xcd_remap);
  if (w >= a.n_blocks) {  // packed halo-band cells
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      int idx = (w - a.n_blocks) * 256 + c * NT + threadIdx.x;
      if (idx < a.n_band) band_cell<ST>(a, a.band[idx]);
    }
    return;
  }
  const int b = a.list ? a.list[w] : a.b0 + w;
  const int bl = b - a.b0;
  const Blk k = load_blk(a.meta, b);
  const CaseDev &cp = a.cases[k.cid];
  const bool slow = (k.flags & (BF_CODES | BF_EDGE)) != 0;
  double part[3] = {0.0, 0.0, 0.0};
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    int cell = threadIdx.x + c * NT;
    level_cell<ST>(a, k, cell, cp, slow, part);
    if (a.mode & MODE_READOUT) {
      // fixed-order per-thread partials (hidden cells contribute nothing)
      acc[0] += part[0];
      acc[1] += part[1];
      acc[2] += part[2];
      part[0] = part[1] = part[2] = 0.0;
    }
  }
  if (a.mode & MODE_READOUT) {
    __shared__ double red[3][NT];
#pragma unroll
    for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
#pragma unroll
        for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < 3; ++q) a.partial[(size_t)bl * 3 + q] = red[q][0];
    }
  }
}

// ---- interior blocks: LDS-staged stream + collide ---------------------------
// The block's 9 planes are read with 16-byte vector loads into an LDS tile
// that also holds the one-cell halo each direction needs (188 values from
// the 8 neighbours); every lane then gathers its 9 incoming populations at
// fixed offsets, collides and stores.
template <int ST>
struct Tile {
  using T = typename Store<ST>::T;
  static constexpr int V = 16 / (int)sizeof(T);  // elements per 16-byte vector
  static constexpr int OFF = V;                  // column of x = 0 in a tile row
  static constexpr int RS = 16 + 2 * V;          // row stride
  static constexpr int PS = 18 * RS;             // plane stride
};

template <int ST, bool SLOW>
__device__ __forceinline__ void tile_block(const LevelArgs &a, int b, typename Store<ST>::T *tile) {
#pragma clang fp contract(off)
  using S = Store<ST>;
  using T = typename S::T;
  using C = typename S::C;
  using TL = Tile<ST>;
  const Blk k = load_blk(a.meta, b);
  const CaseDev &cp = a.cases[k.cid];
  const int tid = threadIdx.x;
  const T *src = static_cast<const T *>(a.src);

  // interior of the 9 planes
  constexpr int VPP = 256 / TL::V;      // vectors per plane
  for (int v = tid; v < 9 * VPP; v += 256) {
    int plane = v / VPP, e = (v % VPP) * TL::V;
    int y = e >> 4, x = e & 15;
    uint4 val = *reinterpret_cast<const uint4 *>(src + ((size_t)b * kQ + plane) * kCells + e);
    *reinterpret_cast<uint4 *>(&tile[plane * TL::PS + (y + 1) * TL::RS + TL::OFF + x]) = val;
  }
  // halo: 16 cells for each axis direction, 31 for each diagonal
  if (tid < 188) {
    int plane, hx, hy;
    if (tid < 64) {
      int s = tid & 15;
      plane = 1 + (tid >> 4);
      hx = plane == 1 ? -1 : (plane == 3 ? 16 : s);
      hy = plane == 2 ? -1 : (plane == 4 ? 16 : s);
    } else {
      int d = (tid - 64) / 31, s = (tid - 64) % 31;
      plane = 5 + d;
      bool col = s < 16;
      if (plane == 5) { hx = col ? -1 : s - 16; hy = col ? s - 1 : -1; }
      else if (plane == 6) { hx = col ? 16 : s - 15; hy = col ? s - 1 : -1; }
      else if (plane == 7) { hx = col ? 16 : s - 15; hy = col ? s + 1 : 16; }
      else { hx = col ? -1 : s - 16; hy = col ? s + 1 : 16; }
    }
    int nb = pick_nbr(k, hx, hy);
    T v = nb < 0 ? S::st(C(__builtin_nan(""))) : src[((size_t)nb * kQ + plane) * kCells + (hy & 15) * 16 + (hx & 15)];
    tile[plane * TL::PS + (hy + 1) * TL::RS + TL::OFF + hx] = v;
  }
  __syncthreads();

  const int x = tid & 15, y = tid >> 4;
  const int l = k.level;
  uint16_t code = 0;
  if (SLOW) {
    code = (k.flags & BF_CODES) ? a.codes[(size_t)k.code * kCells + tid] : (uint16_t)0;
    if (code & CC_HIDDEN) return;  // covered by the finer level
  }
  C f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i)
    f[i] = S::ld(tile[i * TL::PS + (y - CY[i] + 1) * TL::RS + TL::OFF + x - CX[i]]);
  if (SLOW) {
    const int gx = k.ox + x, gy = k.oy + y;
    const bool edge = (k.flags & BF_EDGE) != 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      if (code & (1u << i)) {
        f[i] = coalesce<ST>(a, k, x, y, i);
      } else if (edge) {
        int sx = gx - CX[i], sy = gy - CY[i];
        bool out = (!cp.per_x && (sx < 0 || sx >= cp.nx[0])) || (!cp.per_y && (sy < 0 || sy >= cp.ny[0]));
        if (out) f[i] = edge_value<ST>(cp, a.src, k, x, y, gx, gy, i);
      }
    }
    if ((code & CC_HSRC) && cp.cf_mode == 1) {  // RESCALE the coalesced populations
      C r, jx, jy;
      frame_moments<ST>(cp, f, r, jx, jy);
      C ux = jx / r, uy = jy / r;
      C sf;
      if constexpr (!S::kShift) sf = cp.s_fc[l];
      else sf = cp.s_fc_f[l];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        C fe = feq_frame<ST>(cp, i, r, ux, uy);
        C v = fe + sf * (f[i] - fe);
        f[i] = (code & (1u << i)) ? v : f[i];
      }
    }
  }

  C Fx, Fy;
  if constexpr (!S::kShift) {
    Fx = cp.fx[l];
    Fy = cp.fy[l];
  } else {
    Fx = cp.fx_f[l];
    Fy = cp.fy_f[l];
  }
  if (k.flags & BF_IBM) {
    const IbmWindow win = *cp.win;
    int wx = k.ox + x - win.x0, wy = k.oy + y - win.y0;
    if (wx >= 0 && wx < win.w && wy >= 0 && wy < win.h) {
      size_t wi = (size_t)wy * win.w + wx;
      Fx = Fx + (C)cp.wF[wi];
      Fy = Fy + (C)cp.wF[(size_t)cp.win_cap + wi];
    }
  }
  C rho, ux, uy;
  Collide<ST>::run(cp, l, f, Fx, Fy, rho, ux, uy);
  if (!(rho == rho) || rho > C(1e30) || rho < C(-1e30)) atomicOr(a.err, ERR_NONFINITE);
  T *dst = static_cast<T *>(a.dst);
#pragma unroll
  for (int i = 0; i < 9; ++i) dst[((size_t)b * kQ + i) * kCells + tid] = S::st(f[i]);
  if (SLOW && (code & CC_IFACE)) {  // coarse-to-fine: explode f* into the 4 halo children
    int cb = pick_child(k, x, y);
    if (cb >= 0) {
      C sc;
      if constexpr (!S::kShift) sc = cp.s_cf[l + 1];
      else sc = cp.s_cf_f[l + 1];
      const bool resc = cp.cf_mode == 1;
      T *fd = static_cast<T *>(a.fcur);
      int fx0 = (2 * x) & 15, fy0 = (2 * y) & 15;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        C e = f[i];
        if (resc) {
          C fe = feq_frame<ST>(cp, i, rho, ux, uy);
          e = fe + sc * (f[i] - fe);
        }
        T v = S::st(e);
        size_t base = ((size_t)cb * kQ + i) * kCells;
        fd[base + fy0 * 16 + fx0] = v;
        fd[base + fy0 * 16 + fx0 + 1] = v;
        fd[base + (fy0 + 1) * 16 + fx0] = v;
        fd[base + (fy0 + 1) * 16 + fx0 + 1] = v;
      }
    }
  }
}

// One launch per level substep: the first n_fast list entries are interior
// blocks, the rest of the list are blocks next to a finer level or a domain
// edge, and workgroups past the list gather packed halo-band cells.
template <int ST>
__global__ __launch_bounds__(256) void level_tile_kernel(LevelArgs a) {
  using T = typename Store<ST>::T;
  __shared__ __attribute__((aligned(16))) T tile[9 * Tile<ST>::PS];
  const int w = remap_block(blockIdx.x, gridDim.x, a.xcd_remap);
  if (w < a.n_fast) {
    tile_block<ST, false>(a, a.list[w], tile);
  } else if (w < a.n_blocks) {
    tile_block<ST, true>(a, a.list[w], tile);
  } else {
    int idx = (w - a.n_blocks) * 256 + threadIdx.x;
    if (idx < a.n_band) band_cell<ST>(a, a.band[idx]);
  }
}

// ---- IBM: multi-direct forcing, one workgroup per body --------------------
constexpr int MDF_THREADS = kMaxMarkers;

__device__ __forceinline__ double peskin(double r) {
#pragma clang fp contract(off)
  double a = fabs(r);
  if (a <= 1.0) return 0.125 * (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a));
  if (a <= 2.0) return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
  return 0.0;
}

__device__ __forceinline__ int tap0(double X) { return (int)floor(X - 1.5); }

// Rigid motion of the body at finest substep k: centre and the rotation by
// alpha (FIXED bodies: identity rotation about (p0, p1)).
struct Pose {
  double xc, yc, ca, sa;
};

__device__ Pose body_pose(const CaseDev &cp, double k) {
#pragma clang fp contract(off)
  const double *p = cp.bp;
  Pose r;
  if (cp.body_kind == 0) {
    r.xc = p[0];
    r.yc = p[1];
    r.ca = 1.0;
    r.sa = 0.0;
    return r;
  }
  double tstar = k * p[8] / p[9];
  double theta = 2.0 * M_PI * tstar / p[6];
  double alpha = p[2] - p[3] * sin(theta + p[7]);
  double h = 0.5 * p[4] * cos(theta);
  r.xc = p[0] + h * cos(p[5]);
  r.yc = p[1] + h * sin(p[5]);
  r.ca = cos(alpha);
  r.sa = sin(alpha);
  return r;
}

__device__ __forceinline__ void marker_position(const CaseDev &cp, const Pose &q, int j, double &X, double &Y) {
#pragma clang fp contract(off)
  if (cp.body_kind == 0) {
    X = q.xc + cp.xb[j];
    Y = q.yc + cp.yb[j];
    return;
  }
  X = q.xc + cp.xb[j] * q.ca + cp.yb[j] * q.sa;
  Y = q.yc - cp.xb[j] * q.sa + cp.yb[j] * q.ca;
}

// Owned finest-level block of the case holding cell (gx, gy), -1 if none.
__device__ __forceinline__ int finest_block(const CaseDev &cp, int gx, int gy) {
  const int l = cp.n_levels - 1;
  if (gx < 0 || gy < 0 || gx >= cp.nx[l] || gy >= cp.ny[l]) return -1;
  int rx = (gx >> 4) - cp.bm_x0, ry = (gy >> 4) - cp.bm_y0;
  if (rx < 0 || ry < 0 || rx >= cp.bm_w || ry >= cp.bm_h) return -1;
  return cp.bmap[(size_t)ry * cp.bm_w + rx];
}

// A stencil cell and its 8 streaming sources must be owned finest cells; the
// 3x3 neighbourhood spans at most 2x2 blocks, all found at its corners.
__device__ __forceinline__ bool stencil_ok(const CaseDev &cp, int gx, int gy) {
  return finest_block(cp, gx - 1, gy - 1) >= 0 && finest_block(cp, gx + 1, gy - 1) >= 0 &&
         finest_block(cp, gx - 1, gy + 1) >= 0 && finest_block(cp, gx + 1, gy + 1) >= 0;
}

// rho and the uncorrected velocity of finest cell (gx, gy) from its
// post-stream populations (the initial state is read in place).
template <int ST>
__device__ __forceinline__ void cell_moments(const MdfArgs &a, const CaseDev &cp, int gx, int gy, double &rho,
                                             double &ux, double &uy) {
#pragma clang fp contract(off)
  double f[9];
  if (a.first) {
    int b = finest_block(cp, gx, gy);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = (double)ldv<ST>(a.src, b, i, (gy & 15) * 16 + (gx & 15));
  } else {
    int nb[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) nb[i] = finest_block(cp, gx - CX[i], gy - CY[i]);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      int sx = gx - CX[i], sy = gy - CY[i];
      f[i] = (double)ldv<ST>(a.src, nb[i], i, (sy & 15) * 16 + (sx & 15));
    }
  }
  double jx, jy;
  moments64(f, rho, jx, jy);
  if constexpr (Store<ST>::kShift) rho = cp.rho0 + rho;
  int l = cp.n_levels - 1;
  ux = (jx + 0.5 * cp.fx[l]) / rho;
  uy = (jy + 0.5 * cp.fy[l]) / rho;
}

// Ascending sort of up to N marker indices held in registers (bitonic
// network; every index is a compile-time constant, so nothing spills).
template <int N>
__device__ __forceinline__ void sort_net(int (&v)[N]) {
#pragma unroll
  for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        int j = i ^ stride;
        if (j > i) {
          bool up = (i & size) == 0;
          int lo = min(v[i], v[j]), hi = max(v[i], v[j]);
          v[i] = up ? lo : hi;
          v[j] = up ? hi : lo;
        }
      }
    }
  }
}

template <int N>
__device__ __forceinline__ void sorted_copy(const int32_t *L, int cnt, int32_t *out) {
  int v[N];
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] = r < cnt ? L[r] : 0x7fffffff;
  sort_net<N>(v);
#pragma unroll
  for (int r = 0; r < N; ++r)
    if (r < cnt) out[r] = v[r];
}

__device__ __forceinline__ void mdf_fail(const CaseDev &cp, int *err, int code, int64_t k) {
  atomicOr(err, code);
  IbmWindow e = {0, 0, 0, 0};
  *cp.win = e;
  *cp.kcount = k + 1;
}

template <int ST>
__global__ __launch_bounds__(MDF_THREADS) void mdf_kernel(MdfArgs a) {
#pragma clang fp contract(off)
  const int ci = a.body_cases[blockIdx.x];
  const CaseDev &cp = a.cases[ci];
  const int n = cp.n_markers;
  const int tid = threadIdx.x, lane = tid & 63;
  const int NM = a.max_markers;
  // LDS marker tables: Peskin weights of the 4 x and 4 y taps, current force,
  // arc length, first tap, and the compact stencil-cell index of each tap.
  extern __shared__ double lds[];
  double *s_wx = lds;               // [4][NM]
  double *s_wy = s_wx + 4 * NM;     // [4][NM]
  double *s_dFx = s_wy + 4 * NM;    // [NM]
  double *s_dFy = s_dFx + NM;
  double *s_ds = s_dFy + NM;
  int *s_i0 = (int *)(s_ds + NM);   // [NM]
  int *s_j0 = s_i0 + NM;
  int *s_tap = s_j0 + NM;           // [16][NM]
  int *s_cnt = s_tap + 16 * NM;     // [lds_window] window counters
  __shared__ int s_box[4];
  __shared__ int s_bad;
  __shared__ Pose s_pose[2];
  const int64_t k = *cp.kcount;

  // 1. kinematics: r_j(t_k), desired velocity (r_j(t_k+1) - r_j(t_k)) / dt,
  //    and the Peskin weights of the marker's 4x4 stencil (Eqs. (13), (14))
  if (tid == 0) {
    s_box[0] = 1 << 30; s_box[1] = 1 << 30; s_box[2] = -(1 << 30); s_box[3] = -(1 << 30);
    s_bad = 0;
    s_pose[0] = body_pose(cp, (double)k);
  } else if (tid == 64) {
    s_pose[1] = body_pose(cp, (double)(k + 1));
  }
  __syncthreads();
  double udx = 0.0, udy = 0.0, ftx = 0.0, fty = 0.0;
  const bool own = tid < n;
  int bx0 = 1 << 30, by0 = 1 << 30, bx1 = -(1 << 30), by1 = -(1 << 30);
  if (own) {
    double X, Y, X1, Y1;
    marker_position(cp, s_pose[0], tid, X, Y);
    marker_position(cp, s_pose[1], tid, X1, Y1);
    udx = X1 - X;
    udy = Y1 - Y;
    int i0 = tap0(X), j0 = tap0(Y);
    s_i0[tid] = i0;
    s_j0[tid] = j0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      s_wx[t * NM + tid] = peskin(i0 + t + 0.5 - X);
      s_wy[t * NM + tid] = peskin(j0 + t + 0.5 - Y);
    }
    s_ds[tid] = cp.ds[tid];
    bx0 = i0; by0 = j0; bx1 = i0 + 4; by1 = j0 + 4;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    bx0 = min(bx0, __shfl_xor(bx0, o, 64));
    by0 = min(by0, __shfl_xor(by0, o, 64));
    bx1 = max(bx1, __shfl_xor(bx1, o, 64));
    by1 = max(by1, __shfl_xor(by1, o, 64));
  }
  if (lane == 0) {
    atomicMin(&s_box[0], bx0);
    atomicMin(&s_box[1], by0);
    atomicMax(&s_box[2], bx1);
    atomicMax(&s_box[3], by1);
  }
  __syncthreads();
  const int wx0 = s_box[0], wy0 = s_box[1];
  const int ww = s_box[2] - wx0, wh = s_box[3] - wy0;
  const int ncell = ww * wh;
  if (ncell > cp.win_cap || ww <= 0 || wh <= 0) {
    if (tid == 0) mdf_fail(cp, a.err, ERR_WINDOW, k);
    return;
  }
  if (tid == 0) {
    IbmWindow w = {wx0, wy0, ww, wh};
    *cp.win = w;
    *cp.sCount = 0;
  }
  // 2. clear the window (counts and force; the level kernel reads the force
  //    over the whole window).  Counters live in LDS when the window fits.
  const bool lds_cnt = ncell <= a.lds_window;
  int *wcnt = lds_cnt ? s_cnt : cp.wCnt;
  for (int c = tid; c < ncell; c += MDF_THREADS) {
    wcnt[c] = 0;
    cp.wF[c] = 0.0;
    cp.wF[(size_t)cp.win_cap + c] = 0.0;
  }
  __syncthreads();
  // 3. each marker lane registers its 16 taps at once: contributor lists of
  //    the cells, and a compact list of the distinct stencil cells (the first
  //    toucher of a cell appends it; a wavefront prefix sum sizes the append)
  {
    int cidx[16], pos[16];
    int nf = 0;
    if (own) {
      const int i0 = s_i0[tid], j0 = s_j0[tid];
#pragma unroll
      for (int t = 0; t < 16; ++t) cidx[t] = (j0 + (t >> 2) - wy0) * ww + (i0 + (t & 3) - wx0);
#pragma unroll
      for (int t = 0; t < 16; ++t) pos[t] = atomicAdd(&wcnt[cidx[t]], 1);
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        if (pos[t] < kMaxContrib) cp.wList[(size_t)cidx[t] * kMaxContrib + pos[t]] = tid;
        else s_bad = 2;
        nf += pos[t] == 0;
      }
    }
    int incl = nf;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    const int total = __shfl(incl, 63, 64);
    int base = 0;
    if (lane == 63 && total > 0) base = atomicAdd(cp.sCount, total);
    base = __shfl(base, 63, 64);
    if (own) {
      int q = base + incl - nf;
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (pos[t] == 0) {
          cp.sCells[q] = cidx[t];
          cp.wIdx[cidx[t]] = q;
          ++q;
        }
    }
  }
  __syncthreads();
  const int ns = atomicAdd(cp.sCount, 0);
  // 4. taps -> compact cell index (LDS); per stencil cell: ownership check,
  //    marker list in index order (spreading sums in index order), rho and
  //    the uncorrected velocity
  if (own) {
    const int i0 = s_i0[tid], j0 = s_j0[tid];
    int qi[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) qi[t] = cp.wIdx[(j0 + (t >> 2) - wy0) * ww + (i0 + (t & 3) - wx0)];
#pragma unroll
    for (int t = 0; t < 16; ++t) s_tap[t * NM + tid] = qi[t];
  }
  for (int q = tid; q < ns; q += MDF_THREADS) {
    const int c = cp.sCells[q];
    const int gx = wx0 + c % ww, gy = wy0 + c / ww;
    const int cnt = min(wcnt[c], kMaxContrib);
    if (!stencil_ok(cp, gx, gy)) {
      s_bad = 1;
      continue;
    }
    const int32_t *L = cp.wList + (size_t)c * kMaxContrib;
    int32_t *O = cp.sList + (size_t)q * kMaxContrib;
    if (cnt <= 16) {
      sorted_copy<16>(L, cnt, O);
    } else {  // rare: more than 16 markers over one cell
      for (int r = 0; r < cnt; ++r) {
        int v = L[r], w = r - 1;
        while (w >= 0 && O[w] > v) {
          O[w + 1] = O[w];
          --w;
        }
        O[w + 1] = v;
      }
    }
    double rho, ux, uy;
    cell_moments<ST>(a, cp, gx, gy, rho, ux, uy);
    cp.sRho[q] = rho;
    cp.sU[q] = ux;
    cp.sV[q] = uy;
    cp.sFx[q] = 0.0;
    cp.sFy[q] = 0.0;
    int4 meta = {cnt, gx, gy, c};
    *reinterpret_cast<int4 *>(cp.sMeta + 4 * (size_t)q) = meta;
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) mdf_fail(cp, a.err, s_bad == 2 ? ERR_CONTRIB : ERR_MARKER, k);
    return;
  }
  // 5. N_F iterations: interpolate (Eq. 12), boundary force (Eq. 11),
  //    spread (Eq. 15), correct velocity and accumulate force
  for (int it = 0; it < cp.mdf_iters; ++it) {
    if (own) {
      double su = 0.0, sv = 0.0, sr = 0.0;
#pragma unroll
      for (int half = 0; half < 2; ++half) {  // two rows of taps per round of loads
        double uq[8], vq[8], rq[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          int q = s_tap[(half * 8 + t) * NM + tid];
          uq[t] = cp.sU[q];
          vq[t] = cp.sV[q];
          rq[t] = cp.sRho[q];
        }
#pragma unroll
        for (int bh = 0; bh < 2; ++bh) {
          const int bb = half * 2 + bh;
          double py = s_wy[bb * NM + tid];
#pragma unroll
          for (int aa = 0; aa < 4; ++aa) {
            double w = s_wx[aa * NM + tid] * py;
            su += uq[bh * 4 + aa] * w;
            sv += vq[bh * 4 + aa] * w;
            sr += rq[bh * 4 + aa] * w;
          }
        }
      }
      double gx = 2.0 * sr * (udx - su);
      double gy = 2.0 * sr * (udy - sv);
      s_dFx[tid] = gx;
      s_dFy[tid] = gy;
      ftx += gx;
      fty += gy;
    }
    __syncthreads();
    for (int q = tid; q < ns; q += MDF_THREADS) {
      const int4 meta = *reinterpret_cast<const int4 *>(cp.sMeta + 4 * (size_t)q);
      const int cnt = meta.x, gx = meta.y, gy = meta.z;
      const int32_t *L = cp.sList + (size_t)q * kMaxContrib;
      const double rho = cp.sRho[q], u0 = cp.sU[q], v0 = cp.sV[q], fx0 = cp.sFx[q], fy0 = cp.sFy[q];
      double dfx = 0.0, dfy = 0.0;
      for (int r0 = 0; r0 < cnt; r0 += 4) {
        const int4 v4 = *reinterpret_cast<const int4 *>(L + r0);
        const int js[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (r0 + r < cnt) {
            int j = js[r];
            double w = s_wx[(gx - s_i0[j]) * NM + j] * s_wy[(gy - s_j0[j]) * NM + j];
            dfx += s_dFx[j] * w * s_ds[j];
            dfy += s_dFy[j] * w * s_ds[j];
          }
        }
      }
      cp.sFx[q] = fx0 + dfx;
      cp.sFy[q] = fy0 + dfy;
      double r2 = 2.0 * rho;
      cp.sU[q] = u0 + dfx / r2;
      cp.sV[q] = v0 + dfy / r2;
    }
    __syncthreads();
  }
  // 6. force density of the stencil cells for the collision, total marker
  //    forces, and the body force of Eq. (16) summed in marker order
  for (int q = tid; q < ns; q += MDF_THREADS) {
    const int c = cp.sMeta[4 * (size_t)q + 3];
    cp.wF[c] = cp.sFx[q];
    cp.wF[(size_t)cp.win_cap + c] = cp.sFy[q];
  }
  double *gtx = cp.ftot + (size_t)(k & 1) * 2 * n;
  double *gty = gtx + n;
  if (own) {
    gtx[tid] = ftx;
    gty[tid] = fty;
    s_dFx[tid] = ftx * s_ds[tid];
    s_dFy[tid] = fty * s_ds[tid];
  }
  __syncthreads();
  if (tid == 0) {
    double fsx = 0.0, fsy = 0.0;
    int j = 0;
    for (; j + 8 <= n; j += 8) {
      double vx[8], vy[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        vx[r] = s_dFx[j + r];
        vy[r] = s_dFy[j + r];
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        fsx -= vx[r];
        fsy -= vy[r];
      }
    }
    for (; j < n; ++j) {
      fsx -= s_dFx[j];
      fsy -= s_dFy[j];
    }
    int64_t slot = k % cp.hist_cap;
    cp.hist[2 * slot] = fsx;
    cp.hist[2 * slot + 1] = fsy;
    *cp.kcount = k + 1;
  }
}

// ---- small helpers ---------------------------------------------------------
__global__ void reduce_kernel(const double *partial, int n, double vol, double *out, int accumulate) {
  __shared__ double red[3][256];
  double acc[3] = {0.0, 0.0, 0.0};
  int per = (n + 255) / 256;
  int b0 = threadIdx.x * per, b1 = min(n, b0 + per);
  for (int b = b0; b < b1; ++b)
    for (int k = 0; k < 3; ++k) acc[k] += partial[(size_t)b * 3 + k];
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) out[k] = (accumulate ? out[k] : 0.0) + vol * red[k][0];
}

// f = f^eq(rho, u) (Eq. (7)) on owned cells, in the storage frame.
template <int ST>
__global__ __launch_bounds__(256) void init_kernel(const BlockMeta *meta, const uint16_t *codes,
                                                  const CaseDev *cases, void *lat, int b0,
                                                  const double *fields, double r0, double u0, double v0) {
#pragma clang fp contract(off)
  using S = Store<ST>;
  using T = typename S::T;
  const int b = b0 + blockIdx.x, cell = threadIdx.x;
  const BlockMeta m = meta[b];
  const CaseDev &cp = cases[m.case_id];
  uint16_t code = (m.flags & BF_CODES) ? codes[(size_t)m.code * kCells + cell] : (uint16_t)0;
  if ((m.flags & BF_GHOST) || (code & CC_HIDDEN)) return;
  double rho = r0 < 0.0 ? cp.rho0 : r0, ux = u0, uy = v0;
  if (fields) {
    const double *f = fields + (size_t)blockIdx.x * 3 * kCells;
    rho = f[cell];
    ux = f[kCells + cell];
    uy = f[2 * kCells + cell];
  }
  double usq = ux * ux + uy * uy;
  T *d = static_cast<T *>(lat);
  for (int i = 0; i < 9; ++i) {
    double v = feq64(i, rho, ux, uy, usq);
    if constexpr (S::kShift) v = v - wgt<double>(i) * cp.rho0;
    d[((size_t)b * kQ + i) * kCells + cell] = S::st((typename S::C)v);
  }
}

template <typename T>
__global__ void fill_nan_kernel(T *p, size_t n, T v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

template <int ST>
hipError_t launch_level_st(int tile, const LevelArgs *a, hipStream_t s) {
  int groups = a->n_blocks + (a->n_band + 255) / 256;
  if (groups <= 0) return hipSuccess;
  dim3 grid(groups);
  switch (tile) {
    case 1:
      hipLaunchKernelGGL((level_kernel<ST, 2>), grid, dim3(128), 0, s, *a);
      break;
    case 2:
      hipLaunchKernelGGL((level_kernel<ST, 4>), grid, dim3(64), 0, s, *a);
      break;
    default:
      hipLaunchKernelGGL((level_kernel<ST, 1>), grid, dim3(256), 0, s, *a);
      break;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" hipError_t sbt_launch_level_tile(int storage, const LevelArgs *a, hipStream_t s) {
  int groups = a->n_blocks + (a->n_band + 255) / 256;
  if (groups <= 0) return hipSuccess;
  dim3 grid(groups);
  switch (storage) {
    case 0: hipLaunchKernelGGL(level_tile_kernel<0>, grid, dim3(256), 0, s, *a); break;
    case 1: hipLaunchKernelGGL(level_tile_kernel<1>, grid, dim3(256), 0, s, *a); break;
    case 2: hipLaunchKernelGGL(level_tile_kernel<2>, grid, dim3(256), 0, s, *a); break;
    case 3: hipLaunchKernelGGL(level_tile_kernel<3>, grid, dim3(256), 0, s, *a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

extern "C" hipError_t sbt_launch_level(int storage, int tile, const LevelArgs *a, hipStream_t s) {
  switch (storage) {
    case 0: return launch_level_st<0>(tile, a, s);
    case 1: return launch_level_st<1>(tile, a, s);
    case 2: return launch_level_st<2>(tile, a, s);
    case 3: return launch_level_st<3>(tile, a, s);
  }
  return hipErrorInvalidValue;
}

extern "C" size_t sbt_mdf_lds_bytes(int max_markers, int lds_window) {
  return (size_t)max_markers * (11 * sizeof(double) + 18 * sizeof(int)) + (size_t)lds_window * sizeof(int);
}

extern "C" hipError_t sbt_launch_mdf(int storage, const MdfArgs *a, int n_bodies, hipStream_t s) {
  if (n_bodies <= 0) return hipSuccess;
  size_t lds = sbt_mdf_lds_bytes(a->max_markers, a->lds_window);
  switch (storage) {
    case 0: hipLaunchKernelGGL(mdf_kernel<0>, dim3(n_bodies), dim3(MDF_THREADS), lds, s, *a); break;
    case 1: hipLaunchKernelGGL(mdf_kernel<1>, dim3(n_bodies), dim3(MDF_THREADS), lds, s, *a); break;
    case 2: hipLaunchKernelGGL(mdf_kernel<2>, dim3(n_bodies), dim3(MDF_THREADS), lds, s, *a); break;
    case 3: hipLaunchKernelGGL(mdf_kernel<3>, dim3(n_bodies), dim3(MDF_THREADS), lds, s, *a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

extern "C" hipError_t sbt_launch_reduce(const double *partial, int n_blocks, double vol, double *out,
                                        int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, s, partial, n_blocks, vol, out, accumulate);
  return hipGetLastError();
}

extern "C" hipError_t sbt_launch_init(int storage, const BlockMeta *meta, const uint16_t *codes,
                                      const CaseDev *cases, void *lat, int b0, int n,
                                      const double *fields, const double *u, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  double r0 = u ? u[0] : -1.0, u0 = u ? u[1] : 0.0, v0 = u ? u[2] : 0.0;
  switch (storage) {
    case 0: hipLaunchKernelGGL(init_kernel<0>, dim3(n), dim3(256), 0, s, meta, codes, cases, lat, b0, fields, r0, u0, v0); break;
    case 1: hipLaunchKernelGGL(init_kernel<1>, dim3(n), dim3(256), 0, s, meta, codes, cases, lat, b0, fields, r0, u0, v0); break;
    case 2: hipLaunchKernelGGL(init_kernel<2>, dim3(n), dim3(256), 0, s, meta, codes, cases, lat, b0, fields, r0, u0, v0); break;
    case 3: hipLaunchKernelGGL(init_kernel<3>, dim3(n), dim3(256), 0, s, meta, codes, cases, lat, b0, fields, r0, u0, v0); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

extern "C" hipError_t sbt_launch_fill_nan(void *p, size_t n, int storage, hipStream_t s) {
  if (n == 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536));
  switch (storage) {
    case 0:
      hipLaunchKernelGGL(fill_nan_kernel<double>, grid, dim3(256), 0, s, (double *)p, n,
                         (double)__builtin_nan(""));
      break;
    case 1:
      hipLaunchKernelGGL(fill_nan_kernel<float>, grid, dim3(256), 0, s, (float *)p, n,
                         (float)__builtin_nanf(""));
      break;
    case 2:
    case 3:  // 0x7e00 is a quiet NaN in FP16; 0x7fc0 in BF16
      hipLaunchKernelGGL(fill_nan_kernel<uint16_t>, grid, dim3(256), 0, s, (uint16_t *)p, n,
                         (uint16_t)(storage == 2 ? 0x7e00 : 0x7fc0));
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
