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

// c_x, c_y of a direction known only at run time, from 2-bit fields (c + 1)
// of a constant: no table load
__device__ __forceinline__ int cx_of(int p) { return (int)((0x20919u >> (2 * p)) & 3u) - 1; }
__device__ __forceinline__ int cy_of(int p) { return (int)((0x2865u >> (2 * p)) & 3u) - 1; }

template <typename C>
__device__ __forceinline__ C wgt(int i) {
  return i == 0 ? C(4.0 / 9.0) : (i < 5 ? C(1.0 / 9.0) : C(1.0 / 36.0));
}

// ---- storage types ---------------------------------------------------------
// Kernel variant ST = storage | (collision model << 2): bits 0-1 select the
// storage form, bit 2 the MRT collision (kMrt).
template <int SB> struct StoreOf;
template <> struct StoreOf<0> {  // FP64: f itself, FP64 arithmetic
  using T = double;
  using C = double;
  static constexpr bool kShift = false;
  __device__ static C ld(T v) { return v; }
  __device__ static T st(C v) { return v; }
};
template <> struct StoreOf<1> {  // FP32 deviation
  using T = float;
  using C = float;
  static constexpr bool kShift = true;
  __device__ static C ld(T v) { return v; }
  __device__ static T st(C v) { return v; }
};
template <> struct StoreOf<2> {  // FP16 deviation, round to nearest even
  using T = _Float16;
  using C = float;
  static constexpr bool kShift = true;
  __device__ static C ld(T v) { return (float)v; }
  __device__ static T st(C v) { return (_Float16)v; }
};
template <> struct StoreOf<3> {  // BF16 deviation, round to nearest even
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
template <int ST> struct Store : StoreOf<ST & 3> {
  static constexpr bool kMrt = (ST & 4) != 0;
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
template <int SB>
struct CollideBGK;

template <>
struct CollideBGK<0> {
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

template <int SB>
struct CollideBGK {
  // Deviation form (f = w rho0 + d): rho = rho0 + sum d, sum c f = sum c d,
  // and d^eq = w (drho + rho (3 cu + 4.5 cu^2 - 1.5 u^2)), evaluated with
  // the shared terms of the D2Q9 directions.  The Guo term is added only
  // where the force is nonzero.
  __device__ __forceinline__ static void run(const CaseDev &cp, int l, float d[9], float Fx, float Fy, float &rho,
                                             float &ux, float &uy) {
    const float e = d[1] + d[5] + d[8], w = d[3] + d[6] + d[7];   // c_x = +1, -1
    const float n = d[2] + d[5] + d[6], s = d[4] + d[7] + d[8];   // c_y = +1, -1
    const float jx = e - w, jy = n - s;
    const float drho = d[0] + (e + w) + (d[2] + d[4]);
    rho = (float)cp.rho0 + drho;
    const float ir = __builtin_amdgcn_rcpf(rho);
    ux = (jx + 0.5f * Fx) * ir;
    uy = (jy + 0.5f * Fy) * ir;
    const float om = cp.omega_f[l];
    const float A = drho - rho * (1.5f * (ux * ux + uy * uy));
    const float W1 = 1.0f / 9.0f, W2 = 1.0f / 36.0f;
    auto relax = [&](int i, float wi, float cu) {
      const float fe = wi * fmaf(rho * cu, fmaf(4.5f, cu, 3.0f), A);
      d[i] = fmaf(om, fe - d[i], d[i]);
    };
    d[0] = fmaf(om, (4.0f / 9.0f) * A - d[0], d[0]);
    relax(1, W1, ux);
    relax(2, W1, uy);
    relax(3, W1, -ux);
    relax(4, W1, -uy);
    const float pp = ux + uy, pm = ux - uy;
    relax(5, W2, pp);
    relax(6, W2, -pm);
    relax(7, W2, -pp);
    relax(8, W2, pm);
    if (Fx != 0.f || Fy != 0.f) {
      const float pre = cp.pre_f[l];
      const float uF = ux * Fx + uy * Fy;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const float cu = CX[i] * ux + CY[i] * uy;
        const float cF = CX[i] * Fx + CY[i] * Fy;
        d[i] += wgt<float>(i) * pre * (3.f * cF + 9.f * cu * cF - 3.f * uF);
      }
      d[0] += wgt<float>(0) * pre * (-3.f * uF);
    }
  }
};

// MRT collision, the option Sec. 2.1 names for low viscosity: the D2Q9
// moments e, eps (energy and its square), qx, qy (energy flux) and pxx, pxy
// (stresses) relax toward the moments of the Eq. (7) equilibrium at rates
// s_e, s_eps, s_q and 1/tau; density and momentum are conserved except for
// the force, which enters in moment space as (1 - s/2) times the moments of
// Guo's term: (6 u.F, -6 u.F, -Fx, -Fy, 2 (ux Fx - uy Fy), ux Fy + uy Fx),
// and adds exactly F to the momentum.  The change of each moment goes back
// through the orthogonal basis (row norms 36, 36, 6, 12, 6, 12, 4, 4):
//   axis i (c = (+-1, 0), (0, +-1)): -De/36 - Deps/18 +- (Dj - Dq)/6 +- Dxx/4
//   diagonal i:  De/18 + Deps/36 + cx (Djx/6 + Dqx/12) + cy (Djy/6 + Dqy/12)
//                + cx cy Dxy/4
//   rest:        (Deps - De)/9
// so equal rates 1/tau give Eqs. (2)-(3).  Direction order of Eq. (1):
// 1 (+x), 2 (+y), 3 (-x), 4 (-y), 5 (+x+y), 6 (-x+y), 7 (-x-y), 8 (+x-y).
template <typename C>
__device__ __forceinline__ void mrt_update(C f[9], C rho, C ux, C uy, C Fx, C Fy, C e_eq, C ep_eq, C se, C sp, C sq,
                                           C sn) {
#pragma clang fp contract(off)
  const C h = C(0.5);
  const C ax = f[1] + f[3], ay = f[2] + f[4];
  const C sa = ax + ay, sd = (f[5] + f[6]) + (f[7] + f[8]);
  const C e = (C(-4) * f[0] - sa) + C(2) * sd;
  const C ep = (C(4) * f[0] - C(2) * sa) + sd;
  const C qx = C(-2) * (f[1] - f[3]) + ((f[5] - f[6]) - (f[7] - f[8]));
  const C qy = C(-2) * (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
  const C pxx = ax - ay;
  const C pxy = (f[5] - f[6]) + (f[7] - f[8]);
  const C rux = rho * ux, ruy = rho * uy;
  C De = -se * (e - e_eq), Dp = -sp * (ep - ep_eq);
  C Dqx = -sq * (qx + rux), Dqy = -sq * (qy + ruy);
  C Dxx = -sn * (pxx - rho * (ux * ux - uy * uy)), Dxy = -sn * (pxy - rux * uy);
  C Djx = C(0), Djy = C(0);
  if (Fx != C(0) || Fy != C(0)) {
    const C uF = ux * Fx + uy * Fy;
    De = De + (C(1) - h * se) * (C(6) * uF);
    Dp = Dp + (C(1) - h * sp) * (C(-6) * uF);
    Dqx = Dqx + (C(1) - h * sq) * (-Fx);
    Dqy = Dqy + (C(1) - h * sq) * (-Fy);
    Dxx = Dxx + (C(1) - h * sn) * (C(2) * (ux * Fx - uy * Fy));
    Dxy = Dxy + (C(1) - h * sn) * (ux * Fy + uy * Fx);
    Djx = Fx;
    Djy = Fy;
  }
  const C a0 = -De / C(36) - Dp / C(18);
  const C gx = (Djx - Dqx) / C(6), gy = (Djy - Dqy) / C(6), P = Dxx / C(4);
  const C d0 = De / C(18) + Dp / C(36);
  const C hx = Djx / C(6) + Dqx / C(12), hy = Djy / C(6) + Dqy / C(12), X = Dxy / C(4);
  f[0] = f[0] + (Dp - De) / C(9);
  f[1] = f[1] + ((a0 + gx) + P);
  f[3] = f[3] + ((a0 - gx) + P);
  f[2] = f[2] + ((a0 + gy) - P);
  f[4] = f[4] + ((a0 - gy) - P);
  f[5] = f[5] + (((d0 + hx) + hy) + X);
  f[6] = f[6] + (((d0 - hx) + hy) - X);
  f[7] = f[7] + (((d0 - hx) - hy) + X);
  f[8] = f[8] + (((d0 + hx) - hy) - X);
}

template <int SB>
struct CollideMRT {
  // Deviation form: the moments of d = f - w rho0 differ from those of f by
  // rho0 (1, -2, 1, 0, ...), so e_eq and eps_eq shift by 2 rho0 and -rho0.
  __device__ __forceinline__ static void run(const CaseDev &cp, int l, float d[9], float Fx, float Fy, float &rho,
                                             float &ux, float &uy) {
    const float e = d[1] + d[5] + d[8], w = d[3] + d[6] + d[7];
    const float n = d[2] + d[5] + d[6], s = d[4] + d[7] + d[8];
    const float jx = e - w, jy = n - s;
    const float drho = d[0] + (e + w) + (d[2] + d[4]);
    rho = (float)cp.rho0 + drho;
    const float ir = __builtin_amdgcn_rcpf(rho);
    ux = (jx + 0.5f * Fx) * ir;
    uy = (jy + 0.5f * Fy) * ir;
    const float ru2 = rho * (3.0f * (ux * ux + uy * uy));
    mrt_update<float>(d, rho, ux, uy, Fx, Fy, -2.0f * drho + ru2, drho - ru2, cp.mrt_s_f[0], cp.mrt_s_f[1],
                      cp.mrt_s_f[2], cp.omega_f[l]);
  }
};

template <>
struct CollideMRT<0> {
  __device__ __forceinline__ static void run(const CaseDev &cp, int l, double f[9], double Fx, double Fy, double &rho,
                                             double &ux, double &uy) {
#pragma clang fp contract(off)
    double jx, jy;
    moments64(f, rho, jx, jy);
    ux = (jx + 0.5 * Fx) / rho;
    uy = (jy + 0.5 * Fy) / rho;
    const double u2 = ux * ux + uy * uy;
    mrt_update<double>(f, rho, ux, uy, Fx, Fy, rho * (-2.0 + 3.0 * u2), rho * (1.0 - 3.0 * u2), cp.mrt_s[0],
                       cp.mrt_s[1], cp.mrt_s[2], 1.0 / cp.tau[l]);
  }
};

template <bool B, class A, class Z> struct PickT { using type = A; };
template <class A, class Z> struct PickT<false, A, Z> { using type = Z; };
template <int ST>
struct Collide : PickT<(ST & 4) != 0, CollideMRT<ST & 3>, CollideBGK<ST & 3>>::type {};

// IBM force density at cell (x, y) of the finest block at (ox, oy) for the
// collision of the substep the last forcing loop ran for (zero outside its
// window).  `parity` is that substep's plan buffer (negative: derived from
// the forcing-loop counter).  The window test is per block, on wave-uniform
// values.
// The window and the plan counter are written by other launches, never by
// the kernels that read them here, so they are read through the constant
// address space (scalar loads); the force density through the global one.
// Generic (flat) loads would make the compiler wait for every outstanding
// direct-to-LDS copy first, since a flat access may alias LDS.
typedef __attribute__((address_space(4))) const int32_t ci32_t;
typedef __attribute__((address_space(4))) const int64_t ci64_t;
typedef __attribute__((address_space(1))) const double gdbl_t;

// A value another workgroup of the same launch may have written (used in
// the persistent step's module): a vector load at agent scope, never a
// scalar one (the scalar cache is not kept coherent with vector stores).
template <typename T>
__device__ __forceinline__ T ld_fresh(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// In the persistent step's module the window and counter may have been
// written earlier in the same launch: vector loads there.
template <typename C>
__device__ __forceinline__ void add_ibm_force(const CaseDev &cp, int parity, int ox, int oy, int x, int y, C &Fx,
                                              C &Fy) {
#ifdef SBT_PERSISTENT_TU
  const int b = parity >= 0 ? parity : __builtin_amdgcn_readfirstlane((int)((ld_fresh(cp.kcount) - 1) & cp.plan_mask));
  const int32_t *w = reinterpret_cast<const int32_t *>(cp.win + b);
  const int x0 = __builtin_amdgcn_readfirstlane(ld_fresh(w)), y0 = __builtin_amdgcn_readfirstlane(ld_fresh(w + 1));
  const int ww = __builtin_amdgcn_readfirstlane(ld_fresh(w + 2)), wh = __builtin_amdgcn_readfirstlane(ld_fresh(w + 3));
#else
  const int b = parity >= 0 ? parity
                            : __builtin_amdgcn_readfirstlane((int)((*(ci64_t *)cp.kcount - 1) & cp.plan_mask));
  ci32_t *w = (ci32_t *)cp.win + 4 * b;   // IbmWindow {x0, y0, w, h}
  const int x0 = __builtin_amdgcn_readfirstlane(w[0]), y0 = __builtin_amdgcn_readfirstlane(w[1]);
  const int ww = __builtin_amdgcn_readfirstlane(w[2]), wh = __builtin_amdgcn_readfirstlane(w[3]);
#endif
  if (ox + kB <= x0 || ox >= x0 + ww || oy + kB <= y0 || oy >= y0 + wh) return;
  const int wx = ox + x - x0, wy = oy + y - y0;
  if (wx >= 0 && wx < ww && wy >= 0 && wy < wh) {
    gdbl_t *F = (gdbl_t *)cp.wF + (size_t)b * 2 * cp.win_cap;
    const size_t wi = (size_t)wy * ww + wx;
    Fx = Fx + (C)F[wi];
    Fy = Fy + (C)F[(size_t)cp.win_cap + wi];
  }
}

// Equilibrium in the storage frame for the interface / boundary operators.
template <int ST>
__device__ __forceinline__ typename Store<ST>::C feq_frame(const CaseDev &cp, int i,
                                                          typename Store<ST>::C rho,
                                                          typename Store<ST>::C ux,
                                                          typename Store<ST>::C uy) {
#pragma clang fp contract(off)
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
// rd(lx, ly, p) reads the post-collision population p of the cell at local
// coordinates (lx, ly) (block `self` or a neighbour).  The edge kinds and
// velocities are read at constant indices (scalar loads of the wave-uniform
// case) and selected per lane, never indexed by the lane's edge.
// The case parameters every edge decision uses, read once per block and
// packed into three registers.  An empty asm statement that takes
// them as operands pins the loads before the per-direction branches (sunk
// into those branches, each scalar load would wait on its own).  The wall
// and inflow velocities and rho0 are read where those rules apply.
struct EdgeParams {
  int nx, ny;
  int bits;  // per_x | per_y << 1 | bc[e] << (4 + 4 e)
  const CaseDev *cp;
  __device__ int per_x() const { return bits & 1; }
  __device__ int per_y() const { return (bits >> 1) & 1; }
  __device__ int bc(int e) const { return (bits >> (4 + 4 * e)) & 15; }
};

__device__ __forceinline__ EdgeParams edge_params(const CaseDev &cp) {
  EdgeParams ep;
  int nx = cp.nx[0], ny = cp.ny[0];
  int bits = (cp.per_x ? 1 : 0) | (cp.per_y ? 2 : 0);
#pragma unroll
  for (int e = 0; e < 4; ++e) bits |= (cp.bc[e] & 15) << (4 + 4 * e);
  asm volatile("" : "+v"(nx), "+v"(ny), "+v"(bits));
  ep.nx = nx;
  ep.ny = ny;
  ep.bits = bits;
  ep.cp = &cp;
  return ep;
}

template <int ST, class Reader>
__device__ __forceinline__ typename Store<ST>::C edge_value_rd(const EdgeParams &ep, int x, int y, int gx, int gy, int q,
                                                               Reader &&rd) {
#pragma clang fp contract(off)
  using C = typename Store<ST>::C;
  const int nx = ep.nx, ny = ep.ny;
  const int bc0 = ep.bc(0), bc1 = ep.bc(1), bc2 = ep.bc(2), bc3 = ep.bc(3);
  const CaseDev &cp = *ep.cp;
  auto pick = [](int e, auto v0, auto v1, auto v2, auto v3) { return e == 0 ? v0 : (e == 1 ? v1 : (e == 2 ? v2 : v3)); };
  int sx = gx - CX[q], sy = gy - CY[q];
  bool outx = (sx < 0 || sx >= nx) && !ep.per_x();
  bool outy = (sy < 0 || sy >= ny) && !ep.per_y();
  int ex = sx < 0 ? 0 : 1, ey = sy < 0 ? 2 : 3;
  int e = outx ? ex : ey;
  if (outx && outy) {
    int kx = ex == 0 ? bc0 : bc1, ky = ey == 2 ? bc2 : bc3;
    bool lx = kx == 1 || kx == 2, ly = ky == 1 || ky == 2;
    if (!lx && ly) e = ey;
  }
  const int kind = pick(e, bc0, bc1, bc2, bc3);
  auto uwall = [&](int c) { return pick(e, cp.bcu[0][c], cp.bcu[1][c], cp.bcu[2][c], cp.bcu[3][c]); };
  switch (kind) {
    case 1: {  // wall: half-way bounce-back with moving-wall term
      const double uwx = uwall(0), uwy = uwall(1);
      C fs = rd(x, y, OPP[q]);
      if constexpr (!Store<ST>::kShift) {
        return fs + 6.0 * wgt<double>(q) * cp.rho0 * (CX[q] * uwx + CY[q] * uwy);
      } else {
        return fs + (float)(6.0 * wgt<double>(q) * cp.rho0 * (CX[q] * uwx + CY[q] * uwy));
      }
    }
    case 2: {  // equilibrium inflow at (rho0, u_in)
      const double uwx = uwall(0), uwy = uwall(1);
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
      if (kind == 3) {
        px = gx - nrx - CX[q];
        py = gy - nry - CY[q];
      } else {
        px = gx - (xn ? 0 : CX[q]);
        py = gy - (xn ? CY[q] : 0);
        qq = xn ? MIRX[q] : MIRY[q];
      }
      // periodic axes wrap through the neighbour table; others clamp (corners)
      if (!ep.per_x()) px = px < 0 ? 0 : (px >= nx ? nx - 1 : px);
      if (!ep.per_y()) py = py < 0 ? 0 : (py >= ny ? ny - 1 : py);
      return rd(x + (px - gx), y + (py - gy), qq);
    }
    default:
      return C(__builtin_nan(""));
  }
}

// The same, reading every source from the lattice in memory.
template <int ST>
__device__ __forceinline__ typename Store<ST>::C edge_value(const CaseDev &cp, const void *src, const Blk &k, int x, int y,
                                                            int gx, int gy, int q) {
  return edge_value_rd<ST>(edge_params(cp), x, y, gx, gy, q,
                           [&](int lx, int ly, int p) { return fetch<ST>(src, k, lx, ly, p); });
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

// The same mean, for a block whose 4 finer blocks' neighbour tables sit in
// LDS: cn[c * 9 + d] = neighbour d (the block table's order) of the finer
// block under quadrant c = (x >= 8) + 2 (y >= 8), cn[c * 9 + 8] = that block
// (-1 if none).  The 4 loads are issued together (a missing block reads
// block 0 and is replaced by NaN after the load), so a coalesced direction
// costs one memory round trip.
__device__ __forceinline__ int nbr_dir(int x, int y) {
  if (x < 0) return y < 0 ? 6 : (y > 15 ? 5 : 2);
  if (x > 15) return y < 0 ? 7 : (y > 15 ? 4 : 0);
  if (y < 0) return 3;
  if (y > 15) return 1;
  return 8;
}

template <int ST>
__device__ __forceinline__ typename Store<ST>::C coalesce_lds(const LevelArgs &a, const int *cn, int x, int y,
                                                               int q) {
#pragma clang fp contract(off)
  using C = typename Store<ST>::C;
  const int c = (x >= 8) + 2 * (y >= 8);
  const int fx0 = (2 * x) & 15, fy0 = (2 * y) & 15;
  C v[4];
  bool miss[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int sx = fx0 + (s & 1) - CX[q], sy = fy0 + (s >> 1) - CY[q];
    const int nb = cn[c * 9 + nbr_dir(sx, sy)];
    miss[s] = nb < 0;
    v[s] = ldv<ST>(a.fprev, nb < 0 ? 0 : nb, q, (sy & 15) * 16 + (sx & 15));
  }
  C sum = miss[0] ? C(__builtin_nan("")) : v[0];
  sum += miss[1] ? C(__builtin_nan("")) : v[1];
  sum += miss[2] ? C(__builtin_nan("")) : v[2];
  sum += miss[3] ? C(__builtin_nan("")) : v[3];
  return C(0.25) * sum;
}

// Interpolated bounce-back (linear Bouzidi form, resting wall) of pulled
// direction i at cell (x, y) of block k, whose source x - c_i is solid: the
// population o = opposite(i) that the cell sent toward the wall, at wall
// fraction q of its link, comes back as
//   q <  1/2:  2q f*_o(x) + (1 - 2q) f*_o(x + c_i)
//   q >= 1/2:  f*_o(x) / (2q) + (2q - 1)/(2q) f*_i(x).
// Both forms are affine with weights summing to 1 and w_o = w_i, so they
// hold unchanged for the deviation storage forms.
template <int ST>
__device__ __forceinline__ typename Store<ST>::C bouzidi(const LevelArgs &a, const Blk &k, int srec, int x, int y,
                                                         int i) {
#pragma clang fp contract(off)
  using C = typename Store<ST>::C;
  const int cell = y * 16 + x, o = OPP[i];
  const double q = a.sq[((size_t)srec * kQ + i) * kCells + cell];
  const C fo = ldv<ST>(a.src, k.self, o, cell);
  if (q < 0.5) {
    const int ux = x + CX[i], uy = y + CY[i];
    const int nb = pick_nbr(k, ux, uy);
    const C fu = ldv<ST>(a.src, nb, o, (uy & 15) * 16 + (ux & 15));
    return C(2.0 * q) * fo + C(1.0 - 2.0 * q) * fu;
  }
  const C fi = ldv<ST>(a.src, k.self, i, cell);
  return fo / C(2.0 * q) + C((2.0 * q - 1.0) / (2.0 * q)) * fi;
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
  const int srec = (k.flags & BF_SOLID) ? a.meta[b].solid : -1;
  const uint16_t sb = srec >= 0 ? a.sbits[(size_t)srec * kCells + cell] : (uint16_t)0;

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
  if ((code & CC_HIDDEN) || (sb & SB_SOLID)) {  // covered by the finer level, or solid
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
      if (sb & (1u << i)) {
        f[i] = bouzidi<ST>(a, k, srec, x, y, i);
      } else if (code & (1u << i)) {
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
  if (k.flags & BF_IBM) add_ibm_force<C>(cp, a.ibm_parity, k.ox, k.oy, x, y, Fx, Fy);

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

// Work item of tile-launch workgroup `bid` (roles: 0 interior run, 1 edge or
// interface block, 2 band-cell group, -1 none).  Workgroups go to the 8
// XCDs round-robin; XCD x takes the x-th eighth of each role (contiguous in
// Morton order, so its halo reads stay in its own L2), band groups and
// edge/interface blocks first: they are latency-bound and slower, so they
// are spread over all XCDs and overlap the streaming runs instead of
// trailing at the end.  Without the remap the grid is plain
// [runs | blocks | band groups].
__device__ __forceinline__ int tile_role(int bid, int n_run, int n_blk, int n_bnd, int enable, int &idx) {
  if (!enable) {
    if (bid < n_run) { idx = bid; return 0; }
    bid -= n_run;
    if (bid < n_blk) { idx = bid; return 1; }
    bid -= n_blk;
    idx = bid;
    return bid < n_bnd ? 2 : -1;
  }
  const int x = bid & 7, k = bid >> 3;
  const int b0 = n_bnd * x / 8, b1 = n_bnd * (x + 1) / 8;
  if (k < b1 - b0) { idx = b0 + k; return 2; }
  const int k1 = k - (b1 - b0);
  const int s0 = n_blk * x / 8, s1 = n_blk * (x + 1) / 8;
  if (k1 < s1 - s0) { idx = s0 + k1; return 1; }
  const int k2 = k1 - (s1 - s0);
  const int r0 = n_run * x / 8, r1 = n_run * (x + 1) / 8;
  if (k2 < r1 - r0) { idx = r0 + k2; return 0; }
  return -1;
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
  const bool slow = (k.flags & (BF_CODES | BF_EDGE | BF_SOLID)) != 0;
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
// LDS image of one block: the 9 planes dense (256 cells each, the same
// byte order as in HBM, so a 16-byte-per-lane direct copy fills them), then
// 188 halo populations that stream in from the 8 neighbours.
template <int ST>
struct Tile {
  using T = typename Store<ST>::T;
  static constexpr int DENSE = kQ * kCells;                   // elements
  static constexpr int HALO = 192;                            // 188 used
  // Halo populations of 4 bytes or less arrive by direct global->LDS copy,
  // which puts each lane's value in a 32-bit slot (low bytes); 8-byte ones
  // go through a register into dense slots.
  static constexpr bool kDmaHalo = sizeof(T) <= 4;
  static constexpr int HSTRIDE = kDmaHalo ? 4 / (int)sizeof(T) : 1;  // elements per halo slot
  static constexpr int SIZE = DENSE + HALO * HSTRIDE;
  static constexpr int NVEC = DENSE * (int)sizeof(T) / 16;    // 16-byte vectors
  static constexpr int NOPS = (NVEC + 255) / 256;             // copies per lane
};

typedef __attribute__((address_space(3))) void lds_void;

// Halo slot t (0..187): the plane it feeds and the local cell (x, y in
// -1..16) just outside the block that the plane streams in from.  Slots
// 0..63 are the four axis directions (16 each), 64..187 the four diagonals
// (31 each: a column of 16, then a row of 15).
constexpr void halo_slot(int t, int &plane, int &hx, int &hy) {
  if (t < 64) {
    int s = t & 15;
    plane = 1 + (t >> 4);
    hx = plane == 1 ? -1 : (plane == 3 ? 16 : s);
    hy = plane == 2 ? -1 : (plane == 4 ? 16 : s);
  } else {
    int d = (t - 64) / 31, s = (t - 64) % 31;
    plane = 5 + d;
    bool col = s < 16;
    if (plane == 5) { hx = col ? -1 : s - 16; hy = col ? s - 1 : -1; }
    else if (plane == 6) { hx = col ? 16 : s - 15; hy = col ? s - 1 : -1; }
    else if (plane == 7) { hx = col ? 16 : s - 15; hy = col ? s + 1 : 16; }
    else { hx = col ? -1 : s - 16; hy = col ? s + 1 : 16; }
  }
}

// Halo slot t as (neighbour << 16) | element: the neighbour in BlockMeta.nbr
// order (E, N, W, S, NE, NW, SW, SE) that holds the source cell, and the
// element (plane * 256 + cell) of that population inside it.  A table
// built at compile time from halo_slot, so a lane does one lookup instead
// of the slot arithmetic.
struct HaloTable {
  uint32_t e[192];
  constexpr HaloTable() : e() {
    for (int t = 0; t < 192; ++t) {
      int plane = 0, hx = 0, hy = 0;
      halo_slot(t < 188 ? t : 187, plane, hx, hy);
      int nb = 0;
      if (hx < 0) nb = hy < 0 ? 6 : (hy > 15 ? 5 : 2);
      else if (hx > 15) nb = hy < 0 ? 7 : (hy > 15 ? 4 : 0);
      else nb = hy < 0 ? 3 : 1;
      e[t] = ((uint32_t)nb << 16) | (uint32_t)(plane * kCells + (hy & 15) * 16 + (hx & 15));
    }
  }
};
__constant__ constexpr HaloTable kHalo{};

__device__ __forceinline__ int halo_nbr(const Blk &k, int code) {
  int v = vsel(code == 1, k.nN, k.nE);
  v = vsel(code == 2, k.nW, v);
  v = vsel(code == 3, k.nS, v);
  v = vsel(code == 4, k.nNE, v);
  v = vsel(code == 5, k.nNW, v);
  v = vsel(code == 6, k.nSW, v);
  return vsel(code == 7, k.nSE, v);
}

// LDS element holding the population of direction i that streams into
// local cell (x, y): the dense plane when its source cell is inside the
// block, else the halo slot of that source (inverse of halo_slot).
template <int HSTRIDE>
__device__ __forceinline__ int tile_index(int i, int x, int y) {
  const int sx = x - cx_of(i), sy = y - cy_of(i);
  if ((unsigned)sx < 16u && (unsigned)sy < 16u) return i * kCells + sy * 16 + sx;
  int slot;
  switch (i) {
    case 1: slot = y; break;
    case 2: slot = 16 + x; break;
    case 3: slot = 32 + y; break;
    case 4: slot = 48 + x; break;
    case 5: slot = 64 + (x == 0 ? y : 15 + x); break;
    case 6: slot = 95 + (x == 15 ? y : 16 + x); break;
    case 7: slot = 126 + (x == 15 ? y : 16 + x); break;
    default: slot = 157 + (x == 0 ? y : 15 + x); break;
  }
  return kQ * kCells + slot * HSTRIDE;
}

// Source of the halo population of a missing neighbour: NaN in each storage
// type (f32 word 0; bf16 high half of word 0; f16 low half of word 1).
__device__ uint32_t kNanSrc[2] = {0x7FC00000u, 0x7FC07E00u};

template <int ST>
__device__ __forceinline__ const typename Store<ST>::T *nan_src() {
  using T = typename Store<ST>::T;
  const char *p = reinterpret_cast<const char *>(kNanSrc);
  if constexpr (sizeof(T) == 4) return reinterpret_cast<const T *>(p);
  else if constexpr ((ST & 3) == 3) return reinterpret_cast<const T *>(p + 2);  // bf16
  else return reinterpret_cast<const T *>(p + 4);
}

// Issue the loads of block k into LDS image `buf`: the dense planes by
// direct global->LDS copies (16 bytes per lane, no registers), and this
// lane's halo population (NaN where the neighbour is missing) by a direct
// copy too, or into h for 8-byte storage.
template <int ST>
__device__ __forceinline__ void fetch_tile(const LevelArgs &a, const Blk &k, typename Store<ST>::T *buf,
                                           typename Store<ST>::T &h, uint32_t he) {
  using S = Store<ST>;
  using T = typename S::T;
  using C = typename S::C;
  using TL = Tile<ST>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const T *src = static_cast<const T *>(a.src);
  const char *g = reinterpret_cast<const char *>(src + (size_t)k.self * kQ * kCells);
#pragma unroll
  for (int r = 0; r < TL::NOPS; ++r) {
    const int v0 = r * 256 + wv * 64;  // wave-uniform first vector
    if (v0 < TL::NVEC && v0 + lane < TL::NVEC)
      __builtin_amdgcn_global_load_lds(g + (size_t)(v0 + lane) * 16, (lds_void *)(reinterpret_cast<char *>(buf) + v0 * 16),
                                       16, 0, 0);
  }
  if (tid < 188) {
    const uint32_t e = he;
    const int nb = halo_nbr(k, (int)(e >> 16));
    if constexpr (TL::kDmaHalo) {
      const T *p = nb < 0 ? nan_src<ST>() : src + (size_t)nb * kQ * kCells + (e & 0xffff);
      __builtin_amdgcn_global_load_lds(p, (lds_void *)(reinterpret_cast<char *>(buf + TL::DENSE) + wv * 64 * 4),
                                       (int)sizeof(T), 0, 0);
    } else {
      h = nb < 0 ? S::st(C(__builtin_nan(""))) : src[(size_t)nb * kQ * kCells + (e & 0xffff)];
    }
  }
}

// Make buf complete for every lane: this lane's halo value (8-byte
// storage), then wait for this wave's direct copies before the barrier
// (other waves read them).  Vector memory operations complete in issue
// order, so when at least `after` were issued after this buffer's copies
// (later blocks' copies, earlier blocks' 9 stores), vmcnt(after) covers the
// copies without waiting for those.  The barrier then carries no memory fence: a fence
// would wait for the stores too.  Only LDS is shared across it, and every
// LDS access before it has completed (the copies by the wait, the reads
// because their values were used); the empty asm statements keep the
// compiler from moving memory accesses across it.
template <int ST>
__device__ __forceinline__ void commit_tile(typename Store<ST>::T *buf, typename Store<ST>::T h, int after = 0) {
  if constexpr (!Tile<ST>::kDmaHalo) {
    if (threadIdx.x < 188) buf[Tile<ST>::DENSE + threadIdx.x] = h;
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
  } else {
    // vmcnt(n) with lgkmcnt and expcnt left at their maxima
    if (after >= 9) __builtin_amdgcn_s_waitcnt(0x0F79);        // vmcnt(9)
    else __builtin_amdgcn_s_waitcnt(0x0F70);                   // vmcnt(0)
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  }
}

// Stream (from the staged tile) + collide of block k; interface, edge and
// explosion work only when SLOW.
template <int ST, bool SLOW>
__device__ __forceinline__ void compute_block(const LevelArgs &a, const CaseDev *__restrict__ cases, const Blk &k,
                                              const typename Store<ST>::T *tile, double ibm_fx, double ibm_fy,
                                              uint16_t code_in = 0, const int *cn = nullptr) {
#pragma clang fp contract(off)
  using S = Store<ST>;
  using T = typename S::T;
  using C = typename S::C;
  // block fields are wave-uniform: keep the case parameters on the scalar
  // path (a vector load here would wait for the next block's copies)
  const CaseDev &cp = cases[__builtin_amdgcn_readfirstlane(k.cid)];
  const int tid = threadIdx.x;
  const int b = __builtin_amdgcn_readfirstlane(k.self);

  const int x = tid & 15, y = tid >> 4;
  const int l = __builtin_amdgcn_readfirstlane(k.level);
  uint16_t code = 0;
  if (SLOW) {
    code = code_in;  // loaded by the caller while the tile copies were in flight
    if (code & CC_HIDDEN) return;  // covered by the finer level
  }
  C f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i)
    f[i] = S::ld(tile[tile_index<Tile<ST>::HSTRIDE>(i, x, y)]);
  if (SLOW) {
    const int gx = k.ox + x, gy = k.oy + y;
    const bool edge = (k.flags & BF_EDGE) != 0;
    // post-collision population p of local cell (lx, ly): from the staged
    // tile when the block holds it or when it is the halo value that some
    // cell of the block streams in, else from memory (block corners)
    const EdgeParams ep = edge_params(cp);
    auto tile_reader = [&](int lx, int ly, int p) -> C {
      if ((unsigned)lx < 16u && (unsigned)ly < 16u) return S::ld(tile[p * kCells + ly * 16 + lx]);
      const int cx = lx + cx_of(p), cy = ly + cy_of(p);
      if ((unsigned)cx < 16u && (unsigned)cy < 16u) return S::ld(tile[tile_index<Tile<ST>::HSTRIDE>(p, cx, cy)]);
      return fetch<ST>(a.src, k, lx, ly, p);
    };
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      if (code & (1u << i)) {
        f[i] = coalesce_lds<ST>(a, cn, x, y, i);
      } else if (edge) {
        int sx = gx - CX[i], sy = gy - CY[i];
        bool out = (!ep.per_x() && (sx < 0 || sx >= ep.nx)) || (!ep.per_y() && (sy < 0 || sy >= ep.ny));
        if (out) f[i] = edge_value_rd<ST>(ep, x, y, gx, gy, i, tile_reader);
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
    Fx = Fx + (C)ibm_fx;
    Fy = Fy + (C)ibm_fy;
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

// IBM force density of this lane's cell of block k for the collision of
// this substep (zero outside the body's window, and for blocks of levels
// without a body).  Its loads are issued where the caller puts this call:
// before a block's tile copies, so that waiting for them never waits for
// the copies.
// The window and counter reads are scalar, so a block outside the window
// issues no vector load; the few blocks inside it load their cells' values
// before the next block's copies are issued.
template <int ST>
__device__ __forceinline__ void ibm_force_of(const LevelArgs &a, const CaseDev *__restrict__ cases, const Blk &k,
                                             double &fx, double &fy) {
  fx = 0.0;
  fy = 0.0;
  if (k.flags & BF_IBM) {
    const CaseDev &cp = cases[__builtin_amdgcn_readfirstlane(k.cid)];
    const int b = a.ibm_parity >= 0
                      ? a.ibm_parity
                      : __builtin_amdgcn_readfirstlane((int)((*(ci64_t *)cp.kcount - 1) & cp.plan_mask));
    ci32_t *w = (ci32_t *)cp.win + 4 * b;   // IbmWindow {x0, y0, w, h}
    const int x0 = __builtin_amdgcn_readfirstlane(w[0]), y0 = __builtin_amdgcn_readfirstlane(w[1]);
    const int ww = __builtin_amdgcn_readfirstlane(w[2]), wh = __builtin_amdgcn_readfirstlane(w[3]);
    if (k.ox + kB <= x0 || k.ox >= x0 + ww || k.oy + kB <= y0 || k.oy >= y0 + wh) return;
    const int wx = k.ox + (int)(threadIdx.x & 15) - x0, wy = k.oy + (int)(threadIdx.x >> 4) - y0;
    if (wx >= 0 && wx < ww && wy >= 0 && wy < wh) {
      gdbl_t *F = (gdbl_t *)cp.wF + (size_t)b * 2 * cp.win_cap + (size_t)wy * ww + wx;
      fx = F[0];
      fy = F[cp.win_cap];
    }
  }
}


// One pipelined step over a run of interior blocks: make `cur` (block j)
// complete, issue the loads of block j's IBM force, start block j+1's copies
// into `nxt`, stream + collide block j from `cur`, then issue the scalar
// load of block j+2's metadata (used after the next barrier).  No vector
// load whose value the step needs is issued after the copies, so nothing
// waits for them before the barrier of the next step.
template <int ST>
__device__ __forceinline__ void pipe_step(const LevelArgs &a, const CaseDev *__restrict__ cases,
                                          const BlockMeta *__restrict__ meta, Blk &kc, Blk &kn, int lv, int j, int cnt,
                                          typename Store<ST>::T *cur, typename Store<ST>::T *nxt,
                                          typename Store<ST>::T &h, uint32_t he) {
  // after the first block, the previous block's 9 stores were issued after
  // this buffer's copies
  commit_tile<ST>(cur, h, j > 0 ? 9 : 0);
  double fx, fy;
  ibm_force_of<ST>(a, cases, kc, fx, fy);
  if (j + 1 < cnt) fetch_tile<ST>(a, kn, nxt, h, he);
  compute_block<ST, false>(a, cases, kc, cur, fx, fy);
  kc = kn;
  if (j + 2 < cnt) kn = load_blk(meta, __builtin_amdgcn_readlane(lv, j + 2));
}

// One launch per level substep.  With NBUF = 2, workgroups [0, n_fast_wg)
// each take a run of up to `kpw` consecutive interior blocks (no cell
// codes, no domain edge, all eight neighbours) and copy block j+1 into the
// second LDS image while block j is computed from the first.  The next
// n_blocks - n_fast workgroups take one block next to a finer level or a
// domain edge each; the rest gather packed halo-band cells.
template <int ST, int NBUF>
__global__ __launch_bounds__(256) void level_tile_kernel(LevelArgs a, const CaseDev *__restrict__ cases,
                                                        const BlockMeta *__restrict__ meta, const int32_t *__restrict__ list) {
  using T = typename Store<ST>::T;
  using TL = Tile<ST>;
  __shared__ __attribute__((aligned(16))) T bufA[TL::SIZE];
  __shared__ __attribute__((aligned(16))) T bufB[NBUF == 2 ? TL::SIZE : 8];
  const int kpw = NBUF == 2 ? a.kpw : 1;
  const int n_fast_wg = (a.n_fast + kpw - 1) / kpw;
  const int n_band_wg = (a.n_band + 255) / 256;
  int w0;
  const int role = __builtin_amdgcn_readfirstlane(
      tile_role(blockIdx.x, n_fast_wg, a.n_blocks - a.n_fast, n_band_wg, a.xcd_remap, w0));
  const int w = __builtin_amdgcn_readfirstlane(w0);  // wave-uniform: keeps block metadata on the scalar path
  const int lane = threadIdx.x & 63;
  // this lane's halo slot (neighbour code, element), the same for every
  // block: loaded before any copy is in flight
  const uint32_t he = threadIdx.x < 188 ? kHalo.e[threadIdx.x] : 0u;
  T h;
  if (role == 0) {
    const int first = w * kpw;
    const int cnt = min(kpw, a.n_fast - first);
    if (NBUF == 1 || cnt == 1) {
      const Blk k = load_blk(meta, list[first]);
      double fx, fy;
      ibm_force_of<ST>(a, cases, k, fx, fy);
      fetch_tile<ST>(a, k, bufA, h, he);
      commit_tile<ST>(bufA, h);
      compute_block<ST, false>(a, cases, k, bufA, fx, fy);
      return;
    }
    // the run's block ids (one per lane) and the first two blocks' metadata
    // (scalar loads)
    const int lv = list[first + min(lane, cnt - 1)];
    Blk kc = load_blk(meta, __builtin_amdgcn_readlane(lv, 0));
    Blk kn = load_blk(meta, __builtin_amdgcn_readlane(lv, 1));
    fetch_tile<ST>(a, kc, bufA, h, he);
    for (int j = 0; j < cnt; j += 2) {
      pipe_step<ST>(a, cases, meta, kc, kn, lv, j, cnt, bufA, bufB, h, he);
      if (j + 1 < cnt) pipe_step<ST>(a, cases, meta, kc, kn, lv, j + 1, cnt, bufB, bufA, h, he);
    }
    return;
  }
  if (role == 1) {
    __shared__ int cn[36];  // the finer blocks' neighbour tables (coalescence)
    const Blk k = load_blk(meta, list[a.n_fast + w]);
    double fx, fy;
    ibm_force_of<ST>(a, cases, k, fx, fy);
    int cv = -1;
    if ((k.flags & BF_CODES) && a.fmeta && threadIdx.x < 36) {
      const int c = threadIdx.x / 9, d = threadIdx.x % 9;
      const int cb = c == 0 ? k.c0 : (c == 1 ? k.c1 : (c == 2 ? k.c2 : k.c3));
      cv = cb < 0 ? -1 : (d == 8 ? cb : a.fmeta[cb].nbr[d]);
    }
    fetch_tile<ST>(a, k, bufA, h, he);
    const uint16_t code = (k.flags & BF_CODES) ? a.codes[(size_t)k.code * kCells + threadIdx.x] : (uint16_t)0;
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the table entry (and the copies) have landed
    if (threadIdx.x < 36) cn[threadIdx.x] = cv;
    commit_tile<ST>(bufA, h);
    compute_block<ST, true>(a, cases, k, bufA, fx, fy, code, cn);
  } else if (role == 2) {
    int idx = w * 256 + threadIdx.x;
    if (idx < a.n_band) band_cell<ST>(a, a.band[idx]);
  }
}

// ---- IBM: multi-direct forcing (Sec. 2.2), one workgroup per body ----------
// Two kernels per finest substep k of every body:
//  * ibm_prep_kernel builds the plan of substep k one substep ahead.  It
//    needs only the prescribed kinematics and the block map: marker
//    positions, desired velocities and Peskin weights (Eqs. (13), (14)), the
//    IBM window, the compact list of stencil cells with the blocks their
//    streaming sources lie in, and for every stencil cell the markers whose
//    stencil covers it, in ascending marker index (CSR).
//  * mdf_kernel runs the forcing loop of substep k on that plan: cell
//    moments, N_F iterations of interpolation (Eq. (12)), boundary force
//    (Eq. (11)) and spreading (Eq. (15)), with the moments and the marker
//    tables in LDS and each stencil cell's force in its owner's registers,
//    then the force density for the collision and the body force (Eq. (16)).
// Plans live in plan_mask + 1 buffers (index k & plan_mask), and so do the
// window and its force density that the collision of substep k reads: one
// launch builds the plans of all finest substeps of a coarse step.
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

// log cosh x without the overflow of cosh: |x| - log 2 + log1p(e^-2|x|).
__device__ __forceinline__ double log_cosh(double x) {
#pragma clang fp contract(off)
  const double a = fabs(x);
  return a - 0.69314718055994530942 + log1p(exp(-2.0 * a));
}

// Pitch angle at nondimensional time ts (= k U_ref / c) of the moving kinds.
//  FLAP (Sec. 3.6): alpha0 - A_pitch sin(2 pi ts / T + phi).
//  RAMP (Sec. 3.5): A G(ts) / sup G with Eldredge's smoothing
//    G = log cosh(a_s (ts - t1)) - log cosh(a_s (ts - t2)) + a_s (t2 - t1),
//    t2 = t1 + A / (2K), sup G = 2 a_s (t2 - t1); p = {x0, y0, A, a_s, K, t1}.
//  TRI (Sec. 3.6, E5): period T of two straight ramps (rates r1 > 0, r2 < 0)
//    blended into the extremes +-alpha0 by quartics of duration ta on both
//    sides of t2 = xi T / 2 and t5 = T (1 - xi / 2); p = {x0, y0, alpha0, xi,
//    T, ta / T}.  Every blend is r (s^3 / ta^2 +- s^4 / (2 ta^3)) away from the
//    extreme, s = t - t_extreme, which keeps alpha and its rate continuous.
__device__ __forceinline__ double pitch_angle(const CaseDev &cp, double ts) {
#pragma clang fp contract(off)
  const double *p = cp.bp;
  if (cp.body_kind == 1) return p[2] - p[3] * sin(2.0 * M_PI * ts / p[6] + p[7]);
  if (cp.body_kind == 3) {
    const double A = p[2], as = p[3];
    const double t1 = p[5], t2 = t1 + A / (2.0 * p[4]);
    const double g = log_cosh(as * (ts - t1)) - log_cosh(as * (ts - t2)) - as * (t1 - t2);
    return A * g / (2.0 * as * (t2 - t1));
  }
  // kind 4
  const double a0 = p[2], xi = p[3], T = p[4], ta = p[5] * p[4];
  const double r1 = 2.0 * a0 / (xi * T - ta);
  const double r2 = -2.0 * a0 / ((1.0 - xi) * T - ta);
  const double te = 0.5 * xi * T;            // +alpha0
  const double tm = T * (1.0 - 0.5 * xi);    // -alpha0
  double t = fmod(ts, T);
  if (t < 0.0) t += T;
  if (t < te - ta) return r1 * t;
  if (t >= tm + ta) return r1 * (t - T);
  if (t >= te + ta && t < tm - ta) return r2 * (t - (tm - ta)) - r2 * ta / 2.0 - a0;
  // one of the four blends: extreme e, incoming/outgoing rate r, sign of s^4
  const bool up = t < te + ta;
  const double s = t - (up ? te : tm);
  const double r = (up ? (s < 0.0 ? r1 : r2) : (s < 0.0 ? r2 : r1));
  const double q = s < 0.0 ? 1.0 : -1.0;
  const double ta2 = ta * ta, ta3 = ta2 * ta;
  return q * r / (2.0 * ta3) * s * s * s * s + r / ta2 * s * s * s + (up ? a0 : -a0);
}

__device__ Pose body_pose(const CaseDev &cp, double k) {
#pragma clang fp contract(off)
  const double *p = cp.bp;
  Pose r;
  r.xc = p[0];
  r.yc = p[1];
  if (cp.body_kind == 0) {
    r.ca = 1.0;
    r.sa = 0.0;
    return r;
  }
  const double tstar = k * p[8] / p[9];
  const double alpha = pitch_angle(cp, tstar);
  if (cp.body_kind == 1) {  // plunge along the stroke angle
    const double h = 0.5 * p[4] * cos(2.0 * M_PI * tstar / p[6]);
    r.xc = p[0] + h * cos(p[5]);
    r.yc = p[1] + h * sin(p[5]);
  }
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

// Plan buffer b of a case: element offsets of its arrays.
struct PlanView {
  int32_t *i0, *j0;      // first tap of each marker
  double *w;             // [8][nm]: wx[0..3], wy[0..3]
  double *ud;            // [2][nm]: desired velocity (x, y)
  uint16_t *tap;         // [16][nm]: stencil cell of each tap (y outer, x inner)
  int32_t *cell;         // [cell_cap][8]: window index, 4 source blocks, csr start, count, 0
  uint16_t *list;        // [16 nm]: contributors of the stencil cells, CSR
  int32_t *hdr;          // [4]: stamp (low 32 bits of k), stencil cells, status, 0
};

__device__ __forceinline__ PlanView plan_view(const CaseDev &cp, int b) {
  const size_t nm = (size_t)cp.nm_cap;
  PlanView v;
  v.i0 = cp.p_ij + (size_t)b * 2 * nm;
  v.j0 = v.i0 + nm;
  v.w = cp.p_w + (size_t)b * 8 * nm;
  v.ud = cp.p_ud + (size_t)b * 2 * nm;
  v.tap = cp.p_tap + (size_t)b * 16 * nm;
  v.cell = cp.p_cell + (size_t)b * 8 * cp.cell_cap;
  v.list = cp.p_list + (size_t)b * 16 * nm;
  v.hdr = cp.phdr + 4 * b;
  return v;
}

// Plan builder.  LDS: window counters and compact indices (when the window
// fits), the stencil cells' window indices and CSR starts, the contributor
// lists while they are filled.
// Plan `item` of the launch: substep item / n_bodies of body item % n_bodies.
// The arguments come by value, as a kernel's do: taken by reference they
// cost the plan builder 4 more VGPRs (one builder per CU instead of two).
__device__ __forceinline__ void prep_item(const IbmArgs a, unsigned item) {
#pragma clang fp contract(off)
  const int64_t j = item / a.n_bodies;  // plan of the launch's j-th substep
  const CaseDev &cp = a.bodies[item % a.n_bodies];
  const int n = cp.n_markers;
  const int nm = cp.nm_cap, cap = cp.cell_cap;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  extern __shared__ int lds_i[];
  const int NMa = a.max_markers, CCa = a.cell_cap;  // LDS table sizes
  int *s_cells = lds_i;                  // [CCa] window index of stencil cell q
  int *s_start = s_cells + CCa;          // [CCa] CSR start of stencil cell q
  uint16_t *s_list = reinterpret_cast<uint16_t *>(s_start + CCa);  // [16 NMa]
  // window cells' contributor counters, two 16-bit counters per word, and
  // their compact indices (16 bits)
  uint32_t *s_cnt = reinterpret_cast<uint32_t *>(s_list + 16 * NMa);  // [(lds_window + 1) / 2]
  uint16_t *s_idx = reinterpret_cast<uint16_t *>(s_cnt + (a.lds_window + 1) / 2);  // [lds_window]
  __shared__ int s_box[4];
  __shared__ int s_ns, s_bad;
  __shared__ int s_wsum[MDF_THREADS / 64];
  __shared__ Pose s_pose[2];
  // the forcing loop of substep kcount runs next, in stream order after this
#ifdef SBT_PERSISTENT_TU
  const int64_t k = ld_fresh(cp.kcount) + j;  // written earlier in the same launch
#else
  const int64_t k = *cp.kcount + j;
#endif
  const int b = (int)(k & cp.plan_mask);
  const PlanView P = plan_view(cp, b);

  // 1. kinematics: r_j(t_k), desired velocity (r_j(t_k+1) - r_j(t_k)) / dt,
  //    and the Peskin weights of the marker's 4x4 stencil
  if (tid == 0) {
    s_box[0] = 1 << 30; s_box[1] = 1 << 30; s_box[2] = -(1 << 30); s_box[3] = -(1 << 30);
    s_ns = 0;
    s_bad = 0;
    s_pose[0] = body_pose(cp, (double)k);
  } else if (tid == 64) {
    s_pose[1] = body_pose(cp, (double)(k + 1));
  }
  __syncthreads();
  const bool own = tid < n;
  int i0 = 0, j0 = 0;
  int bx0 = 1 << 30, by0 = 1 << 30, bx1 = -(1 << 30), by1 = -(1 << 30);
  if (own) {
    double X, Y;
    if (cp.body_kind == 2) {  // caller-placed markers with given desired velocity
      X = cp.xb[tid];
      Y = cp.yb[tid];
      P.ud[tid] = cp.hud[tid];
      P.ud[nm + tid] = cp.hud[nm + tid];
    } else {
      double X1, Y1;
      marker_position(cp, s_pose[0], tid, X, Y);
      marker_position(cp, s_pose[1], tid, X1, Y1);
      P.ud[tid] = X1 - X;
      P.ud[nm + tid] = Y1 - Y;
    }
    i0 = tap0(X);
    j0 = tap0(Y);
    P.i0[tid] = i0;
    P.j0[tid] = j0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      P.w[(size_t)t * nm + tid] = peskin(i0 + t + 0.5 - X);
      P.w[(size_t)(4 + t) * nm + tid] = peskin(j0 + t + 0.5 - Y);
    }
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
    if (tid == 0) {
      IbmWindow e = {0, 0, 0, 0};
      cp.win[b] = e;
      P.hdr[0] = (int)k; P.hdr[1] = 0; P.hdr[2] = ERR_WINDOW;
    }
    return;
  }
  if (tid == 0) {
    IbmWindow w = {wx0, wy0, ww, wh};
    cp.win[b] = w;
  }
  // 2. clear the window's force density (the collision reads all of it) and
  //    the per-cell counters
  const bool in_lds = ncell <= a.lds_window;
  uint32_t *cnt = in_lds ? s_cnt : reinterpret_cast<uint32_t *>(cp.wCnt + (size_t)b * cp.win_cap);
  uint16_t *idx = in_lds ? s_idx : reinterpret_cast<uint16_t *>(cp.wIdx + (size_t)b * cp.win_cap);
  auto count_of = [&](int c) -> int { return (int)((cnt[c >> 1] >> ((c & 1) << 4)) & 0xffffu); };
  {
    double *F = cp.wF + (size_t)b * 2 * cp.win_cap;
    for (int c = tid; c < ncell; c += MDF_THREADS) {
      F[c] = 0.0;
      F[(size_t)cp.win_cap + c] = 0.0;
    }
    for (int w = tid; w < (ncell + 1) / 2; w += MDF_THREADS) cnt[w] = 0u;
  }
  __syncthreads();
  // 3. every marker lane registers its 16 taps: its slot in each cell's
  //    contributor list, and the first toucher of a cell appends the cell
  //    to the compact list (a wavefront prefix sum sizes the append).
  //    cidx(t): window index of tap t; pos(t): its slot in that cell's
  //    contributor list (16 bits, two per word)
  auto cidx = [&](int t) { return (j0 + (t >> 2) - wy0) * ww + (i0 + (t & 3) - wx0); };
  uint32_t pos2[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  auto pos = [&](int t) { return (int)((pos2[t >> 1] >> ((t & 1) << 4)) & 0xffffu); };
  {
    int nf = 0;
    if (own) {
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int c = cidx(t), sh = (c & 1) << 4;  // counts stay below 2^16 (at most one per marker)
        const uint32_t p = (atomicAdd(&cnt[c >> 1], 1u << sh) >> sh) & 0xffffu;
        if (t & 1) pos2[t >> 1] |= p << 16;
        else pos2[t >> 1] = p;
      }
#pragma unroll
      for (int t = 0; t < 16; ++t) nf += pos(t) == 0;
    }
    int incl = nf;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    const int total = __shfl(incl, 63, 64);
    int base = 0;
    if (lane == 63 && total > 0) base = atomicAdd(&s_ns, total);
    base = __shfl(base, 63, 64);
    if (own) {
      int q = base + incl - nf;
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (pos(t) == 0) {
          if (q < cap) s_cells[q] = cidx(t);
          idx[cidx(t)] = (uint16_t)q;
          ++q;
        }
    }
  }
  __syncthreads();
  const int ns = s_ns;
  if (ns > cap) {
    if (tid == 0) {
      P.hdr[0] = (int)k; P.hdr[1] = 0; P.hdr[2] = ERR_CONTRIB;
    }
    return;
  }
  // 4. CSR starts: exclusive prefix sum of the contributor counts over the
  //    compact cells (each lane sums a contiguous run, then a block scan)
  {
    const int per = (ns + MDF_THREADS - 1) / MDF_THREADS;
    const int q0 = min(ns, tid * per), q1 = min(ns, q0 + per);
    int sum = 0;
    for (int q = q0; q < q1; ++q) sum += count_of(s_cells[q]);
    int incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += s_wsum[w];
    int run = wbase + incl - sum;
    for (int q = q0; q < q1; ++q) {
      s_start[q] = run;
      run += count_of(s_cells[q]);
    }
  }
  __syncthreads();
  // 5. fill the contributor lists (slot order is arbitrary) and the
  //    marker-side map from each tap to its stencil cell
  if (own) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int q = idx[cidx(t)];
      s_list[s_start[q] + pos(t)] = (uint16_t)tid;
      P.tap[(size_t)t * nm + tid] = (uint16_t)q;
    }
  }
  __syncthreads();
  // 6. per stencil cell: contributors in ascending marker index (the
  //    spreading sums in marker order), the blocks holding the cell and its
  //    streaming sources (the 3x3 neighbourhood spans at most 2x2 blocks,
  //    found at its corners; all must be owned finest blocks)
  for (int q = tid; q < ns; q += MDF_THREADS) {
    const int c = s_cells[q];
    const int n_c = count_of(c), st = s_start[q];
    const int gx = wx0 + c % ww, gy = wy0 + c / ww;
    uint16_t *L = s_list + st;
    uint16_t *O = P.list + st;
    if (n_c <= 16) {
      int v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = r < n_c ? (int)L[r] : 0x7fffffff;
      sort_net<16>(v);
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (r < n_c) O[r] = (uint16_t)v[r];
    } else {  // rare: more than 16 markers over one cell (insertion sort in LDS)
      for (int r = 1; r < n_c; ++r) {
        uint16_t v = L[r];
        int w = r - 1;
        while (w >= 0 && L[w] > v) {
          L[w + 1] = L[w];
          --w;
        }
        L[w + 1] = v;
      }
      for (int r = 0; r < n_c; ++r) O[r] = L[r];
    }
    const int sw = finest_block(cp, gx - 1, gy - 1), se = finest_block(cp, gx + 1, gy - 1);
    const int nw = finest_block(cp, gx - 1, gy + 1), ne = finest_block(cp, gx + 1, gy + 1);
    if (sw < 0 || se < 0 || nw < 0 || ne < 0) s_bad = 1;
    int4 r0 = {c, sw, se, nw};
    int4 r1 = {ne, st, n_c, 0};
    int4 *R = reinterpret_cast<int4 *>(P.cell + (size_t)q * 8);
    R[0] = r0;
    R[1] = r1;
  }
  __syncthreads();
  if (tid == 0) {
    P.hdr[0] = (int)k;
    P.hdr[1] = ns;
    P.hdr[2] = s_bad ? ERR_MARKER : 0;
  }
}

#ifndef SBT_PERSISTENT_TU
__global__ __launch_bounds__(MDF_THREADS, 8) void ibm_prep_kernel(IbmArgs a) { prep_item(a, blockIdx.x); }
#endif

__device__ __forceinline__ void mdf_fail(const CaseDev &cp, int *err, int code, int64_t k) {
  atomicOr(err, code);
  IbmWindow e = {0, 0, 0, 0};
  cp.win[k & cp.plan_mask] = e;
  *cp.kcount = k + 1;
}

constexpr int kCellsPerLane = 4;  // stencil cells owned per lane (cell_cap <= 4096)
#ifndef SBT_MDF_CACHED
#define SBT_MDF_CACHED 12
#endif
constexpr int kCached = SBT_MDF_CACHED;  // contributors whose weights a lane keeps in registers

// Block of the finest cell (sx, sy) inside the 3x3 neighbourhood of (gx, gy),
// from the four corner blocks of that neighbourhood.
__device__ __forceinline__ int corner_block(int gx, int gy, int sx, int sy, int sw, int se, int nw, int ne) {
  const bool west = (sx >> 4) == ((gx - 1) >> 4), south = (sy >> 4) == ((gy - 1) >> 4);
  return west ? (south ? sw : nw) : (south ? se : ne);
}

// The forcing loop of body `body` (one 1024-lane workgroup); arguments by
// value for the same reason as prep_item's.
template <int ST>
__device__ __forceinline__ void mdf_body(const MdfArgs a, unsigned body) {
#pragma clang fp contract(off)
  const CaseDev &cp = a.bodies[body];
  const int n = cp.n_markers;
  const int nm = cp.nm_cap;
  const int tid = threadIdx.x;
  const int NM = a.max_markers, CC = a.cell_cap;  // LDS table strides
  extern __shared__ __align__(16) double lds[];
  double2 *s_dF = reinterpret_cast<double2 *>(lds);  // [NM] marker force of the iteration
  double2 *s_uv = s_dF + NM;        // [CC] corrected velocity of the cell
  double *s_wx = reinterpret_cast<double *>(s_uv + CC);  // [4][NM]
  double *s_wy = s_wx + 4 * NM;     // [4][NM]
  double *s_ds = s_wy + 4 * NM;     // [NM]
  double *s_rho = s_ds + NM;        // [CC]
  double *s_fx = s_rho + CC;        // [CC] accumulated force of the cell
  double *s_fy = s_fx + CC;         // [CC]
  int *s_i0 = reinterpret_cast<int *>(s_fy + CC);  // [NM]
  int *s_j0 = s_i0 + NM;
  uint16_t *s_list = reinterpret_cast<uint16_t *>(s_j0 + NM);  // [16 NM]
  // The plan buffer is the substep's parity (known to the launcher), so the
  // plan loads below do not wait for the substep counter.
  const int b = a.parity;
  const PlanView P = plan_view(cp, b);
#ifdef SBT_PERSISTENT_TU
  // written earlier in the same launch (the persistent step)
  const int64_t k = ld_fresh(cp.kcount);
  const int4 hdr = make_int4(ld_fresh(P.hdr), ld_fresh(P.hdr + 1), ld_fresh(P.hdr + 2), ld_fresh(P.hdr + 3));
  const int32_t *wq = reinterpret_cast<const int32_t *>(cp.win + b);
  const IbmWindow win = {ld_fresh(wq), ld_fresh(wq + 1), ld_fresh(wq + 2), ld_fresh(wq + 3)};
#else
  const int64_t k = *cp.kcount;
  const int4 hdr = *reinterpret_cast<const int4 *>(P.hdr);
  const IbmWindow win = cp.win[b];
#endif
  // 1. load the plan before the header is known, all in one round: this
  //    lane's first stencil-cell record, the contributor lists (direct
  //    global->LDS copies, 16 bytes per lane) and the marker tables
  const int cap = min(cp.cell_cap, min(CC, kCellsPerLane * MDF_THREADS));
  int4 rec0[kCellsPerLane], rec1[kCellsPerLane];
  if (tid < cap) {
    const int4 *R = reinterpret_cast<const int4 *>(P.cell + (size_t)tid * 8);
    rec0[0] = R[0];
    rec1[0] = R[1];
  }
  {
    const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const char *src = reinterpret_cast<const char *>(P.list);
#pragma unroll
    for (int r = 0; r < 2; ++r) {  // 32 n bytes = 2 n vectors, n <= 1024
      const int v0 = r * MDF_THREADS + wv * 64;  // wave-uniform first vector
      if (v0 < 2 * n && v0 + lane < 2 * n)
        __builtin_amdgcn_global_load_lds(src + (size_t)(v0 + lane) * 16,
                                         (lds_void *)(reinterpret_cast<char *>(s_list) + (size_t)v0 * 16), 16, 0, 0);
    }
  }
  const bool own = tid < n;
  double wxr[4] = {0.0, 0.0, 0.0, 0.0}, wyr[4] = {0.0, 0.0, 0.0, 0.0};
  double udx = 0.0, udy = 0.0, dsr = 0.0;
  int i0r = 0, j0r = 0;
  uint32_t taps[8];  // stencil cells of the 16 taps, two per word
  if (own) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      wxr[t] = P.w[(size_t)t * nm + tid];
      wyr[t] = P.w[(size_t)(4 + t) * nm + tid];
    }
    udx = P.ud[tid];
    udy = P.ud[nm + tid];
#pragma unroll
    for (int t = 0; t < 8; ++t)
      taps[t] = (uint32_t)P.tap[(size_t)(2 * t) * nm + tid] | ((uint32_t)P.tap[(size_t)(2 * t + 1) * nm + tid] << 16);
    i0r = P.i0[tid];
    j0r = P.j0[tid];
    dsr = cp.ds[tid];
  }
  const int ns = hdr.y;
  int status = hdr.z;
  if (hdr.x != (int)k || (k & cp.plan_mask) != b) status = ERR_PLAN;
  if (!status && ns > cap) status = ERR_CONTRIB;
  if (status) {
    if (tid == 0) mdf_fail(cp, a.err, status, k);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // the list copies land before the LDS is released
    return;
  }
  // 2. moments of the owned stencil cells from the post-stream populations
  //    (the initial state is read in place): rho and the uncorrected
  //    velocity to LDS
  const int l = cp.n_levels - 1;
  int cxy[kCellsPerLane], csc[kCellsPerLane];  // gx | gy << 16, list start | count << 16
#pragma unroll
  for (int r = 0; r < kCellsPerLane; ++r) {
    const int q = tid + r * MDF_THREADS;
    cxy[r] = 0;
    csc[r] = 0;
    if (q < ns) {
      if (r > 0) {
        const int4 *R = reinterpret_cast<const int4 *>(P.cell + (size_t)q * 8);
        rec0[r] = R[0];
        rec1[r] = R[1];
      }
      const int4 r0 = rec0[r], r1 = rec1[r];
      const int c = r0.x;
      const int gx = win.x0 + c % win.w, gy = win.y0 + c / win.w;
      cxy[r] = gx | (gy << 16);
      csc[r] = r1.y | (r1.z << 16);
      double f[9];
      if (a.first) {
        const int ob = corner_block(gx, gy, gx, gy, r0.y, r0.z, r0.w, r1.x);
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = (double)ldv<ST>(a.src, ob, i, (gy & 15) * 16 + (gx & 15));
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          const int sx = gx - CX[i], sy = gy - CY[i];
          const int nb = corner_block(gx, gy, sx, sy, r0.y, r0.z, r0.w, r1.x);
          f[i] = (double)ldv<ST>(a.src, nb, i, (sy & 15) * 16 + (sx & 15));
        }
      }
      double rho, jx, jy;
      moments64(f, rho, jx, jy);
      if constexpr (Store<ST>::kShift) rho = cp.rho0 + rho;
      s_rho[q] = rho;
      s_uv[q] = make_double2((jx + 0.5 * cp.fx[l]) / rho, (jy + 0.5 * cp.fy[l]) / rho);
      s_fx[q] = 0.0;
      s_fy[q] = 0.0;
    }
  }
  // the marker tables to LDS
  if (own) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      s_wx[t * NM + tid] = wxr[t];
      s_wy[t * NM + tid] = wyr[t];
    }
    s_i0[tid] = i0r;
    s_j0[tid] = j0r;
    s_ds[tid] = dsr;
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the list copies
  __syncthreads();
  // Loop invariants.  A marker's interpolated density (the densities do not
  // change in the loop).  A stencil cell's Peskin weights w_x w_y of its
  // first kCached contributors (ascending marker order), with the markers'
  // indices: held in registers for the lane's first cell, so such a
  // contribution of an iteration reads only the marker's force and arc
  // length (LDS); further contributors are looked up in LDS.
  double sr = 0.0;
  if (own) {
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const double py = s_wy[bb * NM + tid];
#pragma unroll
      for (int aa = 0; aa < 4; ++aa) {
        const int t = bb * 4 + aa;
        const int q = (taps[t >> 1] >> ((t & 1) * 16)) & 0xffff;
        sr += s_rho[q] * (s_wx[aa * NM + tid] * py);
      }
    }
  }
  auto weight = [&](int j, int gx, int gy) -> double {
    return s_wx[(gx - s_i0[j]) * NM + j] * s_wy[(gy - s_j0[j]) * NM + j];
  };
  const int cnt0 = tid < ns ? csc[0] >> 16 : 0;
  double cw[kCached];
  uint32_t cj[kCached / 2];
#pragma unroll
  for (int e = 0; e < kCached / 2; ++e) cj[e] = 0;
#pragma unroll
  for (int e = 0; e < kCached; ++e) {
    cw[e] = 0.0;
    if (e < cnt0) {
      const int j = s_list[(csc[0] & 0xffff) + e];
      cw[e] = weight(j, cxy[0] & 0xffff, cxy[0] >> 16);
      cj[e >> 1] |= (uint32_t)j << ((e & 1) * 16);
    }
  }
  // 3. N_F iterations: interpolate (Eq. 12), boundary force (Eq. 11),
  //    spread (Eq. 15), correct velocity and accumulate force
  double ftx = 0.0, fty = 0.0;
  for (int it = 0; it < cp.mdf_iters; ++it) {
    if (own) {
      double su = 0.0, sv = 0.0;
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const double py = s_wy[bb * NM + tid];
#pragma unroll
        for (int aa = 0; aa < 4; ++aa) {
          const int t = bb * 4 + aa;
          const int q = (taps[t >> 1] >> ((t & 1) * 16)) & 0xffff;
          const double w = s_wx[aa * NM + tid] * py;
          const double2 uv = s_uv[q];
          su += uv.x * w;
          sv += uv.y * w;
        }
      }
      const double gx = 2.0 * sr * (udx - su);
      const double gy = 2.0 * sr * (udy - sv);
      s_dF[tid] = make_double2(gx, gy);
      ftx += gx;
      fty += gy;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kCellsPerLane; ++r) {
      const int q = tid + r * MDF_THREADS;
      if (q < ns) {
        double dfx = 0.0, dfy = 0.0;
        if (r == 0) {
#pragma unroll
          for (int e = 0; e < kCached; ++e)
            if (e < cnt0) {
              const int j = (cj[e >> 1] >> ((e & 1) * 16)) & 0xffff;
              const double2 d = s_dF[j];
              const double dsj = s_ds[j];
              dfx += d.x * cw[e] * dsj;
              dfy += d.y * cw[e] * dsj;
            }
          // contributors beyond the cached ones, in the same ascending order
          const int gx = cxy[0] & 0xffff, gy = cxy[0] >> 16, st = csc[0] & 0xffff;
          for (int e = kCached; e < cnt0; ++e) {
            const int j = s_list[st + e];
            const double2 d = s_dF[j];
            const double w = weight(j, gx, gy), dsj = s_ds[j];
            dfx += d.x * w * dsj;
            dfy += d.y * w * dsj;
          }
        } else {  // a lane's further cells
          const int gx = cxy[r] & 0xffff, gy = cxy[r] >> 16;
          const int st = csc[r] & 0xffff, cnt = csc[r] >> 16;
          for (int e = 0; e < cnt; ++e) {
            const int j = s_list[st + e];
            const double2 d = s_dF[j];
            const double w = weight(j, gx, gy), dsj = s_ds[j];
            dfx += d.x * w * dsj;
            dfy += d.y * w * dsj;
          }
        }
        s_fx[q] = s_fx[q] + dfx;
        s_fy[q] = s_fy[q] + dfy;
        const double r2 = 2.0 * s_rho[q];
        const double2 uv = s_uv[q];
        s_uv[q] = make_double2(uv.x + dfx / r2, uv.y + dfy / r2);
      }
    }
    __syncthreads();
  }
  // 4. body force of Eq. (16) summed in marker order by the last two lanes
  //    (their wave rarely owns markers or cells), while the other lanes
  //    write the force density of the stencil cells and the total marker
  //    forces
  if (own) s_dF[tid] = make_double2(ftx * s_ds[tid], fty * s_ds[tid]);
  __syncthreads();
  if (tid >= MDF_THREADS - 2) {
    // the x sum on the second-to-last lane and the y sum on the last: one
    // instruction stream carries both serial chains
    const int comp = tid & 1;
    const double *v = reinterpret_cast<const double *>(s_dF) + comp;
    double fs = 0.0;
    int j = 0;
    for (; j + 16 <= n; j += 16) {
      double t[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) t[r] = v[2 * (j + r)];
#pragma unroll
      for (int r = 0; r < 16; ++r) fs -= t[r];
    }
    for (; j < n; ++j) fs -= v[2 * j];
    const int64_t slot = k % cp.hist_cap;
    cp.hist[2 * slot + comp] = fs;
  }
  {
    double *F = cp.wF + (size_t)b * 2 * cp.win_cap;
#pragma unroll
    for (int r = 0; r < kCellsPerLane; ++r)
      if (tid + r * MDF_THREADS < ns) {
        const int wi = ((cxy[r] >> 16) - win.y0) * win.w + ((cxy[r] & 0xffff) - win.x0);
        F[wi] = s_fx[tid + r * MDF_THREADS];
        F[(size_t)cp.win_cap + wi] = s_fy[tid + r * MDF_THREADS];
      }
  }
  if (own) {
    double *gtx = cp.ftot + (size_t)(k & 1) * 2 * n;
    gtx[tid] = ftx;
    gtx[n + tid] = fty;
  }
  if (tid == 0) *cp.kcount = k + 1;
}

#ifndef SBT_PERSISTENT_TU
template <int ST>
__global__ __launch_bounds__(MDF_THREADS) void mdf_kernel(MdfArgs a) { mdf_body<ST>(a, blockIdx.x); }
#endif

#ifdef SBT_PERSISTENT_TU
// ---- the persistent step ----------------------------------------------------
// Compiled in a module of its own (sbt_persist.hip includes this file with
// SBT_PERSISTENT_TU defined and keeps only this part and its launchers): a
// kernel that runs the plan builder and the forcing loop next to their own
// kernels in one module would change how those kernels address their LDS.
// One launch runs a whole step: the phase table holds the plan builder, the
// forcing loops and the level substeps in the order of the launch chain, and
// a grid barrier separates consecutive phases (every workgroup resident).
// Level substeps go through the generic per-cell path, four blocks at a
// time per workgroup (one per 256 lanes), which needs no workgroup barrier;
// the plan builder and the forcing loop use all 1024 lanes as in their own
// launches.

// Grid barrier number `idx` (1, 2, ...) of the launch: bar[0] counts
// arrivals, so it is passed when bar[0] >= idx * gridDim.x.  The release
// makes this workgroup's writes visible at agent scope and the acquire
// invalidates what this CU cached before.  A wait of `spins` polls without
// the barrier passing raises ERR_BARRIER and sets bar[1], which ends every
// other wait.  Returns false when the launch is aborted.
__device__ bool grid_barrier(uint32_t *bar, uint32_t idx, int32_t *err, uint32_t spins_max) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t target = idx * gridDim.x;
    uint32_t spins = 0;
    while (__hip_atomic_load(&bar[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        ok = 0;
        break;
      }
      if (++spins >= spins_max) {
        atomicOr(err, ERR_BARRIER);
        __hip_atomic_store(&bar[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

template <int ST>
__device__ __forceinline__ void level_phase(const PPhase &P) {
  const LevelArgs &a = P.lv;
  const int sub = threadIdx.x >> 8, cell = threadIdx.x & 255;
  const int n_blk = P.n_list + P.n_solid;
  const int n_work = n_blk + (a.n_band + 255) / 256;
  for (int base = blockIdx.x * 4; base < n_work; base += gridDim.x * 4) {
    const int i = base + sub;  // uniform over the 4 waves of this quarter
    if (i < n_blk) {
      const int b = __builtin_amdgcn_readfirstlane(i < P.n_list ? a.list[i] : P.solid[i - P.n_list]);
      const Blk k = load_blk(a.meta, b);
      const CaseDev &cp = a.cases[k.cid];
      const bool slow = (k.flags & (BF_CODES | BF_EDGE | BF_SOLID)) != 0;
      double part[3] = {0.0, 0.0, 0.0};
      level_cell<ST>(a, k, cell, cp, slow, part);
    } else if (i < n_work) {
      const int idx = (i - n_blk) * 256 + cell;
      if (idx < a.n_band) band_cell<ST>(a, a.band[idx]);
    }
  }
}

template <int ST>
__global__ __launch_bounds__(MDF_THREADS) void step_persistent_kernel(const PPhase *__restrict__ ph, int n_ph,
                                                                      uint32_t *bar, int32_t *err, uint32_t spins) {
  bool ok = true;
  for (int p = 0; p < n_ph && ok; ++p) {
    const PPhase &P = ph[p];
    if (P.type == PP_PREP) {
      for (unsigned it = blockIdx.x; it < (unsigned)P.n_items; it += gridDim.x) {
        prep_item(P.ibm, it);
        __syncthreads();
      }
    } else if (P.type == PP_MDF) {
      for (unsigned it = blockIdx.x; it < (unsigned)P.n_items; it += gridDim.x) {
        mdf_body<ST & 3>(P.mdf, it);
        __syncthreads();
      }
    } else {
      level_phase<ST>(P);
    }
    if (p + 1 < n_ph) ok = grid_barrier(bar, (uint32_t)(p + 1), err, spins);
  }
  // the last workgroup out puts the barrier state back to zero for the next
  // launch (every other workgroup has passed its last barrier)
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t done = __hip_atomic_fetch_add(&bar[2], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (done == gridDim.x - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&bar[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&bar[2], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

#endif  // SBT_PERSISTENT_TU

#ifndef SBT_PERSISTENT_TU
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

#endif  // !SBT_PERSISTENT_TU

}  // namespace

#ifndef SBT_PERSISTENT_TU
extern "C" hipError_t sbt_launch_level_tile(int storage, const LevelArgs *a, hipStream_t s) {
  if (a->kpw < 1) return hipErrorInvalidValue;
  const bool pipe = a->kpw > 1;
  const int kpw = pipe ? a->kpw : 1;
  const int n_run = (a->n_fast + kpw - 1) / kpw, n_blk = a->n_blocks - a->n_fast, n_bnd = (a->n_band + 255) / 256;
  int groups = n_run + n_blk + n_bnd;
  if (groups <= 0) return hipSuccess;
  if (a->xcd_remap) {  // 8 x the largest per-XCD share (see tile_role)
    int most = 0;
    for (int x = 0; x < 8; ++x) {
      int c = (n_run * (x + 1) / 8 - n_run * x / 8) + (n_blk * (x + 1) / 8 - n_blk * x / 8) +
              (n_bnd * (x + 1) / 8 - n_bnd * x / 8);
      most = c > most ? c : most;
    }
    groups = 8 * most;
  }
  dim3 grid(groups);
#define SBT_TILE_LAUNCH(S)                                                               \
  if (pipe) hipLaunchKernelGGL((level_tile_kernel<S, 2>), grid, dim3(256), 0, s, *a, a->cases, a->meta, a->list); \
  else hipLaunchKernelGGL((level_tile_kernel<S, 1>), grid, dim3(256), 0, s, *a, a->cases, a->meta, a->list);
  switch (storage) {
    case 0: SBT_TILE_LAUNCH(0); break;
    case 1: SBT_TILE_LAUNCH(1); break;
    case 2: SBT_TILE_LAUNCH(2); break;
    case 3: SBT_TILE_LAUNCH(3); break;
    case 4: SBT_TILE_LAUNCH(4); break;
    case 5: SBT_TILE_LAUNCH(5); break;
    case 6: SBT_TILE_LAUNCH(6); break;
    case 7: SBT_TILE_LAUNCH(7); break;
    default: return hipErrorInvalidValue;
  }
#undef SBT_TILE_LAUNCH
  return hipGetLastError();
}

extern "C" hipError_t sbt_launch_level(int storage, int tile, const LevelArgs *a, hipStream_t s) {
  switch (storage) {
    case 0: return launch_level_st<0>(tile, a, s);
    case 1: return launch_level_st<1>(tile, a, s);
    case 2: return launch_level_st<2>(tile, a, s);
    case 3: return launch_level_st<3>(tile, a, s);
    case 4: return launch_level_st<4>(tile, a, s);
    case 5: return launch_level_st<5>(tile, a, s);
    case 6: return launch_level_st<6>(tile, a, s);
    case 7: return launch_level_st<7>(tile, a, s);
  }
  return hipErrorInvalidValue;
}

extern "C" size_t sbt_mdf_lds_bytes(int max_markers, int cell_cap) {
  return (size_t)max_markers * (11 * sizeof(double) + 2 * sizeof(int) + 16 * sizeof(uint16_t)) +
         (size_t)cell_cap * 5 * sizeof(double);
}

extern "C" size_t sbt_prep_lds_bytes(int max_markers, int cell_cap, int lds_window) {
  return (size_t)cell_cap * 2 * sizeof(int) + (size_t)max_markers * 16 * sizeof(uint16_t) +
         (size_t)(lds_window + 1) / 2 * sizeof(uint32_t) + (size_t)lds_window * sizeof(uint16_t);
}

extern "C" hipError_t sbt_launch_ibm_prep(const IbmArgs *a, hipStream_t s) {
  if (a->n_bodies <= 0 || a->n_plans <= 0) return hipSuccess;
  size_t lds = sbt_prep_lds_bytes(a->max_markers, a->cell_cap, a->lds_window);
  hipLaunchKernelGGL(ibm_prep_kernel, dim3(a->n_bodies * a->n_plans), dim3(MDF_THREADS), lds, s, *a);
  return hipGetLastError();
}

extern "C" hipError_t sbt_launch_mdf(int storage, const MdfArgs *a, int n_bodies, hipStream_t s) {
  if (n_bodies <= 0) return hipSuccess;
  size_t lds = sbt_mdf_lds_bytes(a->max_markers, a->cell_cap);
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
#endif  // !SBT_PERSISTENT_TU

#ifdef SBT_PERSISTENT_TU
#define SBT_PERSIST_CASES(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)

extern "C" hipError_t sbt_launch_step_persistent(int storage, const PPhase *ph, int n_ph, uint32_t *bar, int32_t *err,
                                                 uint32_t spins, int groups, size_t lds_bytes, hipStream_t s) {
  if (n_ph <= 0 || groups <= 0) return hipSuccess;
  switch (storage) {
#define SBT_P(S)                                                                                              \
  case S:                                                                                                     \
    hipLaunchKernelGGL((step_persistent_kernel<S>), dim3(groups), dim3(MDF_THREADS), lds_bytes, s, ph, n_ph, bar, err, spins); \
    break;
    SBT_PERSIST_CASES(SBT_P)
#undef SBT_P
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

extern "C" int sbt_step_persistent_occupancy(int storage, size_t lds_bytes) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (storage) {
#define SBT_P(S)                                                                                              \
  case S:                                                                                                     \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_persistent_kernel<S>, MDF_THREADS, lds_bytes); \
    break;
    SBT_PERSIST_CASES(SBT_P)
#undef SBT_P
    default: break;
  }
  return e == hipSuccess ? n : 0;
}
#endif  // SBT_PERSISTENT_TU
