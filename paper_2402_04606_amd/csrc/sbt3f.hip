// The 3D block forest (Sec. 2.3-2.4 with the D3Q19 / D3Q27 lattices, fully
// periodic) on gfx950.
//
// Layout in HBM: per level a pool of 8^3-cell blocks -- first the blocks
// holding owned cells (Morton order), then the halo blocks -- with two
// lattices [block][Q][512] in the storage type (cell = (z * 8 + y) * 8 + x),
// a block table (origin, the 26 neighbours and the block itself, the 8 finer
// blocks under its octants) and one 32-bit code per cell for the blocks
// that need one (hidden cells, hidden sources, interface and halo cells).
//
// One launch per level substep, two workgroups per block (one per 4 z-planes), one thread per
// cell, pull scheme (as the 2D level kernel): a lattice holds f*; a launch
// gathers f(x, i) = f*(x - c_i, i) through the neighbour table, replaces the
// populations whose source is hidden by the mean over the cell's 8 children
// of the finer level's post-stream values (coalescence on read, from the
// finer lattice its last substep read), collides (BGK + Guo, half-force
// velocity) and stores f*; an owned cell with halo children also writes its
// f* into them in the finer lattice its next substep reads (explosion).  In
// the first of a fine level's two substeps the halo blocks gather their halo
// cells (never collided): what the second substep pulls from them is then
// their own post-stream value.  HBM-bound: 2 Q s bytes per cell update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "lattice3.h"
#include "sbt3f.h"
#include "sbt_internal.h"

namespace {

constexpr int kB3 = 8;                    // block edge
constexpr int kC3 = kB3 * kB3 * kB3;      // cells per block (one workgroup)
constexpr int kMaxLev3 = 6;
constexpr int kWG3 = kC3 / 2;             // lanes per workgroup: half a block (4 z-planes)

// Per-cell codes.
enum : uint32_t {
  K3_HSRC = (1u << 27) - 1u,  // bit i: the source x - c_i is hidden (covered by the finer level)
  K3_HIDDEN = 1u << 27,       // the cell itself is hidden
  K3_IFACE = 1u << 28,        // owned cell with halo children: explodes into them
  K3_BAND = 1u << 29,         // halo block: the cell is a halo cell
};
enum : int32_t { B3_GHOST = 1 };
enum : int32_t { M3_LOCAL = 1, M3_READOUT = 2 };

struct alignas(16) Blk3 {
  int32_t ox, oy, oz;   // origin, cells of the block's level
  int32_t flags;        // B3_GHOST: halo block
  int32_t code;         // row of the per-cell code table, or -1 (all cells owned, no hidden source)
  int32_t nbr[27];      // pool blocks at block offsets (dx, dy, dz): index (dx+1) + 3 (dy+1) + 9 (dz+1); -1 none
  int32_t child[8];     // finer pool's blocks under octant (x >= 4) + 2 (y >= 4) + 4 (z >= 4); -1 none
};
static_assert(sizeof(Blk3) == 160, "block table entries stay 160 bytes");
constexpr int kBlkInts = (int)(sizeof(Blk3) / 4);

struct Lev3 {
  double tau, pre, rho0, F[3];
  double s_cf;   // explosion into the next finer level
  double s_fc;   // coalescence from the next finer level
  float om_f, pre_f, rho0_f, F_f[3], s_cf_f, s_fc_f;
  int32_t rescale;
};

struct Args3 {
  const Blk3 *meta;
  const uint32_t *codes;
  const void *src;      // lattice read
  void *dst;            // lattice written
  const Blk3 *fmeta;    // next finer pool, or null
  const void *fprev;    // its lattice read by its last substep (coalescence)
  void *fcur;           // its lattice its next substep reads (explosion)
  const int32_t *list;  // pool blocks of the launch
  int32_t n_blocks;     // list entries
  int32_t n_fast;       // leading list entries taking the interior path (step launches)
  const int32_t *band;  // halo cells gathered in the launch (block * 512 + cell), after the blocks
  int32_t n_band;
  int32_t mode;
  int32_t xcd;
  int32_t off32;        // the lattice read is under 4 GiB: 32-bit byte offsets
  Lev3 L;
  double *out;          // readout [n][4][512]: rho, ux, uy, uz
  double *part;         // readout [2 n][4]: mass, jx, jy, jz of the owned cells of each half block
  int32_t *err;
};

// Work item of workgroup bid: an entry of the launch's sequence [interior
// blocks (n_fast) | other blocks | groups of 512 halo cells] (n entries), or
// -1.  Workgroups go to the 8 XCDs round-robin; XCD x takes the x-th eighth
// of the entries after the interior blocks (interface blocks and halo
// groups: latency-bound, so they start first and are spread over all XCDs)
// and then the x-th eighth of the interior blocks (contiguous in Morton
// order, so neighbour reads stay in its own L2).  Without the remap the
// entry is bid.
__device__ __forceinline__ int remap3(int bid, int n, int n_fast, int enable) {
  if (!enable) return bid < n ? bid : -1;
  const int x = bid & 7, k = bid >> 3, ns = n - n_fast;
  const int s0 = ns * x / 8, s1 = ns * (x + 1) / 8;
  if (k < s1 - s0) return n_fast + s0 + k;
  const int k2 = k - (s1 - s0);
  const int r0 = n_fast * x / 8, r1 = n_fast * (x + 1) / 8;
  return k2 < r1 - r0 ? r0 + k2 : -1;
}

__device__ __forceinline__ int nbr_slot(int sx, int sy, int sz) {
  const int ix = sx < 0 ? 0 : (sx >= kB3 ? 2 : 1);
  const int iy = sy < 0 ? 0 : (sy >= kB3 ? 2 : 1);
  const int iz = sz < 0 ? 0 : (sz >= kB3 ? 2 : 1);
  return ix + 3 * iy + 9 * iz;
}

__device__ __forceinline__ int wrap_cell(int sx, int sy, int sz) {
  return (((sz & 7) * kB3) + (sy & 7)) * kB3 + (sx & 7);
}

template <int ST> using Calc3 = std::conditional_t<ST == 0, double, float>;

// Mean over the 8 children g of coarse cell (x, y, z) of the finer level's
// post-stream value f(g, i) = f*(g - c_i, i) (coalescence, step (6) of Sec.
// 2.4), children in z, y, x order.
template <int ST, int Q>
__device__ __forceinline__ Calc3<ST> coalesce3(const Args3 &a, const Blk3 &k, const int32_t (*cnb)[27], int x, int y,
                                               int z, int i) {
#pragma clang fp contract(off)
  using S = Store3<ST>;
  using T = typename S::T;
  using C = Calc3<ST>;
  const int o = (x >> 2) + 2 * (y >> 2) + 4 * (z >> 2);
  const int cb = k.child[o];
  if (cb < 0) return C(__builtin_nan(""));
  const T *fp = static_cast<const T *>(a.fprev);
  const int fx0 = (2 * x) & 7, fy0 = (2 * y) & 7, fz0 = (2 * z) & 7;
  // the 8 loads first (an absent block reads the child block; its value is
  // replaced by NaN), then the sum in z, y, x order
  C v[8];
  bool miss[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int sx = fx0 + (c & 1) - E3X[i], sy = fy0 + ((c >> 1) & 1) - E3Y[i], sz = fz0 + (c >> 2) - E3Z[i];
    const int nb = cnb[o][nbr_slot(sx, sy, sz)];
    miss[c] = nb < 0;
    v[c] = (C)S::ld(fp[((size_t)(nb < 0 ? cb : nb) * Q + i) * kC3 + wrap_cell(sx, sy, sz)]);
  }
  C sum = C(0);
#pragma unroll
  for (int c = 0; c < 8; ++c) sum += miss[c] ? C(__builtin_nan("")) : v[c];
  return C(0.125) * sum;
}

// f^eq (Eq. (7) in 3D) of direction i in the storage frame: f itself (FP64)
// or the deviation f - w rho0 (FP32), written as the oracle's FP64 form.
template <int ST, int Q>
__device__ __forceinline__ Calc3<ST> feq3(const Lev3 &L, int i, Calc3<ST> rho, Calc3<ST> dr, Calc3<ST> ux,
                                          Calc3<ST> uy, Calc3<ST> uz, Calc3<ST> usq) {
#pragma clang fp contract(off)
  using C = Calc3<ST>;
  const C cu = E3X[i] * ux + E3Y[i] * uy + E3Z[i] * uz;
  if constexpr (ST == 0) {
    return w3<double, Q>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
  } else {
    const float A = dr - rho * (1.5f * usq);
    return w3<float, Q>(i) * fmaf(rho * cu, fmaf(4.5f, cu, 3.0f), A);
  }
}

// One cell of a level launch; part gets its mass and first moment in a
// readout.
template <int ST, int Q>
__device__ __forceinline__ void cell3(const Args3 &a, const Blk3 &k, const int32_t (*cnb)[27], int b, int w, int cell,
                                      double part[4]) {
#pragma clang fp contract(off)
  using S = Store3<ST>;
  using T = typename S::T;
  using C = Calc3<ST>;
  const int x = cell & 7, y = (cell >> 3) & 7, z = cell >> 6;
  const uint32_t code = k.code >= 0 ? a.codes[(size_t)k.code * kC3 + cell] : 0u;
  const T *src = static_cast<const T *>(a.src);
  T *dst = static_cast<T *>(a.dst);

  if (k.flags & B3_GHOST) return;  // halo blocks: their cells go through band3
  if (code & K3_HIDDEN) {
    if (a.mode & M3_READOUT) {
#pragma unroll
      for (int q = 0; q < 4; ++q) a.out[((size_t)w * 4 + q) * kC3 + cell] = __builtin_nan("");
    }
    return;
  }

  C f[Q];
  if (a.mode & M3_LOCAL) {
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = (C)S::ld(src[((size_t)b * Q + i) * kC3 + cell]);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {  // every source first (absent blocks as in the halo gather)
      const int sx = x - E3X[i], sy = y - E3Y[i], sz = z - E3Z[i];
      const int nb = k.nbr[nbr_slot(sx, sy, sz)];
      const C v = (C)S::ld(src[((size_t)(nb < 0 ? b : nb) * Q + i) * kC3 + wrap_cell(sx, sy, sz)]);
      f[i] = nb < 0 ? C(__builtin_nan("")) : v;
    }
    if (code & K3_HSRC) {  // then the coalesced populations
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (code & (1u << i)) f[i] = coalesce3<ST, Q>(a, k, cnb, x, y, z, i);
    }
    if ((code & K3_HSRC) && a.L.rescale) {  // RESCALE the coalesced populations
      C r = C(0), jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        r += f[i];
        jx += E3X[i] * f[i];
        jy += E3Y[i] * f[i];
        jz += E3Z[i] * f[i];
      }
      C dr = r;
      if constexpr (ST != 0) r = a.L.rho0_f + dr;
      const C ux = jx / r, uy = jy / r, uz = jz / r;
      const C usq = ux * ux + uy * uy + uz * uz;
      C s;
      if constexpr (ST == 0) s = a.L.s_fc;
      else s = a.L.s_fc_f;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (code & (1u << i)) {
          const C fe = feq3<ST, Q>(a.L, i, r, dr, ux, uy, uz, usq);
          f[i] = fe + s * (f[i] - fe);
        }
      }
    }
  }

  if (a.mode & M3_READOUT) {  // moments of the streamed state, FP64
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double v = (double)f[i];
      rho += v;
      jx += E3X[i] * v;
      jy += E3Y[i] * v;
      jz += E3Z[i] * v;
    }
    if constexpr (ST != 0) rho = a.L.rho0 + rho;
    a.out[((size_t)w * 4 + 0) * kC3 + cell] = rho;
    a.out[((size_t)w * 4 + 1) * kC3 + cell] = (jx + 0.5 * a.L.F[0]) / rho;
    a.out[((size_t)w * 4 + 2) * kC3 + cell] = (jy + 0.5 * a.L.F[1]) / rho;
    a.out[((size_t)w * 4 + 3) * kC3 + cell] = (jz + 0.5 * a.L.F[2]) / rho;
    part[0] = rho;
    part[1] = jx;
    part[2] = jy;
    part[3] = jz;
    return;
  }

  // BGK collision with Guo's term (Eqs. (2)-(8) in 3D).
  C rho = C(0), jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    jx += E3X[i] * f[i];
    jy += E3Y[i] * f[i];
    jz += E3Z[i] * f[i];
  }
  C ux, uy, uz, usq, dr = rho;
  if constexpr (ST == 0) {
    const double Fx = a.L.F[0], Fy = a.L.F[1], Fz = a.L.F[2];
    ux = (jx + 0.5 * Fx) / rho;
    uy = (jy + 0.5 * Fy) / rho;
    uz = (jz + 0.5 * Fz) / rho;
    usq = ux * ux + uy * uy + uz * uz;
    const double uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double cu = E3X[i] * ux + E3Y[i] * uy + E3Z[i] * uz;
      const double cF = E3X[i] * Fx + E3Y[i] * Fy + E3Z[i] * Fz;
      const double fe = w3<double, Q>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
      const double fi = w3<double, Q>(i) * a.L.pre * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF);
      f[i] = f[i] - (f[i] - fe) / a.L.tau + fi;
    }
  } else {
    rho = a.L.rho0_f + dr;
    const float ir = __builtin_amdgcn_rcpf(rho);
    const float Fx = a.L.F_f[0], Fy = a.L.F_f[1], Fz = a.L.F_f[2];
    ux = (jx + 0.5f * Fx) * ir;
    uy = (jy + 0.5f * Fy) * ir;
    uz = (jz + 0.5f * Fz) * ir;
    usq = ux * ux + uy * uy + uz * uz;
    const float A = dr - rho * (1.5f * usq);
    const bool forced = Fx != 0.f || Fy != 0.f || Fz != 0.f;
    const float uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float cu = E3X[i] * ux + E3Y[i] * uy + E3Z[i] * uz;
      const float de = w3<float, Q>(i) * fmaf(rho * cu, fmaf(4.5f, cu, 3.0f), A);
      float v = fmaf(a.L.om_f, de - f[i], f[i]);
      if (forced) {
        const float cF = E3X[i] * Fx + E3Y[i] * Fy + E3Z[i] * Fz;
        v += w3<float, Q>(i) * a.L.pre_f * (3.f * cF + 9.f * cu * cF - 3.f * uF);
      }
      f[i] = v;
    }
  }
  if (!(rho == rho) || rho > C(1e30) || rho < C(-1e30)) atomicOr(a.err, sbt::ERR_NONFINITE);
#pragma unroll
  for (int i = 0; i < Q; ++i) dst[((size_t)b * Q + i) * kC3 + cell] = S::st(f[i]);

  if (code & K3_IFACE) {  // explosion into the 8 halo children (step (2) of Sec. 2.4)
    const int cb = k.child[(x >> 2) + 2 * (y >> 2) + 4 * (z >> 2)];
    if (cb >= 0) {
      T *fd = static_cast<T *>(a.fcur);
      const int c0 = wrap_cell(2 * x, 2 * y, 2 * z);
      C s;
      if constexpr (ST == 0) s = a.L.s_cf;
      else s = a.L.s_cf_f;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        C e = f[i];
        if (a.L.rescale) {
          const C fe = feq3<ST, Q>(a.L, i, rho, dr, ux, uy, uz, usq);
          e = fe + s * (f[i] - fe);
        }
        const T v = S::st(e);
        T *row = fd + ((size_t)cb * Q + i) * kC3 + c0;
        row[0] = v;
        row[1] = v;
        row[kB3] = v;
        row[kB3 + 1] = v;
        row[kB3 * kB3] = v;
        row[kB3 * kB3 + 1] = v;
        row[kB3 * kB3 + kB3] = v;
        row[kB3 * kB3 + kB3 + 1] = v;
      }
    }
  }
}

typedef __attribute__((address_space(4))) const int32_t ci32_3;

// Interior block (no per-cell code: every cell owned, every source in the
// pool): the straight-line gather + collide.  The neighbour indices come
// through scalar loads; each lane picks its source block per direction with
// selects among the (at most 8) candidates the direction can reach, so the Q
// loads issue back to back.
template <int ST, int Q, bool O32>
__device__ __forceinline__ void interior3(const Args3 &a, int b, int cell) {
#pragma clang fp contract(off)
  using S = Store3<ST>;
  using T = typename S::T;
  using C = Calc3<ST>;
  ci32_3 *nbp = (ci32_3 *)(a.meta + b) + 5;   // Blk3::nbr, 27 scalar loads
  int nb[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) nb[k] = __builtin_amdgcn_readfirstlane(nbp[k]);
  const int x = cell & 7, y = (cell >> 3) & 7, z = cell >> 6;
  const T *src = static_cast<const T *>(a.src);
  T *dst = static_cast<T *>(a.dst);
  C f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = E3X[i], cy = E3Y[i], cz = E3Z[i];
    // the lane's source leaves the block along an axis only at one face
    const bool ox = cx != 0 && x == (cx > 0 ? 0 : 7);
    const bool oy = cy != 0 && y == (cy > 0 ? 0 : 7);
    const bool oz = cz != 0 && z == (cz > 0 ? 0 : 7);
    // select among the candidates of this direction (compile-time slots)
    const int s0 = 13, sx = -cx, sy = -3 * cy, sz = -9 * cz;
    const int p00 = ox ? nb[s0 + sx] : nb[s0];
    const int p10 = ox ? nb[s0 + sx + sy] : nb[s0 + sy];
    const int p01 = ox ? nb[s0 + sx + sz] : nb[s0 + sz];
    const int p11 = ox ? nb[s0 + sx + sy + sz] : nb[s0 + sy + sz];
    const int q0 = oy ? p10 : p00, q1 = oy ? p11 : p01;
    const int blk = oz ? q1 : q0;
    const uint32_t off = ((uint32_t)blk * Q + i) * kC3 + (uint32_t)wrap_cell(x - cx, y - cy, z - cz);
    if constexpr (O32)  // pool under 4 GiB: a 32-bit byte offset from the scalar base, one VGPR per load
      f[i] = (C)S::ld(*reinterpret_cast<const T *>(reinterpret_cast<const char *>(src) + off * (uint32_t)sizeof(T)));
    else
      f[i] = (C)S::ld(src[off]);
  }
  C rho = C(0), jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    jx += E3X[i] * f[i];
    jy += E3Y[i] * f[i];
    jz += E3Z[i] * f[i];
  }
  if constexpr (ST == 0) {
    const double Fx = a.L.F[0], Fy = a.L.F[1], Fz = a.L.F[2];
    const double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho, uz = (jz + 0.5 * Fz) / rho;
    const double usq = ux * ux + uy * uy + uz * uz;
    const double uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double cu = E3X[i] * ux + E3Y[i] * uy + E3Z[i] * uz;
      const double cF = E3X[i] * Fx + E3Y[i] * Fy + E3Z[i] * Fz;
      const double fe = w3<double, Q>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
      const double fi = w3<double, Q>(i) * a.L.pre * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF);
      f[i] = f[i] - (f[i] - fe) / a.L.tau + fi;
    }
  } else {
    const float dr = rho;
    rho = a.L.rho0_f + dr;
    const float ir = __builtin_amdgcn_rcpf(rho);
    const float Fx = a.L.F_f[0], Fy = a.L.F_f[1], Fz = a.L.F_f[2];
    const float ux = (jx + 0.5f * Fx) * ir, uy = (jy + 0.5f * Fy) * ir, uz = (jz + 0.5f * Fz) * ir;
    const float usq = ux * ux + uy * uy + uz * uz;
    const float A = dr - rho * (1.5f * usq);
    const bool forced = Fx != 0.f || Fy != 0.f || Fz != 0.f;
    const float uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const float cu = E3X[i] * ux + E3Y[i] * uy + E3Z[i] * uz;
      const float de = w3<float, Q>(i) * fmaf(rho * cu, fmaf(4.5f, cu, 3.0f), A);
      float v = fmaf(a.L.om_f, de - f[i], f[i]);
      if (forced) {
        const float cF = E3X[i] * Fx + E3Y[i] * Fy + E3Z[i] * Fz;
        v += w3<float, Q>(i) * a.L.pre_f * (3.f * cF + 9.f * cu * cF - 3.f * uF);
      }
      f[i] = v;
    }
  }
  if (!(rho == rho) || rho > C(1e30) || rho < C(-1e30)) atomicOr(a.err, sbt::ERR_NONFINITE);
#pragma unroll
  for (int i = 0; i < Q; ++i) dst[((size_t)b * Q + i) * kC3 + cell] = S::st(f[i]);
}

// A halo cell of the level (first of a fine level's two substeps): streamed,
// never collided; a source outside the level's blocks gives NaN.
template <int ST, int Q>
__device__ __forceinline__ void band3(const Args3 &a, int packed) {
  using S = Store3<ST>;
  using T = typename S::T;
  using C = Calc3<ST>;
  const int b = packed >> 9, cell = packed & (kC3 - 1);
  const int x = cell & 7, y = (cell >> 3) & 7, z = cell >> 6;
  const T *src = static_cast<const T *>(a.src);
  T *dst = static_cast<T *>(a.dst);
  const int32_t *nbr = a.meta[b].nbr;
  int nb[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) nb[i] = nbr[nbr_slot(x - E3X[i], y - E3Y[i], z - E3Z[i])];
  T g[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {  // an absent block reads the cell's own block; NaN replaces the value
    const T v = src[((size_t)(nb[i] < 0 ? b : nb[i]) * Q + i) * kC3 + wrap_cell(x - E3X[i], y - E3Y[i], z - E3Z[i])];
    g[i] = nb[i] < 0 ? S::st(C(__builtin_nan(""))) : v;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) dst[((size_t)b * Q + i) * kC3 + cell] = g[i];
}

// MODE: 0 step (interior blocks first, then the rest, then halo cells),
// M3_LOCAL, M3_READOUT or both.
template <int ST, int Q, int MODE>
__global__ __launch_bounds__(kWG3) void forest3_kernel(Args3 a) {
  // work items: the two halves (z < 4, z >= 4) of each listed block, then
  // groups of kWG3 halo cells
  const int n_bg = (a.n_band + kWG3 - 1) / kWG3;
  const int w2 = remap3(blockIdx.x, 2 * a.n_blocks + n_bg, 2 * a.n_fast, a.xcd);
  if (w2 < 0) return;
  if (w2 >= 2 * a.n_blocks) {
    const int idx = (w2 - 2 * a.n_blocks) * kWG3 + threadIdx.x;
    if (idx < a.n_band) band3<ST, Q>(a, a.band[idx]);
    return;
  }
  const int w = w2 >> 1;
  const int cell = (w2 & 1) * kWG3 + threadIdx.x;
  const int b = __builtin_amdgcn_readfirstlane(a.list[w]);
  if constexpr (MODE == 0) {
    if (w < a.n_fast) {
      if (a.off32) interior3<ST, Q, true>(a, b, cell);
      else interior3<ST, Q, false>(a, b, cell);
      return;
    }
  }
  // the block's table and the neighbour tables of the 8 finer blocks under
  // its octants (coalescence), in LDS
  __shared__ Blk3 sk;
  __shared__ int32_t cnb[8][27];
  const int t = threadIdx.x;
  if (t < kBlkInts) reinterpret_cast<int32_t *>(&sk)[t] = reinterpret_cast<const int32_t *>(a.meta + b)[t];
  if (t < 8 * 27) {
    const int o = t / 27, sl = t % 27;
    const int cb = a.fmeta ? a.meta[b].child[o] : -1;
    cnb[o][sl] = cb >= 0 ? a.fmeta[cb].nbr[sl] : -1;
  }
  __syncthreads();
  double part[4] = {0.0, 0.0, 0.0, 0.0};
  Args3 m = a;
  m.mode = MODE;
  cell3<ST, Q>(m, sk, cnb, b, w, cell, part);
  if constexpr ((MODE & M3_READOUT) != 0) {  // fixed-order tree over the half block's cells
    __shared__ double red[4][kWG3];
#pragma unroll
    for (int q = 0; q < 4; ++q) red[q][t] = part[q];
    __syncthreads();
    for (int h = kWG3 / 2; h > 0; h >>= 1) {
      if (t < h) {
#pragma unroll
        for (int q = 0; q < 4; ++q) red[q][t] += red[q][t + h];
      }
      __syncthreads();
    }
    if (t < 4) a.part[(size_t)w2 * 4 + t] = red[t][0];
  }
}

// f = f^eq(rho, u) on the owned cells of the listed blocks from staged FP64
// fields [n][4][512] (a NaN density leaves the cell as it is), or rest at
// rho0 when fld is null.
template <int ST, int Q>
__global__ __launch_bounds__(kC3) void init3f_kernel(const int32_t *list, const Blk3 *meta, const uint32_t *codes,
                                                     void *lat_, const double *fld, Lev3 L) {
#pragma clang fp contract(off)
  using S = Store3<ST>;
  using T = typename S::T;
  const int w = blockIdx.x, cell = threadIdx.x;
  const int b = list[w];
  const int code_row = meta[b].code;
  const uint32_t code = code_row >= 0 ? codes[(size_t)code_row * kC3 + cell] : 0u;
  if (code & K3_HIDDEN) return;
  double rho = L.rho0, ux = 0.0, uy = 0.0, uz = 0.0;
  if (fld) {
    rho = fld[((size_t)w * 4 + 0) * kC3 + cell];
    if (rho != rho) return;
    ux = fld[((size_t)w * 4 + 1) * kC3 + cell];
    uy = fld[((size_t)w * 4 + 2) * kC3 + cell];
    uz = fld[((size_t)w * 4 + 3) * kC3 + cell];
  }
  T *lat = static_cast<T *>(lat_);
  const double usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double cu = E3X[i] * ux + E3Y[i] * uy + E3Z[i] * uz;
    const double fe = w3<double, Q>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    if constexpr (ST == 0) lat[((size_t)b * Q + i) * kC3 + cell] = S::st(fe);
    else lat[((size_t)b * Q + i) * kC3 + cell] = S::st((float)(fe - w3<double, Q>(i) * L.rho0));
  }
}

// Workgroups of a launch over n list entries: with the XCD remap, 8 times
// the largest share of one XCD.
int grid3(int n, int n_fast, int remap) {
  if (!remap) return n;
  int most = 0;
  for (int x = 0; x < 8; ++x) {
    const int ns = n - n_fast;
    most = std::max(most, (ns * (x + 1) / 8 - ns * x / 8) + (n_fast * (x + 1) / 8 - n_fast * x / 8));
  }
  return 8 * most;
}

template <int ST, int Q>
hipError_t launch_forest3(const Args3 &a, hipStream_t s) {
  const int n = grid3(2 * a.n_blocks + (a.n_band + kWG3 - 1) / kWG3, 2 * a.n_fast, a.xcd);
  if (n <= 0) return hipSuccess;
  switch (a.mode) {
    case 0: hipLaunchKernelGGL((forest3_kernel<ST, Q, 0>), dim3(n), dim3(kWG3), 0, s, a); break;
    case M3_LOCAL: hipLaunchKernelGGL((forest3_kernel<ST, Q, M3_LOCAL>), dim3(n), dim3(kWG3), 0, s, a); break;
    case M3_READOUT: hipLaunchKernelGGL((forest3_kernel<ST, Q, M3_READOUT>), dim3(n), dim3(kWG3), 0, s, a); break;
    default:
      hipLaunchKernelGGL((forest3_kernel<ST, Q, M3_LOCAL | M3_READOUT>), dim3(n), dim3(kWG3), 0, s, a);
  }
  return hipGetLastError();
}

template <int ST, int Q>
hipError_t launch_init3f(const int32_t *list, int n, const Blk3 *meta, const uint32_t *codes, void *lat,
                         const double *fld, const Lev3 &L, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((init3f_kernel<ST, Q>), dim3(n), dim3(kC3), 0, s, list, meta, codes, lat, fld, L);
  return hipGetLastError();
}

hipError_t forest3_dispatch(int st, int q, const Args3 &a, hipStream_t s) {
  if (q == 19) {
    switch (st) {
      case 0: return launch_forest3<0, 19>(a, s);
      case 1: return launch_forest3<1, 19>(a, s);
      case 2: return launch_forest3<2, 19>(a, s);
      default: return launch_forest3<3, 19>(a, s);
    }
  }
  switch (st) {
    case 0: return launch_forest3<0, 27>(a, s);
    case 1: return launch_forest3<1, 27>(a, s);
    case 2: return launch_forest3<2, 27>(a, s);
    default: return launch_forest3<3, 27>(a, s);
  }
}

hipError_t init3f_dispatch(int st, int q, const int32_t *list, int n, const Blk3 *meta, const uint32_t *codes,
                           void *lat, const double *fld, const Lev3 &L, hipStream_t s) {
  if (q == 19) {
    switch (st) {
      case 0: return launch_init3f<0, 19>(list, n, meta, codes, lat, fld, L, s);
      case 1: return launch_init3f<1, 19>(list, n, meta, codes, lat, fld, L, s);
      case 2: return launch_init3f<2, 19>(list, n, meta, codes, lat, fld, L, s);
      default: return launch_init3f<3, 19>(list, n, meta, codes, lat, fld, L, s);
    }
  }
  switch (st) {
    case 0: return launch_init3f<0, 27>(list, n, meta, codes, lat, fld, L, s);
    case 1: return launch_init3f<1, 27>(list, n, meta, codes, lat, fld, L, s);
    case 2: return launch_init3f<2, 27>(list, n, meta, codes, lat, fld, L, s);
    default: return launch_init3f<3, 27>(list, n, meta, codes, lat, fld, L, s);
  }
}

// ---------------------------------------------------------------------------
// Host: the forest.
// ---------------------------------------------------------------------------

constexpr int kDX[3] = {-1, 0, 1};

// Interleaved bits of (x, y, z): Morton order of the blocks.
uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  auto spread = [](uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffull;
    v = (v | v << 16) & 0x1f0000ff0000ffull;
    v = (v | v << 8) & 0x100f00f00f00f00full;
    v = (v | v << 4) & 0x10c30c30c30c30c3ull;
    v = (v | v << 2) & 0x1249249249249249ull;
    return v;
  };
  return spread(x) | spread(y) << 1 | spread(z) << 2;
}

using Mask512 = std::vector<uint8_t>;  // one byte per cell of a block

struct LevelHost {
  int n[3] = {0, 0, 0};    // cells per axis
  int nb[3] = {0, 0, 0};   // blocks per axis
  std::unordered_map<int64_t, int> region;   // region block key -> 1 (level 0: implicit)
  bool all = false;                          // level 0: every block is a region block
  std::unordered_map<int64_t, Mask512> ghost;  // halo block key -> halo-cell mask
  std::vector<int64_t> own_keys, halo_keys;  // pool order
  std::unordered_map<int64_t, int> index;    // block key -> pool index
  int64_t n_own = 0, n_ghost = 0, n_hidden = 0;
  double tau = 0, F[3] = {0, 0, 0};

  int64_t key(int bx, int by, int bz) const { return ((int64_t)bz * nb[1] + by) * nb[0] + bx; }
  void unkey(int64_t k, int &bx, int &by, int &bz) const {
    bx = (int)(k % nb[0]);
    by = (int)((k / nb[0]) % nb[1]);
    bz = (int)(k / ((int64_t)nb[0] * nb[1]));
  }
  bool in_region_blk(int bx, int by, int bz) const { return all || region.count(key(bx, by, bz)) > 0; }
};

struct Forest {
  sbt3f_desc d{};
  std::vector<int32_t> boxes;
  int m = 0;
  std::vector<LevelHost> L;

  int wrap(int v, int n) const { return ((v % n) + n) % n; }
  // cell of level l (wrapped coordinates) in the region / hidden / owned
  bool region_cell(int l, int x, int y, int z) const { return L[l].in_region_blk(x >> 3, y >> 3, z >> 3); }
  bool hidden_cell(int l, int x, int y, int z) const {
    return l + 1 < m && region_cell(l, x, y, z) && L[l + 1].in_region_blk(x >> 2, y >> 2, z >> 2);
  }
  bool own_cell(int l, int x, int y, int z) const { return region_cell(l, x, y, z) && !hidden_cell(l, x, y, z); }
  bool ghost_cell(int l, int x, int y, int z) const {
    if (l == 0) return false;
    const LevelHost &H = L[l];
    auto it = H.ghost.find(H.key(x >> 3, y >> 3, z >> 3));
    return it != H.ghost.end() && it->second[((z & 7) * 8 + (y & 7)) * 8 + (x & 7)];
  }
  uint8_t kind(int l, int x, int y, int z) const {
    if (region_cell(l, x, y, z)) return hidden_cell(l, x, y, z) ? 3 : 1;
    return ghost_cell(l, x, y, z) ? 2 : 0;
  }
};

sbt_status fail3(sbt_status c, const std::string &m) { return sbt_set_error(c, m.c_str()); }

sbt_status check_desc3f(const sbt3f_desc *d) {
  if (!d) return fail3(SBT_ERR_ARG, "null descriptor");
  if (d->n_levels < 1 || d->n_levels > kMaxLev3) return fail3(SBT_ERR_ARG, "n_levels must be 1 .. 6");
  if (d->nx0 < kB3 || d->ny0 < kB3 || d->nz0 < kB3 || d->nx0 % kB3 || d->ny0 % kB3 || d->nz0 % kB3)
    return fail3(SBT_ERR_ARG, "level-0 cells per axis must be positive multiples of 8");
  const int64_t top = (int64_t)1 << (d->n_levels - 1);
  if ((int64_t)d->nx0 * top > (1 << 20) || (int64_t)d->ny0 * top > (1 << 20) || (int64_t)d->nz0 * top > (1 << 20))
    return fail3(SBT_ERR_ARG, "grid too large");
  if (!(d->tau0 > 0.5)) return fail3(SBT_ERR_ARG, "tau0 must exceed 1/2");
  if (!(d->rho0 > 0.0)) return fail3(SBT_ERR_ARG, "rho0 must be positive");
  if (d->storage < SBT_F64 || d->storage > SBT_BF16S) return fail3(SBT_ERR_ARG, "bad storage");
  if (d->lattice != 19 && d->lattice != 27) return fail3(SBT_ERR_ARG, "lattice must be 19 or 27");
  if (d->cf_mode != SBT_CF_HOMOGENEOUS && d->cf_mode != SBT_CF_RESCALE) return fail3(SBT_ERR_ARG, "bad cf_mode");
  if (d->n_boxes < 0 || (d->n_boxes > 0 && !d->boxes)) return fail3(SBT_ERR_ARG, "bad boxes");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(d->fext[k])) return fail3(SBT_ERR_ARG, "fext must be finite");
  return SBT_OK;
}

// Separable Chebyshev dilation of radius 2 on a 12^3 byte cube.
void dilate2(std::vector<uint8_t> &a) {
  std::vector<uint8_t> t(a.size());
  auto at = [](int x, int y, int z) { return (z * 12 + y) * 12 + x; };
  for (int axis = 0; axis < 3; ++axis) {
    for (int z = 0; z < 12; ++z)
      for (int y = 0; y < 12; ++y)
        for (int x = 0; x < 12; ++x) {
          uint8_t v = 0;
          for (int dd = -2; dd <= 2 && !v; ++dd) {
            int xx = x, yy = y, zz = z;
            (axis == 0 ? xx : axis == 1 ? yy : zz) += dd;
            if (xx < 0 || yy < 0 || zz < 0 || xx >= 12 || yy >= 12 || zz >= 12) continue;
            v = a[at(xx, yy, zz)];
          }
          t[at(x, y, z)] = v;
        }
    a.swap(t);
  }
}

sbt_status build_forest(const sbt3f_desc *din, Forest &Fo) {
  sbt_status st = check_desc3f(din);
  if (st) return st;
  Fo.d = *din;
  Fo.m = din->n_levels;
  Fo.boxes.assign(din->boxes, din->boxes + 7 * (size_t)din->n_boxes);
  Fo.d.boxes = Fo.boxes.data();
  Fo.L.assign(Fo.m, LevelHost{});
  const int n0[3] = {din->nx0, din->ny0, din->nz0};
  for (int l = 0; l < Fo.m; ++l) {
    LevelHost &H = Fo.L[l];
    for (int a = 0; a < 3; ++a) {
      H.n[a] = n0[a] << l;
      H.nb[a] = H.n[a] / kB3;
    }
    H.tau = 0.5 + (double)(1 << l) * (din->tau0 - 0.5);
    for (int a = 0; a < 3; ++a) H.F[a] = din->fext[a] / (double)(1 << l);
    H.all = l == 0;
  }
  if (din->cf_mode == SBT_CF_RESCALE)
    for (int l = 0; l + 1 < Fo.m; ++l)
      if (std::fabs(Fo.L[l].tau - 1.0) < 1e-6) return fail3(SBT_ERR_ARG, "RESCALE needs tau_l != 1 below the finest level");
  // region blocks
  for (int b = 0; b < din->n_boxes; ++b) {
    const int32_t *q = Fo.boxes.data() + 7 * b;
    const int l = q[0];
    if (l < 1 || l >= Fo.m) return fail3(SBT_ERR_ARG, "box level must be 1 .. n_levels - 1");
    LevelHost &H = Fo.L[l];
    for (int a = 0; a < 3; ++a)
      if (q[1 + a] < 0 || q[4 + a] > H.nb[a] || q[1 + a] >= q[4 + a]) return fail3(SBT_ERR_ARG, "box outside its level's grid or empty");
    for (int bz = q[3]; bz < q[6]; ++bz)
      for (int by = q[2]; by < q[5]; ++by)
        for (int bx = q[1]; bx < q[4]; ++bx) H.region[H.key(bx, by, bz)] = 1;
  }
  for (int l = 1; l < Fo.m; ++l) {
    if (Fo.L[l].region.empty()) return fail3(SBT_ERR_TOPOLOGY, "a refined level has no box");
    for (const auto &kv : Fo.L[l].region) {  // nesting: the parent block is a region block
      int bx, by, bz;
      Fo.L[l].unkey(kv.first, bx, by, bz);
      if (!Fo.L[l - 1].in_region_blk(bx >> 1, by >> 1, bz >> 1))
        return fail3(SBT_ERR_TOPOLOGY, "level " + std::to_string(l) + " leaves its parent level's region");
    }
  }
  // halo cells: outside the region, within Chebyshev distance 2 of an owned cell
  for (int l = 1; l < Fo.m; ++l) {
    LevelHost &H = Fo.L[l];
    std::unordered_map<int64_t, int> cand;
    for (const auto &kv : H.region) {
      int bx, by, bz;
      H.unkey(kv.first, bx, by, bz);
      for (int dz : kDX)
        for (int dy : kDX)
          for (int dx : kDX) {
            const int nx = Fo.wrap(bx + dx, H.nb[0]), ny = Fo.wrap(by + dy, H.nb[1]), nz = Fo.wrap(bz + dz, H.nb[2]);
            if (!H.in_region_blk(nx, ny, nz)) cand[H.key(nx, ny, nz)] = 1;
          }
    }
    for (const auto &kv : cand) {
      int bx, by, bz;
      H.unkey(kv.first, bx, by, bz);
      std::vector<uint8_t> own(12 * 12 * 12, 0);
      for (int z = 0; z < 12; ++z)
        for (int y = 0; y < 12; ++y)
          for (int x = 0; x < 12; ++x) {
            const int gx = Fo.wrap(bx * 8 + x - 2, H.n[0]), gy = Fo.wrap(by * 8 + y - 2, H.n[1]),
                      gz = Fo.wrap(bz * 8 + z - 2, H.n[2]);
            own[(z * 12 + y) * 12 + x] = Fo.own_cell(l, gx, gy, gz);
          }
      dilate2(own);
      Mask512 g(kC3, 0);
      bool any = false;
      for (int z = 0; z < 8; ++z)
        for (int y = 0; y < 8; ++y)
          for (int x = 0; x < 8; ++x)
            if (own[((z + 2) * 12 + y + 2) * 12 + x + 2]) {
              g[(z * 8 + y) * 8 + x] = 1;
              any = true;
              const int px = (bx * 8 + x) >> 1, py = (by * 8 + y) >> 1, pz = (bz * 8 + z) >> 1;
              if (!Fo.own_cell(l - 1, px, py, pz))
                return fail3(SBT_ERR_TOPOLOGY, "a halo cell of level " + std::to_string(l) + " has no owned parent");
            }
      if (any) H.ghost[kv.first] = std::move(g);
    }
  }
  // pools: blocks with owned cells (Morton order), then halo blocks
  for (int l = 0; l < Fo.m; ++l) {
    LevelHost &H = Fo.L[l];
    std::vector<std::pair<uint64_t, int64_t>> own, halo;
    auto visit = [&](int64_t k) {
      int bx, by, bz;
      H.unkey(k, bx, by, bz);
      int64_t no = 0, nh = 0;
      for (int z = 0; z < 8; ++z)
        for (int y = 0; y < 8; ++y)
          for (int x = 0; x < 8; ++x) {
            if (Fo.hidden_cell(l, bx * 8 + x, by * 8 + y, bz * 8 + z)) ++nh;
            else ++no;
          }
      H.n_own += no;
      H.n_hidden += nh;
      if (no > 0) own.push_back({morton3(bx, by, bz), k});
    };
    if (H.all) {
      for (int64_t k = 0; k < (int64_t)H.nb[0] * H.nb[1] * H.nb[2]; ++k) visit(k);
    } else {
      for (const auto &kv : H.region) visit(kv.first);
    }
    for (const auto &kv : H.ghost) {
      int bx, by, bz;
      H.unkey(kv.first, bx, by, bz);
      for (uint8_t v : kv.second) H.n_ghost += v;
      halo.push_back({morton3(bx, by, bz), kv.first});
    }
    std::sort(own.begin(), own.end());
    std::sort(halo.begin(), halo.end());
    for (auto &p : own) H.own_keys.push_back(p.second);
    for (auto &p : halo) H.halo_keys.push_back(p.second);
    int i = 0;
    for (int64_t k : H.own_keys) H.index[k] = i++;
    for (int64_t k : H.halo_keys) H.index[k] = i++;
  }
  return SBT_OK;
}

// Whether a block of level l or one of its 26 neighbours has hidden cells
// (only such blocks can hold hidden cells, hidden sources or interface cells).
bool near_finer(const Forest &Fo, int l, int bx, int by, int bz) {
  const LevelHost &H = Fo.L[l], &Fn = Fo.L[l + 1];
  for (int dz : kDX)
    for (int dy : kDX)
      for (int dx : kDX) {
        const int nx = Fo.wrap(bx + dx, H.nb[0]), ny = Fo.wrap(by + dy, H.nb[1]), nz = Fo.wrap(bz + dz, H.nb[2]);
        for (int o = 0; o < 8; ++o)
          if (Fn.in_region_blk(2 * nx + (o & 1), 2 * ny + ((o >> 1) & 1), 2 * nz + (o >> 2))) return true;
      }
  return false;
}

// Block tables and per-cell codes of level l's pool.
void build_tables(const Forest &Fo, int l, std::vector<Blk3> &meta, std::vector<uint32_t> &codes) {
  const LevelHost &H = Fo.L[l];
  const int Q = Fo.d.lattice;
  const int n_pool = (int)(H.own_keys.size() + H.halo_keys.size());
  meta.assign(n_pool, Blk3{});
  codes.clear();
  int rows = 0;
  for (int p = 0; p < n_pool; ++p) {
    const bool halo = p >= (int)H.own_keys.size();
    const int64_t k = halo ? H.halo_keys[p - H.own_keys.size()] : H.own_keys[p];
    int bx, by, bz;
    H.unkey(k, bx, by, bz);
    Blk3 &M = meta[p];
    M.ox = bx * 8;
    M.oy = by * 8;
    M.oz = bz * 8;
    M.flags = halo ? B3_GHOST : 0;
    M.code = -1;
    for (int dz : kDX)
      for (int dy : kDX)
        for (int dx : kDX) {
          const int64_t nk = H.key(Fo.wrap(bx + dx, H.nb[0]), Fo.wrap(by + dy, H.nb[1]), Fo.wrap(bz + dz, H.nb[2]));
          auto it = H.index.find(nk);
          M.nbr[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] = it == H.index.end() ? -1 : it->second;
        }
    for (int o = 0; o < 8; ++o) {
      M.child[o] = -1;
      if (halo || l + 1 >= Fo.m) continue;
      const LevelHost &Fn = Fo.L[l + 1];
      auto it = Fn.index.find(Fn.key(2 * bx + (o & 1), 2 * by + ((o >> 1) & 1), 2 * bz + (o >> 2)));
      if (it != Fn.index.end()) M.child[o] = it->second;
    }
    std::vector<uint32_t> row(kC3, 0u);
    bool any = false;
    if (halo) {
      const Mask512 &g = H.ghost.at(k);
      for (int c = 0; c < kC3; ++c) row[c] = g[c] ? K3_BAND : 0u;
      any = true;
    } else if (l + 1 < Fo.m && near_finer(Fo, l, bx, by, bz)) {
      for (int z = 0; z < 8; ++z)
        for (int y = 0; y < 8; ++y)
          for (int x = 0; x < 8; ++x) {
            const int gx = bx * 8 + x, gy = by * 8 + y, gz = bz * 8 + z;
            uint32_t c = 0;
            if (Fo.hidden_cell(l, gx, gy, gz)) {
              c = K3_HIDDEN;
            } else {
              for (int i = 0; i < Q; ++i) {
                static const int ex[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                           1, -1, 1, -1, 1, -1, 1, -1};
                static const int ey[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1,
                                           1, 1, -1, -1, 1, 1, -1, -1};
                static const int ez[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1,
                                           1, 1, 1, 1, -1, -1, -1, -1};
                const int sx = Fo.wrap(gx - ex[i], H.n[0]), sy = Fo.wrap(gy - ey[i], H.n[1]),
                          sz = Fo.wrap(gz - ez[i], H.n[2]);
                if (Fo.hidden_cell(l, sx, sy, sz)) c |= 1u << i;
              }
              bool gchild = false;
              for (int o = 0; o < 8 && !gchild; ++o)
                gchild = Fo.ghost_cell(l + 1, 2 * gx + (o & 1), 2 * gy + ((o >> 1) & 1), 2 * gz + (o >> 2));
              if (gchild) c |= K3_IFACE;
            }
            row[(z * 8 + y) * 8 + x] = c;
            any |= c != 0u;
          }
    }
    if (any) {
      M.code = rows++;
      codes.insert(codes.end(), row.begin(), row.end());
    }
  }
}

size_t stor_bytes3(int st) { return st == 0 ? 8 : (st == 1 ? 4 : 2); }
size_t al256(size_t b) { return (b + 255) / 256 * 256; }
constexpr int kStageBlocks = 2048;

struct Pool3 {
  int n_own = 0, n_halo = 0, code_rows = 0;
  int n_fast = 0;            // interior blocks: the first n_fast entries of the list
  int32_t *d_band = nullptr; // halo cells: pool block * 512 + cell
  int n_band = 0;
  Blk3 *d_meta = nullptr;
  uint32_t *d_codes = nullptr;
  int32_t *d_list = nullptr;
  void *lat[2] = {nullptr, nullptr};
  int cur = 0;
  Lev3 L{};
};

struct Carve {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t bytes) {
    T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
    off += al256(bytes);
    return p;
  }
};

}  // namespace

struct sbt3f_ctx {
  Forest fo;
  std::vector<Pool3> pools;
  int storage = 0, q = 19;
  hipStream_t stream = nullptr;
  double *d_stage = nullptr, *d_part = nullptr;
  int32_t *d_stage_list = nullptr;
  int32_t *d_err = nullptr;
  bool post = false;   // false: the lattices hold the initial pre-collision state
  std::vector<std::pair<int, int>> phases;  // (level, substep parity 1 or 2) of one coarse step
};

namespace {

#define HIPCHK3(x)                                                                   \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) return fail3(SBT_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Layout of the device buffer (null base: sizes only).
size_t layout(sbt3f_ctx &X, char *base, const std::vector<std::vector<Blk3>> &metas,
              const std::vector<std::vector<uint32_t>> &codes) {
  Carve cv{base};
  const size_t s = stor_bytes3(X.storage);
  X.pools.assign(X.fo.m, Pool3{});
  int max_pool = 1;
  for (int l = 0; l < X.fo.m; ++l) {
    Pool3 &P = X.pools[l];
    const LevelHost &H = X.fo.L[l];
    P.n_own = (int)H.own_keys.size();
    P.n_halo = (int)H.halo_keys.size();
    const size_t n = (size_t)P.n_own + P.n_halo;
    max_pool = std::max<int>(max_pool, (int)n);
    P.code_rows = (int)(codes[l].size() / kC3);
    for (int h = 0; h < 2; ++h) P.lat[h] = cv.take<void>(n * X.q * kC3 * s);
    P.d_meta = cv.take<Blk3>(n * sizeof(Blk3));
    P.d_codes = cv.take<uint32_t>(std::max<size_t>(1, codes[l].size()) * 4);
    P.d_list = cv.take<int32_t>(n * 4);
    P.n_band = (int)H.n_ghost;
    P.d_band = cv.take<int32_t>(std::max<size_t>(1, (size_t)P.n_band) * 4);
  }
  const int sb = std::min(kStageBlocks, max_pool);
  X.d_stage = cv.take<double>((size_t)sb * 4 * kC3 * 8);
  X.d_part = cv.take<double>((size_t)max_pool * 2 * 4 * 8);
  X.d_stage_list = cv.take<int32_t>((size_t)sb * 4);
  X.d_err = cv.take<int32_t>(256);
  return cv.off;
}

int stage_blocks(const sbt3f_ctx &X) {
  int mx = 1;
  for (const Pool3 &P : X.pools) mx = std::max(mx, P.n_own + P.n_halo);
  return std::min(kStageBlocks, mx);
}

void set_level_params(sbt3f_ctx &X) {
  const Forest &Fo = X.fo;
  for (int l = 0; l < Fo.m; ++l) {
    Lev3 &L = X.pools[l].L;
    const LevelHost &H = Fo.L[l];
    L.tau = H.tau;
    L.pre = 1.0 - 0.5 / H.tau;
    L.rho0 = Fo.d.rho0;
    for (int a = 0; a < 3; ++a) {
      L.F[a] = H.F[a];
      L.F_f[a] = (float)H.F[a];
    }
    L.s_cf = L.s_fc = 1.0;
    if (l + 1 < Fo.m) {  // the pair (l, l + 1): tau_c = tau_l, tau_f = tau_{l+1}
      const double tc = H.tau, tf = Fo.L[l + 1].tau;
      L.s_cf = (tf - 1.0) / (2.0 * (tc - 1.0));
      L.s_fc = 2.0 * tc / tf;
    }
    L.om_f = (float)(1.0 / H.tau);
    L.pre_f = (float)L.pre;
    L.rho0_f = (float)Fo.d.rho0;
    L.s_cf_f = (float)L.s_cf;
    L.s_fc_f = (float)L.s_fc;
    L.rescale = Fo.d.cf_mode == SBT_CF_RESCALE;
  }
}

// Algorithm 1 unrolled: a level launch streams the previous collision's
// output and performs the next collision, so the launches follow the order
// of the paper's streaming calls: streams(l) = streams(l+1), S_l(first),
// streams(l+1), S_l(second).
void rec3(int l, int V, std::vector<std::pair<int, int>> &out) {
  if (l == V - 1) {
    out.push_back({l, 1});
    out.push_back({l, 2});
    return;
  }
  rec3(l + 1, V, out);
  out.push_back({l, 1});
  rec3(l + 1, V, out);
  out.push_back({l, 2});
}

// One launch of level l over n blocks of `list` (pool indices) and, in a
// step launch, n_band halo cells.
sbt_status launch_level3(sbt3f_ctx &X, int l, const int32_t *list, int n, int mode, bool flip, int n_band = 0) {
  Pool3 &P = X.pools[l];
  Args3 a{};
  a.meta = P.d_meta;
  a.codes = P.d_codes;
  a.src = P.lat[P.cur];
  a.dst = P.lat[1 - P.cur];
  // a readout after a step gathers from the lattice the level's last launch
  // read: its streamed state is the oracle's pre-collision state
  if ((mode & M3_READOUT) && !(mode & M3_LOCAL)) a.src = P.lat[1 - P.cur];
  if (l + 1 < X.fo.m) {
    Pool3 &F = X.pools[l + 1];
    a.fmeta = F.d_meta;
    a.fprev = F.lat[1 - F.cur];
    a.fcur = F.lat[F.cur];
  }
  a.list = list;
  a.n_blocks = n;
  a.n_fast = mode == 0 ? P.n_fast : 0;
  a.band = P.d_band;
  a.n_band = mode == 0 ? n_band : 0;
  a.mode = mode;
  a.xcd = mode == 0 ? 1 : 0;
  a.off32 = ((size_t)P.n_own + P.n_halo) * X.q * kC3 * stor_bytes3(X.storage) < ((size_t)1 << 32);
  a.L = P.L;
  a.out = X.d_stage;
  a.part = X.d_part;
  a.err = X.d_err;
  HIPCHK3(forest3_dispatch(X.storage, X.q, a, X.stream));
  if (flip) P.cur ^= 1;
  return SBT_OK;
}

// Substep p (1 or 2) of level l: the blocks with owned cells, and in the
// first of a fine level's two substeps its halo cells.
sbt_status substep3(sbt3f_ctx &X, int l, int p) {
  Pool3 &P = X.pools[l];
  return launch_level3(X, l, P.d_list, P.n_own, 0, true, (p == 1 && l > 0) ? P.n_band : 0);
}

// The first collision of every level from the initial pre-collision state,
// finest first so that each coarse level explodes into its finer level's
// current lattice.
sbt_status prologue3(sbt3f_ctx &X) {
  for (int l = X.fo.m - 1; l >= 0; --l) {
    sbt_status st = launch_level3(X, l, X.pools[l].d_list, X.pools[l].n_own, M3_LOCAL, true);
    if (st) return st;
  }
  X.post = true;
  return SBT_OK;
}

sbt_status check_box(const sbt3f_ctx &X, int level, const int32_t *box) {
  if (level < 0 || level >= X.fo.m) return fail3(SBT_ERR_ARG, "level out of range");
  if (!box) return fail3(SBT_ERR_ARG, "null box");
  const LevelHost &H = X.fo.L[level];
  for (int a = 0; a < 3; ++a)
    if (box[a] < 0 || box[3 + a] < 1 || (int64_t)box[a] + box[3 + a] > H.n[a])
      return fail3(SBT_ERR_ARG, "box outside the level's grid");
  return SBT_OK;
}

// Pool blocks of a level's owned part that meet the box.
std::vector<int32_t> blocks_in_box(const sbt3f_ctx &X, int level, const int32_t *box) {
  const LevelHost &H = X.fo.L[level];
  std::vector<int32_t> out;
  for (int p = 0; p < (int)H.own_keys.size(); ++p) {
    int bx, by, bz;
    H.unkey(H.own_keys[p], bx, by, bz);
    const int o[3] = {bx * 8, by * 8, bz * 8};
    bool hit = true;
    for (int a = 0; a < 3; ++a) hit = hit && o[a] + 8 > box[a] && o[a] < box[a] + box[3 + a];
    if (hit) out.push_back(p);
  }
  return out;
}

}  // namespace

extern "C" {

sbt_status sbt3f_plan(const sbt3f_desc *desc, size_t *device_bytes) {
  if (!device_bytes) return fail3(SBT_ERR_ARG, "null output");
  sbt3f_ctx X;
  sbt_status st = build_forest(desc, X.fo);
  if (st) return st;
  X.storage = desc->storage;
  X.q = desc->lattice;
  std::vector<std::vector<Blk3>> metas(X.fo.m);
  std::vector<std::vector<uint32_t>> codes(X.fo.m);
  for (int l = 0; l < X.fo.m; ++l) build_tables(X.fo, l, metas[l], codes[l]);
  *device_bytes = layout(X, nullptr, metas, codes);
  return SBT_OK;
}

sbt_status sbt3f_level_kinds(const sbt3f_desc *desc, int32_t level, const int32_t box[6], uint8_t *kind,
                             int64_t info[6]) {
  Forest Fo;
  sbt_status st = build_forest(desc, Fo);
  if (st) return st;
  if (level < 0 || level >= Fo.m) return fail3(SBT_ERR_ARG, "level out of range");
  const LevelHost &H = Fo.L[level];
  if (info) {
    for (int a = 0; a < 3; ++a) info[a] = H.n[a];
    info[3] = H.n_own;
    info[4] = H.n_ghost;
    info[5] = H.n_hidden;
  }
  if (!kind) return SBT_OK;
  if (!box) return fail3(SBT_ERR_ARG, "null box");
  for (int a = 0; a < 3; ++a)
    if (box[a] < 0 || box[3 + a] < 1 || (int64_t)box[a] + box[3 + a] > H.n[a])
      return fail3(SBT_ERR_ARG, "box outside the level's grid");
  size_t c = 0;
  for (int z = box[2]; z < box[2] + box[5]; ++z)
    for (int y = box[1]; y < box[1] + box[4]; ++y)
      for (int x = box[0]; x < box[0] + box[3]; ++x) kind[c++] = Fo.kind(level, x, y, z);
  return SBT_OK;
}

sbt_status sbt3f_create(const sbt3f_desc *desc, void *device_buf, size_t bytes, void *hip_stream,
                        sbt3f_ctx **out) {
  if (!out) return fail3(SBT_ERR_ARG, "null output");
  *out = nullptr;
  if (!device_buf || ((uintptr_t)device_buf & 255)) return fail3(SBT_ERR_ARG, "device buffer null or not 256-byte aligned");
  auto X = new sbt3f_ctx();
  sbt_status st = build_forest(desc, X->fo);
  if (st) {
    delete X;
    return st;
  }
  X->storage = desc->storage;
  X->q = desc->lattice;
  X->stream = static_cast<hipStream_t>(hip_stream);
  std::vector<std::vector<Blk3>> metas(X->fo.m);
  std::vector<std::vector<uint32_t>> codes(X->fo.m);
  for (int l = 0; l < X->fo.m; ++l) build_tables(X->fo, l, metas[l], codes[l]);
  const size_t need = layout(*X, nullptr, metas, codes);
  if (bytes < need) {
    delete X;
    return fail3(SBT_ERR_NOMEM, "device buffer smaller than sbt3f_plan asked");
  }
  layout(*X, static_cast<char *>(device_buf), metas, codes);
  set_level_params(*X);
  auto cleanup = [&](sbt_status s) {
    delete X;
    return s;
  };
  for (int l = 0; l < X->fo.m; ++l) {
    Pool3 &P = X->pools[l];
    const size_t n = (size_t)P.n_own + P.n_halo;
    // launch order: interior blocks, the other blocks with owned cells, halo blocks
    std::vector<int32_t> list;
    list.reserve(n);
    for (int i = 0; i < P.n_own; ++i)
      if (metas[l][i].code < 0) list.push_back(i);
    P.n_fast = (int)list.size();
    for (int i = 0; i < P.n_own; ++i)
      if (metas[l][i].code >= 0) list.push_back(i);
    for (size_t i = P.n_own; i < n; ++i) list.push_back((int32_t)i);
    std::vector<int32_t> band;
    band.reserve(P.n_band);
    for (size_t i = P.n_own; i < n; ++i) {
      const int32_t code = metas[l][i].code;
      for (int c = 0; c < kC3; ++c)
        if (codes[l][(size_t)code * kC3 + c] & K3_BAND) band.push_back((int32_t)(i * kC3 + c));
    }
    if ((int)band.size() != P.n_band) return cleanup(fail3(SBT_ERR_STATE, "halo cell count mismatch"));
    if (!band.empty() && hipMemcpyAsync(P.d_band, band.data(), band.size() * 4, hipMemcpyHostToDevice, X->stream) != hipSuccess)
      return cleanup(fail3(SBT_ERR_DEVICE, "upload of the halo cells failed"));
    if (hipMemcpyAsync(P.d_meta, metas[l].data(), n * sizeof(Blk3), hipMemcpyHostToDevice, X->stream) != hipSuccess ||
        (!codes[l].empty() && hipMemcpyAsync(P.d_codes, codes[l].data(), codes[l].size() * 4, hipMemcpyHostToDevice,
                                             X->stream) != hipSuccess) ||
        hipMemcpyAsync(P.d_list, list.data(), n * 4, hipMemcpyHostToDevice, X->stream) != hipSuccess)
      return cleanup(fail3(SBT_ERR_DEVICE, "upload of the block tables failed"));
    for (int h = 0; h < 2; ++h)
      if (sbt_launch_fill_nan(P.lat[h], n * X->q * kC3, X->storage, X->stream) != hipSuccess)
        return cleanup(fail3(SBT_ERR_DEVICE, "lattice fill failed"));
    if (init3f_dispatch(X->storage, X->q, P.d_list, P.n_own, P.d_meta, P.d_codes, P.lat[0], nullptr, P.L,
                        X->stream) != hipSuccess)
      return cleanup(fail3(SBT_ERR_DEVICE, "initial state failed"));
    if (hipStreamSynchronize(X->stream) != hipSuccess)  // the host vectors go out of scope
      return cleanup(fail3(SBT_ERR_DEVICE, "create synchronisation failed"));
  }
  if (hipMemsetAsync(X->d_err, 0, 4, X->stream) != hipSuccess || hipStreamSynchronize(X->stream) != hipSuccess)
    return cleanup(fail3(SBT_ERR_DEVICE, "error flag reset failed"));
  rec3(1, X->fo.m, X->phases);
  if (X->fo.m == 1) X->phases.clear();
  X->phases.push_back({0, 1});
  *out = X;
  return SBT_OK;
}

sbt_status sbt3f_destroy(sbt3f_ctx *ctx) {
  if (!ctx) return SBT_OK;
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
  return SBT_OK;
}

sbt_status sbt3f_init_box(sbt3f_ctx *ctx, int32_t level, const int32_t box[6], const double *rho, const double *ux,
                          const double *uy, const double *uz) {
  if (!ctx) return fail3(SBT_ERR_ARG, "null context");
  sbt_status st = check_box(*ctx, level, box);
  if (st) return st;
  if (!rho || !ux || !uy || !uz) return fail3(SBT_ERR_ARG, "null field array");
  sbt3f_ctx &X = *ctx;
  HIPCHK3(hipStreamSynchronize(X.stream));
  if (X.post) {  // after a step: every level starts over from rest, then takes this box
    for (int l = 0; l < X.fo.m; ++l) {
      Pool3 &P = X.pools[l];
      P.cur = 0;
      HIPCHK3(init3f_dispatch(X.storage, X.q, P.d_list, P.n_own, P.d_meta, P.d_codes, P.lat[0], nullptr, P.L,
                              X.stream));
    }
    X.post = false;
  }
  Pool3 &P = X.pools[level];
  const std::vector<int32_t> blocks = blocks_in_box(X, level, box);
  const LevelHost &H = X.fo.L[level];
  const int sb = stage_blocks(X);
  std::vector<double> stage((size_t)sb * 4 * kC3);
  for (size_t b0 = 0; b0 < blocks.size(); b0 += sb) {
    const int nb = (int)std::min<size_t>(sb, blocks.size() - b0);
    for (int w = 0; w < nb; ++w) {
      int bx, by, bz;
      H.unkey(H.own_keys[blocks[b0 + w]], bx, by, bz);
      for (int c = 0; c < kC3; ++c) {
        const int x = bx * 8 + (c & 7) - box[0], y = by * 8 + ((c >> 3) & 7) - box[1], z = bz * 8 + (c >> 6) - box[2];
        double *s = stage.data() + (size_t)w * 4 * kC3 + c;
        if (x < 0 || y < 0 || z < 0 || x >= box[3] || y >= box[4] || z >= box[5]) {
          s[0] = __builtin_nan("");
          continue;
        }
        const size_t i = ((size_t)z * box[4] + y) * box[3] + x;
        s[0] = rho[i];
        s[kC3] = ux[i];
        s[2 * kC3] = uy[i];
        s[3 * kC3] = uz[i];
        if (!std::isfinite(rho[i]) || !(rho[i] > 0.0)) return fail3(SBT_ERR_ARG, "densities must be positive and finite");
      }
    }
    HIPCHK3(hipMemcpyAsync(X.d_stage, stage.data(), (size_t)nb * 4 * kC3 * 8, hipMemcpyHostToDevice, X.stream));
    HIPCHK3(hipMemcpyAsync(X.d_stage_list, blocks.data() + b0, (size_t)nb * 4, hipMemcpyHostToDevice, X.stream));
    HIPCHK3(init3f_dispatch(X.storage, X.q, X.d_stage_list, nb, P.d_meta, P.d_codes, P.lat[P.cur], X.d_stage, P.L,
                            X.stream));
    HIPCHK3(hipStreamSynchronize(X.stream));
  }
  return SBT_OK;
}

sbt_status sbt3f_step(sbt3f_ctx *ctx, int32_t n) {
  if (!ctx) return fail3(SBT_ERR_ARG, "null context");
  if (n < 0) return fail3(SBT_ERR_ARG, "negative step count");
  sbt3f_ctx &X = *ctx;
  if (n > 0 && !X.post) {
    sbt_status st = prologue3(X);
    if (st) return st;
  }
  for (int t = 0; t < n; ++t)
    for (const auto &ph : X.phases) {
      sbt_status st = substep3(X, ph.first, ph.second);
      if (st) return st;
    }
  return SBT_OK;
}

sbt_status sbt3f_synchronize(sbt3f_ctx *ctx) {
  if (!ctx) return fail3(SBT_ERR_ARG, "null context");
  HIPCHK3(hipStreamSynchronize(ctx->stream));
  int32_t err = 0;
  HIPCHK3(hipMemcpy(&err, ctx->d_err, 4, hipMemcpyDeviceToHost));
  if (err & sbt::ERR_NONFINITE) return fail3(SBT_ERR_NONFINITE, "a density became NaN or Inf");
  return SBT_OK;
}

sbt_status sbt3f_read_box(sbt3f_ctx *ctx, int32_t level, const int32_t box[6], double *rho, double *ux, double *uy,
                          double *uz) {
  if (!ctx) return fail3(SBT_ERR_ARG, "null context");
  sbt_status st = check_box(*ctx, level, box);
  if (st) return st;
  if (!rho || !ux || !uy || !uz) return fail3(SBT_ERR_ARG, "null field array");
  sbt3f_ctx &X = *ctx;
  const size_t nc = (size_t)box[3] * box[4] * box[5];
  for (size_t i = 0; i < nc; ++i) rho[i] = ux[i] = uy[i] = uz[i] = __builtin_nan("");
  const LevelHost &H = X.fo.L[level];
  const std::vector<int32_t> blocks = blocks_in_box(X, level, box);
  const int sb = stage_blocks(X);
  std::vector<double> stage((size_t)sb * 4 * kC3);
  for (size_t b0 = 0; b0 < blocks.size(); b0 += sb) {
    const int nb = (int)std::min<size_t>(sb, blocks.size() - b0);
    HIPCHK3(hipMemcpyAsync(X.d_stage_list, blocks.data() + b0, (size_t)nb * 4, hipMemcpyHostToDevice, X.stream));
    st = launch_level3(X, level, X.d_stage_list, nb, M3_READOUT | (X.post ? 0 : M3_LOCAL), false);
    if (st) return st;
    HIPCHK3(hipMemcpyAsync(stage.data(), X.d_stage, (size_t)nb * 4 * kC3 * 8, hipMemcpyDeviceToHost, X.stream));
    HIPCHK3(hipStreamSynchronize(X.stream));
    for (int w = 0; w < nb; ++w) {
      int bx, by, bz;
      H.unkey(H.own_keys[blocks[b0 + w]], bx, by, bz);
      for (int c = 0; c < kC3; ++c) {
        const int x = bx * 8 + (c & 7) - box[0], y = by * 8 + ((c >> 3) & 7) - box[1], z = bz * 8 + (c >> 6) - box[2];
        if (x < 0 || y < 0 || z < 0 || x >= box[3] || y >= box[4] || z >= box[5]) continue;
        const size_t i = ((size_t)z * box[4] + y) * box[3] + x;
        const double *s = stage.data() + (size_t)w * 4 * kC3 + c;
        rho[i] = s[0];
        ux[i] = s[kC3];
        uy[i] = s[2 * kC3];
        uz[i] = s[3 * kC3];
      }
    }
  }
  return SBT_OK;
}

sbt_status sbt3f_diagnostics(sbt3f_ctx *ctx, double out[4]) {
  if (!ctx || !out) return fail3(SBT_ERR_ARG, "null argument");
  sbt3f_ctx &X = *ctx;
  for (int k = 0; k < 4; ++k) out[k] = 0.0;
  const int sb = stage_blocks(X);
  std::vector<double> part((size_t)sb * 2 * 4);
  for (int l = 0; l < X.fo.m; ++l) {
    Pool3 &P = X.pools[l];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b0 = 0; b0 < P.n_own; b0 += sb) {
      const int nb = std::min(sb, P.n_own - b0);
      std::vector<int32_t> list(nb);
      for (int i = 0; i < nb; ++i) list[i] = b0 + i;
      HIPCHK3(hipMemcpyAsync(X.d_stage_list, list.data(), (size_t)nb * 4, hipMemcpyHostToDevice, X.stream));
      sbt_status st = launch_level3(X, l, X.d_stage_list, nb, M3_READOUT | (X.post ? 0 : M3_LOCAL), false);
      if (st) return st;
      HIPCHK3(hipMemcpyAsync(part.data(), X.d_part, (size_t)nb * 2 * 4 * 8, hipMemcpyDeviceToHost, X.stream));
      HIPCHK3(hipStreamSynchronize(X.stream));
      for (int w = 0; w < 2 * nb; ++w)
        for (int k = 0; k < 4; ++k) acc[k] += part[(size_t)w * 4 + k];
    }
    const double wgt = 1.0 / (double)((int64_t)1 << (3 * l));
    for (int k = 0; k < 4; ++k) out[k] += wgt * acc[k];
  }
  return SBT_OK;
}

}  // extern "C"
