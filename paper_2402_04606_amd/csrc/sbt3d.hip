// D3Q19 / D3Q27 stream + collide on one periodic level (the 3D form of Sec. 2.1),
// fused into one launch per step with the pull scheme: a lattice holds
// post-collision populations f*; each thread gathers f*(x - c_i, i) (the
// streamed, pre-collision state of its cell), collides it (BGK + Guo,
// Eqs. (2)-(3), (6)-(8)) and stores f*(x) at its own cell, coalesced along
// x.  The first launch after an initialisation collides the cells' own
// populations in place of the gather.  HBM-bound: 2 * Q * s bytes per cell
// update (D3Q19 or D3Q27).  (Measured against the push form -- own loads, scattered stores
// -- the gather is 7 % faster in FP32 and 17 % in FP16.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "lattice3.h"
#include "sbt3d.h"
#include "sbt_internal.h"

namespace {

constexpr int kThreads = 256;

constexpr uint32_t kSolidBit = 1u << 31;  // solid-record bits: the cell itself is solid

struct Params {
  int nx, ny, nz, walls;
  const int32_t *scode;        // solid cells: per cell 0, or 1 + its record; null without solids
  const uint32_t *rbits;       // per record: bit i = the source of direction i is solid; kSolidBit
  const double *rq;            // per record [Q]: wall fraction of the link of pulled direction i
  long long n;
  double tau, pre, rho0, F[3];
  double uw[2][3];             // bottom and top wall velocities (walls across z)
  const double *ibm_F;         // immersed body: force density [3][box] over its current box, or null
  const int *ibm_box;          // [6] that box: origin x, y, z and size x, y, z
  // the body force of the forcing loop that precedes this launch, summed by
  // the launch's first workgroup beside the cells' work (fs_n = 0: none)
  const double *fs_ft, *fs_dA; // [3][n] total marker force of the loop, [n] surface elements
  double *fs_out;              // [3] F_s = -sum_j F_j dA_j, marker order
  int fs_n;
  float om_f, pre_f, rho0_f, F_f[3];
};

// Neighbour offsets of cell c along each axis (periodic): o[0] = -1, o[2] = +1.
struct Offsets {
  long long ox[3], oy[3], oz[3];
};

__device__ __forceinline__ Offsets offsets(const Params &p, long long c) {
  const int x = (int)(c % p.nx);
  const int y = (int)((c / p.nx) % p.ny);
  const int z = (int)(c / ((long long)p.nx * p.ny));
  const long long plane = (long long)p.nx * p.ny;
  Offsets o;
  o.ox[0] = x == 0 ? (long long)(p.nx - 1) : -1;
  o.ox[1] = 0;
  o.ox[2] = x == p.nx - 1 ? -(long long)(p.nx - 1) : 1;
  o.oy[0] = y == 0 ? (long long)(p.ny - 1) * p.nx : -(long long)p.nx;
  o.oy[1] = 0;
  o.oy[2] = y == p.ny - 1 ? -(long long)(p.ny - 1) * p.nx : (long long)p.nx;
  o.oz[0] = z == 0 ? (long long)(p.nz - 1) * plane : -plane;
  o.oz[1] = 0;
  o.oz[2] = z == p.nz - 1 ? -(long long)(p.nz - 1) * plane : plane;
  return o;
}

// Index of the source x - c_i of direction i (pull), or the cell itself.
__device__ __forceinline__ long long source(const Offsets &o, long long c, int i, bool pull) {
  return pull ? c + o.ox[1 - E3X[i]] + o.oy[1 - E3Y[i]] + o.oz[1 - E3Z[i]] : c;
}

// Walls across z: a population whose source lies below z = 0 or above
// z = nz - 1 is the opposite population o of the same cell bounced back
// half-way, with the moving-wall term f_i = f*_o - 6 w_i rho0 (c_o . u_wall)
// (the same in the deviation frame, w_i = w_o).  The choice of address is a
// select, so the 19 or 27 loads of a thread stay one unbranched batch; the
// term is applied after them.
struct WallSide {
  bool lo, hi;  // the cell's sources below z = 0 / above z = nz - 1 are walls
};

__device__ __forceinline__ WallSide wall_side(const Params &p, long long c, bool pull) {
  const int z = (int)(c / ((long long)p.nx * p.ny));
  WallSide w;
  w.lo = pull && p.walls && z == 0;
  w.hi = pull && p.walls && z == p.nz - 1;
  return w;
}

__device__ __forceinline__ bool bounced(const WallSide &w, int i) {
  return (E3Z[i] > 0 && w.lo) || (E3Z[i] < 0 && w.hi);
}

__device__ __forceinline__ long long gather_index(const Params &p, const Offsets &o, long long c, int i, bool pull,
                                                  const WallSide &w) {
  return bounced(w, i) ? (long long)OPP3[i] * p.n + c : (long long)i * p.n + source(o, c, i, pull);
}

// Interpolated bounce-back (linear Bouzidi form, resting wall) of pulled
// direction i, whose source x - c_i is solid: o = opposite(i) at wall
// fraction q of the link x -> x + c_o,
//   q <  1/2:  2q f*_o(x) + (1 - 2q) f*_o(x + c_i)
//   q >= 1/2:  f*_o(x) / (2q) + (2q - 1)/(2q) f*_i(x)
// (affine with weights summing to 1 and w_o = w_i, so it holds for the
// deviation storage forms too).
template <int ST, int Q>
__device__ __forceinline__ auto bouzidi3(const Params &p, const typename Store3<ST>::T *src, const Offsets &o,
                                         long long c, int rec, int i) {
#pragma clang fp contract(off)
  using S = Store3<ST>;
  using C = decltype(S::ld(src[0]));
  const double q = p.rq[(long long)rec * Q + i];
  const int oi = OPP3[i];
  const C fo = S::ld(src[(long long)oi * p.n + c]);
  if (q < 0.5) {
    const C fu = S::ld(src[(long long)oi * p.n + source(o, c, oi, true)]);
    return C(2.0 * q) * fo + C(1.0 - 2.0 * q) * fu;
  }
  const C fi = S::ld(src[(long long)i * p.n + c]);
  return fo / C(2.0 * q) + C((2.0 * q - 1.0) / (2.0 * q)) * fi;
}

// Index of cell c in the immersed body's force box, or -1 (no body, or outside).
__device__ __forceinline__ long long ibm_box_index(const Params &p, long long c) {
  if (!p.ibm_F) return -1;
  const int *B = p.ibm_box;
  const int x = (int)(c % p.nx) - B[0], y = (int)((c / p.nx) % p.ny) - B[1];
  const int z = (int)(c / ((long long)p.nx * p.ny)) - B[2];
  if (x < 0 || y < 0 || z < 0 || x >= B[3] || y >= B[4] || z >= B[5]) return -1;
  return ((long long)z * B[4] + y) * B[3] + x;
}

template <int Q>
__device__ __forceinline__ double wall_term(const Params &p, int i) {
#pragma clang fp contract(off)
  const int oi = OPP3[i];
  const double *u = p.uw[E3Z[i] > 0 ? 0 : 1];
  const double cu = E3X[oi] * u[0] + E3Y[oi] * u[1] + E3Z[oi] * u[2];
  return 6.0 * w3<double, Q>(i) * p.rho0 * cu;
}

// F_s = -sum_j F_j dA_j of the forcing loop that precedes the launch, in
// marker order (Eq. (16) in 3D): the products formed in parallel 256 at a
// time, then summed in order by one lane per component.
__device__ __forceinline__ void body_force_sum(const Params &p) {
#pragma clang fp contract(off)
  __shared__ double s_prod[3][kThreads];
  const int tid = threadIdx.x, n = p.fs_n;
  double fsum = 0.0;
  for (int j0 = 0; j0 < n; j0 += kThreads) {
    const int j = j0 + tid;
    if (j < n)
      for (int a = 0; a < 3; ++a) s_prod[a][tid] = p.fs_ft[a * n + j] * p.fs_dA[j];
    __syncthreads();
    if (tid < 3) {
      const int m = min(kThreads, n - j0);
      int i = 0;
      for (; i + 8 <= m; i += 8) {  // loads ahead of the (ordered) subtractions
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = s_prod[tid][i + q];
#pragma unroll
        for (int q = 0; q < 8; ++q) fsum -= v[q];
      }
      for (; i < m; ++i) fsum -= s_prod[tid][i];
    }
    __syncthreads();
  }
  if (tid < 3) p.fs_out[tid] = fsum;
}

template <int ST, int kQ3>
__global__ __launch_bounds__(kThreads) void step3_kernel(Params p, const void *src_, void *dst_, int pull,
                                                         int *err) {
#pragma clang fp contract(off)
  using S = Store3<ST>;
  using T = typename S::T;
  const int fsw = p.fs_n > 0;  // workgroup 0 sums the body force (it starts first)
  if (fsw && blockIdx.x == 0) {
    body_force_sum(p);
    return;
  }
  const long long c = (long long)(blockIdx.x - fsw) * kThreads + threadIdx.x;
  if (c >= p.n) return;
  const T *src = static_cast<const T *>(src_);
  T *dst = static_cast<T *>(dst_);
  const Offsets o = offsets(p, c);
  const WallSide ws = wall_side(p, c, pull);
  const int rec = p.scode ? p.scode[c] - 1 : -1;
  const uint32_t sbits = rec >= 0 ? p.rbits[rec] : 0u;
  if (sbits & kSolidBit) return;  // solid cells are not collided
  const bool bz = pull && sbits != 0u;
  if constexpr (ST == 0) {
    double f[kQ3];
#pragma unroll
    for (int i = 0; i < kQ3; ++i) f[i] = S::ld(src[gather_index(p, o, c, i, pull, ws)]);
    if (ws.lo || ws.hi) {
#pragma unroll
      for (int i = 0; i < kQ3; ++i)
        if (bounced(ws, i)) f[i] = f[i] - wall_term<kQ3>(p, i);
    }
    if (bz) {
#pragma unroll
      for (int i = 1; i < kQ3; ++i)
        if (sbits & (1u << i)) f[i] = bouzidi3<ST, kQ3>(p, src, o, c, rec, i);
    }
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < kQ3; ++i) {
      rho += f[i];
      jx += E3X[i] * f[i];
      jy += E3Y[i] * f[i];
      jz += E3Z[i] * f[i];
    }
    double Fx = p.F[0], Fy = p.F[1], Fz = p.F[2];
    const long long bi = ibm_box_index(p, c);
    if (bi >= 0) {
      const long long bn = (long long)p.ibm_box[3] * p.ibm_box[4] * p.ibm_box[5];
      Fx = Fx + p.ibm_F[bi];
      Fy = Fy + p.ibm_F[bn + bi];
      Fz = Fz + p.ibm_F[2 * bn + bi];
    }
    const double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho, uz = (jz + 0.5 * Fz) / rho;
    const double usq = ux * ux + uy * uy + uz * uz;
    const double uF = ux * Fx + uy * Fy + uz * Fz;
    if (!(rho == rho) || rho > 1e30 || rho < -1e30) atomicOr(err, 1);
#pragma unroll
    for (int i = 0; i < kQ3; ++i) {
      const double cu = E3X[i] * ux + E3Y[i] * uy + E3Z[i] * uz;
      const double cF = E3X[i] * Fx + E3Y[i] * Fy + E3Z[i] * Fz;
      const double fe = w3<double, kQ3>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
      const double fi = w3<double, kQ3>(i) * p.pre * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF);
      const double v = f[i] - (f[i] - fe) / p.tau + fi;
      dst[(long long)i * p.n + c] = S::st(v);
    }
  } else {
    // deviation form d = f - w rho0 (FP32 arithmetic)
    float d[kQ3];
#pragma unroll
    for (int i = 0; i < kQ3; ++i) d[i] = S::ld(src[gather_index(p, o, c, i, pull, ws)]);
    if (ws.lo || ws.hi) {
#pragma unroll
      for (int i = 0; i < kQ3; ++i)
        if (bounced(ws, i)) d[i] = d[i] - (float)wall_term<kQ3>(p, i);
    }
    if (bz) {
#pragma unroll
      for (int i = 1; i < kQ3; ++i)
        if (sbits & (1u << i)) d[i] = bouzidi3<ST, kQ3>(p, src, o, c, rec, i);
    }
    float dr = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < kQ3; ++i) {
      dr += d[i];
      jx += E3X[i] * d[i];
      jy += E3Y[i] * d[i];
      jz += E3Z[i] * d[i];
    }
    const float rho = p.rho0_f + dr;
    const float ir = __builtin_amdgcn_rcpf(rho);
    float Fx = p.F_f[0], Fy = p.F_f[1], Fz = p.F_f[2];
    const long long bi = ibm_box_index(p, c);
    if (bi >= 0) {
      const long long bn = (long long)p.ibm_box[3] * p.ibm_box[4] * p.ibm_box[5];
      Fx += (float)p.ibm_F[bi];
      Fy += (float)p.ibm_F[bn + bi];
      Fz += (float)p.ibm_F[2 * bn + bi];
    }
    const float ux = (jx + 0.5f * Fx) * ir, uy = (jy + 0.5f * Fy) * ir, uz = (jz + 0.5f * Fz) * ir;
    const float A = dr - rho * (1.5f * (ux * ux + uy * uy + uz * uz));
    const bool forced = Fx != 0.f || Fy != 0.f || Fz != 0.f;
    const float uF = ux * Fx + uy * Fy + uz * Fz;
    if (!(rho == rho) || rho > 1e30f || rho < -1e30f) atomicOr(err, 1);
#pragma unroll
    for (int i = 0; i < kQ3; ++i) {
      const float cu = E3X[i] * ux + E3Y[i] * uy + E3Z[i] * uz;
      const float de = w3<float, kQ3>(i) * fmaf(rho * cu, fmaf(4.5f, cu, 3.0f), A);
      float v = fmaf(p.om_f, de - d[i], d[i]);
      if (forced) {
        const float cF = E3X[i] * Fx + E3Y[i] * Fy + E3Z[i] * Fz;
        v += w3<float, kQ3>(i) * p.pre_f * (3.f * cF + 9.f * cu * cF - 3.f * uF);
      }
      dst[(long long)i * p.n + c] = S::st(v);
    }
  }
}

// An immersed body: its markers and the device work arrays of its forcing
// loop.  Marker positions are rebuilt every step from the motion law.  The
// box arrays hold K = box[3] box[4] box[5] <= cap cells, x fastest.
struct Ibm3 {
  int n, iters, kind;          // markers, N_F, motion (0 fixed, 1 pitch about y + plunge along z)
  long long cap;               // cells the box arrays hold
  double mp[10];               // kind 1: x0, y0, z0, alpha0, A_pitch, A0, T, phi, U_ref, chord
  const double *xb, *yb, *zb;  // [n] absolute (kind 0) or body-frame (kind 1) positions
  const double *dA;            // [n] surface element
  int *tap;                    // [3][n] first tap cell per axis
  double *phi;                 // [12][n] the 4 weights per axis (x, y, z)
  double *ud;                  // [3][n] desired velocity r(t + 1) - r(t)
  double *rho, *u;             // [K], [3][K] box moments
  double *g, *ft;              // [3][n] force of the pass, total force per marker
  double *Fbox;                // [3][K] force density the step kernel adds
  int *box;                    // [6] the box: origin and size (size 0: no force this step)
  int *lohi;                   // [6] tap bounds reduced over the markers
  double *fs;                  // [2][3] F_s of forcing loop L in slot L & 1
  int *err;                    // bit 2: the box outgrew cap or left the lattice
};

__device__ __forceinline__ double peskin3d(double r) {
#pragma clang fp contract(off)
  const double a = fabs(r);
  if (a <= 1.0) return 0.125 * (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a));
  if (a <= 2.0) return 0.125 * (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a));
  return 0.0;
}

// Position of marker j at step t (the Sec. 3.6 law in the x-z plane for
// kind 1: t* = t U_ref / c, theta = 2 pi t* / T, alpha = alpha0 -
// A_pitch sin(theta + phi), centre (x0, y0, z0 + (A0/2) cos theta),
// X = xc + xb cos a + zb sin a, Y = yc + yb, Z = zc - xb sin a + zb cos a).
struct Pose3 {
  double zc, ca, sa;
};

// Evaluated on the host (C library sin / cos) once per forcing loop and
// passed to the marker kernel.
Pose3 pose3(const Ibm3 &b, double t) {
#pragma clang fp contract(off)
  Pose3 q;
  const double *p = b.mp;
  const double tstar = t * p[8] / p[9];
  const double theta = 2.0 * M_PI * tstar / p[6];
  const double alpha = p[3] - p[4] * sin(theta + p[7]);
  q.zc = p[2] + 0.5 * p[5] * cos(theta);
  q.ca = cos(alpha);
  q.sa = sin(alpha);
  return q;
}

__device__ __forceinline__ void marker3(const Ibm3 &b, const Pose3 &q, int j, double &X, double &Y, double &Z) {
#pragma clang fp contract(off)
  if (b.kind == 0) {
    X = b.xb[j];
    Y = b.yb[j];
    Z = b.zb[j];
    return;
  }
  X = b.mp[0] + b.xb[j] * q.ca + b.zb[j] * q.sa;
  Y = b.mp[1] + b.yb[j];
  Z = q.zc - b.xb[j] * q.sa + b.zb[j] * q.ca;
}

__device__ __forceinline__ long long box_cells(const int *B) { return (long long)B[3] * B[4] * B[5]; }

// Sec. 2.2 in 3D, the forcing loop before the collision of step t, as a
// chain of launches on the stream: ibm3_markers_kernel (markers, desired
// velocities, 4x4x4 taps with weight phi_x (phi_y phi_z)), ibm3_box_kernel
// (the box they cover; it also resets the bounds for the next loop),
// ibm3_moments_kernel (rho, u of the box cells from
// the state the step collides), then N_F times ibm3_interp_kernel (U_j,
// rho_j over the taps, z outer, y, x inner; g_j = 2 rho_j (u_d - U_j)) and
// ibm3_spread_kernel (each box cell sums g_j phi dA_j over the markers in
// marker order, then F += dF, u += dF / (2 rho)).  The loop's body force F_s is summed by the first
// workgroup of the step kernel that follows it.
// Marker j at step t: position, desired velocity, taps and weights; clears
// its force total; the workgroup's tap bounds go into lohi.
__global__ __launch_bounds__(kThreads) void ibm3_markers_kernel(Pose3 q0, Pose3 q1, Ibm3 b) {
#pragma clang fp contract(off)
  __shared__ int s_lo[3], s_hi[3];
  const int tid = threadIdx.x, n = b.n, j = blockIdx.x * blockDim.x + tid;
  if (tid < 3) {
    s_lo[tid] = 1 << 30;
    s_hi[tid] = -(1 << 30);
  }
  __syncthreads();
  if (j < n) {
    double X, Y, Z, X1, Y1, Z1;
    marker3(b, q0, j, X, Y, Z);
    if (b.kind == 0) {
      X1 = X;
      Y1 = Y;
      Z1 = Z;
    } else {
      marker3(b, q1, j, X1, Y1, Z1);
    }
    b.ud[j] = X1 - X;
    b.ud[n + j] = Y1 - Y;
    b.ud[2 * n + j] = Z1 - Z;
    b.ft[j] = b.ft[n + j] = b.ft[2 * n + j] = 0.0;
    const double P[3] = {X, Y, Z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int t0 = (int)floor(P[a] - 1.5);
      b.tap[a * n + j] = t0;
#pragma unroll
      for (int k = 0; k < 4; ++k) b.phi[(a * 4 + k) * n + j] = peskin3d(t0 + k + 0.5 - P[a]);
      atomicMin(&s_lo[a], t0);
      atomicMax(&s_hi[a], t0 + 4);
    }
  }
  __syncthreads();
  if (tid < 3) {
    atomicMin(&b.lohi[tid], s_lo[tid]);
    atomicMax(&b.lohi[3 + tid], s_hi[tid]);
  }
}

// The box of this loop from the reduced bounds; a box outside the lattice
// or above cap gives no force this step (the host reports it at the next
// synchronisation).
__global__ __launch_bounds__(64) void ibm3_box_kernel(Params p, Ibm3 b) {
  if (threadIdx.x != 0) return;
  const int dims[3] = {p.nx, p.ny, p.nz};
  long long K = 1;
  bool bad = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int lo = b.lohi[a], hi = b.lohi[3 + a];
    K *= hi - lo;
    bad |= lo < 0 || hi > dims[a];
  }
  int box[6] = {0, 0, 0, 0, 0, 0};
  if (bad || K > b.cap) {
    atomicOr(b.err, 2);
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      box[a] = b.lohi[a];
      box[3 + a] = b.lohi[3 + a] - b.lohi[a];
    }
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) b.box[a] = box[a];
  // the bounds start over for the next loop's marker kernel
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    b.lohi[a] = 1 << 30;
    b.lohi[3 + a] = -(1 << 30);
  }
}

// rho, u of box cell k from the state the next step collides (gathered when
// the lattice holds post-collision populations); clears the box force.
template <int ST, int kQ3>
__global__ __launch_bounds__(kThreads) void ibm3_moments_kernel(Params p, const void *lat_, int pull, Ibm3 b) {
#pragma clang fp contract(off)
  using S = Store3<ST>;
  using T = typename S::T;
  const int *B = b.box;
  const long long K = box_cells(B), k = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (k >= K) return;
  const T *lat = static_cast<const T *>(lat_);
  const int x = B[0] + (int)(k % B[3]), y = B[1] + (int)((k / B[3]) % B[4]), z = B[2] + (int)(k / ((long long)B[3] * B[4]));
  const long long c = ((long long)z * p.ny + y) * p.nx + x;
  const Offsets o = offsets(p, c);
  double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
  for (int i = 0; i < kQ3; ++i) {
    const double f = (double)S::ld(lat[(long long)i * p.n + source(o, c, i, pull)]);
    r += f;
    jx += E3X[i] * f;
    jy += E3Y[i] * f;
    jz += E3Z[i] * f;
  }
  if constexpr (ST != 0) r = p.rho0 + r;
  b.rho[k] = r;
  b.u[k] = (jx + 0.5 * p.F[0]) / r;
  b.u[K + k] = (jy + 0.5 * p.F[1]) / r;
  b.u[2 * K + k] = (jz + 0.5 * p.F[2]) / r;
  b.Fbox[k] = b.Fbox[K + k] = b.Fbox[2 * K + k] = 0.0;
}

// One pass's interpolation for marker j: U_j, rho_j, g_j; ft_j += g_j.
__global__ __launch_bounds__(kThreads) void ibm3_interp_kernel(Ibm3 b) {
#pragma clang fp contract(off)
  const int *B = b.box;
  const int n = b.n, j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || B[3] == 0) return;
  const int bwx = B[3], bwy = B[4];
  const int i0 = b.tap[j] - B[0], j0 = b.tap[n + j] - B[1], k0 = b.tap[2 * n + j] - B[2];
  const long long K = box_cells(B);
  double U0 = 0.0, U1 = 0.0, U2 = 0.0, R = 0.0;
  for (int cz = 0; cz < 4; ++cz) {
    const double pz = b.phi[(8 + cz) * n + j];
    for (int cy = 0; cy < 4; ++cy) {
      const double pyz = b.phi[(4 + cy) * n + j] * pz;
      for (int cx = 0; cx < 4; ++cx) {
        const double w = b.phi[cx * n + j] * pyz;
        const long long k = ((long long)(k0 + cz) * bwy + (j0 + cy)) * bwx + (i0 + cx);
        U0 += b.u[k] * w;
        U1 += b.u[K + k] * w;
        U2 += b.u[2 * K + k] * w;
        R += b.rho[k] * w;
      }
    }
  }
  const double g0 = 2.0 * R * (b.ud[j] - U0), g1 = 2.0 * R * (b.ud[n + j] - U1);
  const double g2 = 2.0 * R * (b.ud[2 * n + j] - U2);
  b.g[j] = g0;
  b.g[n + j] = g1;
  b.g[2 * n + j] = g2;
  b.ft[j] += g0;
  b.ft[n + j] += g1;
  b.ft[2 * n + j] += g2;
}

// One pass's spreading, markers in order.  A one-wave workgroup takes 4x4x4
// tiles of the box (grid-stride).  For each tile it stages the taps of up to
// kSpBlock markers in LDS at once and lists, in marker order, the markers
// whose 4x4x4 stencil reaches the tile (no global load in this scan); then
// it stages the listed markers' weights, g_j and dA_j 64 at a time (one
// round of loads per 64 listed markers) and each cell sums over them.
constexpr int kSpThreads = 64, kSpTx = 4, kSpTy = 4, kSpTz = kSpThreads / (kSpTx * kSpTy), kSpBlock = 1024;
static_assert(kSpTz * kSpTx * kSpTy == kSpThreads && kSpThreads == 64, "one wave, one cell per lane");

__global__ __launch_bounds__(kSpThreads) void ibm3_spread_kernel(Ibm3 b) {
#pragma clang fp contract(off)
  __shared__ int s_tap[3][kSpBlock];
  __shared__ int s_rel[kSpBlock];
  __shared__ int s_t[3][kSpThreads];
  __shared__ double s_phi[12][kSpThreads];
  __shared__ double s_g[3][kSpThreads];
  __shared__ double s_dA[kSpThreads];
  const int *B = b.box;
  const int lane = threadIdx.x, n = b.n;
  const int bwx = B[3], bwy = B[4], bwz = B[5];
  if (bwx == 0) return;  // the whole grid: no force this step
  const long long K = box_cells(B);
  const int ntx = (bwx + kSpTx - 1) / kSpTx, nty = (bwy + kSpTy - 1) / kSpTy, ntz = (bwz + kSpTz - 1) / kSpTz;
  const int tiles = ntx * nty * ntz;
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int xlo = (tile % ntx) * kSpTx, ylo = ((tile / ntx) % nty) * kSpTy, zlo = (tile / (ntx * nty)) * kSpTz;
    const int xhi = min(xlo + kSpTx, bwx) - 1, yhi = min(ylo + kSpTy, bwy) - 1, zhi = min(zlo + kSpTz, bwz) - 1;
    const int x = xlo + lane % kSpTx, y = ylo + (lane / kSpTx) % kSpTy, z = zlo + lane / (kSpTx * kSpTy);
    const bool live = x <= xhi && y <= yhi && z <= zhi;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int b0 = 0; b0 < n; b0 += kSpBlock) {
      const int bn = min(kSpBlock, n - b0);
      {  // taps in the box frame: all loads issued before the LDS stores
        constexpr int kPer = kSpBlock / kSpThreads;
        int v[3][kPer];
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
          const int i = r * kSpThreads + lane;
#pragma unroll
          for (int a = 0; a < 3; ++a) v[a][r] = i < bn ? b.tap[a * n + b0 + i] : 0;
        }
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
          const int i = r * kSpThreads + lane;
#pragma unroll
          for (int a = 0; a < 3; ++a) s_tap[a][i] = v[a][r] - B[a];
        }
      }
      __syncthreads();
      // the markers of this block that reach the tile, in marker order
      int cnt = 0;
      for (int c0 = 0; c0 < bn; c0 += kSpThreads) {
        const int i = c0 + lane;
        bool f = false;
        if (i < bn) {
          const int tx = s_tap[0][i], ty = s_tap[1][i], tz = s_tap[2][i];
          f = tx <= xhi && tx + 3 >= xlo && ty <= yhi && ty + 3 >= ylo && tz <= zhi && tz + 3 >= zlo;
        }
        const unsigned long long m = __ballot(f);
        if (f) s_rel[cnt + __popcll(m & ((1ull << lane) - 1ull))] = i;
        cnt += __popcll(m);
      }
      __syncthreads();
      for (int g0 = 0; g0 < cnt; g0 += kSpThreads) {
        const int total = min(kSpThreads, cnt - g0);
        if (lane < total) {
          const int i = s_rel[g0 + lane], jc = b0 + i;
          s_t[0][lane] = s_tap[0][i];
          s_t[1][lane] = s_tap[1][i];
          s_t[2][lane] = s_tap[2][i];
          double w[12], gg[3];
#pragma unroll
          for (int q = 0; q < 12; ++q) w[q] = b.phi[q * n + jc];
#pragma unroll
          for (int a = 0; a < 3; ++a) gg[a] = b.g[a * n + jc];
          const double dA = b.dA[jc];
#pragma unroll
          for (int q = 0; q < 12; ++q) s_phi[q][lane] = w[q];
#pragma unroll
          for (int a = 0; a < 3; ++a) s_g[a][lane] = gg[a];
          s_dA[lane] = dA;
        }
        __syncthreads();
        if (live) {
          for (int c = 0; c < total; ++c) {
            const int dx = x - s_t[0][c], dy = y - s_t[1][c], dz = z - s_t[2][c];
            if ((unsigned)dx > 3u || (unsigned)dy > 3u || (unsigned)dz > 3u) continue;
            const double w = s_phi[dx][c] * (s_phi[4 + dy][c] * s_phi[8 + dz][c]);
            d0 += s_g[0][c] * w * s_dA[c];
            d1 += s_g[1][c] * w * s_dA[c];
            d2 += s_g[2][c] * w * s_dA[c];
          }
        }
        __syncthreads();  // the group is restaged by the next one
      }
    }
    if (!live || (d0 == 0.0 && d1 == 0.0 && d2 == 0.0)) continue;
    const long long k = ((long long)z * bwy + y) * bwx + x;
    b.Fbox[k] += d0;
    b.Fbox[K + k] += d1;
    b.Fbox[2 * K + k] += d2;
    b.u[k] += d0 / (2.0 * b.rho[k]);
    b.u[K + k] += d1 / (2.0 * b.rho[k]);
    b.u[2 * K + k] += d2 / (2.0 * b.rho[k]);
  }
}

// f = f^eq(rho, u) of cells [c0, c0 + m) from staged FP64 fields [4][m].
template <int ST, int kQ3>
__global__ __launch_bounds__(kThreads) void init3_kernel(Params p, void *lat_, const double *fld, long long c0,
                                                         long long m) {
#pragma clang fp contract(off)
  using S = Store3<ST>;
  using T = typename S::T;
  const long long k = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (k >= m) return;
  T *lat = static_cast<T *>(lat_);
  const double rho = fld[k], ux = fld[m + k], uy = fld[2 * m + k], uz = fld[3 * m + k];
  const double usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int i = 0; i < kQ3; ++i) {
    const double cu = E3X[i] * ux + E3Y[i] * uy + E3Z[i] * uz;
    const double fe = w3<double, kQ3>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    if constexpr (ST == 0) lat[(long long)i * p.n + c0 + k] = S::st(fe);
    else lat[(long long)i * p.n + c0 + k] = S::st((float)(fe - w3<double, kQ3>(i) * p.rho0));
  }
}

// rho, u of cells [c0, c0 + m) into [4][m] (FP64), from the streamed state:
// gathered from the post-collision lattice the last step read (pull), or the
// cells' own populations before the first step.
template <int ST, int kQ3>
__global__ __launch_bounds__(kThreads) void read3_kernel(Params p, const void *lat_, double *fld, long long c0,
                                                         long long m, int pull) {
#pragma clang fp contract(off)
  using S = Store3<ST>;
  using T = typename S::T;
  const long long k = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (k >= m) return;
  const T *lat = static_cast<const T *>(lat_);
  const Offsets o = offsets(p, c0 + k);
  const WallSide ws = wall_side(p, c0 + k, pull);
  const int rec = p.scode ? p.scode[c0 + k] - 1 : -1;
  const uint32_t sbits = rec >= 0 ? p.rbits[rec] : 0u;
  if (sbits & kSolidBit) {
    for (int q = 0; q < 4; ++q) fld[q * m + k] = __builtin_nan("");
    return;
  }
  double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
  for (int i = 0; i < kQ3; ++i) {
    auto v = S::ld(lat[gather_index(p, o, c0 + k, i, pull, ws)]);
    if (bounced(ws, i)) v = v - (decltype(v))wall_term<kQ3>(p, i);
    if (pull && (sbits & (1u << i))) v = bouzidi3<ST, kQ3>(p, lat, o, c0 + k, rec, i);
    const double f = (double)v;
    r += f;
    jx += E3X[i] * f;
    jy += E3Y[i] * f;
    jz += E3Z[i] * f;
  }
  if constexpr (ST != 0) r = p.rho0 + r;
  fld[k] = r;
  fld[m + k] = (jx + 0.5 * p.F[0]) / r;
  fld[2 * m + k] = (jy + 0.5 * p.F[1]) / r;
  fld[3 * m + k] = (jz + 0.5 * p.F[2]) / r;
}

size_t storage_bytes3(int st) { return st == 0 ? 8 : (st == 1 ? 4 : 2); }

constexpr long long kStageCells = 1ll << 22;

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

struct sbt3_ctx {
  sbt3_desc d;
  Params p;
  void *lat[2];
  double *stage;
  int *err;
  long long stage_cells;
  int cur = 0;
  bool post = false;  // the lattices hold post-collision populations (a step has run)
  hipStream_t stream;
  long long n_records = 0;
  Ibm3 ibm{};                 // immersed body (ibm.n == 0: none)
  long long ibm_t = 0;        // step of the next forcing loop
};

namespace {

sbt_status check_desc(const sbt3_desc *d) {
  if (!d) return sbt_set_error(SBT_ERR_ARG, "null descriptor");
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return sbt_set_error(SBT_ERR_ARG, "nx, ny, nz must be >= 1");
  if ((long long)d->nx * d->ny * d->nz * 27 >= (1ll << 40)) return sbt_set_error(SBT_ERR_ARG, "grid too large");
  if (!(d->tau > 0.5)) return sbt_set_error(SBT_ERR_ARG, "tau must exceed 1/2");
  if (!(d->rho0 > 0.0)) return sbt_set_error(SBT_ERR_ARG, "rho0 must be positive");
  if (d->storage < SBT_F64 || d->storage > SBT_BF16S) return sbt_set_error(SBT_ERR_ARG, "bad storage");
  if (d->lattice != 19 && d->lattice != 27) return sbt_set_error(SBT_ERR_ARG, "lattice must be 19 or 27");
  if (d->n_markers < 0 || (d->n_markers > 0 && (!d->marker_xyz || !d->marker_dA || d->mdf_iters < 0)))
    return sbt_set_error(SBT_ERR_ARG, "bad immersed body");
  if (d->n_markers > 0 && (d->walls_z || d->solid_mask))
    return sbt_set_error(SBT_ERR_ARG, "an immersed body needs a fully periodic box without solid cells");
  if (d->n_markers > 0 && (d->ibm_box_cells < 64 || (d->body_motion != 0 && d->body_motion != 1)))
    return sbt_set_error(SBT_ERR_ARG, "an immersed body needs ibm_box_cells 0 or >= 64 and motion 0 or 1");
  if (d->n_markers > 0 && d->body_motion == 1 && (d->motion_p[6] == 0.0 || d->motion_p[9] == 0.0))
    return sbt_set_error(SBT_ERR_ARG, "motion period and chord must be nonzero");
  if (d->n_markers > 0) {
    // the stencils at t = 0 (every step's are checked again on the device)
    const int n = d->n_markers;
    const int dims[3] = {d->nx, d->ny, d->nz};
    const double *mp = d->motion_p;
    double ca = 1.0, sa = 0.0, zc = 0.0;
    if (d->body_motion == 1) {
      const double alpha = mp[3] - mp[4] * std::sin(mp[7]);
      ca = std::cos(alpha);
      sa = std::sin(alpha);
      zc = mp[2] + 0.5 * mp[5];
    }
    long long cells = 1;
    for (int a = 0; a < 3; ++a) {
      int lo = 1 << 30, hi = -(1 << 30);
      for (int j = 0; j < n; ++j) {
        const double xb = d->marker_xyz[j], yb = d->marker_xyz[n + j], zb = d->marker_xyz[2 * n + j];
        double P = d->marker_xyz[a * n + j];
        if (d->body_motion == 1)
          P = a == 0 ? mp[0] + xb * ca + zb * sa : a == 1 ? mp[1] + yb : zc - xb * sa + zb * ca;
        if (!std::isfinite(P)) return sbt_set_error(SBT_ERR_ARG, "marker positions must be finite");
        const int t0 = (int)std::floor(P - 1.5);
        lo = std::min(lo, t0);
        hi = std::max(hi, t0 + 4);
      }
      if (lo < 0 || hi > dims[a])
        return sbt_set_error(SBT_ERR_ARG, "an immersed body's stencils must not wrap across a face");
      cells *= hi - lo;
    }
    if (cells > d->ibm_box_cells) return sbt_set_error(SBT_ERR_ARG, "the body's stencil box exceeds ibm_box_cells");
  }
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(d->fext[k]) || !std::isfinite(d->wall_u[0][k]) || !std::isfinite(d->wall_u[1][k]))
      return sbt_set_error(SBT_ERR_ARG, "body force and wall velocities must be finite");
  return SBT_OK;
}

constexpr int H3X[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int H3Y[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int H3Z[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
constexpr int HOPP[27] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15, 26, 25, 24, 23, 22, 21, 20, 19};

// Solid records of a descriptor's mask: code[c] = 0 for a plain cell, else
// 1 + record; a record per solid cell (kSolidBit) and per fluid cell with a
// solid source.  The wall fraction of pulled direction i is the caller's
// q of the link toward the wall (direction opposite(i)); a short link with
// no fluid cell behind it takes 1/2.  Counts only when code is null.
sbt_status solid_records(const sbt3_desc *d, std::vector<int32_t> *code, std::vector<uint32_t> *bits,
                         std::vector<double> *rq, long long *count) {
  const int nx = d->nx, ny = d->ny, nz = d->nz, Q = d->lattice;
  const long long n = (long long)nx * ny * nz;
  auto cell = [&](int x, int y, int z, long long &out) -> bool {
    if (z < 0 || z >= nz) {
      if (d->walls_z) return false;
      z = (z + nz) % nz;
    }
    x = (x + nx) % nx;
    y = (y + ny) % ny;
    out = ((long long)z * ny + y) * nx + x;
    return true;
  };
  long long r = 0;
  if (code) code->assign(n, 0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const long long c = ((long long)z * ny + y) * nx + x;
        uint32_t b = 0;
        double qv[27];
        if (d->solid_mask[c]) {
          b = kSolidBit;
        } else {
          for (int i = 1; i < Q; ++i) {
            long long s;
            if (!cell(x - H3X[i], y - H3Y[i], z - H3Z[i], s) || !d->solid_mask[s]) continue;
            const int o = HOPP[i];
            double v = d->solid_q ? d->solid_q[c * Q + o] : 0.5;
            if (!(v > 0.0 && v <= 1.0)) return sbt_set_error(SBT_ERR_ARG, "wall fractions must lie in (0, 1]");
            long long u;
            if (v < 0.5 && (!cell(x + H3X[i], y + H3Y[i], z + H3Z[i], u) || d->solid_mask[u])) v = 0.5;
            b |= 1u << i;
            qv[i] = v;
          }
        }
        if (!b) continue;
        if (code) {
          (*code)[c] = (int32_t)(r + 1);
          bits->push_back(b);
          for (int i = 0; i < Q; ++i) rq->push_back((b & (1u << i)) && i > 0 ? qv[i] : 0.5);
        }
        ++r;
      }
  if (r >= (1ll << 31) - 1) return sbt_set_error(SBT_ERR_ARG, "too many solid records");
  *count = r;
  return SBT_OK;
}

// ibm_box_cells = 0 asks for the box of every cell the body's stencils can
// reach over its motion: the markers' extent (for the pitch/plunge motion,
// the disc their distance from the pivot sweeps in x and z, widened by the
// plunge along z) plus the 4-cell stencil and a cell of margin on each
// side, capped at the lattice.
sbt3_desc with_box(sbt3_desc d) {
  if (d.n_markers <= 0 || d.ibm_box_cells != 0 || !d.marker_xyz) return d;
  const int n = d.n_markers;
  double ext[3];
  for (int a = 0; a < 3; ++a) {
    double lo = 1e300, hi = -1e300;
    for (int j = 0; j < n; ++j) {
      lo = std::min(lo, d.marker_xyz[a * n + j]);
      hi = std::max(hi, d.marker_xyz[a * n + j]);
    }
    ext[a] = hi - lo;
  }
  if (d.body_motion == 1) {
    double r = 0.0;
    for (int j = 0; j < n; ++j) r = std::max(r, std::hypot(d.marker_xyz[j], d.marker_xyz[2 * n + j]));
    ext[0] = 2.0 * r;
    ext[2] = 2.0 * r + std::fabs(d.motion_p[5]);
  }
  const long long all = (long long)d.nx * d.ny * d.nz;
  long long cells = 1;
  for (int a = 0; a < 3; ++a) cells *= std::isfinite(ext[a]) ? (long long)std::ceil(ext[a]) + 6 : all;
  d.ibm_box_cells = std::max<long long>(64, std::min(cells, all));
  return d;
}

size_t body_bytes(const sbt3_desc *d) {
  const size_t n = d->n_markers, cap = (size_t)d->ibm_box_cells;
  return 4 * align256(n * 8) + align256(3 * n * 4) + align256(12 * n * 8) + 3 * align256(3 * n * 8) +
         align256(cap * 8) + 2 * align256(3 * cap * 8) + 2 * align256(6 * 4) + align256(6 * 8) + align256(4);
}

size_t plan_bytes(const sbt3_desc *d, long long *stage, long long records) {
  const long long n = (long long)d->nx * d->ny * d->nz;
  *stage = std::min<long long>(n, std::max<long long>(kStageCells, (long long)d->nx * d->ny));
  size_t b = 2 * align256((size_t)n * d->lattice * storage_bytes3(d->storage)) +
             align256((size_t)*stage * 4 * sizeof(double)) + 256;
  if (d->solid_mask)
    b += align256((size_t)n * sizeof(int32_t)) + align256((size_t)records * sizeof(uint32_t)) +
         align256((size_t)records * d->lattice * sizeof(double));
  if (d->n_markers > 0) b += body_bytes(d);
  return b;
}

#define HIP3(x)                                                                   \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) return sbt_set_error(SBT_ERR_DEVICE, hipGetErrorString(e_)); \
  } while (0)

#define SBT3_LAUNCH(K, st, q, g, s, ...)                                                          \
  [&]() -> hipError_t {                                                                             \
    switch ((st) + 4 * ((q) == 27)) {                                                               \
      case 0: hipLaunchKernelGGL((K<0, 19>), g, dim3(kThreads), 0, s, __VA_ARGS__); break;          \
      case 1: hipLaunchKernelGGL((K<1, 19>), g, dim3(kThreads), 0, s, __VA_ARGS__); break;          \
      case 2: hipLaunchKernelGGL((K<2, 19>), g, dim3(kThreads), 0, s, __VA_ARGS__); break;          \
      case 3: hipLaunchKernelGGL((K<3, 19>), g, dim3(kThreads), 0, s, __VA_ARGS__); break;          \
      case 4: hipLaunchKernelGGL((K<0, 27>), g, dim3(kThreads), 0, s, __VA_ARGS__); break;          \
      case 5: hipLaunchKernelGGL((K<1, 27>), g, dim3(kThreads), 0, s, __VA_ARGS__); break;          \
      case 6: hipLaunchKernelGGL((K<2, 27>), g, dim3(kThreads), 0, s, __VA_ARGS__); break;          \
      case 7: hipLaunchKernelGGL((K<3, 27>), g, dim3(kThreads), 0, s, __VA_ARGS__); break;          \
      default: return hipErrorInvalidValue;                                                         \
    }                                                                                               \
    return hipGetLastError();                                                                       \
  }()

hipError_t launch_ibm(sbt3_ctx &X, int pull) {
  const Ibm3 &B = X.ibm;
  // one wave per workgroup for the per-marker kernels: their threads are
  // few and latency-bound, so they are spread over as many CUs as possible
  const dim3 gk((unsigned)((B.cap + kThreads - 1) / kThreads)), gn((unsigned)((B.n + 63) / 64));
  // tiles, grid-stride: the box is known only on the device and is mostly
  // smaller than cap, and workgroups that find no tile still cost dispatch
  // time, so the grid is capped at two small workgroups per CU
  const dim3 gs((unsigned)std::min<long long>(512, (B.cap + kSpThreads - 1) / kSpThreads));
  const Pose3 q0 = B.kind ? pose3(B, (double)X.ibm_t) : Pose3{}, q1 = B.kind ? pose3(B, (double)(X.ibm_t + 1)) : Pose3{};
  hipLaunchKernelGGL(ibm3_markers_kernel, gn, dim3(64), 0, X.stream, q0, q1, B);
  hipLaunchKernelGGL(ibm3_box_kernel, dim3(1), dim3(64), 0, X.stream, X.p, B);
  const void *lat = X.lat[X.cur];
  switch (X.d.storage + 4 * (X.d.lattice == 27)) {
    case 0: hipLaunchKernelGGL((ibm3_moments_kernel<0, 19>), gk, dim3(kThreads), 0, X.stream, X.p, lat, pull, B); break;
    case 1: hipLaunchKernelGGL((ibm3_moments_kernel<1, 19>), gk, dim3(kThreads), 0, X.stream, X.p, lat, pull, B); break;
    case 2: hipLaunchKernelGGL((ibm3_moments_kernel<2, 19>), gk, dim3(kThreads), 0, X.stream, X.p, lat, pull, B); break;
    case 3: hipLaunchKernelGGL((ibm3_moments_kernel<3, 19>), gk, dim3(kThreads), 0, X.stream, X.p, lat, pull, B); break;
    case 4: hipLaunchKernelGGL((ibm3_moments_kernel<0, 27>), gk, dim3(kThreads), 0, X.stream, X.p, lat, pull, B); break;
    case 5: hipLaunchKernelGGL((ibm3_moments_kernel<1, 27>), gk, dim3(kThreads), 0, X.stream, X.p, lat, pull, B); break;
    case 6: hipLaunchKernelGGL((ibm3_moments_kernel<2, 27>), gk, dim3(kThreads), 0, X.stream, X.p, lat, pull, B); break;
    case 7: hipLaunchKernelGGL((ibm3_moments_kernel<3, 27>), gk, dim3(kThreads), 0, X.stream, X.p, lat, pull, B); break;
    default: return hipErrorInvalidValue;
  }
  for (int it = 0; it < B.iters; ++it) {
    hipLaunchKernelGGL(ibm3_interp_kernel, gn, dim3(64), 0, X.stream, B);
    hipLaunchKernelGGL(ibm3_spread_kernel, gs, dim3(kSpThreads), 0, X.stream, B);
  }
  return hipGetLastError();
}

sbt_status check_slab(sbt3_ctx *ctx, int32_t z0, int32_t nz, const void *a, const void *b, const void *c,
                      const void *e) {
  if (!ctx) return sbt_set_error(SBT_ERR_ARG, "null context");
  if (z0 < 0 || nz < 1 || z0 + nz > ctx->d.nz) return sbt_set_error(SBT_ERR_ARG, "planes out of range");
  if (!a || !b || !c || !e) return sbt_set_error(SBT_ERR_ARG, "null field");
  return SBT_OK;
}

}  // namespace

extern "C" {

sbt_status sbt3_plan(const sbt3_desc *desc_in, size_t *device_bytes) {
  if (!desc_in) return sbt_set_error(SBT_ERR_ARG, "null descriptor");
  const sbt3_desc dd = with_box(*desc_in);
  const sbt3_desc *desc = &dd;
  sbt_status st = check_desc(desc);
  if (st) return st;
  if (!device_bytes) return sbt_set_error(SBT_ERR_ARG, "null output");
  long long stage, records = 0;
  if (desc->solid_mask) {
    st = solid_records(desc, nullptr, nullptr, nullptr, &records);
    if (st) return st;
  }
  *device_bytes = plan_bytes(desc, &stage, records);
  return SBT_OK;
}

sbt_status sbt3_create(const sbt3_desc *desc_in, void *device_buf, size_t bytes, void *hip_stream,
                       sbt3_ctx **out) {
  if (!desc_in) return sbt_set_error(SBT_ERR_ARG, "null descriptor");
  const sbt3_desc dd = with_box(*desc_in);
  const sbt3_desc *desc = &dd;
  sbt_status st = check_desc(desc);
  if (st) return st;
  if (!out) return sbt_set_error(SBT_ERR_ARG, "null output");
  *out = nullptr;
  long long stage, records = 0;
  std::vector<int32_t> code;
  std::vector<uint32_t> bits;
  std::vector<double> rq;
  if (desc->solid_mask) {
    st = solid_records(desc, &code, &bits, &rq, &records);
    if (st) return st;
  }
  const size_t need = plan_bytes(desc, &stage, records);
  if (!device_buf || bytes < need) return sbt_set_error(SBT_ERR_BUFSIZE, "device buffer smaller than planned");
  if ((uintptr_t)device_buf & 255) return sbt_set_error(SBT_ERR_ARG, "device buffer must be 256-byte aligned");
  sbt3_ctx *X = new sbt3_ctx();
  X->d = *desc;
  Params &p = X->p;
  p.nx = desc->nx;
  p.ny = desc->ny;
  p.nz = desc->nz;
  p.n = (long long)desc->nx * desc->ny * desc->nz;
  p.tau = desc->tau;
  p.pre = 1.0 - 0.5 / desc->tau;
  p.rho0 = desc->rho0;
  p.om_f = (float)(1.0 / desc->tau);
  p.pre_f = (float)p.pre;
  p.rho0_f = (float)desc->rho0;
  for (int k = 0; k < 3; ++k) {
    p.F[k] = desc->fext[k];
    p.F_f[k] = (float)desc->fext[k];
    p.uw[0][k] = desc->wall_u[0][k];
    p.uw[1][k] = desc->wall_u[1][k];
  }
  p.walls = desc->walls_z ? 1 : 0;
  char *b = static_cast<char *>(device_buf);
  const size_t lat = align256((size_t)p.n * desc->lattice * storage_bytes3(desc->storage));
  X->lat[0] = b;
  X->lat[1] = b + lat;
  X->stage = reinterpret_cast<double *>(b + 2 * lat);
  X->err = reinterpret_cast<int *>(b + 2 * lat + align256((size_t)stage * 4 * sizeof(double)));
  X->stage_cells = stage;
  X->stream = static_cast<hipStream_t>(hip_stream);
  X->d.solid_mask = nullptr;  // borrowed for this call only
  X->d.solid_q = nullptr;
  p.scode = nullptr;
  p.rbits = nullptr;
  p.rq = nullptr;
  if (desc->solid_mask) {
    char *sb = b + 2 * lat + align256((size_t)stage * 4 * sizeof(double)) + 256;
    int32_t *dcode = reinterpret_cast<int32_t *>(sb);
    uint32_t *dbits = reinterpret_cast<uint32_t *>(sb + align256((size_t)p.n * sizeof(int32_t)));
    double *dq = reinterpret_cast<double *>(sb + align256((size_t)p.n * sizeof(int32_t)) +
                                            align256((size_t)records * sizeof(uint32_t)));
    bool ok = hipMemcpy(dcode, code.data(), sizeof(int32_t) * code.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (records > 0) {
      ok &= hipMemcpy(dbits, bits.data(), sizeof(uint32_t) * bits.size(), hipMemcpyHostToDevice) == hipSuccess;
      ok &= hipMemcpy(dq, rq.data(), sizeof(double) * rq.size(), hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!ok) {
      delete X;
      return sbt_set_error(SBT_ERR_DEVICE, "solid table upload");
    }
    p.scode = dcode;
    p.rbits = dbits;
    p.rq = dq;
    X->n_records = records;
  }
  p.ibm_F = nullptr;
  p.ibm_box = nullptr;
  if (desc->n_markers > 0) {
    size_t off = 2 * lat + align256((size_t)stage * 4 * sizeof(double)) + 256;
    if (desc->solid_mask)
      off += align256((size_t)p.n * sizeof(int32_t)) + align256((size_t)records * sizeof(uint32_t)) +
             align256((size_t)records * desc->lattice * sizeof(double));
    char *q = b + off;
    auto take = [&](size_t bytes) {
      char *r = q;
      q += align256(bytes);
      return r;
    };
    const int n = desc->n_markers;
    const size_t cap = (size_t)desc->ibm_box_cells;
    Ibm3 &B = X->ibm;
    B.n = n;
    B.iters = desc->mdf_iters;
    B.kind = desc->body_motion;
    B.cap = (long long)cap;
    for (int i = 0; i < 10; ++i) B.mp[i] = desc->motion_p[i];
    double *xb = reinterpret_cast<double *>(take(n * 8));
    double *yb = reinterpret_cast<double *>(take(n * 8));
    double *zb = reinterpret_cast<double *>(take(n * 8));
    double *dA = reinterpret_cast<double *>(take(n * 8));
    B.xb = xb;
    B.yb = yb;
    B.zb = zb;
    B.dA = dA;
    B.tap = reinterpret_cast<int *>(take(3 * n * 4));
    B.phi = reinterpret_cast<double *>(take(12 * n * 8));
    B.ud = reinterpret_cast<double *>(take(3 * n * 8));
    B.g = reinterpret_cast<double *>(take(3 * n * 8));
    B.ft = reinterpret_cast<double *>(take(3 * n * 8));
    B.rho = reinterpret_cast<double *>(take(cap * 8));
    B.u = reinterpret_cast<double *>(take(3 * cap * 8));
    B.Fbox = reinterpret_cast<double *>(take(3 * cap * 8));
    B.box = reinterpret_cast<int *>(take(6 * 4));
    B.lohi = reinterpret_cast<int *>(take(6 * 4));
    B.fs = reinterpret_cast<double *>(take(6 * 8));
    B.err = X->err;
    bool ok = hipMemcpy(xb, desc->marker_xyz, n * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy(yb, desc->marker_xyz + n, n * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy(zb, desc->marker_xyz + 2 * n, n * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy(dA, desc->marker_dA, n * 8, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemset(B.box, 0, 6 * 4) == hipSuccess;
    ok &= hipMemset(B.fs, 0, 6 * 8) == hipSuccess;
    const int lohi0[6] = {1 << 30, 1 << 30, 1 << 30, -(1 << 30), -(1 << 30), -(1 << 30)};
    ok &= hipMemcpy(B.lohi, lohi0, sizeof lohi0, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemset(B.ft, 0, 3 * n * 8) == hipSuccess;
    if (!ok) {
      delete X;
      return sbt_set_error(SBT_ERR_DEVICE, "immersed-body upload");
    }
    p.ibm_F = B.Fbox;
    p.ibm_box = B.box;
  }
  X->d.marker_xyz = nullptr;  // borrowed for this call only
  X->d.marker_dA = nullptr;
  if (hipMemsetAsync(X->err, 0, sizeof(int), X->stream) != hipSuccess) {
    delete X;
    return sbt_set_error(SBT_ERR_DEVICE, "error flag clear");
  }
  *out = X;
  return SBT_OK;
}

sbt_status sbt3_destroy(sbt3_ctx *ctx) {
  delete ctx;
  return SBT_OK;
}

sbt_status sbt3_init_slab(sbt3_ctx *ctx, int32_t z0, int32_t nz, const double *rho, const double *ux,
                          const double *uy, const double *uz) {
  sbt_status st = check_slab(ctx, z0, nz, rho, ux, uy, uz);
  if (st) return st;
  sbt3_ctx &X = *ctx;
  const long long plane = (long long)X.p.nx * X.p.ny, total = plane * nz;
  for (long long k0 = 0; k0 < total; k0 += X.stage_cells) {
    const long long m = std::min(X.stage_cells, total - k0);
    const double *src[4] = {rho, ux, uy, uz};
    for (int q = 0; q < 4; ++q)
      HIP3(hipMemcpyAsync(X.stage + q * m, src[q] + k0, sizeof(double) * m, hipMemcpyHostToDevice, X.stream));
    X.post = false;  // the lattice holds an initial, pre-collision state again
    HIP3(SBT3_LAUNCH(init3_kernel, X.d.storage, X.d.lattice, dim3((unsigned)((m + kThreads - 1) / kThreads)), X.stream, X.p,
                     X.lat[X.cur], (const double *)X.stage, (long long)z0 * plane + k0, m));
    HIP3(hipStreamSynchronize(X.stream));
  }
  return SBT_OK;
}

// The step kernel's launch after forcing loop L (its first workgroup sums
// that loop's F_s into slot L & 1).
hipError_t launch_step3(sbt3_ctx &X, int pull) {
  Params p = X.p;
  long long wgs = (X.p.n + kThreads - 1) / kThreads;
  if (X.ibm.n > 0) {
    p.fs_n = X.ibm.n;
    p.fs_ft = X.ibm.ft;
    p.fs_dA = X.ibm.dA;
    p.fs_out = X.ibm.fs + 3 * ((X.ibm_t - 1) & 1);
    ++wgs;
  }
  return SBT3_LAUNCH(step3_kernel, X.d.storage, X.d.lattice, dim3((unsigned)wgs), X.stream, p,
                     (const void *)X.lat[X.cur], X.lat[1 - X.cur], pull, X.err);
}

sbt_status sbt3_step(sbt3_ctx *ctx, int32_t n) {
  if (!ctx || n < 0) return sbt_set_error(SBT_ERR_ARG, "bad argument");
  sbt3_ctx &X = *ctx;
  if (n == 0) return SBT_OK;
  if (!X.post) {  // collide the initial state in place: the lattice then holds f*
    if (X.ibm.n > 0) {
      X.ibm_t = 0;
      HIP3(launch_ibm(X, 0));
      ++X.ibm_t;
    }
    HIP3(launch_step3(X, 0));
    X.cur = 1 - X.cur;
    X.post = true;
  }
  for (int t = 0; t < n; ++t) {
    if (X.ibm.n > 0) {
      HIP3(launch_ibm(X, 1));
      ++X.ibm_t;
    }
    HIP3(launch_step3(X, 1));
    X.cur = 1 - X.cur;
  }
  return SBT_OK;
}

sbt_status sbt3_synchronize(sbt3_ctx *ctx) {
  if (!ctx) return sbt_set_error(SBT_ERR_ARG, "null context");
  HIP3(hipStreamSynchronize(ctx->stream));
  int e = 0;
  HIP3(hipMemcpy(&e, ctx->err, sizeof(int), hipMemcpyDeviceToHost));
  if (e) {
    HIP3(hipMemset(ctx->err, 0, sizeof(int)));
    if (e & 1) return sbt_set_error(SBT_ERR_NONFINITE, "a density became NaN or Inf");
    return sbt_set_error(SBT_ERR_MARKER_OUTSIDE, "the immersed body's stencils outgrew ibm_box_cells or left the box");
  }
  return SBT_OK;
}

sbt_status sbt3_body_force(sbt3_ctx *ctx, double out[3]) {
  if (!ctx || !out) return sbt_set_error(SBT_ERR_ARG, "null argument");
  if (ctx->ibm.n == 0) return sbt_set_error(SBT_ERR_STATE, "no immersed body");
  if (!ctx->post) return sbt_set_error(SBT_ERR_STATE, "no completed step");
  // the last launch ran the forcing loop of the step after the last completed
  // one: the completed step's loop is the one before it
  HIP3(hipMemcpyAsync(out, ctx->ibm.fs + 3 * ((ctx->ibm_t - 2) & 1), 3 * sizeof(double), hipMemcpyDeviceToHost,
                      ctx->stream));
  HIP3(hipStreamSynchronize(ctx->stream));
  // a step whose stencils left the box ran without the body force: its F_s
  // is not a result (the flag stays set for sbt3_synchronize)
  int e = 0;
  HIP3(hipMemcpy(&e, ctx->err, sizeof(int), hipMemcpyDeviceToHost));
  if (e & 2) return sbt_set_error(SBT_ERR_MARKER_OUTSIDE, "the immersed body's stencils outgrew ibm_box_cells or left the box");
  return SBT_OK;
}

sbt_status sbt3_read_slab(sbt3_ctx *ctx, int32_t z0, int32_t nz, double *rho, double *ux, double *uy, double *uz) {
  sbt_status st = check_slab(ctx, z0, nz, rho, ux, uy, uz);
  if (st) return st;
  sbt3_ctx &X = *ctx;
  const long long plane = (long long)X.p.nx * X.p.ny, total = plane * nz;
  for (long long k0 = 0; k0 < total; k0 += X.stage_cells) {
    const long long m = std::min(X.stage_cells, total - k0);
    // after a step the streamed state is gathered from the lattice the last step read
    const void *src = X.post ? X.lat[1 - X.cur] : X.lat[X.cur];
    HIP3(SBT3_LAUNCH(read3_kernel, X.d.storage, X.d.lattice, dim3((unsigned)((m + kThreads - 1) / kThreads)), X.stream, X.p, src,
                     X.stage, (long long)z0 * plane + k0, m, X.post ? 1 : 0));
    double *dst[4] = {rho, ux, uy, uz};
    for (int q = 0; q < 4; ++q)
      HIP3(hipMemcpyAsync(dst[q] + k0, X.stage + q * m, sizeof(double) * m, hipMemcpyDeviceToHost, X.stream));
    HIP3(hipStreamSynchronize(X.stream));
  }
  return SBT_OK;
}

}  // extern "C"
