// Run statistics on the device: the force-coefficient statistics of
// Sec. 3.3 (Eq. (21): mean drag, rms lift, Strouhal number) over the force
// history ring, and the velocity-change measure E of the Sec. 3.2
// convergence criterion over the leaf cells of every level.
#include "sbt_internal.h"

namespace {
using namespace sbt;

constexpr int kStatThreads = 1024;

// Sum over the workgroup in a fixed order (per-thread partials, then a tree).
__device__ double wg_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kStatThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double wg_min(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kStatThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// History entry i (0 .. n-1) of the window: substep first + i, ring slot
// (first + i) mod cap, stored as {Fx, Fy}.
__device__ __forceinline__ double2 hist_at(const double *hist, int64_t cap, int64_t first, int64_t i) {
  const int64_t slot = (first + i) % cap;
  return make_double2(hist[2 * slot], hist[2 * slot + 1]);
}

// out = {mean C_D, mean C_L, rms(C_D - mean), rms(C_L - mean), St, upward
// crossings of C_L through its mean, samples}.  C = F * scale with
// scale = 1 / (rho0 U^2 L / 2).  The shedding frequency is the number of
// full periods between the first and the last upward crossing over the time
// between them; crossing times are interpolated linearly between substeps.
__global__ __launch_bounds__(kStatThreads) void force_stats_kernel(const double *hist, int64_t cap, int64_t first,
                                                                   int64_t n, double scale, double l_over_u,
                                                                   double *out) {
#pragma clang fp contract(off)
  __shared__ double red[kStatThreads];
  const int tid = threadIdx.x;
  double sd = 0.0, sl = 0.0;
  for (int64_t i = tid; i < n; i += kStatThreads) {
    const double2 f = hist_at(hist, cap, first, i);
    sd += f.x * scale;
    sl += f.y * scale;
  }
  const double md = wg_sum(sd, red) / (double)n;
  const double ml = wg_sum(sl, red) / (double)n;
  double vd = 0.0, vl = 0.0;
  for (int64_t i = tid; i < n; i += kStatThreads) {
    const double2 f = hist_at(hist, cap, first, i);
    const double dd = f.x * scale - md, dl = f.y * scale - ml;
    vd += dd * dd;
    vl += dl * dl;
  }
  const double rd = sqrt(wg_sum(vd, red) / (double)n);
  const double rl = sqrt(wg_sum(vl, red) / (double)n);
  double cnt = 0.0, t0 = INFINITY, t1 = INFINITY;  // t1 holds -(last crossing)
  for (int64_t i = tid; i + 1 < n; i += kStatThreads) {
    const double c0 = hist_at(hist, cap, first, i).y * scale - ml;
    const double c1 = hist_at(hist, cap, first, i + 1).y * scale - ml;
    if (c0 < 0.0 && c1 >= 0.0) {
      const double t = (double)i + c0 / (c0 - c1);
      cnt += 1.0;
      t0 = fmin(t0, t);
      t1 = fmin(t1, -t);
    }
  }
  const double ncr = wg_sum(cnt, red);
  const double tf = wg_min(t0, red), tl = -wg_min(t1, red);
  if (tid == 0) {
    out[0] = md;
    out[1] = ml;
    out[2] = rd;
    out[3] = rl;
    out[4] = ncr >= 2.0 ? (ncr - 1.0) / (tl - tf) * l_over_u : 0.0;
    out[5] = ncr;
    out[6] = (double)n;
  }
}

// One workgroup per owned block of a level, one thread per cell.  fields is
// the level's readout [block][rho, ux, uy][256]; snap holds [block][ux, uy][256].
// mode 2: per-block partial {sum |u - u_snap|, sum |u|, leaf cells} over the
// block's leaf cells (cells neither covered by the finer level nor solid); mode 1: the
// snapshot takes the current velocity; mode 3 does both (compare first).
__global__ __launch_bounds__(256) void velocity_change_kernel(const BlockMeta *meta, const uint16_t *codes,
                                                              const uint16_t *sbits, int b0, const double *fields,
                                                              double *snap, int mode, double *partial) {
#pragma clang fp contract(off)
  __shared__ double red[3][256];
  const int ob = blockIdx.x, cell = threadIdx.x;
  const BlockMeta m = meta[b0 + ob];
  const uint16_t code = (m.flags & BF_CODES) ? codes[(size_t)m.code * kCells + cell] : (uint16_t)0;
  const uint16_t sb = (m.flags & BF_SOLID) ? sbits[(size_t)m.solid * kCells + cell] : (uint16_t)0;
  const bool leaf = !(code & CC_HIDDEN) && !(sb & SB_SOLID);
  const double ux = fields[((size_t)ob * 3 + 1) * kCells + cell];
  const double uy = fields[((size_t)ob * 3 + 2) * kCells + cell];
  double *sp = snap + (size_t)ob * 2 * kCells;
  double d = 0.0, u = 0.0, w = 0.0;
  if (leaf && (mode & 2)) {
    const double dx = ux - sp[cell], dy = uy - sp[kCells + cell];
    d = sqrt(dx * dx + dy * dy);
    u = sqrt(ux * ux + uy * uy);
    w = 1.0;
  }
  if (mode & 1) {
    sp[cell] = leaf ? ux : 0.0;
    sp[kCells + cell] = leaf ? uy : 0.0;
  }
  if (!(mode & 2)) return;
  red[0][cell] = d;
  red[1][cell] = u;
  red[2][cell] = w;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (cell < s)
      for (int q = 0; q < 3; ++q) red[q][cell] += red[q][cell + s];
    __syncthreads();
  }
  if (cell == 0)
    for (int q = 0; q < 3; ++q) partial[(size_t)ob * 3 + q] = red[q][0];
}

}  // namespace

extern "C" hipError_t sbt_launch_force_stats(const double *hist, int64_t cap, int64_t first, int64_t n, double scale,
                                             double l_over_u, double *out, hipStream_t s) {
  if (n <= 0 || cap <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(force_stats_kernel, dim3(1), dim3(kStatThreads), 0, s, hist, cap, first, n, scale, l_over_u,
                     out);
  return hipGetLastError();
}

extern "C" hipError_t sbt_launch_velocity_change(const BlockMeta *meta, const uint16_t *codes, const uint16_t *sbits,
                                                 int b0, int n, const double *fields, double *snap, int mode,
                                                 double *partial, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(velocity_change_kernel, dim3(n), dim3(256), 0, s, meta, codes, sbits, b0, fields, snap, mode,
                     partial);
  return hipGetLastError();
}
