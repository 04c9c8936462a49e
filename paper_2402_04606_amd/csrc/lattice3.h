// D3Q19 / D3Q27 velocity sets, weights and storage forms shared by the 3D
// kernels (the uniform level and the block forest).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// Rest, +x -x +y -y +z -z, the 12 edges (+-1, +-1, 0), (+-1, 0, +-1),
// (0, +-1, +-1), then (D3Q27 only) the 8 corners.
__device__ constexpr int E3X[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                    1, -1, 1, -1, 1, -1, 1, -1};
__device__ constexpr int E3Y[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1,
                                    1, 1, -1, -1, 1, 1, -1, -1};
__device__ constexpr int E3Z[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1,
                                    1, 1, 1, 1, -1, -1, -1, -1};

__device__ constexpr int OPP3[27] = {0,  2,  1,  4,  3,  6,  5,  10, 9,  8,  7,  14, 13, 12,
                                     11, 18, 17, 16, 15, 26, 25, 24, 23, 22, 21, 20, 19};

// Weights: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216.
template <typename C, int Q>
__device__ __forceinline__ C w3(int i) {
  if constexpr (Q == 19) return i == 0 ? C(1.0 / 3.0) : (i < 7 ? C(1.0 / 18.0) : C(1.0 / 36.0));
  return i == 0 ? C(8.0 / 27.0) : (i < 7 ? C(2.0 / 27.0) : (i < 19 ? C(1.0 / 54.0) : C(1.0 / 216.0)));
}

template <int ST> struct Store3;
template <> struct Store3<0> {
  using T = double;
  __device__ static double ld(T v) { return v; }
  __device__ static T st(double v) { return v; }
};
template <> struct Store3<1> {
  using T = float;
  __device__ static float ld(T v) { return v; }
  __device__ static T st(float v) { return v; }
};
template <> struct Store3<2> {
  using T = _Float16;
  __device__ static float ld(T v) { return (float)v; }
  __device__ static T st(float v) { return (_Float16)v; }
};
template <> struct Store3<3> {  // bf16, round to nearest even
  using T = uint16_t;
  __device__ static float ld(T v) { return __uint_as_float(((uint32_t)v) << 16); }
  __device__ static T st(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (T)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (T)(u >> 16);
  }
};

}  // namespace
