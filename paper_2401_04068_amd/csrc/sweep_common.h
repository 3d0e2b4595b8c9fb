// Helpers shared by the sweep kernels (sweep.hip: one frequency per
// wavefront; sweep16.hip: four frequencies per wavefront).
#pragma once

#include <hip/hip_runtime.h>

#include "lti_kernels.h"

namespace lti {
namespace sweep_detail {

constexpr int kWaves = 4;  // wavefronts per workgroup, one tile each

template <typename T>
using gptr = const T __attribute__((address_space(1)))*;  // global
template <typename T>
using cptr = const T __attribute__((address_space(4)))*;  // constant (scalar loads)
template <typename T>
using lptr = const T __attribute__((address_space(3)))*;  // LDS
template <typename T>
using gmut = T __attribute__((address_space(1)))*;  // global, written

// Stores through the global address space (a generic store also counts
// against the LDS wait counter).
__device__ __forceinline__ void store_c(double* G, int idx, double2 v) {
  gmut<double> g = (gmut<double>)G + 2 * idx;
  g[0] = v.x;
  g[1] = v.y;
}
__device__ __forceinline__ void store_info(lti_point_info* info, int64_t k, const lti_point_info& v) {
  uint64_t bits;
  __builtin_memcpy(&bits, &v, sizeof(bits));
  ((gmut<uint64_t>)info)[k] = bits;
}

// Launch tile t (wave-uniform) of a sweep launch: its segment, and the
// frequencies and columns it covers.
struct Tile {
  uint32_t start, count;
  int j0, mc;
};

__device__ __forceinline__ int seg_of(const SweepLaunch& L, int t) {
  int s = 0;
#pragma unroll
  for (int i = 1; i < kMaxSegs; ++i)
    if (i < L.nseg && t >= (int)L.seg[i].tile0) s = i;
  return s;
}

__device__ __forceinline__ Tile tile_of(const SweepSeg& g, int t) {
  const uint32_t local = g.first + (uint32_t)(t - (int)g.tile0);
  const uint32_t fb = local / g.S, grp = local % g.S;
  Tile x;
  x.start = fb * g.F;
  x.count = min((uint32_t)g.F, g.K - x.start);
  x.j0 = (int)grp * g.mc;
  x.mc = min((int)g.mc, g.rd.m - x.j0);
  return x;
}

// Read-only view of one array of the reduced model, staged in LDS (kLds) or
// read from global memory.
template <typename T, bool kLds>
struct Src {
  const T* p;
  __device__ __forceinline__ T operator[](int i) const {
    if constexpr (kLds)
      return ((lptr<T>)p)[i];
    else
      return ((gptr<T>)p)[i];
  }
  // an entry every lane reads at once (a scalar load from global memory)
  __device__ __forceinline__ T uniform(int i) const {
    if constexpr (kLds)
      return ((lptr<T>)p)[i];
    else
      return ((cptr<T>)p)[i];
  }
};

template <bool kLds>
struct ModelSrc {
  Src<double, kLds> H, Bt, Ct;
  Src<float, kLds> H32, Bt32;
};

__device__ __forceinline__ double readlane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double rsqrt_t(double x) { return rsqrt(x); }
__device__ __forceinline__ float rsqrt_t(float x) { return rsqrtf(x); }

__device__ __forceinline__ int hoff32(int j) { return j * (j + 3) / 2; }

__device__ __forceinline__ int xcd_swizzle(int b, int nb) {
  // Workgroups are dealt to the 8 XCDs round-robin; renumber them so that each
  // XCD works on a contiguous range of tiles (tiles of one request share H in
  // that XCD's L2).
  const int per = nb / 8, rem = nb % 8;
  const int xcd = b % 8, pos = b / 8;
  return (xcd < rem) ? xcd * (per + 1) + pos : rem * (per + 1) + (xcd - rem) * per + pos;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = fmax(x, __shfl_xor(x, d, 64));
  return x;
}


}  // namespace sweep_detail
}  // namespace lti
