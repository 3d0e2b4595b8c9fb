// Helpers shared by the sweep kernels (sweep.hip: one frequency per
// wavefront; sweep16.hip: four frequencies per wavefront).
#pragma once

#include <cfloat>

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

// A point's record: plain store, or (columns split over tiles) merged with
// the other column groups' records by atomic maxima on its two 32-bit words:
// the larger error estimate, and the worse path (FP64 < REFINED < FALLBACK <
// SINGULAR < FP64_DD order of the codes), then the larger solve count.
// Merged records start from zero (the runtime clears them).
__device__ __forceinline__ void put_info(const ReqDesc& rd, int64_t k, const lti_point_info& v) {
  if (rd.flags & kFlagMergeInfo) {
    gmut<uint32_t> w = (gmut<uint32_t>)rd.info + 2 * k;
    const uint32_t w0 = __float_as_uint(v.est_rel_err);
    const uint32_t w1 = (uint32_t)v.iters | ((uint32_t)v.path << 8);
    atomicMax((uint32_t*)&w[0], w0);
    atomicMax((uint32_t*)&w[1], w1);
  } else {
    store_info(rd.info, k, v);
  }
}

// Estimated relative error of a float64 point from its triangular factor:
// (u / 2) sqrt(n) max|R(k,k)| / min|R(k,k)|.  The diagonal spread alone is a
// lower bound on kappa(s I - H) that falls short by about 0.6 / sqrt(n) on
// an isolated near-resonance (measured on reduced models with random
// orthogonal bases, n = 16 .. 300), hence the sqrt(n).  A point whose
// estimate exceeds kFP64QueueFraction * rtol is finished by the
// double-double refinement against A.
constexpr double kFP64QueueFraction = 0.25;
__device__ __forceinline__ double fp64_estimate(int n, double diag_spread) {
  return 0.5 * DBL_EPSILON * sqrt((double)n) * diag_spread;
}
__device__ __forceinline__ bool fp64_needs_dd(const ReqDesc& rd, double est) {
  return !(est <= kFP64QueueFraction * rd.rtol) || (rd.flags & kFlagForceDD);
}

// Hand point k, columns j0 .. j0+mc-1, to the extended-precision refinement
// (one lane calls this).
__device__ __forceinline__ void enqueue_dd(const ReqDesc& rd, int64_t k, int j0, int mc, int fp32_solves,
                                           int reason) {
  const uint32_t e = atomicAdd(rd.fbq, 1u);
  gmut<uint32_t> q = (gmut<uint32_t>)rd.fbq + 2 + 2 * (size_t)e;
  q[0] = (uint32_t)k;
  q[1] = (uint32_t)j0 | ((uint32_t)mc << 8) | ((uint32_t)min(fp32_solves, 255) << 16) | ((uint32_t)reason << 24);
}

// Evaluation point s_k = sr + j si of a request (see ReqDesc).
struct SPoint {
  double re, im;
};
__device__ __forceinline__ SPoint point_of(const ReqDesc& rd, int64_t k) {
  const gptr<double> w = (gptr<double>)rd.omega;
  const int kind = (int)((rd.flags >> 8) & 3u);
  SPoint s;
  if (kind == kPointsS) {
    s.re = w[2 * k];
    s.im = w[2 * k + 1];
  } else if (kind == kPointsZ) {
    sincos(w[k], &s.im, &s.re);
  } else {
    s.re = 0.0;
    s.im = w[k];
  }
  return s;
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
// A squared norm usable for a rotation or a reciprocal: a normal number of
// the format (not zero, not subnormal, not infinite, not NaN).  A step whose
// norm falls outside that range -- a zero column, or a model whose scale
// squares out of the format -- is treated as singular, so that the point is
// flagged (the float32 solves then hand it to the float64 refinement)
// instead of returning a silently wrong value.
__device__ __forceinline__ bool norm2_ok(double x) { return x >= DBL_MIN && x <= DBL_MAX; }
__device__ __forceinline__ bool norm2_ok(float x) { return x >= FLT_MIN && x <= FLT_MAX; }
// float32 (the refined path's solves, which its float64 residuals check):
// the hardware reciprocal square root (1 ulp), with the input held at the
// smallest normal number instead of the library's rescaling of denormal
// inputs, which the instruction does not take.
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(fmaxf(x, FLT_MIN)); }

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
