// Cross-lane moves within a wavefront through DPP (data-parallel primitives:
// a VALU operand modifier, no LDS round trip).  CDNA4 DPP works on 32-bit
// lanes, so doubles move as two halves.
//
// Control codes (GCN/CDNA ISA, DPP_CTRL field):
//   quad_perm [a,b,c,d] = a | b << 2 | c << 4 | d << 6   (within groups of 4)
//   row_shl:n = 0x100 + n, row_shr:n = 0x110 + n       (within rows of 16)
//   row_mirror = 0x140 (lane i <- 15 - i), row_half_mirror = 0x141 (i <- 7 - i)
//   row_bcast:15 = 0x142, row_bcast:31 = 0x143
//   row_newbcast:n = 0x150 + n (every lane of a row <- lane n of that row)
// Lanes whose source falls outside their row keep `old`.
#pragma once

#include <hip/hip_runtime.h>

namespace lti {

constexpr int kDppQuadSwap1 = 0xB1;  // quad_perm [1,0,3,2]: i <- i ^ 1
constexpr int kDppQuadSwap2 = 0x4E;  // quad_perm [2,3,0,1]: i <- i ^ 2
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;
constexpr int dpp_row_shl(int n) { return 0x100 + n; }
constexpr int dpp_row_shr(int n) { return 0x110 + n; }
constexpr int dpp_row_newbcast(int n) { return 0x150 + n; }

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i(int old, int x) {
  return __builtin_amdgcn_update_dpp(old, x, CTRL, ROW_MASK, 0xf, false);
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp(float x, float old = 0.0f) {
  return __int_as_float(dpp_i<CTRL, ROW_MASK>(__float_as_int(old), __float_as_int(x)));
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp(double x, double old = 0.0) {
  const int lo = dpp_i<CTRL, ROW_MASK>(__double2loint(old), __double2loint(x));
  const int hi = dpp_i<CTRL, ROW_MASK>(__double2hiint(old), __double2hiint(x));
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of G lanes (G = 1, 2, 4, 8, 16); every lane of the
// group gets the total.  Pairings: i^1, i^2 (quads), 7-i (half rows), 15-i
// (rows) -- each stage pairs the two halves of the next larger group.
template <int G, typename T>
__device__ __forceinline__ T group_sum_dpp(T x) {
  if constexpr (G >= 2) x += dpp<kDppQuadSwap1>(x);
  if constexpr (G >= 4) x += dpp<kDppQuadSwap2>(x);
  if constexpr (G >= 8) x += dpp<kDppRowHalfMirror>(x);
  if constexpr (G >= 16) x += dpp<kDppRowMirror>(x);
  return x;
}

// Variant for code in which every lane of the wavefront is active and the
// pattern has a source inside the row for every lane (quad_perm, mirrors):
// the destination needs no initial value, which saves a move per half.
template <int CTRL>
__device__ __forceinline__ double dpp_full(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over each 16-lane row, every lane active (same pairings and order as
// group_sum_dpp<16>).
__device__ __forceinline__ double row_sum16_full(double x) {
  x += dpp_full<kDppQuadSwap1>(x);
  x += dpp_full<kDppQuadSwap2>(x);
  x += dpp_full<kDppRowHalfMirror>(x);
  return x + dpp_full<kDppRowMirror>(x);
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_d(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Exchanges between 16-lane rows (gfx950 v_permlane16_swap / 32_swap, VALU
// operations): with both operands x, permlane16_swap returns (even row's x,
// odd row's x) at each position of a row pair, permlane32_swap returns (low
// half's x, high half's x).  Summing the pair gives every lane
// x[l] + x[l ^ 16] (resp. x[l ^ 32]), added in the same order on both sides.
__device__ __forceinline__ double xor16_sum(double x) {
  const unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ double xor32_sum(double x) {
  const unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}

// Reduce-scatter steps between halves (32 lanes) or row pairs (16 lanes):
// the swap exchanges complementary parts of u and w, so u + w afterwards
// holds, on half of the lanes, u's total over the two parts and, on the
// other half, w's.  Which lanes get which is read off the same swap applied
// to the tags 0 (u) and 1 (w): swap_tag32/16() return that tag per lane.
__device__ __forceinline__ double rs32_sum(double u, double w) {
  const auto a = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(u), (unsigned)__double2loint(w), false, false);
  const auto b = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(u), (unsigned)__double2hiint(w), false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ double rs16_sum(double u, double w) {
  const auto a = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(u), (unsigned)__double2loint(w), false, false);
  const auto b = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(u), (unsigned)__double2hiint(w), false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ int swap_tag32() { return (int)__builtin_amdgcn_permlane32_swap(0u, 1u, false, false)[0]; }
__device__ __forceinline__ int swap_tag16() { return (int)__builtin_amdgcn_permlane16_swap(0u, 1u, false, false)[0]; }

// Sum over the whole wavefront, returned to every lane (read from lane 63).
template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T x) {
  x = group_sum_dpp<16>(x);          // every lane: its row's total
  x += dpp<kDppRowBcast15, 0xa>(x);  // rows 1, 3 add rows 0, 2
  x += dpp<kDppRowBcast31, 0xc>(x);  // rows 2, 3 add the total of rows 0-1
  return readlane_d(x, 63);
}

}  // namespace lti
