// Shifted Hessenberg solves with several frequencies per wavefront: four
// (16-lane groups) for models of at most 64 states, two (32-lane groups) for
// 64 < n <= 128.
//
// The arithmetic is the one of sweep.hip (right-to-left complex Givens column
// rotations fused with back-substitution, then X = Z y by a scan of the
// rotation recurrence, then G = (CQ) X + D; see the comments there).  Only
// the mapping differs: frequency g = lane / GW of the wavefront owns a group
// of GW lanes (one 16-lane DPP row, or a pair of rows), and row i of its
// system lives on lane GW g + i % GW in register slice i / GW (R <= 4
// slices).  The frequencies of a wavefront (consecutive grid points of one
// request, so they share H, Q^T B and (CQ)^T) advance in lockstep, which
//   * shares the per-step scalar chain (pivot broadcast, rsqrt, rotation) and
//     the column load of H among the wavefront's solves,
//   * keeps idle lanes to the pivot's own slice (slices above the pivot are
//     skipped, not masked), and
//   * keeps the cross-lane moves inside the group: the scan uses row_shr DPP
//     with identity `old` values (and row_bcast:15 from the even to the odd
//     row of a 32-lane group), the output reduce-scatter pairs lanes by row
//     mirrors (after a sum over the row pair by v_permlane16_swap).
// The pivot row's carry entry and right-hand side reach the other lanes of
// its group through a small LDS slot per frequency, which lets the GW steps
// of a slice run as a loop (a fully unrolled step sequence does not fit the
// instruction cache).
#include <cfloat>
#include <cmath>
#include <type_traits>

#include "dpp.h"
#include "lti_kernels.h"
#include "sweep_common.h"

namespace lti {

namespace {

using namespace sweep_detail;

constexpr int kWaves16 = 4;  // wavefronts per workgroup, one tile each

template <int T0, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (T0 < N) {
    f(std::integral_constant<int, T0>{});
    static_for<T0 + 1, N>(f);
  }
}

template <typename T, int R, int MM>
struct SG {
  T cr[R], ci[R];           // carry column
  T br[R][MM], bi[R][MM];   // right-hand side -> y -> x
  T rc[R], rsr[R], rsi[R];  // rotation k on row k (row 0 unused)
  T rinv[R];                // 1 / R(k, k) on row k
  bool singular;            // this lane's frequency
};

// The two 16-lane rows of each 32-lane group, at every lane of the group:
// v_permlane16_swap with both operands x leaves the even row's x in the
// first result and the odd row's x in the second.
__device__ __forceinline__ void row_pair(float x, float& ev, float& od) {
  const unsigned u = __float_as_uint(x);
  const auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  ev = __uint_as_float(a[0]);
  od = __uint_as_float(a[1]);
}
__device__ __forceinline__ void row_pair(double x, double& ev, double& od) {
  const unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  ev = __hiloint2double((int)b[0], (int)a[0]);
  od = __hiloint2double((int)b[1], (int)a[1]);
}

template <int GW, typename T>
__device__ __forceinline__ T group_min(T x) {
  x = fmin(x, dpp<kDppQuadSwap1>(x));
  x = fmin(x, dpp<kDppQuadSwap2>(x));
  x = fmin(x, dpp<kDppRowHalfMirror>(x));
  x = fmin(x, dpp<kDppRowMirror>(x));
  if constexpr (GW == 32) {
    T e, o;
    row_pair(x, e, o);
    x = fmin(e, o);
  }
  return x;
}
template <int GW, typename T>
__device__ __forceinline__ T group_max(T x) {
  x = fmax(x, dpp<kDppQuadSwap1>(x));
  x = fmax(x, dpp<kDppQuadSwap2>(x));
  x = fmax(x, dpp<kDppRowHalfMirror>(x));
  x = fmax(x, dpp<kDppRowMirror>(x));
  if constexpr (GW == 32) {
    T e, o;
    row_pair(x, e, o);
    x = fmax(e, o);
  }
  return x;
}
// Every lane of the group gets the group's total, summed in the same order.
template <int GW>
__device__ __forceinline__ double group_sum(double x) {
  x = group_sum_dpp<16>(x);
  if constexpr (GW == 32) {
    double e, o;
    row_pair(x, e, o);
    x = e + o;
  }
  return x;
}
// Lane 0 (kLast false) or lane GW-1 (kLast true) of each group, at every
// lane of the group.
template <int GW, bool kLast, typename T>
__device__ __forceinline__ T group_bcast(T x) {
  const T y = dpp<dpp_row_newbcast(kLast ? 15 : 0)>(x);
  if constexpr (GW == 16) {
    return y;
  } else {
    T e, o;
    row_pair(y, e, o);
    return kLast ? o : e;
  }
}

// Sweep and back-substitution for the frequencies of the wavefront.  On
// entry br/bi hold the right-hand sides, on exit y.  bcast: this wavefront's
// (64 / GW) x (2 + 2 MM) values of LDS, one slot per frequency for the pivot
// row's carry entry and right-hand side.  Slices are unrolled at compile
// time; the GW steps inside a slice are a loop, so the code stays small.
//
// The float32 sweeps (refined path) keep rotation k and 1 / R(k,k) in a
// table in LDS, rot[k] = (c, Re s, Im s, 1 / R(k,k)), one per frequency,
// written by the lane that publishes the next pivot; the float64 sweeps
// keep them in registers, on the lane of row k.  kReuse (float32 only):
// the rotations are those of the table, left by a sweep of the same matrix
// (the correction solves of the refinement): each step then only reads them
// and updates the carry column and the right-hand side.
template <typename T, int R, int MM, bool kLds, int GW, bool kReuse = false>
__device__ __forceinline__ void sweep_grp(Src<T, kLds> H, int n, T sg, T w, SG<T, R, MM>& st, T* bcast,
                                          float4* rot = nullptr) {
  constexpr bool kRot = std::is_same<T, float>::value;
  static_assert(kRot || !kReuse, "only the float32 sweeps reuse their rotations");
  const int lane = threadIdx.x & 63;
  const int g = lane / GW, gl = lane & (GW - 1);
  T* mine = bcast + g * (2 + 2 * MM);
  if constexpr (!kReuse) st.singular = false;
  {
    const int off = hoff32(n - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = gl + GW * r;
      const T h = (i < n) ? H[off + i] : (T)0;
      st.cr[r] = (i == n - 1) ? sg - h : -h;
      st.ci[r] = (i == n - 1) ? w : (T)0;
      st.rc[r] = (T)0;
      st.rsr[r] = (T)1;
      st.rsi[r] = (T)0;
      st.rinv[r] = (T)1;
    }
  }
  T hc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) hc[r] = (T)0;
  if (n >= 2) {
    const int off = hoff32(n - 2);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = gl + GW * r;
      if (i <= n - 1) hc[r] = H[off + i];
    }
  }
  T sub0 = (n >= 2) ? H.uniform(hoff32(n - 2) + n - 1) : (T)0;
  T sub1 = (n >= 3) ? H.uniform(hoff32(n - 3) + n - 2) : (T)0;

  // The pivot row's carry entry and right-hand side reach the other lanes of
  // its group through this wavefront's LDS slot.  Step k publishes the next
  // pivot row k-1 as soon as the slice holding it is rotated: its carry
  // entry is read back at once (the next step's rotation starts from it), its
  // right-hand side after the other slices' back-substitution, which still
  // needs row k's; the LDS round trip overlaps the other slices' work.  LDS
  // operations of one wavefront complete in program order.
  auto lds_order = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  T par = (T)0, pai = (T)0, pbr[MM], pbi[MM];
  // the lane of row j of slice t publishes it (and `extra`, the rotation of
  // the step that made it the next pivot)
  auto publish = [&](auto TT, int j, auto&& extra) {
    constexpr int t = decltype(TT)::value;
    if (gl == j) {
      if constexpr (!kReuse) {
        mine[0] = st.cr[t];
        mine[1] = st.ci[t];
      }
#pragma unroll
      for (int jj = 0; jj < MM; ++jj) {
        mine[2 + 2 * jj] = st.br[t][jj];
        mine[3 + 2 * jj] = st.bi[t][jj];
      }
      extra();
    }
    lds_order();
    if constexpr (!kReuse) {
      par = mine[0];
      pai = mine[1];
    }
  };
  auto read_rhs = [&] {
    lds_order();
#pragma unroll
    for (int jj = 0; jj < MM; ++jj) {
      pbr[jj] = mine[2 + 2 * jj];
      pbi[jj] = mine[3 + 2 * jj];
    }
  };
  // row n-1 is the first pivot
  static_for<0, R>([&](auto TT) {
    constexpr int t = decltype(TT)::value;
    if ((n - 1) / GW == t) publish(TT, (n - 1) & (GW - 1), [] {});
  });
  read_rhs();

  // Step k = GW s + jl; SP (compile-time) is the slice of row k-1: s for
  // jl >= 1, s - 1 for jl = 0.
  auto step = [&](auto SC, auto SP, int jl) {
    constexpr int s = decltype(SC)::value;
    constexpr int sp = decltype(SP)::value;
    const int k = GW * s + jl;
    // prefetch column k-2 (rows 0..k-1) and the subdiagonal two steps
    // ahead.  The loads of the pivot slice run past row k-1 into the next
    // packed column (at most GW entries, all inside the packed array and its
    // LDS copy); those rows are never used.
    T hn[R];
    if (k >= 2) {
      const int off = hoff32(k - 2) + gl;
#pragma unroll
      for (int t = 0; t <= s; ++t) hn[t] = H[off + GW * t];
    } else {
#pragma unroll
      for (int t = 0; t <= s; ++t) hn[t] = (T)0;
    }
    const T sub2 = (k >= 3) ? H.uniform(hoff32(k - 3) + k - 2) : (T)0;
    T c, sr, si, rinv;
    if constexpr (kReuse) {
      const float4 rt = rot[k];
      c = rt.x;
      sr = rt.y;
      si = rt.z;
      rinv = rt.w;
    } else {
      const T beta = -sub0;
      const T nrm2 = par * par + pai * pai + beta * beta;
      const bool ok = norm2_ok(nrm2);
      const T rq = rsqrt_t(ok ? nrm2 : (T)1);
      // zero column (ok false, then par = pai = beta = 0): a zero rotation
      // and R(k,k) = 0; the frequency is flagged singular (also when the
      // norm is out of the format's range)
      rinv = ok ? rq : (T)INFINITY;
      c = beta * rq;
      sr = par * rq;
      si = pai * rq;
      st.singular = st.singular || !ok;
    }
    const T cw = c * w, sw_r = sr * w, sw_i = si * w;
    // rows of slice t below k: rotate the carry column with column k-1, then
    // b_i -= (R(i,k) / R(k,k)) b_k
    auto rot_slice = [&](auto TT) {
      constexpr int t = decltype(TT)::value;
      if (t < s || gl < jl) {
        const T cr_ = st.cr[t], ci_ = st.ci[t];
        // the diagonal entry of column k-1 (row k-1, in slice sp) also
        // holds s = sg + j w
        T d = (T)0;
        if constexpr (t == sp) d = (gl + GW * t == k - 1) ? (T)1 : (T)0;
        const T o = (t == sp) ? fma(d, sg, -hc[t]) : -hc[t];
        T nkr = c * o + sr * cr_ + si * ci_;
        T nki = sr * ci_ - si * cr_;
        T n1r = sr * o - c * cr_;
        T n1i = si * o - c * ci_;
        if constexpr (t == sp) {
          nki = fma(d, cw, nki);
          // row k-1's new carry entry only matters as the next pivot (whose
          // rotation a reusing sweep reads from the table) and, for k = 1,
          // as R(0,0) (which the table keeps too)
          if constexpr (!kReuse) {
            n1r = fma(-d, sw_i, n1r);
            n1i = fma(d, sw_r, n1i);
          }
        }
        st.cr[t] = n1r;
        st.ci[t] = n1i;
        nkr *= rinv;
        nki *= rinv;
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          st.br[t][j] = fma(-nkr, pbr[j], st.br[t][j]);
          st.br[t][j] = fma(nki, pbi[j], st.br[t][j]);
          st.bi[t][j] = fma(-nkr, pbi[j], st.bi[t][j]);
          st.bi[t][j] = fma(-nki, pbr[j], st.bi[t][j]);
        }
      }
    };
    rot_slice(SP);
    publish(SP, (k - 1) & (GW - 1), [&] {
      if constexpr (kRot && !kReuse) rot[k] = make_float4(c, sr, si, rinv);
    });
    // the other slices (for jl = 0, slice s holds no row below k)
    static_for<0, sp>([&](auto TT) { rot_slice(TT); });
    if constexpr (!kRot) {
      if (gl == jl) {
        st.rc[s] = c;
        st.rsr[s] = sr;
        st.rsi[s] = si;
        st.rinv[s] = rinv;
      }
    }
    read_rhs();
#pragma unroll
    for (int t = 0; t <= s; ++t) hc[t] = hn[t];
    sub0 = sub1;
    sub1 = sub2;
  };

  static_for<0, R>([&](auto sc) {
    constexpr int s = R - 1 - decltype(sc)::value;
    if (GW * s > n - 1) return;  // no pivot row in this slice (uniform)
    const int jhi = (n - 1 - GW * s < GW - 1) ? n - 1 - GW * s : GW - 1;
    using SC = std::integral_constant<int, s>;
    for (int jl = jhi; jl >= 1; --jl) step(SC{}, SC{}, jl);
    if constexpr (s >= 1) step(SC{}, std::integral_constant<int, s - 1>{}, 0);
  });
  // y_k = b_k / R(k,k); R(0,0) is the final carry entry of row 0 (kept in
  // the table's unused entry 0 for the sweeps that reuse the rotations)
  T ar, ai;
  if constexpr (kReuse) {
    const float4 r00 = rot[0];
    ar = r00.x;
    ai = r00.y;
  } else {
    ar = group_bcast<GW, false>(st.cr[0]);
    ai = group_bcast<GW, false>(st.ci[0]);
    if constexpr (kRot) {
      if (gl == 0) rot[0] = make_float4(ar, ai, 0.0f, 0.0f);
    }
  }
  const T d = ar * ar + ai * ai;
  st.singular = st.singular || !norm2_ok(d);
  const T dinv = (T)1 / d;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = gl + GW * r;
    if (i == 0) {
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        const T xr = st.br[0][j], xi = st.bi[0][j];
        st.br[0][j] = (xr * ar + xi * ai) * dinv;
        st.bi[0][j] = (xi * ar - xr * ai) * dinv;
      }
    } else {
      T ri;
      if constexpr (kRot) {
        const float rv = rot[i].w;  // rows n.. hold no rotation of this sweep
        ri = (i < n) ? rv : (T)1;
      } else {
        ri = st.rinv[r];
      }
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        st.br[r][j] *= ri;
        st.bi[r][j] *= ri;
      }
    }
  }
}

// Largest over smallest |R(k,k)| for this lane's frequency.
template <typename T, int R, int MM, int GW>
__device__ __forceinline__ double diag_ratio_grp(int n, const SG<T, R, MM>& st) {
  const int gl = threadIdx.x & (GW - 1);
  double lo = INFINITY, hi = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = gl + GW * r;
    if (i >= 1 && i < n) {
      lo = fmin(lo, (double)st.rinv[r]);
      hi = fmax(hi, (double)st.rinv[r]);
    }
  }
  lo = group_min<GW>(lo);
  hi = group_max<GW>(hi);
  const double ar = (double)group_bcast<GW, false>(st.cr[0]);
  const double ai = (double)group_bcast<GW, false>(st.ci[0]);
  const double r0 = sqrt(ar * ar + ai * ai);
  return fmax(1.0 / lo, r0) / fmin(1.0 / hi, r0);
}

// x := Z y in place (scan of t_k = -c_k t_{k-1} + conj(s_k) y_k within each
// group, slice by slice).  The rotations come from the LDS table (float32)
// or from the registers of their rows (float64).
template <typename T, int R, int MM, int GW>
__device__ __forceinline__ void apply_rotations_grp(int n, SG<T, R, MM>& st, const float4* rot = nullptr) {
  constexpr bool kRot = std::is_same<T, float>::value;
  const int gl = threadIdx.x & (GW - 1);
  T tinr[MM], tini[MM];
#pragma unroll
  for (int j = 0; j < MM; ++j) tinr[j] = tini[j] = (T)0;
  // lane 0 of the odd row of a 32-lane group, at every lane of the group
  auto lane0_of_odd = [](T x) {
    T e, o;
    row_pair(dpp<dpp_row_newbcast(0)>(x), e, o);
    return o;
  };
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (GW * r >= n) break;
    const int i = gl + GW * r;
    const bool inner = (i > 0 && i < n);
    // rotation i of row i and rotation i+1 of the next row (table entries of
    // rows 0 and n.. are not this sweep's; they are not used)
    T rc_, rsr_, rsi_, nc, nsr, nsi;
    if constexpr (kRot) {
      const float4 cur = rot[i];
      const float4 nx = rot[(i + 1 < GW * R) ? i + 1 : i];
      rc_ = cur.x;
      rsr_ = cur.y;
      rsi_ = cur.z;
      nc = nx.x;
      nsr = nx.y;
      nsi = nx.z;
    } else {
      rc_ = st.rc[r];
      rsr_ = st.rsr[r];
      rsi_ = st.rsi[r];
    }
    T a = inner ? -rc_ : (T)0;
    constexpr int NQ = (GW == 32) ? 5 : 4;
    T am[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      am[q] = a;
      T ap;
      if (q == 0) ap = dpp<dpp_row_shr(1)>(a, (T)1);
      if (q == 1) ap = dpp<dpp_row_shr(2)>(a, (T)1);
      if (q == 2) ap = dpp<dpp_row_shr(4)>(a, (T)1);
      if (q == 3) ap = dpp<dpp_row_shr(8)>(a, (T)1);
      if (q == 4) ap = dpp<kDppRowBcast15, 0xa>(a, (T)1);  // odd rows <- lane 15 of the even row
      a = a * ap;
    }
    // rotation of row i+1 (lane 0 of the next slice for the group's last
    // lane; in a 32-lane group, lane 0 of the odd row for lane 15)
    const int rn = (r + 1 < R) ? r + 1 : r;
    if constexpr (!kRot) {
      nc = dpp<dpp_row_shl(1)>(st.rc[r]);
      nsr = dpp<dpp_row_shl(1)>(st.rsr[r]);
      nsi = dpp<dpp_row_shl(1)>(st.rsi[r]);
      if constexpr (GW == 32) {
        const T c1 = lane0_of_odd(st.rc[r]);
        const T s1r = lane0_of_odd(st.rsr[r]);
        const T s1i = lane0_of_odd(st.rsi[r]);
        if (gl == 15) {
          nc = c1;
          nsr = s1r;
          nsi = s1i;
        }
      }
      if (r + 1 < R) {
        const T c0 = group_bcast<GW, false>(st.rc[rn]);
        const T s0r = group_bcast<GW, false>(st.rsr[rn]);
        const T s0i = group_bcast<GW, false>(st.rsi[rn]);
        if (gl == GW - 1) {
          nc = c0;
          nsr = s0r;
          nsi = s0i;
        }
      }
    }
    const T sr = rsr_, si = rsi_;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const T yr = st.br[r][j], yi = st.bi[r][j];
      T ur, ui;
      if (inner) {
        ur = sr * yr + si * yi;
        ui = sr * yi - si * yr;
      } else {
        ur = (i == 0) ? yr : (T)0;
        ui = (i == 0) ? yi : (T)0;
      }
      ur = fma(am[0], dpp<dpp_row_shr(1)>(ur, (T)0), ur);
      ui = fma(am[0], dpp<dpp_row_shr(1)>(ui, (T)0), ui);
      ur = fma(am[1], dpp<dpp_row_shr(2)>(ur, (T)0), ur);
      ui = fma(am[1], dpp<dpp_row_shr(2)>(ui, (T)0), ui);
      ur = fma(am[2], dpp<dpp_row_shr(4)>(ur, (T)0), ur);
      ui = fma(am[2], dpp<dpp_row_shr(4)>(ui, (T)0), ui);
      ur = fma(am[3], dpp<dpp_row_shr(8)>(ur, (T)0), ur);
      ui = fma(am[3], dpp<dpp_row_shr(8)>(ui, (T)0), ui);
      if constexpr (GW == 32) {
        ur = fma(am[4], dpp<kDppRowBcast15, 0xa>(ur, (T)0), ur);
        ui = fma(am[4], dpp<kDppRowBcast15, 0xa>(ui, (T)0), ui);
      }
      const T tr = fma(a, tinr[j], ur);
      const T ti = fma(a, tini[j], ui);
      T nyr = dpp<dpp_row_shl(1)>(yr);
      T nyi = dpp<dpp_row_shl(1)>(yi);
      if constexpr (GW == 32) {
        const T y1r = lane0_of_odd(yr);
        const T y1i = lane0_of_odd(yi);
        if (gl == 15) {
          nyr = y1r;
          nyi = y1i;
        }
      }
      if (r + 1 < R) {
        const T y0r = group_bcast<GW, false>(st.br[rn][j]);
        const T y0i = group_bcast<GW, false>(st.bi[rn][j]);
        if (gl == GW - 1) {
          nyr = y0r;
          nyi = y0i;
        }
      }
      tinr[j] = group_bcast<GW, true>(tr);
      tini[j] = group_bcast<GW, true>(ti);
      if (i < n - 1) {
        st.br[r][j] = nsr * tr - nsi * ti + nc * nyr;
        st.bi[r][j] = nsr * ti + nsi * tr + nc * nyi;
      } else if (i == n - 1) {
        st.br[r][j] = tr;
        st.bi[r][j] = ti;
      }
    }
  }
}

// One halving stage of the 16-lane reduce-scatter; CTRL pairs the lanes,
// `upper` marks the half that keeps the upper H entries.
template <int CTRL, int H>
__device__ __forceinline__ void rs16_stage(double (&vr)[8], double (&vi)[8], bool upper) {
#pragma unroll
  for (int q = 0; q < H; ++q) {
    const double sr = upper ? vr[q] : vr[q + H];
    const double si = upper ? vi[q] : vi[q + H];
    const double kr = upper ? vr[q + H] : vr[q];
    const double ki = upper ? vi[q + H] : vi[q];
    vr[q] = kr + dpp<CTRL>(sr);
    vi[q] = ki + dpp<CTRL>(si);
  }
}

// G(:, j0 .. j0+mc-1) of this lane's frequency = (CQ) X + D; the sum over the
// group's lanes is a reduce-scatter of 8 complex values over each 16-lane
// row (in a 32-lane group after summing the two rows), after which lane gl
// of the (first) row holds entry gl / 2.
template <int R, int MM, int GW>
__device__ __forceinline__ void write_output_grp(const ReqDesc& rd, int j0, int mc, bool valid,
                                                 const double (&xr)[R][MM], const double (&xi)[R][MM],
                                                 double* __restrict__ G, bool deriv = false) {
  const int gl = threadIdx.x & (GW - 1);
  const int rl = gl & 15;
  const int n = rd.n, m = rd.m, p = rd.p;
  const gptr<double> Ct = (gptr<double>)rd.Ct;
  constexpr int PC = (8 / MM > 0) ? 8 / MM : 1;
  constexpr int MC = (MM < 8) ? MM : 8;
  const bool up8 = rl >= 8, up4 = (rl & 7) >= 4, up2 = (rl & 3) >= 2;
  for (int a0 = 0; a0 < p; a0 += PC) {
#pragma unroll
    for (int jb = 0; jb < MM; jb += MC) {
      if (jb >= mc) break;
      double vr[8], vi[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) vr[q] = vi[q] = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = gl + GW * r;
        if (i < n) {
#pragma unroll
          for (int q = 0; q < PC; ++q) {
            const int a = a0 + q;
            const double cq = (a < p) ? Ct[i * p + a] : 0.0;
#pragma unroll
            for (int j = 0; j < MC; ++j) {
              vr[q * MC + j] = fma(cq, xr[r][jb + j], vr[q * MC + j]);
              vi[q * MC + j] = fma(cq, xi[r][jb + j], vi[q * MC + j]);
            }
          }
        }
      }
      if constexpr (GW == 32) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          vr[q] = xor16_sum(vr[q]);
          vi[q] = xor16_sum(vi[q]);
        }
      }
      rs16_stage<kDppRowMirror, 4>(vr, vi, up8);
      rs16_stage<kDppRowHalfMirror, 2>(vr, vi, up4);
      rs16_stage<0x1B, 1>(vr, vi, up2);  // quad_perm [3,2,1,0]
      vr[0] += dpp<kDppQuadSwap1>(vr[0]);
      vi[0] += dpp<kDppQuadSwap1>(vi[0]);
      if (valid && gl < 16 && (gl & 1) == 0) {
        const int idx = gl >> 1;
        const int a = a0 + idx / MC;
        const int j = jb + idx % MC;
        if (a < p && j < mc) {
          double2 gv;
          gv.x = deriv ? -vr[0] : vr[0] + ((gptr<double>)rd.D)[a * m + j0 + j];
          gv.y = deriv ? -vi[0] : vi[0];
          store_c(G, g_index(rd, a, j0 + j), gv);
        }
      }
    }
  }
}

template <int R, int MM, bool kLds, int GW>
__device__ void solve_grp_fp64(const ReqDesc& rd, Src<double, kLds> H, int64_t k, bool valid, int j0, int mc,
                               double* bcast) {
  const int gl = threadIdx.x & (GW - 1);
  const int n = rd.n, m = rd.m;
  const SPoint sp = point_of(rd, k);
  const gptr<double> Bt = (gptr<double>)rd.Bt;
  SG<double, R, MM> st;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = gl + GW * r;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      st.br[r][j] = (i < n && j < mc) ? Bt[i * m + j0 + j] : 0.0;
      st.bi[r][j] = 0.0;
    }
  }
  sweep_grp<double, R, MM, kLds, GW>(H, n, sp.re, sp.im, st, bcast);
  // estimated error from the spread of R's diagonal; points above the
  // request's tolerance are finished by the extended refinement
  const double est = fp64_estimate(n, diag_ratio_grp<double, R, MM, GW>(n, st));
  const bool dd = fp64_needs_dd(rd, est);
  if (dd && valid && gl == 0) enqueue_dd(rd, k, j0, mc, 0, kReasonFP64);
  apply_rotations_grp<double, R, MM, GW>(n, st);
  double* G = rd.G + (size_t)k * rd.p * m * 2;
  write_output_grp<R, MM, GW>(rd, j0, mc, valid && !dd, st.br, st.bi, G);
  if (rd.dG) {
    // dG/ds = -C (sI - A)^{-2} B: the same sweep with X as right-hand side
    sweep_grp<double, R, MM, kLds, GW>(H, n, sp.re, sp.im, st, bcast);
    apply_rotations_grp<double, R, MM, GW>(n, st);
    write_output_grp<R, MM, GW>(rd, j0, mc, valid && !dd, st.br, st.bi, rd.dG + (size_t)k * rd.p * m * 2, true);
  }
  if (valid && !dd && gl == 0) {
    lti_point_info inf;
    inf.est_rel_err = (float)est;
    inf.iters = rd.dG ? 2 : 1;
    inf.path = LTI_PATH_FP64;
    inf.reserved = 0;
    put_info(rd, k, inf);
  }
}

__device__ __forceinline__ double bperm_d(int addr, double v) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// r = Q^T B - (s X - H X) in float64 for this lane's frequency; the row
// X(j, :) reaches the other lanes of its group through ds_bpermute.
template <int R, int MM, bool kLds, int GW>
__device__ __forceinline__ void residual_grp(const ReqDesc& rd, Src<double, kLds> H, double sg, double w, int j0,
                                             int mc, const double (&xr)[R][MM], const double (&xi)[R][MM],
                                             double (&rr)[R][MM], double (&ri)[R][MM]) {
  const int lane = threadIdx.x & 63, gl = lane & (GW - 1);
  const int n = rd.n, m = rd.m;
  const gptr<double> Bt = (gptr<double>)rd.Bt;
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int i = gl + GW * t;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const double b = (i < n && j < mc) ? Bt[i * m + j0 + j] : 0.0;
      rr[t][j] = fma(w, xi[t][j], fma(-sg, xr[t][j], b));
      ri[t][j] = fma(-w, xr[t][j], -sg * xi[t][j]);
    }
  }
  static_for<0, R>([&](auto sc) {
    constexpr int sj = decltype(sc)::value;
    if (GW * sj >= n) return;
    const int jend = (n - GW * sj < GW) ? n - GW * sj : GW;
    for (int jl = 0; jl < jend; ++jl) {
      const int jc = GW * sj + jl;  // column of H
      const int off = hoff32(jc);
      const int len = (jc + 2 < n) ? jc + 2 : n;
      const int addr = ((lane & (64 - GW)) | jl) << 2;
      double xjr[MM], xji[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        xjr[j] = bperm_d(addr, xr[sj][j]);
        xji[j] = bperm_d(addr, xi[sj][j]);
      }
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = gl + GW * t;
        if (i < len) {
          const double h = H[off + i];
#pragma unroll
          for (int j = 0; j < MM; ++j) {
            rr[t][j] = fma(h, xjr[j], rr[t][j]);
            ri[t][j] = fma(h, xji[j], ri[t][j]);
          }
        }
      }
    }
  });
}

// Refined path: complex-float32 solves, float64 residuals and accumulation;
// stalled points go to the extended refinement (see solve_refined in
// sweep.hip).  The frequencies of the wavefront iterate in lockstep until
// all have stopped.
template <int R, int MM, bool kL64, bool kL32, int GW>
__device__ void solve_grp_refined(const ReqDesc& rd, Src<double, kL64> H, Src<float, kL32> H32, int64_t k,
                                  bool valid, int j0, int mc, double* bcast64, float4* rot) {
  const int gl = threadIdx.x & (GW - 1);
  const int n = rd.n, m = rd.m;
  const SPoint sp = point_of(rd, k);
  const float sgf = (float)sp.re, wf = (float)sp.im;
  const double tol = 0.1 * rd.rtol;
  constexpr int kMaxIters = 6;
  float* bcast = reinterpret_cast<float*>(bcast64);
  const gptr<float> Bt32 = (gptr<float>)rd.Bt32;

  double xr[R][MM], xi[R][MM];
  SG<float, R, MM> st;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = gl + GW * r;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      st.br[r][j] = (i < n && j < mc) ? Bt32[i * m + j0 + j] : 0.0f;
      st.bi[r][j] = 0.0f;
    }
  }
  sweep_grp<float, R, MM, kL32, GW>(H32, n, sgf, wf, st, bcast, rot);
  apply_rotations_grp<float, R, MM, GW>(n, st, rot);
  double s2 = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      xr[r][j] = (double)st.br[r][j];
      xi[r][j] = (double)st.bi[r][j];
      s2 += xr[r][j] * xr[r][j] + xi[r][j] * xi[r][j];
    }
  double dprev = sqrt(group_sum<GW>(s2));
  int iters = 1;
  double est = 1.0;
  bool done = false, ok = false;
  // singular or non-finite: the extended refinement takes it
  if (st.singular || !(dprev < INFINITY) || (rd.flags & kFlagForceDD)) done = true;
  for (int it = 0; it < kMaxIters; ++it) {
    if (__all(done)) break;
    double rr[R][MM], ri[R][MM];
    residual_grp<R, MM, kL64, GW>(rd, H, sp.re, sp.im, j0, mc, xr, xi, rr, ri);
    double amax = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < MM; ++j) amax = fmax(amax, fmax(fabs(rr[r][j]), fabs(ri[r][j])));
    amax = group_max<GW>(amax);
    if (!done && amax == 0.0) {  // X solves the float64 system exactly
      est = 0.0;
      ok = true;
      done = true;
    }
    const double scale = (amax > 0.0) ? 1.0 / amax : 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        st.br[r][j] = (float)(rr[r][j] * scale);
        st.bi[r][j] = (float)(ri[r][j] * scale);
      }
    sweep_grp<float, R, MM, kL32, GW, true>(H32, n, sgf, wf, st, bcast, rot);
    apply_rotations_grp<float, R, MM, GW>(n, st, rot);
    double d2 = 0.0, x2 = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        const double dr = done ? 0.0 : (double)st.br[r][j] * amax;
        const double di = done ? 0.0 : (double)st.bi[r][j] * amax;
        xr[r][j] += dr;
        xi[r][j] += di;
        d2 += dr * dr + di * di;
        x2 += xr[r][j] * xr[r][j] + xi[r][j] * xi[r][j];
      }
    const double dn = sqrt(group_sum<GW>(d2));
    const double xn = sqrt(group_sum<GW>(x2));
    if (!done) {
      ++iters;
      if (!(dn < INFINITY) || !(xn > 0.0)) {
        done = true;  // non-finite: stalled
      } else {
        const double rel = dn / xn;
        const double pred = rel * (dn / dprev);
        est = (pred < rel) ? pred : rel;
        if (rel <= tol || pred <= tol) {
          ok = true;
          done = true;
        } else if (dn > 0.5 * dprev || it + 1 == kMaxIters) {
          done = true;  // stalled
        }
        dprev = dn;
      }
    }
  }
  // stalled (or singular) points: the extended refinement finishes them
  if (!ok && valid && gl == 0) enqueue_dd(rd, k, j0, mc, iters, kReasonStall);
  double* G = rd.G + (size_t)k * rd.p * m * 2;
  write_output_grp<R, MM, GW>(rd, j0, mc, valid && ok, xr, xi, G);
  if (valid && ok && gl == 0) {
    lti_point_info inf;
    inf.est_rel_err = (float)est;
    inf.iters = (uint8_t)iters;
    inf.path = LTI_PATH_REFINED;
    inf.reserved = 0;
    put_info(rd, k, inf);
  }
}

// Packed length of the largest H a kernel holds (n = GW R).
constexpr int hlen_max(int R, int GW) { return (GW * R - 1) * (GW * R + 2) / 2 + GW * R; }

template <int PREC, int R, int MM, bool kL64, bool kL32, int GW>
__device__ __forceinline__ void run_tile_grp(const ReqDesc& rd, const Tile& td, Src<double, kL64> H,
                                             Src<float, kL32> H32, double* bcast, float4* rot) {
  constexpr int NG = 64 / GW;
  const int g = (threadIdx.x & 63) / GW;
  for (uint32_t f0 = 0; f0 < td.count; f0 += NG) {
    // group g solves frequency f0 + g; past the tile's end it repeats the
    // last frequency and writes nothing
    const uint32_t f = f0 + g;
    const bool valid = f < td.count;
    const int64_t k = (int64_t)td.start + (valid ? f : td.count - 1);
    if constexpr (PREC == LTI_PREC_FP64)
      solve_grp_fp64<R, MM, kL64, GW>(rd, H, k, valid, td.j0, td.mc, bcast);
    else
      solve_grp_refined<R, MM, kL64, kL32, GW>(rd, H, H32, k, valid, td.j0, td.mc, bcast, rot);
  }
}

// The reduced model's H is staged in LDS when the workgroup's four tiles
// belong to one request, which they do except where two requests meet in a
// launch: both copies of H up to 64 states, above that only the copy the
// sweeps read (the float32 one on the refined path, whose float64
// residuals read H from global memory).
template <int PREC, int R, int MM, int GW>
__device__ __forceinline__ void sweep_grp_body(const SweepLaunch& L) {
  constexpr bool kStage64 = PREC == LTI_PREC_FP64 || GW * R <= 64;
  constexpr bool kStage32 = PREC != LTI_PREC_FP64;
  constexpr bool kRotTab = PREC != LTI_PREC_FP64;
  __shared__ double bcast_all[kWaves16][(64 / GW) * (2 + 2 * MM)];
  __shared__ double sH[kStage64 ? hlen_max(R, GW) : 1];
  __shared__ float sH32[kStage32 ? hlen_max(R, GW) : 1];
  // the refined sweeps' rotation tables, one per frequency of each wavefront
  __shared__ float4 rot_all[kRotTab ? kWaves16 * (64 / GW) : 1][kRotTab ? GW * R : 1];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tb = xcd_swizzle(blockIdx.x, gridDim.x) * kWaves16;  // < ntiles
  const int tile = tb + wave;
  const int s0 = seg_of(L, tb);
  const bool staged = seg_of(L, min(tb + kWaves16, L.ntiles) - 1) == s0;
  if (staged) {
    const ReqDesc& r0 = L.seg[s0].rd;
    const int nh = (int)hlen(r0.n);
    if constexpr (kStage64) {
      const gptr<double> gH = (gptr<double>)r0.H;
      for (int i = threadIdx.x; i < nh; i += 64 * kWaves16) sH[i] = gH[i];
    }
    if constexpr (kStage32) {
      const gptr<float> gH32 = (gptr<float>)r0.H32;
      for (int i = threadIdx.x; i < nh; i += 64 * kWaves16) sH32[i] = gH32[i];
    }
    __syncthreads();
  }
  if (tile >= L.ntiles) return;
  const int s = seg_of(L, tile);
  const ReqDesc rd = L.seg[s].rd;
  const Tile td = tile_of(L.seg[s], tile);
  double* bcast = bcast_all[wave];
  float4* rot = kRotTab ? rot_all[wave * (64 / GW) + (threadIdx.x & 63) / GW] : nullptr;
  if (staged && (kStage64 || kStage32)) {
    if constexpr (kStage64 && kStage32)
      run_tile_grp<PREC, R, MM, true, true, GW>(rd, td, Src<double, true>{sH}, Src<float, true>{sH32}, bcast, rot);
    else if constexpr (kStage64)
      run_tile_grp<PREC, R, MM, true, false, GW>(rd, td, Src<double, true>{sH}, Src<float, false>{rd.H32}, bcast,
                                                 rot);
    else
      run_tile_grp<PREC, R, MM, false, true, GW>(rd, td, Src<double, false>{rd.H}, Src<float, true>{sH32}, bcast,
                                                 rot);
  } else {
    run_tile_grp<PREC, R, MM, false, false, GW>(rd, td, Src<double, false>{rd.H}, Src<float, false>{rd.H32},
                                                bcast, rot);
  }
}

// Occupancy: waves per SIMD, which the register caps buy with a few spills
// outside the step loops (measured on the serving mix: three waves beat two
// by about 8 % refined, four beat three by about 4 % where LDS leaves room).
//   * float64: three (168 registers), except the 32-lane kernels up to 128
//     states, whose 67 KB of staged H leave room for two (256 registers);
//   * refined: four (128 registers) up to 32 (16-lane) or 96 (32-lane)
//     states, three above (33-64 and 97-128 states), where the staged H and
//     the rotation tables take 42-50 KB of LDS per workgroup.
template <int PREC, int R, int MM>
__global__ __launch_bounds__(64 * kWaves16)
__attribute__((amdgpu_waves_per_eu(PREC == LTI_PREC_FP64 || R == 4 ? 3 : 4))) void sweep16_kernel(const SweepLaunch L) {
  sweep_grp_body<PREC, R, MM, 16>(L);
}

template <int PREC, int R, int MM>
__global__ __launch_bounds__(64 * kWaves16)
__attribute__((amdgpu_waves_per_eu(PREC == LTI_PREC_FP64 ? (R == 4 ? 2 : 3) : (R == 4 ? 3 : 4)))) void sweep32_kernel(
    const SweepLaunch L) {
  sweep_grp_body<PREC, R, MM, 32>(L);
}

using KernelGrpFn = void (*)(const SweepLaunch);

template <int PREC, int R>
KernelGrpFn pick16_mm(int mi) {
  return mi == 0 ? sweep16_kernel<PREC, R, 1> : mi == 1 ? sweep16_kernel<PREC, R, 2> : sweep16_kernel<PREC, R, 4>;
}

template <int PREC>
KernelGrpFn pick16(int ri, int mi) {
  return ri == 0 ? pick16_mm<PREC, 1>(mi) : ri == 1 ? pick16_mm<PREC, 2>(mi) : pick16_mm<PREC, 4>(mi);
}

template <int PREC, int R>
KernelGrpFn pick32_mm(int mi) {
  return mi == 0 ? sweep32_kernel<PREC, R, 1> : mi == 1 ? sweep32_kernel<PREC, R, 2> : sweep32_kernel<PREC, R, 4>;
}

template <int PREC>
KernelGrpFn pick32(int ri, int mi) {
  return ri == 0 ? pick32_mm<PREC, 3>(mi) : pick32_mm<PREC, 4>(mi);
}

int rhs_index(int mc) { return (mc <= 1) ? 0 : (mc <= 2) ? 1 : 2; }

}  // namespace

int sweep16_class(int precision, int n, int mc) {
  if (precision != LTI_PREC_FP64 && precision != LTI_PREC_REFINED) return -1;
  if (n < 1 || n > 64 || mc < 1 || mc > 4) return -1;
  const int ri = (n <= 16) ? 0 : (n <= 32) ? 1 : 2;
  return (precision * 3 + ri) * 3 + rhs_index(mc);
}

hipError_t launch_sweep16(int cls, const SweepLaunch& L, hipStream_t s) {
  if (L.ntiles <= 0) return hipSuccess;
  if (cls < 0 || cls >= kNumSweep16Classes) return hipErrorInvalidValue;
  const int prec = cls / 9, ri = (cls / 3) % 3, mi = cls % 3;
  const KernelGrpFn fn = prec == LTI_PREC_FP64 ? pick16<LTI_PREC_FP64>(ri, mi) : pick16<LTI_PREC_REFINED>(ri, mi);
  const int blocks = (L.ntiles + kWaves16 - 1) / kWaves16;
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * kWaves16), 0, s, L);
  return hipGetLastError();
}

int sweep32_class(int precision, int n, int mc) {
  if (precision != LTI_PREC_FP64 && precision != LTI_PREC_REFINED) return -1;
  if (n <= 64 || n > 128 || mc < 1 || mc > 4) return -1;
  const int ri = (n <= 96) ? 0 : 1;
  return (precision * 2 + ri) * 3 + rhs_index(mc);
}

hipError_t launch_sweep32(int cls, const SweepLaunch& L, hipStream_t s) {
  if (L.ntiles <= 0) return hipSuccess;
  if (cls < 0 || cls >= kNumSweep32Classes) return hipErrorInvalidValue;
  const int prec = cls / 6, ri = (cls / 3) % 2, mi = cls % 3;
  const KernelGrpFn fn = prec == LTI_PREC_FP64 ? pick32<LTI_PREC_FP64>(ri, mi) : pick32<LTI_PREC_REFINED>(ri, mi);
  const int blocks = (L.ntiles + kWaves16 - 1) / kWaves16;
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * kWaves16), 0, s, L);
  return hipGetLastError();
}

}  // namespace lti
