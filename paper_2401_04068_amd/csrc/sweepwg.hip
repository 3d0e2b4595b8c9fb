// Shifted Hessenberg solves for models of 257 to 1024 states: one workgroup
// of four wavefronts per frequency.
//
// Same arithmetic as sweep.hip (Givens column rotations fused with
// back-substitution, X = Z y by a scan of the rotation recurrence, then
// G = (CQ) X + D).  Row i lives on thread i % 256 of the workgroup in register
// slice i / 256 (R = 4 slices).  Per step the owner of the pivot row puts its
// carry entry and right-hand side into a double-buffered LDS slot; one
// workgroup barrier per step publishes it.  The scan runs per 64-row segment
// inside each wavefront and links the 16 segments through LDS.
#include <cfloat>
#include <cmath>
#include <type_traits>

#include "lti_kernels.h"
#include "sweep_common.h"

namespace lti {

namespace {

using namespace sweep_detail;

constexpr int kThreadsWG = 256;
constexpr int kRWG = 4;  // n <= 1024

template <int T0, int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (T0 < N) {
    f(std::integral_constant<int, T0>{});
    sfor<T0 + 1, N>(f);
  }
}

template <typename T, int MM>
struct SWG {
  T cr[kRWG], ci[kRWG];
  T br[kRWG][MM], bi[kRWG][MM];
  T rc[kRWG], rsr[kRWG], rsi[kRWG], rinv[kRWG];
  bool singular;
};

// LDS of one workgroup (bytes sized for MM <= 4 and T = double).
struct ShWG {
  double piv[2][2 + 2 * 4];       // carry entry and right-hand side of the pivot row
  double subd[kMaxNWG];           // H(j + 1, j) of the sweep's model (as T)
  double segA[4 * kRWG];          // scan: per-segment products
  double segU[4 * kRWG][2 * 4];   // scan: per-segment sums (complex, per column)
  double tin[4 * kRWG][2 * 4];    // scan: carry into each segment
  double first[4 * kRWG][3 + 2 * 4];  // rotation and y of each segment's first row
  double red[4][8][2];            // per-wavefront partial sums of G
  double misc[4];
  double ring[2][8];              // block reductions (alternating buffers)
  double ringN[2][4 * 24];        // block reductions of up to 24 values
};

// Reductions over the workgroup's four wavefronts; every thread gets the same
// total (same operands, same order).  Consecutive calls alternate between two
// LDS buffers, so one barrier per call suffices: a buffer is written again
// only after the barrier of the call in between.
struct BlockRed {
  ShWG& sh;
  int parity = 0;
  __device__ explicit BlockRed(ShWG& s) : sh(s) {}
  __device__ double sum(double x) {
    double* b = sh.ring[parity];
    parity ^= 1;
    x = wave_sum(x);
    if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = x;
    __syncthreads();
    return (b[0] + b[1]) + (b[2] + b[3]);
  }
  // two sums at once
  __device__ double2 sum2(double x, double y) {
    double* b = sh.ring[parity];
    parity ^= 1;
    x = wave_sum(x);
    y = wave_sum(y);
    if ((threadIdx.x & 63) == 0) {
      b[threadIdx.x >> 6] = x;
      b[4 + (threadIdx.x >> 6)] = y;
    }
    __syncthreads();
    return double2{(b[0] + b[1]) + (b[2] + b[3]), (b[4] + b[5]) + (b[6] + b[7])};
  }
  __device__ double max(double x) {
    double* b = sh.ring[parity];
    parity ^= 1;
    x = wave_max(x);
    if ((threadIdx.x & 63) == 0) b[threadIdx.x >> 6] = x;
    __syncthreads();
    return fmax(fmax(b[0], b[1]), fmax(b[2], b[3]));
  }
  // N (<= 24) sums at once, in place
  template <int N>
  __device__ void sumN(double (&v)[N]) {
    static_assert(N <= 24, "at most 24 sums per call");
    double* b = sh.ringN[parity];
    parity ^= 1;
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = wave_sum(v[q]);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int q = 0; q < N; ++q) b[4 * q + (threadIdx.x >> 6)] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = (b[4 * q] + b[4 * q + 1]) + (b[4 * q + 2] + b[4 * q + 3]);
  }
};

template <typename T, int MM>
__device__ __forceinline__ void sweep_wg(const T* Hg, int n, T sg, T w, SWG<T, MM>& st, ShWG& sh) {
  const int tid = threadIdx.x;
  const gptr<T> H = (gptr<T>)Hg;
  st.singular = false;
  {
    const int off = hoff32(n - 1);
#pragma unroll
    for (int r = 0; r < kRWG; ++r) {
      const int i = tid + kThreadsWG * r;
      const T h = (i < n) ? H[off + i] : (T)0;
      st.cr[r] = (i == n - 1) ? sg - h : -h;
      st.ci[r] = (i == n - 1) ? w : (T)0;
      st.rc[r] = (T)0;
      st.rsr[r] = (T)1;
      st.rsi[r] = (T)0;
      st.rinv[r] = (T)1;
    }
  }
  T hc[kRWG];
#pragma unroll
  for (int r = 0; r < kRWG; ++r) hc[r] = (T)0;
  if (n >= 2) {
    const int off = hoff32(n - 2);
#pragma unroll
    for (int r = 0; r < kRWG; ++r) {
      const int i = tid + kThreadsWG * r;
      if (i <= n - 1) hc[r] = H[off + i];
    }
  }
  // the subdiagonal, read by every step, into LDS (ordered before its first
  // read by the first step's barrier; the previous sweep's reads ended at its
  // closing barrier)
  T* const subd = reinterpret_cast<T*>(sh.subd);
  for (int j = tid; j < n - 1; j += kThreadsWG) subd[j] = H[hoff32(j) + j + 1];
  for (int k = n - 1; k >= 1; --k) {
    const int tk = k % kThreadsWG, rk = k / kThreadsWG;
    T* slot = reinterpret_cast<T*>(sh.piv[k & 1]);
    if (tid == tk) {
      // select the pivot slice's values (selects, not a branch per slice:
      // merged branches turn into pointer phis that keep st in memory)
      T pv[2 + 2 * MM];
      pv[0] = st.cr[0];
      pv[1] = st.ci[0];
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        pv[2 + 2 * j] = st.br[0][j];
        pv[3 + 2 * j] = st.bi[0][j];
      }
#pragma unroll
      for (int r = 1; r < kRWG; ++r) {
        const bool here = r == rk;
        pv[0] = here ? st.cr[r] : pv[0];
        pv[1] = here ? st.ci[r] : pv[1];
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          pv[2 + 2 * j] = here ? st.br[r][j] : pv[2 + 2 * j];
          pv[3 + 2 * j] = here ? st.bi[r][j] : pv[3 + 2 * j];
        }
      }
#pragma unroll
      for (int q = 0; q < 2 + 2 * MM; ++q) slot[q] = pv[q];
    }
    T hn[kRWG];
#pragma unroll
    for (int r = 0; r < kRWG; ++r) hn[r] = (T)0;
    if (k >= 2) {
      const int off = hoff32(k - 2);
#pragma unroll
      for (int r = 0; r < kRWG; ++r) {
        const int i = tid + kThreadsWG * r;
        if (r <= rk && i <= k - 1) hn[r] = H[off + i];
      }
    }
    __syncthreads();
    const T ar = slot[0], ai = slot[1];
    T bkr[MM], bki[MM];
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      bkr[j] = slot[2 + 2 * j];
      bki[j] = slot[3 + 2 * j];
    }
    const T beta = -subd[k - 1];
    const T nrm2 = ar * ar + ai * ai + beta * beta;
    const bool ok = norm2_ok(nrm2);
    const T rq = rsqrt_t(ok ? nrm2 : (T)1);
    const T rinv = ok ? rq : (T)INFINITY;
    const T c = ok ? beta * rq : (T)0;
    const T sr = ok ? ar * rq : (T)1;
    const T si = ok ? ai * rq : (T)0;
    st.singular = st.singular || !ok;
#pragma unroll
    for (int r = 0; r < kRWG; ++r) {
      const int i = tid + kThreadsWG * r;
      if (r <= rk && i < k) {
        const T cr_ = st.cr[r], ci_ = st.ci[r];
        const T o = (i == k - 1) ? sg - hc[r] : -hc[r];  // M(i, k-1)
        T nkr = c * o + sr * cr_ + si * ci_;
        T nki = sr * ci_ - si * cr_;
        T n1r = sr * o - c * cr_;
        T n1i = si * o - c * ci_;
        if (i == k - 1) {
          nki += c * w;
          n1r -= si * w;
          n1i += sr * w;
        }
        st.cr[r] = n1r;
        st.ci[r] = n1i;
        nkr *= rinv;
        nki *= rinv;
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          st.br[r][j] = fma(-nkr, bkr[j], st.br[r][j]);
          st.br[r][j] = fma(nki, bki[j], st.br[r][j]);
          st.bi[r][j] = fma(-nkr, bki[j], st.bi[r][j]);
          st.bi[r][j] = fma(-nki, bkr[j], st.bi[r][j]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kRWG; ++r) {
      const bool here = tid == tk && r == rk;
      st.rc[r] = here ? c : st.rc[r];
      st.rsr[r] = here ? sr : st.rsr[r];
      st.rsi[r] = here ? si : st.rsi[r];
      st.rinv[r] = here ? rinv : st.rinv[r];
    }
#pragma unroll
    for (int r = 0; r < kRWG; ++r) hc[r] = hn[r];
  }
  // R(0,0): the final carry entry of row 0 (thread 0, slice 0)
  if (tid == 0) {
    sh.misc[0] = (double)st.cr[0];
    sh.misc[1] = (double)st.ci[0];
  }
  __syncthreads();
  const T ar = (T)sh.misc[0], ai = (T)sh.misc[1];
  const T d = ar * ar + ai * ai;
  st.singular = st.singular || !norm2_ok(d);
  const T dinv = (T)1 / d;
#pragma unroll
  for (int r = 0; r < kRWG; ++r) {
    const int i = tid + kThreadsWG * r;
    if (i == 0) {
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        const T xr = st.br[0][j], xi = st.bi[0][j];
        st.br[0][j] = (xr * ar + xi * ai) * dinv;
        st.bi[0][j] = (xi * ar - xr * ai) * dinv;
      }
    } else {
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        st.br[r][j] *= st.rinv[r];
        st.bi[r][j] *= st.rinv[r];
      }
    }
  }
  __syncthreads();  // sh.misc is reused
}

// Local scan of one slice's 64-row segment: on return `a` is the product of
// the segment's multipliers up to this row and u[j] the partial sum.
template <int r, typename T, int MM>
__device__ __forceinline__ void segment_scan(int n, const SWG<T, MM>& st, T& a, T (&u_r)[MM], T (&u_i)[MM]) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int i = tid + kThreadsWG * r;
  const bool inner = (i > 0 && i < n);
  a = inner ? -st.rc[r] : (T)0;
  T am[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int dd = 1 << q;
    const T ap = __shfl_up(a, dd, 64);
    am[q] = (lane >= dd) ? a : (T)0;
    if (lane >= dd) a = a * ap;
  }
  const T sr = st.rsr[r], si = st.rsi[r];
#pragma unroll
  for (int j = 0; j < MM; ++j) {
    const T yr = st.br[r][j], yi = st.bi[r][j];
    T xr, xi;
    if (inner) {
      xr = sr * yr + si * yi;
      xi = sr * yi - si * yr;
    } else {
      xr = (i == 0) ? yr : (T)0;
      xi = (i == 0) ? yi : (T)0;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int dd = 1 << q;
      const T pr = __shfl_up(xr, dd, 64);
      const T pi = __shfl_up(xi, dd, 64);
      if (lane >= dd) {
        xr = fma(am[q], pr, xr);
        xi = fma(am[q], pi, xi);
      }
    }
    u_r[j] = xr;
    u_i[j] = xi;
  }
}

// x := Z y.  Segment sg = 4 r + wave holds rows 64 sg .. 64 sg + 63 (lane =
// row within the segment).  Pass 1 scans every segment and publishes its
// totals; the totals are linked in order; pass 2 rescans and finishes.
template <typename T, int MM>
__device__ __forceinline__ void apply_rotations_wg(int n, SWG<T, MM>& st, ShWG& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NS = 4 * kRWG;
  sfor<0, kRWG>([&](auto rc_) {
    constexpr int r = decltype(rc_)::value;
    const int sg = 4 * r + wv;
    T a, ur[MM], ui[MM];
    segment_scan<r>(n, st, a, ur, ui);
    if (lane == 63) {
      sh.segA[sg] = (double)a;
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        sh.segU[sg][2 * j] = (double)ur[j];
        sh.segU[sg][2 * j + 1] = (double)ui[j];
      }
    }
    if (lane == 0) {
      sh.first[sg][0] = (double)st.rc[r];
      sh.first[sg][1] = (double)st.rsr[r];
      sh.first[sg][2] = (double)st.rsi[r];
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        sh.first[sg][3 + 2 * j] = (double)st.br[r][j];
        sh.first[sg][4 + 2 * j] = (double)st.bi[r][j];
      }
    }
  });
  __syncthreads();
  if (tid < MM) {  // link the segments: t_in(sg + 1) = A(sg) t_in(sg) + U(sg)
    double tr = 0.0, ti = 0.0;
    for (int sg = 0; sg < NS; ++sg) {
      sh.tin[sg][2 * tid] = tr;
      sh.tin[sg][2 * tid + 1] = ti;
      const double a = sh.segA[sg];
      const double nr = a * tr + sh.segU[sg][2 * tid];
      const double ni = a * ti + sh.segU[sg][2 * tid + 1];
      tr = nr;
      ti = ni;
    }
  }
  __syncthreads();
  sfor<0, kRWG>([&](auto rc_) {
    constexpr int r = decltype(rc_)::value;
    const int i = tid + kThreadsWG * r;
    const int sg = 4 * r + wv;
    T a, ur[MM], ui[MM];
    segment_scan<r>(n, st, a, ur, ui);
    T nc = __shfl_down(st.rc[r], 1, 64);
    T nsr = __shfl_down(st.rsr[r], 1, 64);
    T nsi = __shfl_down(st.rsi[r], 1, 64);
    if (lane == 63 && sg + 1 < NS) {
      nc = (T)sh.first[sg + 1][0];
      nsr = (T)sh.first[sg + 1][1];
      nsi = (T)sh.first[sg + 1][2];
    }
    T nyr[MM], nyi[MM];
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      nyr[j] = __shfl_down(st.br[r][j], 1, 64);
      nyi[j] = __shfl_down(st.bi[r][j], 1, 64);
      if (lane == 63 && sg + 1 < NS) {
        nyr[j] = (T)sh.first[sg + 1][3 + 2 * j];
        nyi[j] = (T)sh.first[sg + 1][4 + 2 * j];
      }
    }
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const T tr = fma(a, (T)sh.tin[sg][2 * j], ur[j]);
      const T ti = fma(a, (T)sh.tin[sg][2 * j + 1], ui[j]);
      if (i < n - 1) {
        st.br[r][j] = nsr * tr - nsi * ti + nc * nyr[j];
        st.bi[r][j] = nsr * ti + nsi * tr + nc * nyi[j];
      } else if (i == n - 1) {
        st.br[r][j] = tr;
        st.bi[r][j] = ti;
      }
    }
  });
  __syncthreads();
}

// G(:, j0 .. j0+mc-1) = (CQ) X + D, summed over the workgroup: per wavefront
// a shuffle sum of one (row, column) entry at a time, then over the four
// wavefronts through LDS.
template <int MM>
__device__ __forceinline__ void write_output_wg(const ReqDesc& rd, int j0, int mc, const double (&xr)[kRWG][MM],
                                                const double (&xi)[kRWG][MM], double* __restrict__ G,
                                                ShWG& sh, bool deriv = false) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = rd.n, m = rd.m, p = rd.p;
  const gptr<double> Ct = (gptr<double>)rd.Ct;
  for (int a = 0; a < p; ++a) {
    double vr[MM], vi[MM];
#pragma unroll
    for (int j = 0; j < MM; ++j) vr[j] = vi[j] = 0.0;
#pragma unroll
    for (int r = 0; r < kRWG; ++r) {
      const int i = tid + kThreadsWG * r;
      if (i < n) {
        const double cq = Ct[i * p + a];
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          vr[j] = fma(cq, xr[r][j], vr[j]);
          vi[j] = fma(cq, xi[r][j], vi[j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      vr[j] = wave_sum(vr[j]);
      vi[j] = wave_sum(vi[j]);
    }
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        sh.red[wv][j][0] = vr[j];
        sh.red[wv][j][1] = vi[j];
      }
    }
    __syncthreads();
    if (tid < mc) {
      const int j = tid;
      double gr = 0.0, gi = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        gr += sh.red[q][j][0];
        gi += sh.red[q][j][1];
      }
      double2 g;
      g.x = deriv ? -gr : gr + ((gptr<double>)rd.D)[a * m + j0 + j];
      g.y = deriv ? -gi : gi;
      store_c(G, g_index(rd, a, j0 + j), g);
    }
    __syncthreads();
  }
}

// Largest over smallest |R(k,k)| after sweep_wg (1 / R(k,k) sits on the row
// k of its step; R(0,0) is thread 0's final carry entry).
template <typename T, int MM>
__device__ __forceinline__ double diag_ratio_wg(int n, const SWG<T, MM>& st, BlockRed& br) {
  const int tid = threadIdx.x;
  double lo = INFINITY, hi = 0.0;
#pragma unroll
  for (int r = 0; r < kRWG; ++r) {
    const int i = tid + kThreadsWG * r;
    double ri = INFINITY;
    if (i == 0) {
      const double ar = (double)st.cr[0], ai = (double)st.ci[0];
      ri = 1.0 / sqrt(ar * ar + ai * ai);
    } else if (i < n) {
      ri = (double)st.rinv[r];
    }
    if (i < n) {
      lo = fmin(lo, ri);
      hi = fmax(hi, ri);
    }
  }
  lo = -br.max(-lo);
  hi = br.max(hi);
  return hi / lo;
}

template <int MM>
__device__ void solve_wg_fp64(const ReqDesc& rd, int64_t k, int j0, int mc, ShWG& sh) {
  const int tid = threadIdx.x;
  const int n = rd.n, m = rd.m;
  const SPoint sp = point_of(rd, k);
  const gptr<double> Bt = (gptr<double>)rd.Bt;
  SWG<double, MM> st;
#pragma unroll
  for (int r = 0; r < kRWG; ++r) {
    const int i = tid + kThreadsWG * r;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      st.br[r][j] = (i < n && j < mc) ? Bt[i * m + j0 + j] : 0.0;
      st.bi[r][j] = 0.0;
    }
  }
  sweep_wg<double, MM>(rd.H, n, sp.re, sp.im, st, sh);
  BlockRed br(sh);
  // estimated error from the spread of R's diagonal; points above the
  // request's tolerance are finished by the extended refinement
  const double est = fp64_estimate(n, diag_ratio_wg<double, MM>(n, st, br));
  if (fp64_needs_dd(rd, est)) {  // uniform
    if (tid == 0) enqueue_dd(rd, k, j0, mc, 0, kReasonFP64);
    __syncthreads();  // LDS reuse by the next point
    return;
  }
  apply_rotations_wg<double, MM>(n, st, sh);
  double* G = rd.G + (size_t)k * rd.p * m * 2;
  write_output_wg<MM>(rd, j0, mc, st.br, st.bi, G, sh);
  if (rd.dG) {
    // dG/ds = -C (sI - A)^{-2} B: the same sweep with X as right-hand side
    sweep_wg<double, MM>(rd.H, n, sp.re, sp.im, st, sh);
    apply_rotations_wg<double, MM>(n, st, sh);
    write_output_wg<MM>(rd, j0, mc, st.br, st.bi, rd.dG + (size_t)k * rd.p * m * 2, sh, true);
  }
  if (tid == 0) {
    lti_point_info inf;
    inf.est_rel_err = (float)est;
    inf.iters = rd.dG ? 2 : 1;
    inf.path = LTI_PATH_FP64;
    inf.reserved = 0;
    put_info(rd, k, inf);
  }
}

// r = Q^T B - (s X - H X) in float64.  X reaches every thread through LDS,
// one 256-row slice at a time (xs: 256 x MM complex values); thread i sums
// row i of H X over the slice's columns j >= i - 1.
template <int MM>
__device__ __forceinline__ void residual_wg(const ReqDesc& rd, double sg, double w, int j0, int mc,
                                            const double (&xr)[kRWG][MM], const double (&xi)[kRWG][MM],
                                            double (&rr)[kRWG][MM], double (&ri)[kRWG][MM], double2* xs) {
  const int tid = threadIdx.x;
  const int n = rd.n, m = rd.m;
  const gptr<double> Bt = (gptr<double>)rd.Bt;
  const gptr<double> H = (gptr<double>)rd.H;
#pragma unroll
  for (int r = 0; r < kRWG; ++r) {
    const int i = tid + kThreadsWG * r;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const double b = (i < n && j < mc) ? Bt[i * m + j0 + j] : 0.0;
      rr[r][j] = fma(w, xi[r][j], fma(-sg, xr[r][j], b));
      ri[r][j] = fma(-w, xr[r][j], -sg * xi[r][j]);
    }
  }
  sfor<0, kRWG>([&](auto sc_) {
    constexpr int sj = decltype(sc_)::value;
    if (kThreadsWG * sj >= n) return;  // uniform
#pragma unroll
    for (int j = 0; j < MM; ++j) xs[tid * MM + j] = double2{xr[sj][j], xi[sj][j]};
    __syncthreads();
    const int jend = min(kThreadsWG, n - kThreadsWG * sj);
    for (int jl = 0; jl < jend; ++jl) {
      const int jc = kThreadsWG * sj + jl;
      const int64_t off = hoff(jc);
      double2 xj[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) xj[j] = xs[jl * MM + j];
#pragma unroll
      for (int r = 0; r < kRWG; ++r) {
        const int i = tid + kThreadsWG * r;
        if (r <= sj + 1 && i <= jc + 1 && i < n) {  // H(i, jc) = 0 below the subdiagonal
          const double h = H[off + i];
#pragma unroll
          for (int j = 0; j < MM; ++j) {
            rr[r][j] = fma(h, xj[j].x, rr[r][j]);
            ri[r][j] = fma(h, xj[j].y, ri[r][j]);
          }
        }
      }
    }
    __syncthreads();
  });
}

// Refined path for 257 .. 1024 states: complex-float32 solves of the scaled
// residual, float64 residuals and accumulation (Higham, Accuracy and
// Stability of Numerical Algorithms, ch. 12); stalled points go to the
// extended refinement.  Every decision below is uniform over the workgroup.
template <int MM>
__device__ void solve_wg_refined(const ReqDesc& rd, int64_t k, int j0, int mc, ShWG& sh, double2* xs) {
  const int tid = threadIdx.x;
  const int n = rd.n, m = rd.m;
  const SPoint sp = point_of(rd, k);
  const float sgf = (float)sp.re, wf = (float)sp.im;
  const double tol = 0.1 * rd.rtol;
  constexpr int kMaxIters = 6;
  const gptr<float> Bt32 = (gptr<float>)rd.Bt32;
  BlockRed br(sh);
  SWG<float, MM> st;
#pragma unroll
  for (int r = 0; r < kRWG; ++r) {
    const int i = tid + kThreadsWG * r;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      st.br[r][j] = (i < n && j < mc) ? Bt32[i * m + j0 + j] : 0.0f;
      st.bi[r][j] = 0.0f;
    }
  }
  sweep_wg<float, MM>(rd.H32, n, sgf, wf, st, sh);
  apply_rotations_wg<float, MM>(n, st, sh);
  double xr[kRWG][MM], xi[kRWG][MM];
  double s2 = 0.0;
#pragma unroll
  for (int r = 0; r < kRWG; ++r)
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      xr[r][j] = (double)st.br[r][j];
      xi[r][j] = (double)st.bi[r][j];
      s2 += xr[r][j] * xr[r][j] + xi[r][j] * xi[r][j];
    }
  double dprev = sqrt(br.sum(s2));
  const bool singular = br.max(st.singular ? 1.0 : 0.0) > 0.0;
  int iters = 1;
  double est = 1.0;
  bool ok = false;
  if (!singular && dprev < INFINITY && !(rd.flags & kFlagForceDD)) {
    for (int it = 0; it < kMaxIters; ++it) {
      double rr[kRWG][MM], ri[kRWG][MM];
      residual_wg<MM>(rd, sp.re, sp.im, j0, mc, xr, xi, rr, ri, xs);
      double amax = 0.0;
#pragma unroll
      for (int r = 0; r < kRWG; ++r)
#pragma unroll
        for (int j = 0; j < MM; ++j) amax = fmax(amax, fmax(fabs(rr[r][j]), fabs(ri[r][j])));
      amax = br.max(amax);
      if (amax == 0.0) {  // X solves the float64 system exactly
        est = 0.0;
        ok = true;
        break;
      }
      const double scale = 1.0 / amax;
#pragma unroll
      for (int r = 0; r < kRWG; ++r)
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          st.br[r][j] = (float)(rr[r][j] * scale);
          st.bi[r][j] = (float)(ri[r][j] * scale);
        }
      sweep_wg<float, MM>(rd.H32, n, sgf, wf, st, sh);
      apply_rotations_wg<float, MM>(n, st, sh);
      ++iters;
      double d2 = 0.0, x2 = 0.0;
#pragma unroll
      for (int r = 0; r < kRWG; ++r)
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          const double dr = (double)st.br[r][j] * amax;
          const double di = (double)st.bi[r][j] * amax;
          xr[r][j] += dr;
          xi[r][j] += di;
          d2 += dr * dr + di * di;
          x2 += xr[r][j] * xr[r][j] + xi[r][j] * xi[r][j];
        }
      const double2 dx = br.sum2(d2, x2);
      const double dn = sqrt(dx.x), xn = sqrt(dx.y);
      if (!(dn < INFINITY) || !(xn > 0.0)) break;  // non-finite: stalled
      const double rel = dn / xn;
      const double pred = rel * (dn / dprev);
      est = (pred < rel) ? pred : rel;
      if (rel <= tol || pred <= tol) {
        ok = true;
        break;
      }
      if (dn > 0.5 * dprev) break;  // stalled
      dprev = dn;
    }
  }
  if (!ok) {
    if (tid == 0) enqueue_dd(rd, k, j0, mc, iters, kReasonStall);
    __syncthreads();
    return;
  }
  double* G = rd.G + (size_t)k * rd.p * m * 2;
  write_output_wg<MM>(rd, j0, mc, xr, xi, G, sh);
  if (tid == 0) {
    lti_point_info inf;
    inf.est_rel_err = (float)est;
    inf.iters = (uint8_t)iters;
    inf.path = LTI_PATH_REFINED;
    inf.reserved = 0;
    put_info(rd, k, inf);
  }
}

// At most 256 registers per lane, so that two workgroups share a CU (the
// step loop is latency-bound: one barrier and one LDS round trip per step);
// the four-column kernel then keeps a few values of its set-up and output
// phases in scratch memory, none in the step loop.
template <int PREC, int MM>
__global__ __launch_bounds__(kThreadsWG) __attribute__((amdgpu_waves_per_eu(2))) void sweep_wg_kernel(
    const SweepLaunch L) {
  __shared__ ShWG sh;
  __shared__ double2 xs[PREC == LTI_PREC_FP64 ? 1 : kThreadsWG * MM];
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  if (tile >= L.ntiles) return;
  const int s = seg_of(L, tile);
  const ReqDesc rd = L.seg[s].rd;
  const Tile td = tile_of(L.seg[s], tile);
  for (uint32_t f = 0; f < td.count; ++f) {
    if (PREC == LTI_PREC_FP64)
      solve_wg_fp64<MM>(rd, (int64_t)td.start + f, td.j0, td.mc, sh);
    else
      solve_wg_refined<MM>(rd, (int64_t)td.start + f, td.j0, td.mc, sh, xs);
  }
}

// ---------------------------------------------------------------------------
// Extended-precision refinement of queued points.
//
// Near an eigenvalue of A the error of a float64 result is dominated by the
// rounding of the reduction H = Q^T A Q itself (a relative perturbation of A
// of order u is amplified by kappa(s I - A)), which no refinement against H
// can remove.  So the residual is taken against the original model: with x
// in double-double (Dekker's pair arithmetic), r = B - (s I - A) x is formed
// exactly enough (each product split by FMA, sums by two-sum) and rounded,
// and the correction solves (s I - A) d = r through the reduced model,
// d = Q (s I - H)^{-1} Q^T r, by the float64 Givens sweep.  The iteration
// converges while kappa(s I - A) u64 is well below one, to a forward error of
// order u64 (Higham, Accuracy and Stability of Numerical Algorithms, 2nd ed.,
// sec. 12.1, residual in higher precision).  Q is applied as its reflectors.

// The pair operations are error-free transformations only if every sum and
// product in them is rounded on its own: floating-point contraction (which
// HIP enables by default) must not fuse, say, the product x.hi * a with the
// sums that follow it once the functions are inlined -- that counts the
// product's rounding error twice and leaves the residual with float64
// accuracy.  Each function therefore turns contraction off; the fused steps
// they need are written as explicit fma().
struct dd {
  double hi, lo;
};
__device__ __forceinline__ dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  return dd{s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  return dd{s, b - (s - a)};
}
__device__ __forceinline__ dd dd_add(dd x, dd y) {
#pragma clang fp contract(off)
  const dd s = two_sum(x.hi, y.hi);
  return fast_two_sum(s.hi, s.lo + (x.lo + y.lo));
}
// x * a, a a double
__device__ __forceinline__ dd dd_mul_d(dd x, double a) {
#pragma clang fp contract(off)
  const double p = x.hi * a;
  const double e = fma(x.hi, a, -p);
  return fast_two_sum(p, fma(x.lo, a, e));
}

struct DDShared {
  ShWG sh;
  // x (re hi, re lo, im hi, im lo) of the columns solved together, for the
  // row products: entry c * CB + j (n CB <= kMaxNWG)
  double4 x[kMaxNWG];
};

// The refinement works on CB right-hand sides of one point at once (rows
// i = tid + 256 r, r < R, of each), so that every block reduction and every
// float64 sweep serves all of them: (R, CB) = (1, 4) for n <= 256, (2, 2)
// for n <= 512, (4, 1) above.

// v <- Q^T v (forward = true) or Q v, Q = P_0 ... P_{n-3}, P_k = I - tau_k
// u_k u_k^T.  G reflectors per block reduction: applied in order, the j-th
// one's dot product with the vector it meets is d_j = u_j^T v -
// sum_{i<j} tau_i d_i (u_j^T u_i), so one reduction of the u_j^T v and the
// u_j^T u_i serves the group; then v -= sum_j tau_j d_j u_j.
template <int R, int CB>
__device__ __forceinline__ void apply_q(const ReducedModel& rm, bool forward, double (&vr)[R][CB],
                                        double (&vi)[R][CB], BlockRed& br) {
  constexpr int G = CB >= 4 ? 2 : 4;            // reflectors per reduction
  constexpr int NX = 2 * G * CB;                // u_j^T v (re, im) per column
  constexpr int NS = NX + G * (G - 1) / 2;      // and u_j^T u_i, i < j
  const int n = rm.n, tid = threadIdx.x;
  const int nq = n - 2;
  const gptr<double> V = (gptr<double>)rm.V;
  const gptr<double> tau = (gptr<double>)rm.tau;
  for (int q0 = 0; q0 < nq; q0 += G) {
    double u[G][R], t[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const bool live = q0 + j < nq;  // past the last reflector: u = 0, tau = 0
      const int kk = forward ? q0 + j : n - 3 - (q0 + j);
      t[j] = live ? tau[kk] : 0.0;
      const int64_t vo = live ? voff(n, kk) - (kk + 2) : 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + kThreadsWG * r;
        u[j][r] = !live ? 0.0 : (i == kk + 1) ? 1.0 : (i >= kk + 2 && i < n) ? V[vo + i] : 0.0;
      }
    }
    double sm[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) sm[q] = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int j = 0; j < G; ++j)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          sm[2 * (j * CB + c)] = fma(u[j][r], vr[r][c], sm[2 * (j * CB + c)]);
          sm[2 * (j * CB + c) + 1] = fma(u[j][r], vi[r][c], sm[2 * (j * CB + c) + 1]);
        }
#pragma unroll
      for (int j = 1; j < G; ++j)
#pragma unroll
        for (int i = 0; i < j; ++i) sm[NX + j * (j - 1) / 2 + i] = fma(u[j][r], u[i][r], sm[NX + j * (j - 1) / 2 + i]);
    }
    br.sumN<NS>(sm);
    double dr[G][CB], di[G][CB];
#pragma unroll
    for (int j = 0; j < G; ++j)
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        dr[j][c] = sm[2 * (j * CB + c)];
        di[j][c] = sm[2 * (j * CB + c) + 1];
#pragma unroll
        for (int i = 0; i < j; ++i) {
          const double w = t[i] * sm[NX + j * (j - 1) / 2 + i];
          dr[j][c] = fma(-w, dr[i][c], dr[j][c]);
          di[j][c] = fma(-w, di[i][c], di[j][c]);
        }
      }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int j = 0; j < G; ++j) {
          vr[r][c] = fma(-t[j] * dr[j][c], u[j][r], vr[r][c]);
          vi[r][c] = fma(-t[j] * di[j][c], u[j][r], vi[r][c]);
        }
  }
}

// (s I - H) y = c for CB right-hand sides through the float64 sweep; on
// return y = (yr, yi); returns whether R had a zero diagonal entry.
template <int R, int CB>
__device__ __forceinline__ bool hess_solve(const ReducedModel& rm, SPoint sp, double (&yr)[R][CB],
                                           double (&yi)[R][CB], ShWG& sh, BlockRed& br) {
  SWG<double, CB> st;
#pragma unroll
  for (int r = 0; r < kRWG; ++r)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      st.br[r][j] = (r < R) ? yr[r < R ? r : 0][j] : 0.0;
      st.bi[r][j] = (r < R) ? yi[r < R ? r : 0][j] : 0.0;
    }
  sweep_wg<double, CB>(rm.H, rm.n, sp.re, sp.im, st, sh);
  const bool singular = br.max(st.singular ? 1.0 : 0.0) > 0.0;
  apply_rotations_wg<double, CB>(rm.n, st, sh);
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      yr[r][j] = st.br[r][j];
      yi[r][j] = st.bi[r][j];
    }
  return singular;
}

struct DDResult {
  double est;
  int solves;
  bool singular;
};

// x = (s I - A)^{-1} c for CB right-hand sides c (in the model's own
// coordinates, float64), refined with the residual in double-double.  On
// return x = (xr, xi) in double-double; res.est is the largest last
// correction norm ||dx|| / ||x|| over the columns.  If the float64 solve
// meets an exactly zero diagonal entry of R, returns at once with
// res.singular and y = (s I - H)^{-1} Q^T c in (yr, yi), reduced
// coordinates.
template <int R, int CB>
__device__ __forceinline__ DDResult refine_solve(const ReducedModel& rm, SPoint sp, double tol, const double (&cr)[R][CB],
                                 const double (&ci)[R][CB], dd (&xr)[R][CB], dd (&xi)[R][CB],
                                 double (&yr)[R][CB], double (&yi)[R][CB], DDShared& S, BlockRed& br) {
  const int tid = threadIdx.x;
  const int n = rm.n;
  constexpr int kMaxDD = 4;
  const gptr<double> A0 = (gptr<double>)rm.A0;  // column-major
  DDResult res{0.0, 1, false};
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      yr[r][j] = cr[r][j];
      yi[r][j] = ci[r][j];
    }
  apply_q<R, CB>(rm, true, yr, yi, br);  // Q^T c
  res.singular = hess_solve<R, CB>(rm, sp, yr, yi, S.sh, br);
  if (res.singular) {
    res.est = INFINITY;
    return res;
  }
  double tr[R][CB], ti[R][CB];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      tr[r][j] = yr[r][j];
      ti[r][j] = yi[r][j];
    }
  apply_q<R, CB>(rm, false, tr, ti, br);  // x = Q y
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      xr[r][j] = dd{tr[r][j], 0.0};
      xi[r][j] = dd{ti[r][j], 0.0};
    }
  double dprev[CB];
  bool done[CB];
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    dprev[j] = INFINITY;
    done[j] = false;
  }
  double est[CB];
#pragma unroll
  for (int j = 0; j < CB; ++j) est[j] = 0.0;
  for (int it = 0; it < kMaxDD; ++it) {
    // r = c - s x + A0 x, in double-double, then rounded
    __syncthreads();  // S.x of the previous pass has been read
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + kThreadsWG * r;
      if (i < n)
#pragma unroll
        for (int j = 0; j < CB; ++j) S.x[i * CB + j] = double4{xr[r][j].hi, xr[r][j].lo, xi[r][j].hi, xi[r][j].lo};
    }
    __syncthreads();
    dd ar[R][CB], ai[R][CB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        // c - sg x + w i x:  re = c - sg xr + w xi,  im = ci - sg xi - w xr
        ar[r][j] = dd_add(dd_add(dd{cr[r][j], 0.0}, dd_mul_d(xr[r][j], -sp.re)), dd_mul_d(xi[r][j], sp.im));
        ai[r][j] = dd_add(dd_add(dd{ci[r][j], 0.0}, dd_mul_d(xi[r][j], -sp.re)), dd_mul_d(xr[r][j], -sp.im));
      }
    // A0's columns are read two ahead of their use (the loads' latency
    // overlaps two columns' pair arithmetic)
    double an[2][R];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + kThreadsWG * r;
        an[q][r] = (i < n && q < n) ? A0[(size_t)q * n + i] : 0.0;
      }
    for (int c = 0; c < n; ++c) {
      double a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + kThreadsWG * r;
        a[r] = an[0][r];
        an[0][r] = an[1][r];
        an[1][r] = (i < n && c + 2 < n) ? A0[(size_t)(c + 2) * n + i] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + kThreadsWG * r;
        if (i < n) {
#pragma unroll
          for (int j = 0; j < CB; ++j) {
            const double4 xc = S.x[c * CB + j];
            ar[r][j] = dd_add(ar[r][j], dd_mul_d(dd{xc.x, xc.y}, a[r]));
            ai[r][j] = dd_add(ai[r][j], dd_mul_d(dd{xc.z, xc.w}, a[r]));
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        tr[r][j] = ar[r][j].hi + ar[r][j].lo;
        ti[r][j] = ai[r][j].hi + ai[r][j].lo;
      }
    // d = Q (s I - H)^{-1} Q^T r
    apply_q<R, CB>(rm, true, tr, ti, br);
    hess_solve<R, CB>(rm, sp, tr, ti, S.sh, br);
    apply_q<R, CB>(rm, false, tr, ti, br);
    ++res.solves;
    double nrm[2 * CB];
#pragma unroll
    for (int j = 0; j < 2 * CB; ++j) nrm[j] = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        // a column that has stopped keeps its x
        const double dr = done[j] ? 0.0 : tr[r][j], di = done[j] ? 0.0 : ti[r][j];
        xr[r][j] = dd_add(xr[r][j], dd{dr, 0.0});
        xi[r][j] = dd_add(xi[r][j], dd{di, 0.0});
        nrm[2 * j] += dr * dr + di * di;
        nrm[2 * j + 1] += xr[r][j].hi * xr[r][j].hi + xi[r][j].hi * xi[r][j].hi;
      }
    br.sumN<2 * CB>(nrm);
    bool all = true;
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      if (done[j]) continue;
      const double dn = sqrt(nrm[2 * j]), xn = sqrt(nrm[2 * j + 1]);
      est[j] = (xn > 0.0) ? dn / xn : (dn > 0.0 ? INFINITY : 0.0);
      if (!(est[j] > tol) || !(dn < 0.5 * dprev[j])) done[j] = true;  // converged (or x = 0), or stalled
      dprev[j] = dn;
      all = all && done[j];
    }
    if (all) break;
  }
#pragma unroll
  for (int j = 0; j < CB; ++j) res.est = fmax(res.est, est[j]);
  return res;
}

// out(:, j0 + j) = sign * C0 x_j (+ D(:, j0 + j) for G), j < nb: per-thread
// double-double sums, then the workgroup sum of the high and low parts.
template <int R, int CB>
__device__ __forceinline__ void write_cx(const ReqDesc& rd, const ReducedModel& rm, int j0, int nb, const dd (&xr)[R][CB],
                         const dd (&xi)[R][CB], double* out, bool deriv, BlockRed& br) {
  const int tid = threadIdx.x;
  const int n = rm.n, m = rm.m, p = rm.p;
  const gptr<double> C0 = (gptr<double>)rm.C0;  // row-major
  for (int a = 0; a < p; ++a) {
    dd gr[CB], gi[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) gr[j] = gi[j] = dd{0.0, 0.0};
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + kThreadsWG * r;
      if (i < n) {
        const double c = C0[(size_t)a * n + i];
#pragma unroll
        for (int j = 0; j < CB; ++j) {
          gr[j] = dd_add(gr[j], dd_mul_d(xr[r][j], c));
          gi[j] = dd_add(gi[j], dd_mul_d(xi[r][j], c));
        }
      }
    }
    double v[4 * CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      v[4 * j] = gr[j].hi;
      v[4 * j + 1] = gi[j].hi;
      v[4 * j + 2] = gr[j].lo;
      v[4 * j + 3] = gi[j].lo;
    }
    br.sumN<4 * CB>(v);
    if (tid < CB && tid < nb) {
      const int j = j0 + tid;
      double vv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) vv[q] = v[4 * 0 + q];
#pragma unroll
      for (int jj = 1; jj < CB; ++jj)
        if (tid == jj)
#pragma unroll
          for (int q = 0; q < 4; ++q) vv[q] = v[4 * jj + q];
      double2 g;
      if (deriv) {
        g.x = -(vv[0] + vv[2]);
        g.y = -(vv[1] + vv[3]);
      } else {
        g.x = (vv[0] + vv[2]) + ((gptr<double>)rm.D)[a * m + j];
        g.y = vv[1] + vv[3];
      }
      store_c(out, g_index(rd, a, j), g);
    }
  }
}

// Columns j0 .. j0+nb-1 (nb <= CB) of point k: G(:, j) = C0 x + D(:, j) with
// x = (s I - A)^{-1} B0(:, j) refined as above; with a derivative requested,
// also dG/ds(:, j) = -C0 (s I - A)^{-1} x, the second solve refined the same
// way.  Columns past nb solve a zero right-hand side and write nothing.
template <int R, int CB>
__device__ __forceinline__ DDResult refine_block(const ReqDesc& rd, const ReducedModel& rm, int64_t k, int j0, int nb,
                                 DDShared& S, BlockRed& br) {
  const int tid = threadIdx.x;
  const int n = rm.n;
  const SPoint sp = point_of(rd, k);
  const double tol = 0.1 * rd.rtol;
  const gptr<double> B0 = (gptr<double>)rm.B0;  // column-major
  double cr[R][CB], ci[R][CB], yr[R][CB], yi[R][CB];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + kThreadsWG * r;
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      cr[r][j] = (i < n && j < nb) ? B0[(size_t)(j0 + j) * n + i] : 0.0;
      ci[r][j] = 0.0;
    }
  }
  dd xr[R][CB], xi[R][CB];
  DDResult res = refine_solve<R, CB>(rm, sp, tol, cr, ci, xr, xi, yr, yi, S, br);
  double* G = rd.G + (size_t)k * rd.p * rd.m * 2;
  if (res.singular) {  // the float64 solution as it is (IEEE values)
    for (int j = 0; j < nb; ++j) {
      double xr1[kRWG][1], xi1[kRWG][1];
#pragma unroll
      for (int r = 0; r < kRWG; ++r) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int jj = 0; jj < CB; ++jj)
            if (rr == r && jj == j) {
              a = yr[rr][jj];
              b = yi[rr][jj];
            }
        xr1[r][0] = a;
        xi1[r][0] = b;
      }
      write_output_wg<1>(rd, j0 + j, 1, xr1, xi1, G, S.sh);
    }
    return res;
  }
  write_cx<R, CB>(rd, rm, j0, nb, xr, xi, G, false, br);
  if (rd.dG) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        cr[r][j] = xr[r][j].hi + xr[r][j].lo;
        ci[r][j] = xi[r][j].hi + xi[r][j].lo;
      }
    dd x2r[R][CB], x2i[R][CB];
    const DDResult r2 = refine_solve<R, CB>(rm, sp, tol, cr, ci, x2r, x2i, yr, yi, S, br);
    write_cx<R, CB>(rd, rm, j0, nb, x2r, x2i, rd.dG + (size_t)k * rd.p * rd.m * 2, true, br);
    res.est = fmax(res.est, r2.est);
    res.solves += r2.solves;
  }
  return res;
}

// Columns j0 .. j0+mc-1 of point k, CB at a time.
template <int R, int CB>
__device__ __forceinline__ void refine_columns(const ReqDesc& rd, const ReducedModel& rm, int64_t k, int j0, int mc, DDShared& S,
                               BlockRed& br, double& est, int& solves, bool& singular) {
  for (int jb = j0; jb < j0 + mc; jb += CB) {
    const int nb = min(CB, j0 + mc - jb);
    const DDResult rr = refine_block<R, CB>(rd, rm, k, jb, nb, S, br);
    est = fmax(est, rr.est);
    solves = max(solves, rr.solves);
    singular = singular || rr.singular;
  }
}

// Size class of the refinement: (R, CB) = (1, 4), (2, 2), (4, 1).
__host__ __device__ constexpr int dd_class(int n) { return n <= kThreadsWG ? 0 : n <= 2 * kThreadsWG ? 1 : 2; }

// One workgroup per queued entry at a time.  The entries of all segments of
// the kernel's size class are numbered in segment order and dealt out over
// the grid together, so that the few entries of many requests run side by
// side (one kernel per class, so that each is register-allocated for its
// own block shape).
template <int R, int CB>
__global__ __launch_bounds__(kThreadsWG) void refine_dd_kernel(const DDLaunch L) {
  constexpr int kClass = R == 1 ? 0 : R == 2 ? 1 : 2;
  __shared__ DDShared S;
  // queued entries per segment: one per (point, column group) at most, K x m
  uint32_t cnt[kMaxDDSegs];
  uint32_t total = 0;
#pragma unroll
  for (int i = 0; i < kMaxDDSegs; ++i) {
    cnt[i] = 0;
    if (i < L.nseg && dd_class(L.seg[i].rm.n) == kClass && L.seg[i].rd.n > 0) {
      const uint32_t cap = (uint32_t)min((uint64_t)UINT32_MAX, L.seg[i].K * (uint64_t)L.seg[i].rd.m);
      cnt[i] = min(*((const volatile uint32_t*)L.seg[i].rd.fbq), cap);
    }
    total += cnt[i];
  }
  for (uint32_t e = blockIdx.x; e < total; e += gridDim.x) {
    // the segment of entry e and its index there (uniform over the workgroup)
    int sgi = 0;
    uint32_t loc = e;
#pragma unroll
    for (int i = 0; i < kMaxDDSegs - 1; ++i) {
      if (sgi == i && loc >= cnt[i]) {
        loc -= cnt[i];
        sgi = i + 1;
      }
    }
    const DDSeg& g = L.seg[sgi];
    const uint32_t k = ((gptr<uint32_t>)g.rd.fbq)[2 + 2 * (size_t)loc];
    const uint32_t w1 = ((gptr<uint32_t>)g.rd.fbq)[3 + 2 * (size_t)loc];
    const int j0 = (int)(w1 & 0xffu), mc = (int)((w1 >> 8) & 0xffu);
    const int solves32 = (int)((w1 >> 16) & 0xffu), reason = (int)(w1 >> 24);
    BlockRed br(S.sh);
    double est = 0.0;
    int solves = 0;
    bool singular = false;
    refine_columns<R, CB>(g.rd, g.rm, (int64_t)k, j0, mc, S, br, est, solves, singular);
    if (threadIdx.x == 0) {
      lti_point_info inf;
      inf.est_rel_err = (float)est;
      inf.iters = (uint8_t)min(255, solves32 + solves);
      inf.path = singular ? LTI_PATH_SINGULAR : (reason == kReasonStall ? LTI_PATH_FALLBACK : LTI_PATH_FP64_DD);
      inf.reserved = 0;
      put_info(g.rd, (int64_t)k, inf);
    }
    __syncthreads();  // LDS reuse by the next entry
  }
}

}  // namespace

int sweep_wg_class(int precision, int n, int mc) {
  if (precision != LTI_PREC_FP64 && precision != LTI_PREC_REFINED) return -1;
  if (n <= kMaxN || n > kThreadsWG * kRWG || mc < 1 || mc > 4) return -1;
  return precision * 3 + ((mc <= 1) ? 0 : (mc <= 2) ? 1 : 2);
}

hipError_t launch_sweep_wg(int cls, const SweepLaunch& L, hipStream_t s) {
  if (L.ntiles <= 0) return hipSuccess;
  if (cls < 0 || cls >= kNumSweepWGClasses) return hipErrorInvalidValue;
  using Fn = void (*)(const SweepLaunch);
  static const Fn fns[kNumSweepWGClasses] = {
      sweep_wg_kernel<LTI_PREC_FP64, 1>,    sweep_wg_kernel<LTI_PREC_FP64, 2>,
      sweep_wg_kernel<LTI_PREC_FP64, 4>,    sweep_wg_kernel<LTI_PREC_REFINED, 1>,
      sweep_wg_kernel<LTI_PREC_REFINED, 2>, sweep_wg_kernel<LTI_PREC_REFINED, 4>};
  hipLaunchKernelGGL(fns[cls], dim3(L.ntiles), dim3(kThreadsWG), 0, s, L);
  return hipGetLastError();
}

hipError_t launch_refine_dd(const DDLaunch& L, int grid, hipStream_t s) {
  if (L.nseg <= 0) return hipSuccess;
  if (L.nseg > kMaxDDSegs || grid <= 0) return hipErrorInvalidValue;
  bool used[3] = {false, false, false};
  for (int i = 0; i < L.nseg; ++i) used[dd_class(L.seg[i].rm.n)] = true;
  using Fn = void (*)(const DDLaunch);
  static const Fn fns[3] = {refine_dd_kernel<1, 4>, refine_dd_kernel<2, 2>, refine_dd_kernel<4, 1>};
  for (int c = 0; c < 3; ++c) {
    if (!used[c]) continue;
    hipLaunchKernelGGL(fns[c], dim3(grid), dim3(kThreadsWG), 0, s, L);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lti
