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
  double segA[4 * kRWG];          // scan: per-segment products
  double segU[4 * kRWG][2 * 4];   // scan: per-segment sums (complex, per column)
  double tin[4 * kRWG][2 * 4];    // scan: carry into each segment
  double first[4 * kRWG][3 + 2 * 4];  // rotation and y of each segment's first row
  double red[4][8][2];            // per-wavefront partial sums of G
  double misc[4];
};

template <typename T, int MM>
__device__ __forceinline__ void sweep_wg(const T* Hg, int n, T w, SWG<T, MM>& st, ShWG& sh) {
  const int tid = threadIdx.x;
  const gptr<T> H = (gptr<T>)Hg;
  const cptr<T> Hs = (cptr<T>)Hg;
  st.singular = false;
  {
    const int off = hoff32(n - 1);
#pragma unroll
    for (int r = 0; r < kRWG; ++r) {
      const int i = tid + kThreadsWG * r;
      const T h = (i < n) ? H[off + i] : (T)0;
      st.cr[r] = -h;
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
  T sub0 = (n >= 2) ? Hs[hoff32(n - 2) + n - 1] : (T)0;
  T sub1 = (n >= 3) ? Hs[hoff32(n - 3) + n - 2] : (T)0;
  for (int k = n - 1; k >= 1; --k) {
    const int tk = k % kThreadsWG, rk = k / kThreadsWG;
    double* slot = sh.piv[k & 1];
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
      for (int q = 0; q < 2 + 2 * MM; ++q) slot[q] = (double)pv[q];
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
    const T sub2 = (k >= 3) ? Hs[hoff32(k - 3) + k - 2] : (T)0;
    __syncthreads();
    const T ar = (T)slot[0], ai = (T)slot[1];
    T bkr[MM], bki[MM];
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      bkr[j] = (T)slot[2 + 2 * j];
      bki[j] = (T)slot[3 + 2 * j];
    }
    const T beta = -sub0;
    const T nrm2 = ar * ar + ai * ai + beta * beta;
    const bool ok = nrm2 > (T)0;
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
        const T o = -hc[r];
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
    sub0 = sub1;
    sub1 = sub2;
  }
  // R(0,0): the final carry entry of row 0 (thread 0, slice 0)
  if (tid == 0) {
    sh.misc[0] = (double)st.cr[0];
    sh.misc[1] = (double)st.ci[0];
  }
  __syncthreads();
  const T ar = (T)sh.misc[0], ai = (T)sh.misc[1];
  const T d = ar * ar + ai * ai;
  st.singular = st.singular || !(d > (T)0);
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
                                                ShWG& sh) {
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
      g.x = gr + ((gptr<double>)rd.D)[a * m + j0 + j];
      g.y = gi;
      store_c(G, a * m + j0 + j, g);
    }
    __syncthreads();
  }
}

template <int MM>
__device__ void solve_wg_fp64(const ReqDesc& rd, int64_t k, int j0, int mc, ShWG& sh) {
  const int tid = threadIdx.x;
  const int n = rd.n, m = rd.m;
  const double w = ((gptr<double>)rd.omega)[k];
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
  sweep_wg<double, MM>(rd.H, n, w, st, sh);
  apply_rotations_wg<double, MM>(n, st, sh);
  double* G = rd.G + (size_t)k * rd.p * m * 2;
  write_output_wg<MM>(rd, j0, mc, st.br, st.bi, G, sh);
  if (rd.info && tid == 0 && j0 == 0) {
    lti_point_info inf;
    inf.est_rel_err = 0.0f;  // no diagonal-ratio estimate on this path
    inf.iters = 1;
    inf.path = st.singular ? LTI_PATH_SINGULAR : LTI_PATH_FP64;
    inf.reserved = 0;
    store_info(rd.info, k, inf);
  }
}

template <int MM>
// At most 256 registers per lane, so that two workgroups share a CU (the
// step loop is latency-bound: one barrier and one LDS round trip per step);
// the four-column kernel then keeps a few values of its set-up and output
// phases in scratch memory, none in the step loop.
__global__ __launch_bounds__(kThreadsWG) __attribute__((amdgpu_waves_per_eu(2))) void sweep_wg_kernel(
    const SweepLaunch L) {
  __shared__ ShWG sh;
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  if (tile >= L.ntiles) return;
  const int s = seg_of(L, tile);
  const ReqDesc rd = L.seg[s].rd;
  const Tile td = tile_of(L.seg[s], tile);
  for (uint32_t f = 0; f < td.count; ++f) solve_wg_fp64<MM>(rd, (int64_t)td.start + f, td.j0, td.mc, sh);
}

}  // namespace

int sweep_wg_class(int precision, int n, int mc) {
  if (precision != LTI_PREC_FP64) return -1;
  if (n <= kMaxN || n > kThreadsWG * kRWG || mc < 1 || mc > 4) return -1;
  return (mc <= 1) ? 0 : (mc <= 2) ? 1 : 2;
}

hipError_t launch_sweep_wg(int cls, const SweepLaunch& L, hipStream_t s) {
  if (L.ntiles <= 0) return hipSuccess;
  if (cls < 0 || cls > 2) return hipErrorInvalidValue;
  using Fn = void (*)(const SweepLaunch);
  const Fn fn = cls == 0 ? sweep_wg_kernel<1> : cls == 1 ? sweep_wg_kernel<2> : sweep_wg_kernel<4>;
  hipLaunchKernelGGL(fn, dim3(L.ntiles), dim3(kThreadsWG), 0, s, L);
  return hipGetLastError();
}

}  // namespace lti
