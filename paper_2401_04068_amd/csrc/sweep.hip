// Per-frequency shifted Hessenberg solves: one wavefront per tile of
// frequencies (and right-hand-side columns) of one request.
//
// For one frequency w, M = j w I - H is upper Hessenberg with a complex
// diagonal and real off-diagonal entries.  Columns are rotated right to left,
// k = n-1 .. 1: a unitary 2x2 rotation of columns (k-1, k),
//
//     [col_{k-1}, col_k] <- [col_{k-1}, col_k] [[s, c], [-c, conj(s)]] ,
//     r = sqrt(|alpha|^2 + beta^2),  c = beta / r (real),  s = alpha / r ,
//
// with alpha = M(k, k) as modified so far and beta = M(k, k-1), zeroes
// M(k, k-1) and leaves column k final: M Z = R with R upper triangular and
// R(k, k) = r real and positive (Golub & Van Loan, sec. 5.1.8, complex
// Givens rotations; Laub 1981 for the per-frequency Hessenberg solve).  As
// soon as column k of R is final, the back-substitution for R y = B takes
// its step: b_{0..k-1} -= (R(0..k-1, k) / r) b_k, and y_k = b_k / r.  R is
// never stored.  Then X = Z y is formed by applying the rotations in
// increasing order, which is the first-order linear recurrence
//
//     t_0 = y_0,  t_k = -c_k t_{k-1} + conj(s_k) y_k,
//     x_{k-1} = s_k t_{k-1} + c_k y_k,  x_{n-1} = t_{n-1} ,
//
// evaluated as a Kogge-Stone scan across lanes.  Finally G = Ct^T X + D with a
// reduce-scatter over the 64 lanes.
//
// Lane layout: row i lives on lane i % 64 in register slice i / 64 (R slices,
// n <= 64 R); each lane holds its rows' carry entry (the column being
// rotated) and right-hand-side rows (MM complex columns); row k keeps b_k,
// the rotation and 1/r after its step.  Per step the pivot row's carry and
// the subdiagonal entry reach every lane as scalars (readlane and a scalar
// load issued two steps ahead), b_k through an LDS broadcast; the column of
// H (real, read once per step, right to left from the packed column-major
// layout) is loaded one step ahead.  Every frequency of a request reads the
// same H, which stays in L1/L2.
#include <cfloat>
#include <cmath>

#include "lti_kernels.h"
#include "sweep_common.h"

namespace lti {

namespace {

using namespace sweep_detail;

// Register state of one frequency's solve.
template <typename T, int R, int MM>
struct Sweep {
  T cr[R], ci[R];           // carry column (real, imag)
  T br[R][MM], bi[R][MM];   // right-hand side; after the sweep y; after apply_rotations x
  T rc[R], rsr[R], rsi[R];  // rotation k stored on row k (row 0 unused)
  T rinv[R];                // 1 / R(k, k) on row k (row 0 unused)
  bool singular;
};

// Givens RQ sweep fused with back-substitution.  On entry br/bi hold the
// right-hand-side rows; on exit they hold y.  `bcast` is this wavefront's
// 2 * MM values of LDS.
//
// kE (descriptor systems, float64): M = s T - H with T upper triangular
// (packed, column j rows 0 .. j at j (j + 1) / 2), so every entry on and
// above the diagonal is s T(i, k) - H(i, k), complex; the subdiagonal stays
// -H(k+1, k).  The rotations and back-substitution are the same.
template <typename T, int R, int MM, bool kLds, bool kE = false>
__device__ __forceinline__ void givens_sweep(Src<T, kLds> H, int n, T sg, T w, Sweep<T, R, MM>& st, T* bcast,
                                             const T* Tm = nullptr) {
  const int lane = threadIdx.x & 63;
  st.singular = false;
  const gptr<T> TT = (gptr<T>)Tm;
  // the pivot row's right-hand side reaches the lanes through scalar
  // registers when it takes at most 16 of them, else through LDS
  constexpr bool kBcastSgpr = false;
  auto toff = [](int j) { return j * (j + 1) / 2; };
  {
    const int off = hoff32(n - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
      const T h = (i < n) ? H[off + i] : (T)0;
      if constexpr (kE) {
        const T t = (i < n) ? TT[toff(n - 1) + i] : (T)0;
        st.cr[r] = sg * t - h;
        st.ci[r] = w * t;
      } else {
        st.cr[r] = (i == n - 1) ? sg - h : -h;
        st.ci[r] = (i == n - 1) ? w : (T)0;
      }
      st.rc[r] = (T)0;
      st.rsr[r] = (T)1;
      st.rsi[r] = (T)0;
      st.rinv[r] = (T)1;
    }
  }
  // column n-2 (rows 0..n-1) for the first step
  T hc[R], tc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    hc[r] = (T)0;
    tc[r] = (T)0;
  }
  if (n >= 2) {
    const int off = hoff32(n - 2);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
      if (i <= n - 1) hc[r] = H[off + i];
      if constexpr (kE) {
        if (i <= n - 2) tc[r] = TT[toff(n - 2) + i];
      }
    }
  }
  // subdiagonal H(k, k-1) for the next two steps (scalar loads)
  T sub0 = (n >= 2) ? H.uniform(hoff32(n - 2) + n - 1) : (T)0;
  T sub1 = (n >= 3) ? H.uniform(hoff32(n - 3) + n - 2) : (T)0;

#pragma unroll
  for (int s = R - 1; s >= 0; --s) {
    if (64 * s > n - 1) continue;  // no pivot row in this slice
    const int khi = (n - 1 < 64 * s + 63) ? n - 1 : 64 * s + 63;
    const int klo = (64 * s > 1) ? 64 * s : 1;
    for (int k = khi; k >= klo; --k) {
      const int kl = k - 64 * s;
      // b_k to LDS (lane kl), read back below as a broadcast, unless it is
      // small enough to go through scalar registers (readlane)
      if constexpr (!kBcastSgpr) {
        if (lane == kl) {
#pragma unroll
          for (int j = 0; j < MM; ++j) {
            bcast[2 * j] = st.br[s][j];
            bcast[2 * j + 1] = st.bi[s][j];
          }
        }
      }
      // prefetch: column k-2 (rows 0..k-1) and subdiagonal H(k-2, k-3)
      T hn[R], tn[R];
#pragma unroll
      for (int t = 0; t < R; ++t) {
        hn[t] = (T)0;
        tn[t] = (T)0;
      }
      if (k >= 2) {
        const int off = hoff32(k - 2);
#pragma unroll
        for (int t = 0; t <= s; ++t) {
          const int i = lane + 64 * t;
          // with two or more slices (n > 64) the pivot slice's loads past
          // row k-1 stay inside the packed array (its last column k-2 = n-3
          // has 3n - 1 entries after it, n + 62 of them read at most), and
          // those lanes never use the values: no per-lane test
          if constexpr (R >= 2 && !kE) {
            hn[t] = H[off + i];
          } else {
            if (i <= k - 1) hn[t] = H[off + i];
          }
          if constexpr (kE) {
            if (i <= k - 2) tn[t] = TT[toff(k - 2) + i];
          }
        }
      }
      const T sub2 = (k >= 3) ? H.uniform(hoff32(k - 3) + k - 2) : (T)0;

      const T ar = readlane(st.cr[s], kl);
      const T ai = readlane(st.ci[s], kl);
      const T beta = -sub0;
      const T nrm2 = ar * ar + ai * ai + beta * beta;
      T rinv, c, sr, si;
      if (norm2_ok(nrm2)) {
        rinv = rsqrt_t(nrm2);
        c = beta * rinv;
        sr = ar * rinv;
        si = ai * rinv;
      } else {  // zero column (or out of range): identity rotation, flagged
        rinv = (T)INFINITY;
        c = (T)0;
        sr = (T)1;
        si = (T)0;
        st.singular = true;
      }
      T bkr[MM], bki[MM];
      if constexpr (kBcastSgpr) {
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          bkr[j] = readlane(st.br[s][j], kl);
          bki[j] = readlane(st.bi[s][j], kl);
        }
      } else {
        // the LDS write above must land before any lane reads it back
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          bkr[j] = bcast[2 * j];
          bki[j] = bcast[2 * j + 1];
        }
      }
      // the shift s = sg + j w on the diagonal entry of column k-1 (row
      // k-1, in slice s or s-1), added to that row's results afterwards
      const T csg = c * sg, cw = c * w;
      const T d1 = sr * sg - si * w, d2 = si * sg + sr * w;
#pragma unroll
      for (int t = 0; t <= s; ++t) {
        const int i = lane + 64 * t;
        if (t < s || lane < kl) {
          const T cr_ = st.cr[t], ci_ = st.ci[t];
          T nkr, nki, n1r, n1i;
          if constexpr (kE) {
            // M(i, k-1) = s T(i, k-1) - H(i, k-1), complex
            const T orr = sg * tc[t] - hc[t];
            const T oi = w * tc[t];
            nkr = c * orr + sr * cr_ + si * ci_;
            nki = c * oi + sr * ci_ - si * cr_;
            n1r = sr * orr - c * cr_ - si * oi;
            n1i = si * orr + sr * oi - c * ci_;
          } else {
            // M(i, k-1) = -H(i, k-1) off the diagonal; the diagonal entry
            // also holds s: its share is added on row k-1 only
            const T o = -hc[t];
            nkr = c * o + sr * cr_ + si * ci_;
            nki = sr * ci_ - si * cr_;
            n1r = sr * o - c * cr_;
            n1i = si * o - c * ci_;
            if (t >= s - 1) {  // the slices that can hold row k-1
              const T d = (i == k - 1) ? (T)1 : (T)0;
              nkr = fma(d, csg, nkr);
              nki = fma(d, cw, nki);
              n1r = fma(d, d1, n1r);
              n1i = fma(d, d2, n1i);
            }
          }
          st.cr[t] = n1r;
          st.ci[t] = n1i;
          nkr *= rinv;  // R(i, k) / R(k, k)
          nki *= rinv;
#pragma unroll
          for (int j = 0; j < MM; ++j) {
            st.br[t][j] = fma(-nkr, bkr[j], st.br[t][j]);
            st.br[t][j] = fma(nki, bki[j], st.br[t][j]);
            st.bi[t][j] = fma(-nkr, bki[j], st.bi[t][j]);
            st.bi[t][j] = fma(-nki, bkr[j], st.bi[t][j]);
          }
        }
      }
      if (lane == kl) {
        st.rc[s] = c;
        st.rsr[s] = sr;
        st.rsi[s] = si;
        st.rinv[s] = rinv;
      }
      // the next step's LDS write must not overtake this step's reads
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int t = 0; t < R; ++t) {
        hc[t] = hn[t];
        tc[t] = tn[t];
      }
      sub0 = sub1;
      sub1 = sub2;
    }
  }
  // y_k = b_k / R(k,k); row 0: R(0,0) is the final carry entry (complex)
  const T ar = readlane(st.cr[0], 0);
  const T ai = readlane(st.ci[0], 0);
  const T d = ar * ar + ai * ai;
  if (!norm2_ok(d)) st.singular = true;
  const T dinv = (T)1 / d;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
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
}

// Ratio of the largest to the smallest |R(k,k)| (a lower bound on the
// condition number of R), from the per-row 1/R(k,k) and R(0,0).
template <typename T, int R, int MM>
__device__ __forceinline__ double diag_ratio(int n, const Sweep<T, R, MM>& st) {
  const int lane = threadIdx.x & 63;
  double lo = INFINITY, hi = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
    if (i >= 1 && i < n) {
      const double ri = (double)st.rinv[r];
      lo = fmin(lo, ri);  // 1 / largest
      hi = fmax(hi, ri);  // 1 / smallest
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, d, 64));
    hi = fmax(hi, __shfl_xor(hi, d, 64));
  }
  const double ar = (double)readlane(st.cr[0], 0);
  const double ai = (double)readlane(st.ci[0], 0);
  const double r0 = sqrt(ar * ar + ai * ai);
  const double rmax = fmax(1.0 / lo, r0);
  const double rmin = fmin(1.0 / hi, r0);
  return rmax / rmin;
}

// x := Z y, in place in br/bi (see the recurrence at the top of the file).
// The scan's multipliers depend only on the rotations, so they are computed
// once and the right-hand-side columns are then scanned one at a time.
template <typename T, int R, int MM>
__device__ __forceinline__ void apply_rotations(int n, Sweep<T, R, MM>& st) {
  const int lane = threadIdx.x & 63;
  T tinr[MM], tini[MM];  // t at the last row of the previous slice
#pragma unroll
  for (int j = 0; j < MM; ++j) tinr[j] = tini[j] = (T)0;
#pragma unroll
  for (int s = 0; s < R; ++s) {
    if (64 * s >= n) break;
    const int i = lane + 64 * s;
    const bool inner = (i > 0 && i < n);
    // element i is t -> a t + u; a = -c_i (0 for row 0 and past the end)
    T a = inner ? -st.rc[s] : (T)0;
    T am[6];  // multiplier of the shifted partial sum at each scan stage
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int d = 1 << q;
      const T ap = __shfl_up(a, d, 64);
      am[q] = (lane >= d) ? a : (T)0;
      if (lane >= d) a = a * ap;
    }
    // rotation of row i+1 (lane 63 takes row 64(s+1) from the next slice)
    T nc = __shfl_down(st.rc[s], 1, 64);
    T nsr = __shfl_down(st.rsr[s], 1, 64);
    T nsi = __shfl_down(st.rsi[s], 1, 64);
    const int sn = (s + 1 < R) ? s + 1 : s;
    if (s + 1 < R) {
      const T c0 = readlane(st.rc[sn], 0);
      const T s0r = readlane(st.rsr[sn], 0);
      const T s0i = readlane(st.rsi[sn], 0);
      if (lane == 63) {
        nc = c0;
        nsr = s0r;
        nsi = s0i;
      }
    }
    const T sr = st.rsr[s], si = st.rsi[s];
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const T yr = st.br[s][j], yi = st.bi[s][j];
      T ur, ui;
      if (inner) {  // conj(s_i) y_i
        ur = sr * yr + si * yi;
        ui = sr * yi - si * yr;
      } else {
        ur = (i == 0) ? yr : (T)0;
        ui = (i == 0) ? yi : (T)0;
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const int d = 1 << q;
        const T upr = __shfl_up(ur, d, 64);
        const T upi = __shfl_up(ui, d, 64);
        if (lane >= d) {
          ur = fma(am[q], upr, ur);
          ui = fma(am[q], upi, ui);
        }
      }
      const T tr = fma(a, tinr[j], ur);
      const T ti = fma(a, tini[j], ui);
      T nyr = __shfl_down(yr, 1, 64);
      T nyi = __shfl_down(yi, 1, 64);
      if (s + 1 < R) {
        const T y0r = readlane(st.br[sn][j], 0);
        const T y0i = readlane(st.bi[sn][j], 0);
        if (lane == 63) {
          nyr = y0r;
          nyi = y0i;
        }
      }
      tinr[j] = readlane(tr, 63);
      tini[j] = readlane(ti, 63);
      if (i < n - 1) {  // x_i = s_{i+1} t_i + c_{i+1} y_{i+1}
        st.br[s][j] = nsr * tr - nsi * ti + nc * nyr;
        st.bi[s][j] = nsr * ti + nsi * tr + nc * nyi;
      } else if (i == n - 1) {
        st.br[s][j] = tr;
        st.bi[s][j] = ti;
      }
    }
  }
}

// One halving stage of the reduce-scatter: lanes whose bit D is set keep the
// upper H entries and send the lower ones to their partner (and vice versa).
template <int V, int H, int D>
__device__ __forceinline__ void rs_stage(double (&vr)[V], double (&vi)[V]) {
  const bool upper = ((threadIdx.x & 63) & D) != 0;
#pragma unroll
  for (int q = 0; q < H; ++q) {
    const double sr = upper ? vr[q] : vr[q + H];
    const double si = upper ? vi[q] : vi[q + H];
    const double kr = upper ? vr[q + H] : vr[q];
    const double ki = upper ? vi[q + H] : vi[q];
    vr[q] = kr + __shfl_xor(sr, D, 64);
    vi[q] = ki + __shfl_xor(si, D, 64);
  }
}

// Sum over the 64 lanes of kV = 8 complex values at once: after the call
// lane l holds the total of index l >> 3 in vr[0], vi[0].
constexpr int kV = 8;
__device__ __forceinline__ void reduce_scatter8(double (&vr)[kV], double (&vi)[kV]) {
  rs_stage<kV, 4, 32>(vr, vi);
  rs_stage<kV, 2, 16>(vr, vi);
  rs_stage<kV, 1, 8>(vr, vi);
#pragma unroll
  for (int d = 4; d >= 1; d >>= 1) {
    vr[0] += __shfl_xor(vr[0], d, 64);
    vi[0] += __shfl_xor(vi[0], d, 64);
  }
}

// G(:, j0 .. j0+mc-1) = Ct^T X + D for one frequency, X in xr/xi; with
// `deriv`, -Ct^T X (the derivative -C (sI - A)^{-2} B from X = (sI - H)^{-2} Q^T B).
template <int R, int MM, bool kLds>
__device__ __forceinline__ void write_output(const ReqDesc& rd, Src<double, kLds> Ct, int j0, int mc,
                                             const double (&xr)[R][MM], const double (&xi)[R][MM],
                                             double* __restrict__ G, bool deriv = false) {
  const int lane = threadIdx.x & 63;
  const int n = rd.n, m = rd.m, p = rd.p;
  constexpr int PC = (kV / MM > 0) ? kV / MM : 1;  // rows of G per pass
  constexpr int MC = (MM < kV) ? MM : kV;           // columns of G per pass
  for (int a0 = 0; a0 < p; a0 += PC) {
#pragma unroll
    for (int jb = 0; jb < MM; jb += MC) {
      if (jb >= mc) break;
      double vr[kV], vi[kV];
#pragma unroll
      for (int q = 0; q < kV; ++q) vr[q] = vi[q] = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = lane + 64 * r;
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
      reduce_scatter8(vr, vi);
      if ((lane & 7) == 0) {
        const int idx = lane >> 3;
        const int a = a0 + idx / MC;
        const int j = jb + idx % MC;
        if (a < p && j < mc) {
          double2 g;
          g.x = deriv ? -vr[0] : vr[0] + ((gptr<double>)rd.D)[a * m + j0 + j];
          g.y = deriv ? -vi[0] : vi[0];
          store_c(G, g_index(rd, a, j0 + j), g);
        }
      }
    }
  }
}

template <int R, int MM, bool kLds, bool kE = false>
__device__ void solve_fp64(const ReqDesc& rd, const ModelSrc<kLds>& md, int64_t k, int j0, int mc,
                           double* bcast) {
  const int lane = threadIdx.x & 63;
  const int n = rd.n, m = rd.m;
  const SPoint sp = point_of(rd, k);
  const Src<double, kLds> Bt = md.Bt;
  Sweep<double, R, MM> st;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      st.br[r][j] = (i < n && j < mc) ? Bt[i * m + j0 + j] : 0.0;
      st.bi[r][j] = 0.0;
    }
  }
  givens_sweep<double, R, MM, kLds, kE>(md.H, n, sp.re, sp.im, st, bcast, rd.T);
  // estimated error from the spread of R's diagonal; points above the
  // request's tolerance are finished by the extended refinement (not for
  // descriptor systems: their result is written with its estimate)
  const double est = fp64_estimate(n, diag_ratio<double, R, MM>(n, st));
  if (!kE && fp64_needs_dd(rd, est)) {
    if (lane == 0) enqueue_dd(rd, k, j0, mc, 0, kReasonFP64);
    return;
  }
  apply_rotations<double, R, MM>(n, st);
  double* G = rd.G + (size_t)k * rd.p * m * 2;
  write_output<R, MM, kLds>(rd, md.Ct, j0, mc, st.br, st.bi, G);
  if (rd.dG) {
    // dG/ds = -C (sI - A)^{-2} B: the same sweep with X as right-hand side
    givens_sweep<double, R, MM, kLds, kE>(md.H, n, sp.re, sp.im, st, bcast, rd.T);
    apply_rotations<double, R, MM>(n, st);
    write_output<R, MM, kLds>(rd, md.Ct, j0, mc, st.br, st.bi, rd.dG + (size_t)k * rd.p * m * 2, true);
  }
  if (lane == 0) {
    lti_point_info inf;
    inf.est_rel_err = (float)est;
    inf.iters = rd.dG ? 2 : 1;
    inf.path = LTI_PATH_FP64;
    inf.reserved = 0;
    put_info(rd, k, inf);
  }
}

// ---------------------------------------------------------------- refined

// r = Bt - (s X - H X), float64, rows lane + 64 t, columns j0 .. j0+MM-1.
template <int R, int MM, bool kLds>
__device__ __forceinline__ void residual64(const ReqDesc& rd, const ModelSrc<kLds>& md, double sg, double w, int j0,
                                           int mc, const double (&xr)[R][MM], const double (&xi)[R][MM],
                                           double (&rr)[R][MM], double (&ri)[R][MM]) {
  const int lane = threadIdx.x & 63;
  const int n = rd.n, m = rd.m;
  const Src<double, kLds> Bt = md.Bt;
  const Src<double, kLds> H = md.H;
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int i = lane + 64 * t;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const double b = (i < n && j < mc) ? Bt[i * m + j0 + j] : 0.0;
      rr[t][j] = fma(w, xi[t][j], fma(-sg, xr[t][j], b));
      ri[t][j] = fma(-w, xr[t][j], -sg * xi[t][j]);
    }
  }
#pragma unroll
  for (int sj = 0; sj < R; ++sj) {
    if (64 * sj >= n) break;
    const int jend = (n - 64 * sj < 64) ? n - 64 * sj : 64;
    for (int jl = 0; jl < jend; ++jl) {
      const int jc = 64 * sj + jl;  // column of H
      const int off = hoff32(jc);
      const int len = (jc + 2 < n) ? jc + 2 : n;
      double xjr[MM], xji[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        xjr[j] = readlane(xr[sj][j], jl);
        xji[j] = readlane(xi[sj][j], jl);
      }
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = lane + 64 * t;
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
  }
}

template <int R, int MM, bool kLds>
__device__ void solve_refined(const ReqDesc& rd, const ModelSrc<kLds>& md, int64_t k, int j0, int mc,
                              double* bcast64) {
  const int lane = threadIdx.x & 63;
  const int n = rd.n;
  const int m = rd.m;
  const SPoint sp = point_of(rd, k);
  const float sgf = (float)sp.re, wf = (float)sp.im;
  const double tol = 0.1 * rd.rtol;
  constexpr int kMaxIters = 6;
  float* bcast = reinterpret_cast<float*>(bcast64);
  const Src<float, kLds> Bt32 = md.Bt32;

  double xr[R][MM], xi[R][MM];
  Sweep<float, R, MM> st;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      st.br[r][j] = (i < n && j < mc) ? Bt32[i * m + j0 + j] : 0.0f;
      st.bi[r][j] = 0.0f;
    }
  }
  givens_sweep<float, R, MM, kLds>(md.H32, n, sgf, wf, st, bcast);
  apply_rotations<float, R, MM>(n, st);
  double dprev = 0.0;
  {
    double s2 = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        xr[r][j] = (double)st.br[r][j];
        xi[r][j] = (double)st.bi[r][j];
        s2 += xr[r][j] * xr[r][j] + xi[r][j] * xi[r][j];
      }
    dprev = sqrt(wave_sum(s2));
  }
  int iters = 1;
  double est = 1.0;
  bool ok = false;
  if (!st.singular && dprev < INFINITY && !(rd.flags & kFlagForceDD)) {
    for (int it = 0; it < kMaxIters; ++it) {
      double rr[R][MM], ri[R][MM];
      residual64<R, MM, kLds>(rd, md, sp.re, sp.im, j0, mc, xr, xi, rr, ri);
      double amax = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < MM; ++j) amax = fmax(amax, fmax(fabs(rr[r][j]), fabs(ri[r][j])));
      amax = wave_max(amax);
      if (amax == 0.0) {  // X solves the float64 system exactly
        est = 0.0;
        ok = true;
        break;
      }
      const double scale = 1.0 / amax;
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          st.br[r][j] = (float)(rr[r][j] * scale);
          st.bi[r][j] = (float)(ri[r][j] * scale);
        }
      givens_sweep<float, R, MM, kLds>(md.H32, n, sgf, wf, st, bcast);
      apply_rotations<float, R, MM>(n, st);
      ++iters;
      double d2 = 0.0, x2 = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          const double dr = (double)st.br[r][j] * amax;
          const double di = (double)st.bi[r][j] * amax;
          xr[r][j] += dr;
          xi[r][j] += di;
          d2 += dr * dr + di * di;
          x2 += xr[r][j] * xr[r][j] + xi[r][j] * xi[r][j];
        }
      const double dn = sqrt(wave_sum(d2));
      const double xn = sqrt(wave_sum(x2));
      if (!(dn < INFINITY) || !(xn > 0.0)) break;  // non-finite: stalled
      // predicted error after this correction: contraction (dn / dprev) times dn
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
  if (!ok) {  // stalled (or singular): the extended refinement finishes it
    if (lane == 0) enqueue_dd(rd, k, j0, mc, iters, kReasonStall);
    return;
  }
  double* G = rd.G + (size_t)k * rd.p * m * 2;
  write_output<R, MM, kLds>(rd, md.Ct, j0, mc, xr, xi, G);
  if (lane == 0) {
    lti_point_info inf;
    inf.est_rel_err = (float)est;
    inf.iters = (uint8_t)iters;
    inf.path = LTI_PATH_REFINED;
    inf.reserved = 0;
    put_info(rd, k, inf);
  }
}

template <int PREC, int R, int MM, bool kLds>
__device__ __forceinline__ void run_tile(const Tile& td, const ReqDesc& rd, const ModelSrc<kLds>& md,
                                         double* bcast) {
  for (uint32_t f = 0; f < td.count; ++f) {
    const int64_t k = (int64_t)td.start + f;
    if (PREC == LTI_PREC_FP64)
      solve_fp64<R, MM, kLds>(rd, md, k, td.j0, td.mc, bcast);
    else
      solve_refined<R, MM, kLds>(rd, md, k, td.j0, td.mc, bcast);
  }
}

template <int PREC, int R, int MM>
__global__ __launch_bounds__(64 * kWaves) void sweep_kernel(const SweepLaunch L, uint32_t lds_bytes) {
  extern __shared__ __align__(16) char stage[];
  __shared__ double bcast_all[kWaves][2 * MM];
  // the tile index is uniform per wavefront; say so, so that everything
  // derived from it stays in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tb = xcd_swizzle(blockIdx.x, gridDim.x) * kWaves;  // < ntiles
  const int tile = tb + wave;
  // stage the model in LDS when the whole workgroup works on one request
  const int s0 = seg_of(L, tb);
  const bool same = seg_of(L, min(tb + kWaves, L.ntiles) - 1) == s0;
  const ReqDesc rd0 = L.seg[s0].rd;
  const StageLayout SL = stage_layout(PREC, rd0.n, rd0.m, rd0.p);
  // (a model with more than 128 states never fits the staging limit)
  constexpr bool kCanStage = (R <= 2);
  const bool staged = kCanStage && same && lds_bytes > 0 && SL.bytes <= lds_bytes && SL.bytes <= kStageLimit;
  if (kCanStage && staged) {
    const int nh = (int)hlen(rd0.n);
    const int nb = rd0.n * rd0.m, nc = rd0.n * rd0.p;
    double* sH = reinterpret_cast<double*>(stage + SL.H);
    double* sB = reinterpret_cast<double*>(stage + SL.Bt);
    double* sC = reinterpret_cast<double*>(stage + SL.Ct);
    for (int i = threadIdx.x; i < nh; i += 64 * kWaves) sH[i] = rd0.H[i];
    for (int i = threadIdx.x; i < nb; i += 64 * kWaves) sB[i] = rd0.Bt[i];
    for (int i = threadIdx.x; i < nc; i += 64 * kWaves) sC[i] = rd0.Ct[i];
    if (PREC == LTI_PREC_REFINED) {
      float* sH32 = reinterpret_cast<float*>(stage + SL.H32);
      float* sB32 = reinterpret_cast<float*>(stage + SL.Bt32);
      for (int i = threadIdx.x; i < nh; i += 64 * kWaves) sH32[i] = rd0.H32[i];
      for (int i = threadIdx.x; i < nb; i += 64 * kWaves) sB32[i] = rd0.Bt32[i];
    }
    __syncthreads();
  }
  if (tile >= L.ntiles) return;
  const int s = seg_of(L, tile);
  const ReqDesc rd = L.seg[s].rd;
  const Tile td = tile_of(L.seg[s], tile);
  double* bcast = bcast_all[wave];
  if constexpr (kCanStage) {
    if (staged) {
      ModelSrc<true> md;
      md.H.p = reinterpret_cast<const double*>(stage + SL.H);
      md.Bt.p = reinterpret_cast<const double*>(stage + SL.Bt);
      md.Ct.p = reinterpret_cast<const double*>(stage + SL.Ct);
      md.H32.p = reinterpret_cast<const float*>(stage + SL.H32);
      md.Bt32.p = reinterpret_cast<const float*>(stage + SL.Bt32);
      run_tile<PREC, R, MM, true>(td, rd, md, bcast);
      return;
    }
  }
  {
    ModelSrc<false> md;
    md.H.p = rd.H;
    md.Bt.p = rd.Bt;
    md.Ct.p = rd.Ct;
    md.H32.p = rd.H32;
    md.Bt32.p = rd.Bt32;
    run_tile<PREC, R, MM, false>(td, rd, md, bcast);
  }
}

// Descriptor systems (float64 path, model read from global memory).
template <int R, int MM>
__global__ __launch_bounds__(64 * kWaves) void sweep_desc_kernel(const SweepLaunch L, uint32_t) {
  __shared__ double bcast_all[kWaves][2 * MM];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x) * kWaves + wave;
  if (tile >= L.ntiles) return;
  const int s = seg_of(L, tile);
  const ReqDesc rd = L.seg[s].rd;
  const Tile td = tile_of(L.seg[s], tile);
  ModelSrc<false> md;
  md.H.p = rd.H;
  md.Bt.p = rd.Bt;
  md.Ct.p = rd.Ct;
  md.H32.p = rd.H32;
  md.Bt32.p = rd.Bt32;
  for (uint32_t f = 0; f < td.count; ++f)
    solve_fp64<R, MM, false, true>(rd, md, (int64_t)td.start + f, td.j0, td.mc, bcast_all[wave]);
}

using KernelFn = void (*)(const SweepLaunch, uint32_t);

template <int PREC, int R>
constexpr KernelFn pick_mm(int mi) {
  return mi == 0 ? sweep_kernel<PREC, R, 1>
       : mi == 1 ? sweep_kernel<PREC, R, 2>
       : mi == 2 ? sweep_kernel<PREC, R, 4>
       : mi == 3 ? sweep_kernel<PREC, R, 8>
                 : sweep_kernel<PREC, R, 16>;
}

// R * MM <= 32 keeps the per-lane state in registers.
template <int PREC>
KernelFn pick(int ri, int mi) {
  switch (ri) {
    case 0: return pick_mm<PREC, 1>(mi);
    case 1: return pick_mm<PREC, 2>(mi);
    default:
      return mi == 0 ? sweep_kernel<PREC, 4, 1>
           : mi == 1 ? sweep_kernel<PREC, 4, 2>
           : mi == 2 ? sweep_kernel<PREC, 4, 4>
                     : sweep_kernel<PREC, 4, 8>;
  }
}

}  // namespace

int sweep_class(int precision, int n, int m) {
  if (precision != LTI_PREC_FP64 && precision != LTI_PREC_REFINED) return -1;
  if (n < 1 || n > kMaxN || m < 1 || m > kMaxRhs) return -1;
  const int ri = (n <= 64) ? 0 : (n <= 128) ? 1 : 2;
  const int mi = (m <= 1) ? 0 : (m <= 2) ? 1 : (m <= 4) ? 2 : (m <= 8) ? 3 : 4;
  if (ri == 2 && mi == 4) return -1;
  return (precision * kNumRowClasses + ri) * kNumRhsClasses + mi;
}

hipError_t launch_sweep_desc(int kclass, const SweepLaunch& L, hipStream_t s) {
  if (L.ntiles <= 0) return hipSuccess;
  if (kclass < 0 || kclass >= kNumRowClasses * kNumRhsClasses) return hipErrorInvalidValue;
  const int mi = kclass % kNumRhsClasses;
  const int ri = kclass / kNumRhsClasses;
  KernelFn fn;
  switch (ri * 8 + mi) {
    case 0: fn = sweep_desc_kernel<1, 1>; break;
    case 1: fn = sweep_desc_kernel<1, 2>; break;
    case 2: fn = sweep_desc_kernel<1, 4>; break;
    case 3: fn = sweep_desc_kernel<1, 8>; break;
    case 4: fn = sweep_desc_kernel<1, 16>; break;
    case 8: fn = sweep_desc_kernel<2, 1>; break;
    case 9: fn = sweep_desc_kernel<2, 2>; break;
    case 10: fn = sweep_desc_kernel<2, 4>; break;
    case 11: fn = sweep_desc_kernel<2, 8>; break;
    case 12: fn = sweep_desc_kernel<2, 16>; break;
    case 16: fn = sweep_desc_kernel<4, 1>; break;
    case 17: fn = sweep_desc_kernel<4, 2>; break;
    case 18: fn = sweep_desc_kernel<4, 4>; break;
    case 19: fn = sweep_desc_kernel<4, 8>; break;
    default: return hipErrorInvalidValue;
  }
  const int blocks = (L.ntiles + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * kWaves), 0, s, L, 0u);
  return hipGetLastError();
}

hipError_t launch_sweep(int kclass, const SweepLaunch& L, size_t lds_bytes, hipStream_t s) {
  if (L.ntiles <= 0) return hipSuccess;
  if (kclass < 0 || kclass >= kNumSweepClasses) return hipErrorInvalidValue;
  const int mi = kclass % kNumRhsClasses;
  const int ri = (kclass / kNumRhsClasses) % kNumRowClasses;
  const int prec = kclass / (kNumRhsClasses * kNumRowClasses);
  const KernelFn fn = prec == LTI_PREC_FP64 ? pick<LTI_PREC_FP64>(ri, mi) : pick<LTI_PREC_REFINED>(ri, mi);
  const int blocks = (L.ntiles + kWaves - 1) / kWaves;
  if (lds_bytes > kStageLimit) lds_bytes = 0;
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * kWaves), lds_bytes, s, L, (uint32_t)lds_bytes);
  return hipGetLastError();
}

}  // namespace lti
